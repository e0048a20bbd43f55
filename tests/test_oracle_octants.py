"""Pins of the oracle's group walk with one interaction list per 4^3 octant
of a leaf block (list_group 4) in place of one per block (Sec. 2.1's group
walk, with a smaller target group).

* Every accept/open decision of an octant's list is re-derived in numpy from
  the node geometry with the octant's own box: the centres of its 4^3 cells,
  the octant's centre offset by 2 h from the block's per axis (upper half
  where bit a of the octant is set) and half-extent 1.5 h; for BH, APE with
  theta_pix and MPE, isolated and 2P1I.  The list partitions the domain's
  cells, and it coarsens the block's list: every node of the block's list is
  in it or below one of its nodes.
* The walk at each cell sums that cell's octant list: Phi and a recomputed in
  numpy from the node moments with the octant taken from the cell's (i, j, k)
  (isolated, so the pair kernel is Newtonian), to 1e-12.
* The surrogate walk picks the list of the octant that holds each cell group:
  the constant-network closed form of the surrogate pins, with the octant
  lists, to 1e-12 (2^3 and 4^3 groups).
* The adaptive update over octant lists: tolerance 0 is the octant-list walk
  bit for bit, an unchanged density keeps every block, and a local bump's
  decisions follow the corner criterion read from independent full walks.
* Planted mistakes (octant bits transposed, the octant centre mirrored, the
  block's extent kept) are each caught.
"""
import os
import shutil

import numpy as np
import pytest

import oracle
import workloads
from test_oracle_mac import decide, node_geometry, visited
from test_oracle_abu import _perturbed
from test_oracle_mlpwalk import EW_N, closed_form, const_surrogate, lognormal16
from test_oracle_tree import _node_cells

CASES = {
    "bh0.6": (dict(theta=0.6), {}),
    "ape+pix": (dict(mac="ape", a_lim=3e-2, theta_pix=0.5), {}),
    "mpe": (dict(mac="mpe", a_lim=3e-3), {}),
    "bh1.0 2p1i": (dict(theta=1.0), dict(bc=(1, 1, 0), nroot=(1, 1, 2))),
}


def octant_box(g, lb, so):
    """Centre and half-extent of octant so of leaf block lb."""
    s = g.root_size / 2.0 ** (g.level[lb] - 1)
    h = s / 8.0
    bits = np.array([(so >> a) & 1 for a in range(3)])
    cT = np.asarray(g.origin) + (g.coord[lb] + 0.5) * s + np.where(bits == 1, 2.0, -2.0) * h
    return cT, 1.5 * h


def ancestors(parent, i):
    out = []
    while i >= 0:
        out.append(i)
        i = parent[i]
    return out


def check_octants(g, kw, blocks):
    t = oracle.Tree(g, list_group=4, **kw)
    ex, h, gc, parent = node_geometry(t, g)
    B = t.mpe_moments() if kw.get("mac") == "mpe" else None
    L = np.asarray(g.nroot, np.float64) * g.root_size
    per = np.asarray(g.bc, bool)
    ncell0 = t.na + 72 * g.nb
    roots = np.nonzero(ex["alev"] == 1)[0]
    n = 0
    for lb in blocks:
        blk = t.block_list(lb)
        for so in range(8):
            ids = t.octant_list(lb, so)
            cT, ext = octant_box(g, lb, so)
            acc, opened = visited(ids, parent)
            inner = acc[acc < ncell0]
            assert decide(kw, ex, h, gc, B, inner, cT, ext, L, per).all(), (lb, so, "accepted node fails")
            assert not decide(kw, ex, h, gc, B, opened, cT, ext, L, per).any(), (lb, so, "opened node passes")
            assert np.isin(roots, np.concatenate([acc, opened])).all()
            cov = np.zeros(512 * g.nb, np.int64)
            for a in acc:
                np.add.at(cov, _node_cells(t, g, ex, a), 1)
            assert (cov == 1).all()
            # a coarsening of the block's list
            sid = set(ids.tolist())
            assert all(any(a in sid for a in ancestors(parent, b)) for b in blk)
            assert ids.size <= blk.size
            n += inner.size + opened.size
    return n


@pytest.mark.parametrize("case", sorted(CASES))
def test_octant_decisions_rederived(case):
    kw, gkw = CASES[case]
    g = workloads.small_amr(**gkw)
    blocks = np.random.default_rng(5).choice(g.nb, 4, replace=False)
    assert check_octants(g, kw, blocks) > 500


def direct_over_lists(t, g, lb):
    """Phi [512], a [3, 512] of block lb's cells, each from its octant's
    list (isolated: Newtonian pairs)."""
    ex = t.export()
    s = g.root_size / 2.0 ** (g.level[lb] - 1)
    h = s / 8.0
    ci = np.arange(512)
    ijk = np.stack([ci % 8, (ci // 8) % 8, ci // 64], 1)
    x = np.asarray(g.origin) + (8 * g.coord[lb] + ijk + 0.5) * h
    octs = (ijk // 4) @ np.array([1, 2, 4])
    lists = [t.octant_list(lb, so) for so in range(8)]
    phi, acc = np.zeros(512), np.zeros((3, 512))
    for c in range(512):
        ids = lists[octs[c]]
        d = x[c] - ex["com"][ids]
        r2 = (d * d).sum(1)
        k = r2 > 0
        inv = 1.0 / np.sqrt(r2[k])
        M = ex["M"][ids][k]
        phi[c] = -(M * inv).sum()
        acc[:, c] = -(M[:, None] * d[k] * (inv ** 3)[:, None]).sum(0)
    return phi, acc, sum(len(l) for l in lists)


def test_walk_sums_each_cells_octant_list():
    g = workloads.small_amr()
    t = oracle.Tree(g, mac="ape", a_lim=3e-3, list_group=4)
    blocks = np.array([0, 7, g.nb - 1])
    phi, acc, nint = t.walk_group(blocks)
    for q, lb in enumerate(blocks):
        pr, ar, nl = direct_over_lists(t, g, lb)
        sl = slice(512 * q, 512 * (q + 1))
        np.testing.assert_allclose(phi[sl], pr, rtol=1e-12)
        assert np.abs(acc[:, sl] - ar).max() <= 1e-12 * np.abs(ar).max()
        assert nint[q] == nl
    # the octant lists are shorter in total per cell than the block's list
    tb = oracle.Tree(g, mac="ape", a_lim=3e-3)
    _, _, nb = tb.walk_group(blocks)
    assert (nint < 8 * nb).all()


@pytest.mark.parametrize("reach", [1.0, 3.0])
def test_surrogate_walk_with_octant_lists(reach):
    g = lognormal16((1, 1, 1), (1, 1, 1))
    t = oracle.Tree(g, theta=0.5, ewald="table", ew_n=EW_N, mlp_reach=reach, list_group=4)
    params, norm = const_surrogate(np.array([0.5, 0.5, 0.5]))
    blocks = [0, 5, g.nb - 1]
    phi, acc, nint = t.walk_group_mlp(params, norm, blocks)
    for q, lb in enumerate(blocks):
        lists = [t.octant_list(lb, so) for so in range(8)]
        pr, ar, gl = closed_form(t, g, lb, False, reach, lists=lists)
        assert gl == (1 if reach == 1.0 else 2)
        sl = slice(512 * q, 512 * (q + 1))
        np.testing.assert_allclose(phi[sl], pr, rtol=1e-12)
        assert np.abs(acc[:, sl] - ar).max() <= 1e-12 * np.abs(ar).max()
        assert nint[q] == sum(len(l) for l in lists)


def test_list_group_is_validated():
    g = workloads.small_amr()
    for bad in (2, 16, -1):
        with pytest.raises(ValueError):
            oracle.Tree(g, list_group=bad)
    t = oracle.Tree(g, list_group=4)
    with pytest.raises(ValueError):
        t.octant_list(0, 8)


# ------------------------------------------------------------------ mutants
OCT_MUTANTS = {
    "octant bits transposed": (
        "oracle_internal.h",
        "return ((ci & 7) >> 2) | ((((ci >> 3) & 7) >> 2) << 1) | ((ci >> 8) << 2);",
        "return ((ci & 7) >> 2) << 1 | ((((ci >> 3) & 7) >> 2)) | ((ci >> 8) << 2);"),
    "octant centre mirrored": (
        "octoracle.c",
        "for (int k = 0; k < 3; ++k) cT[k] += (((so >> k) & 1) ? 2.0 : -2.0) * h;",
        "for (int k = 0; k < 3; ++k) cT[k] += (((so >> k) & 1) ? -2.0 : 2.0) * h;"),
    "block extent kept": ("octoracle.c", "  *ext = 1.5 * h;\n", "\n"),
}


@pytest.fixture(scope="module")
def oct_mutants(tmp_path_factory):
    libs = {}
    for name, (fn, old, new) in OCT_MUTANTS.items():
        src = open(os.path.join(oracle.HERE, fn)).read()
        assert src.count(old) == 1, name
        d = tmp_path_factory.mktemp("octmutant")
        for f in os.listdir(oracle.HERE):
            if f.endswith((".c", ".h")):
                shutil.copy(os.path.join(oracle.HERE, f), d)
        (d / fn).write_text(src.replace(old, new))
        libs[name] = oracle.build(src_dir=str(d), out=str(d / "liboracle_oct.so"))
    return libs


@pytest.mark.parametrize("name", sorted(OCT_MUTANTS))
def test_octant_pins_catch_planted_mistakes(oct_mutants, name):
    caught = 0
    with oracle.using_library(oct_mutants[name]):
        for check in (lambda: check_octants(workloads.small_amr(), CASES["bh0.6"][0], [0, 9]),
                      test_walk_sums_each_cells_octant_list,
                      lambda: test_surrogate_walk_with_octant_lists(3.0)):
            try:
                check()
            except AssertionError:
                caught += 1
    assert caught, f"no pin catches the mutant '{name}'"


def test_adaptive_update_with_octant_lists():
    """The adaptive update walks each cell over its octant's list too:
    tolerance 0 is the octant-list group walk bit for bit, an unchanged
    density keeps every block, and on a perturbed density the decisions
    follow the corner criterion read from independent full walks."""
    g = workloads.small_amr()
    t = oracle.Tree(g, theta=0.5, list_group=4)
    p0, a0, _ = t.walk_group()
    p, a, upd = t.walk_abu(np.zeros_like(p0), np.zeros_like(a0), 0.0)
    assert upd.all() and np.array_equal(p, p0) and np.array_equal(a, a0)
    p, a, upd = t.walk_abu(p0, a0, 1e-12)
    assert not upd.any() and np.array_equal(p, p0) and np.array_equal(a, a0)
    # a local bump in the density
    g1 = _perturbed(g)
    t1 = oracle.Tree(g1, theta=0.5, list_group=4)
    p1, a1, _ = t1.walk_group()
    tol = 1e-3 * np.sqrt((a1 ** 2).sum(0)).max()
    p, a, upd = t1.walk_abu(p0, a0, tol)
    corners = [7 * (k & 1) + 56 * ((k >> 1) & 1) + 448 * (k >> 2) for k in range(8)]
    da = np.sqrt(((a1 - a0) ** 2).sum(0)).reshape(g.nb, 512)[:, corners].max(1)
    assert np.array_equal(upd.astype(bool), ~(da < tol))
    assert 0 < upd.sum() < g.nb
    pb = p.reshape(g.nb, 512)
    assert np.array_equal(pb[upd == 1], p1.reshape(g.nb, 512)[upd == 1])
    assert np.array_equal(pb[upd == 0], p0.reshape(g.nb, 512)[upd == 0])
