"""Pins of the oracle's MAC suite (Sec. 2.1 safe box and Eq. 1; Eqs. 2-4 and 6
for MPE and APE; Sec. 2.3 for the extra opening angle with columns).

Every decision of the group walk is re-derived here in numpy from the node
geometry alone: the walk visits a root, accepts it or opens it, and visits
the children of every opened node.  So the nodes a block's list implies are
its entries (accepted, or cells, which are always accepted) and their proper
ancestors (opened).  For each visited non-cell node the re-derivation must
give the oracle's decision:

* accepted  <=>  safe box AND gravity MAC AND (with columns) BH at theta_pix;
* safe box: on some axis |delta_k| - ext > eta_SB h / 2, delta from the
  node's geometric centre to the block's centre (minimum image);
* MAC distance d: from the node's centre of mass to the closest point of the
  block's cell-centre box (half-extent ext = 3.5 cell sizes).

The re-derivation is checked to bite: copies of the oracle's sources with a
planted mistake (a safe box about the centre of mass, eta_SB not halved, the
column angle OR'ed instead of AND'ed, a MAC distance to the block centre)
are built and each makes the check fail.
"""
import os
import shutil

import numpy as np
import pytest

import oracle
import workloads


def node_geometry(t, g):
    """Edge h, geometric centre [nn, 3] and parent id of every node, from the
    grid's integer layout (independent of the oracle's own geometry)."""
    ex = t.export()
    na, nb = t.na, g.nb
    rs, org = float(g.root_size), np.asarray(g.origin, np.float64)
    lev, bc = np.asarray(g.level), np.asarray(g.coord, np.int64)
    bs = rs / 2.0 ** (lev - 1)
    nn = na + 72 * nb + 512 * nb
    h = np.empty(nn)
    gc = np.empty((nn, 3))
    parent = np.full(nn, -1, np.int64)
    h[:na] = rs / 2.0 ** (ex["alev"] - 1)
    gc[:na] = org + (ex["acoord"] + 0.5) * h[:na, None]
    for i in range(na):
        if ex["aleaf"][i] < 0:
            parent[ex["achild"][i]] = i
    leaf_node = np.empty(nb, np.int64)
    leaf_node[ex["aleaf"][ex["aleaf"] >= 0]] = np.nonzero(ex["aleaf"] >= 0)[0]
    bits = np.array([[(o >> k) & 1 for k in range(3)] for o in range(8)])
    # +1 nodes
    o1 = np.tile(np.arange(8), nb)
    lb1 = np.repeat(np.arange(nb), 8)
    ids = na + np.arange(8 * nb)
    h[ids] = bs[lb1] / 2
    gc[ids] = org + (2 * bc[lb1] + bits[o1] + 0.5) * h[ids, None]
    parent[ids] = leaf_node[lb1]
    # +2 nodes
    q = np.tile(np.arange(64), nb)
    lb2 = np.repeat(np.arange(nb), 64)
    ids = na + 8 * nb + np.arange(64 * nb)
    h[ids] = bs[lb2] / 4
    gc[ids] = org + (4 * bc[lb2] + 2 * bits[q // 8] + bits[q % 8] + 0.5) * h[ids, None]
    parent[ids] = na + 8 * lb2 + q // 8
    # cells
    ci = np.tile(np.arange(512), nb)
    lbc = np.repeat(np.arange(nb), 512)
    ijk = np.stack([ci % 8, (ci // 8) % 8, ci // 64], 1)
    ids = na + 72 * nb + np.arange(512 * nb)
    h[ids] = bs[lbc] / 8
    gc[ids] = org + (8 * bc[lbc] + ijk + 0.5) * h[ids, None]
    oct1 = ((ijk >> 2) & 1) @ np.array([1, 2, 4])
    oct2 = ((ijk >> 1) & 1) @ np.array([1, 2, 4])
    parent[ids] = na + 8 * nb + 64 * lbc + 8 * oct1 + oct2
    return ex, h, gc, parent


def wrap(d, L, per):
    return np.where(per, d - L * np.floor(d / L + 0.5), d)


def visited(ids, parent):
    """Accepted entries and opened ancestors of one block's list."""
    acc = np.asarray(ids, np.int64)
    opened = set()
    for a in acc:
        p = parent[a]
        while p >= 0 and p not in opened:
            opened.add(p)
            p = parent[p]
    return acc, np.array(sorted(opened), np.int64)


def decide(kw, ex, h, gc, B, nodes, cT, ext, L, per):
    """The MAC suite's decision for each node (True = accept), in numpy."""
    hh = h[nodes]
    dg = wrap(cT - gc[nodes], L, per)
    safe = ((np.abs(dg) - ext) > 0.5 * kw.get("eta_sb", 1.2) * hh[:, None]).any(1)
    dc = wrap(cT - ex["com"][nodes], L, per)
    e = np.maximum(np.abs(dc) - ext, 0.0)
    d2 = (e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1]) + e[:, 2] * e[:, 2]
    mac = kw.get("mac", "bh")
    M = ex["M"][nodes]
    if mac == "bh":
        th = kw.get("theta", 0.5)
        ok = hh * hh < th * th * d2
    elif mac == "ape":
        ok = M * hh * hh < kw["a_lim"] * d2 * d2
    else:
        B2, B3 = B[0][nodes], B[1][nodes]
        b = np.abs(ex["com"][nodes] - gc[nodes]) + 0.5 * hh[:, None]
        bmax = np.sqrt((b[:, 0] * b[:, 0] + b[:, 1] * b[:, 1]) + b[:, 2] * b[:, 2])
        d = np.sqrt(d2)
        qd = d - bmax
        ok = (d > bmax) & (3.0 * B2 * d - 2.0 * B3 < kw["a_lim"] * (d2 * d) * (qd * qd))
    tp = kw.get("theta_pix", 0.0)
    if kw.get("nside", 0) and tp <= 0:
        tp = 1.0 / kw["nside"]
    if tp > 0:
        ok = ok & (hh * hh < tp * tp * d2)
    return safe & ok


def check_lists(g, kw, blocks):
    """Number of decisions re-derived; raises AssertionError on a mismatch."""
    t = oracle.Tree(g, **kw)
    ex, h, gc, parent = node_geometry(t, g)
    B = t.mpe_moments() if kw.get("mac") == "mpe" else None
    L = np.asarray(g.nroot, np.float64) * g.root_size
    per = np.asarray(g.bc, bool)
    ncell0 = t.na + 72 * g.nb
    n = 0
    for lb in blocks:
        s = g.root_size / 2.0 ** (g.level[lb] - 1)
        cT = np.asarray(g.origin) + (g.coord[lb] + 0.5) * s
        ext = 3.5 * (s / 8.0)
        acc, opened = visited(t.block_list(lb), parent)
        inner = acc[acc < ncell0]
        assert decide(kw, ex, h, gc, B, inner, cT, ext, L, per).all(), (lb, "accepted node fails the suite")
        assert not decide(kw, ex, h, gc, B, opened, cT, ext, L, per).any(), (lb, "opened node passes the suite")
        # the walk starts at every root
        roots = np.nonzero(ex["alev"] == 1)[0]
        assert np.isin(roots, np.concatenate([acc, opened])).all()
        n += inner.size + opened.size
    return n


CASES = {
    "bh0.5": (dict(theta=0.5), {}),
    "bh1.0": (dict(theta=1.0), {}),
    "ape": (dict(mac="ape", a_lim=3e-3), {}),
    "ape+pix": (dict(mac="ape", a_lim=3e-2, theta_pix=0.5), {}),
    "mpe": (dict(mac="mpe", a_lim=3e-3), {}),
    "bh1.0 2p1i": (dict(theta=1.0), dict(bc=(1, 1, 0), nroot=(1, 1, 2))),
    "ape+pix 3p": (dict(mac="ape", a_lim=3e-2, theta_pix=0.5), dict(bc=(1, 1, 1))),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_every_decision_rederived(case):
    kw, gkw = CASES[case]
    g = workloads.small_amr(**gkw)
    blocks = np.random.default_rng(3).choice(g.nb, 8, replace=False)
    assert check_lists(g, kw, blocks) > 500


def test_decisions_with_columns_nside2():
    """Columns on (N_side 2): theta_pix = 1/2 joins the APE MAC."""
    g = workloads.c1_sphere()
    kw = dict(mac="ape", a_lim=1e-2, nside=2)
    assert check_lists(g, kw, [0, 9, 27, 42, 63]) > 500


# ------------------------------------------------------------------ mutants
MUTANTS = {
    "safe box about the COM": ("double d = or_wrap(t, k, cT[k] - gc[k]);",
                               "double d = or_wrap(t, k, cT[k] - t->com[3 * id + k]);"),
    "eta_SB not halved": ("double half = 0.5 * p->eta_sb * h;", "double half = p->eta_sb * h;"),
    "theta_pix OR'ed": ("ok = ok && (h * h < p->theta_pix * p->theta_pix * d2);",
                        "ok = ok || (h * h < p->theta_pix * p->theta_pix * d2);"),
    "MAC distance to the block centre": ("double e = fabs(d) - ext;", "double e = fabs(d);"),
}


@pytest.fixture(scope="module")
def mutant_libs(tmp_path_factory):
    src = open(os.path.join(oracle.HERE, "octoracle.c")).read()
    out = {}
    for name, (old, new) in MUTANTS.items():
        assert src.count(old) == 1, name
        d = tmp_path_factory.mktemp("mutant")
        for f in os.listdir(oracle.HERE):
            if f.endswith((".c", ".h")):
                shutil.copy(os.path.join(oracle.HERE, f), d)
        with open(d / "octoracle.c", "w") as fh:
            fh.write(src.replace(old, new))
        out[name] = oracle.build(src_dir=str(d), out=str(d / "liboracle.so"))
    return out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_rederivation_catches_planted_mistakes(mutant_libs, name):
    """Each planted mistake makes at least one case of the check fail."""
    caught = []
    with oracle.using_library(mutant_libs[name]):
        for case in ("bh1.0", "ape", "ape+pix", "bh1.0 2p1i"):
            kw, gkw = CASES[case]
            g = workloads.small_amr(**gkw)
            try:
                check_lists(g, kw, np.random.default_rng(3).choice(g.nb, 8, replace=False))
            except AssertionError:
                caught.append(case)
    assert caught, f"no case catches the mutant '{name}'"
