"""Pins of the oracle's MPE MAC (Sec. 2.2.1, Eqs. (2)-(4), p = 1): the node
moments B_2 and B_3 of Eq. (3) against closed forms, the parallel-axis
identity and brute force; the MAC's bound against the actual error of the
monopole; and the invariant that a vanishing limit opens every node."""
import numpy as np
import pytest

import oracle
import workloads
from test_oracle_tree import _node_cells


def _uniform_grid(n=16, rho=2.0):
    level, coord = workloads.uniform_blocks(n)
    r = np.full((level.shape[0], 8, 8, 8), rho)
    return workloads.Grid((1, 1, 1), 1.0, (0.0, 0.0, 0.0), level, coord, r, (0, 0, 0))


def _cells(g):
    x = workloads.cell_centres(g.root_size, g.origin, g.level, g.coord).reshape(-1, 3)
    h = g.root_size / 2.0 ** (g.level.astype(np.float64) + 2.0)
    m = g.rho.reshape(g.nb, 512) * (h ** 3)[:, None]
    return x, m.ravel()


def test_moments_closed_form_uniform():
    """Uniform density: a node of n^3 cells of size h has B_2 = M h^2 (n^2 - 1) / 4
    (three axes of variance h^2 (n^2 - 1) / 12); the 8 cells of a +2 node all
    lie sqrt(3) h / 2 from the centre, so B_3 = M (sqrt(3) h / 2)^3."""
    g = _uniform_grid()
    t = oracle.Tree(g, mac="mpe", a_lim=1e-3)
    B2, B3 = t.mpe_moments()
    ex = t.export()
    na, nb = t.na, g.nb
    h = 1.0 / 16
    m = 2.0 * h ** 3
    p2 = slice(na + 8 * nb, na + 72 * nb)
    np.testing.assert_allclose(B2[p2], 8 * m * h * h * 3 / 4, rtol=1e-13)
    np.testing.assert_allclose(B3[p2], 8 * m * (np.sqrt(3) * h / 2) ** 3, rtol=1e-13)
    p1 = slice(na, na + 8 * nb)
    np.testing.assert_allclose(B2[p1], 64 * m * h * h * 15 / 4, rtol=1e-13)
    leaf = np.nonzero(ex["aleaf"] >= 0)[0]
    np.testing.assert_allclose(B2[leaf], 512 * m * h * h * 63 / 4, rtol=1e-13)
    root = np.nonzero(ex["alev"] == 1)[0]
    np.testing.assert_allclose(B2[root], 4096 * m * h * h * 255 / 4, rtol=1e-12)


def test_moments_parallel_axis_and_brute_force():
    """Non-uniform AMR grid: B_2 of every internal node equals the sum over its
    children of B_2 + M |r_child - r_a|^2 (exact identity, cells having B = 0);
    B_2 and B_3 of sampled nodes equal a brute-force sum over their cells."""
    g = workloads.small_amr()
    t = oracle.Tree(g, mac="mpe", a_lim=1e-3)
    B2, B3 = t.mpe_moments()
    ex = t.export()
    na, nb = t.na, g.nb
    ncell0 = na + 72 * nb
    Bfull = np.concatenate([B2, np.zeros(512 * nb)])
    M, com = ex["M"], ex["com"]

    def children(i):
        if i < na:
            if ex["aleaf"][i] >= 0:
                return na + 8 * ex["aleaf"][i] + np.arange(8)
            return ex["achild"][i]
        if i < na + 8 * nb:
            lb, o1 = divmod(i - na, 8)
            return na + 8 * nb + 64 * lb + 8 * o1 + np.arange(8)
        lb, q = divmod(i - na - 8 * nb, 64)
        o1, o2 = divmod(q, 8)
        cells = [sum((4 * ((o1 >> k) & 1) + 2 * ((o2 >> k) & 1) + ((o3 >> k) & 1)) * 8 ** k for k in range(3))
                 for o3 in range(8)]
        return ncell0 + 512 * lb + np.array(cells)

    for i in range(ncell0):
        ch = children(i)
        ref = (Bfull[ch] + M[ch] * ((com[ch] - com[i]) ** 2).sum(1)).sum()
        assert abs(B2[i] - ref) <= 1e-12 * max(B2[i], 1e-300), i
    x, m = _cells(g)
    rng = np.random.default_rng(3)
    for i in np.concatenate([np.arange(na), rng.choice(np.arange(na, ncell0), 40, replace=False)]):
        c = _node_cells(t, g, ex, i)
        r = np.sqrt(((x[c] - com[i]) ** 2).sum(1))
        np.testing.assert_allclose(B2[i], (m[c] * r ** 2).sum(), rtol=1e-12)
        np.testing.assert_allclose(B3[i], (m[c] * r ** 3).sum(), rtol=1e-12)


def _mpe_bound(G, d, bmax, B2, B3):
    return G / d ** 2 / (1 - bmax / d) ** 2 * (3 * B2 / d ** 2 - 2 * B3 / d ** 3)


def test_mpe_bound_covers_the_monopole_error():
    """Eq. (2) with p = 1 bounds the acceleration error of a node's monopole
    (about its COM) at any point farther than b_max: checked for every
    internal node of a lognormal-noise AMR grid at random points."""
    g = workloads.small_amr(seed=11)
    t = oracle.Tree(g, mac="mpe", a_lim=1e-3)
    B2, B3 = t.mpe_moments()
    ex = t.export()
    na, nb = t.na, g.nb
    x, m = _cells(g)
    size = np.concatenate([1.0 / 2.0 ** (ex["alev"] - 1), np.repeat(0.5 / 2.0 ** (g.level - 1), 8),
                           np.repeat(0.25 / 2.0 ** (g.level - 1), 64)])
    rng = np.random.default_rng(9)
    worst = 0.0
    for i in range(na + 72 * nb):
        if i >= na and rng.random() > 0.1:
            continue
        c = _node_cells(t, g, ex, i)
        ra, h = ex["com"][i], size[i]
        # geometric centre: the cube holding the node's cells
        gc = (x[c].min(0) + x[c].max(0)) / 2
        bmax = np.sqrt(((np.abs(ra - gc) + h / 2) ** 2).sum())
        for _ in range(6):
            u = rng.normal(size=3)
            u /= np.linalg.norm(u)
            d = bmax * np.exp(rng.uniform(np.log(1.05), np.log(20.0)))
            p = ra + d * u
            v = x[c] - p
            r = np.sqrt((v ** 2).sum(1))
            exact = (m[c, None] * v / r[:, None] ** 3).sum(0)
            w = ra - p
            mono = m[c].sum() * w / d ** 3
            err = np.linalg.norm(exact - mono)
            bound = _mpe_bound(1.0, d, bmax, B2[i], B3[i])
            assert err <= bound * (1 + 1e-9) + 1e-300, (i, d / bmax, err, bound)
            worst = max(worst, err / bound)
    assert worst > 1e-3  # the bound is not vacuous


def test_mpe_lists_respect_the_mac_and_vanishing_limit_opens_all():
    """Each accepted internal node passes Eq. (2) at the block's closest point
    (recomputed with numpy from the moments); with a_lim -> 0 every node is
    opened and the walk equals the direct sum."""
    g = workloads.small_amr()
    a_lim = 2e-3
    t = oracle.Tree(g, mac="mpe", a_lim=a_lim)
    B2, B3 = t.mpe_moments()
    ex = t.export()
    na, nb = t.na, g.nb
    size = np.concatenate([1.0 / 2.0 ** (ex["alev"] - 1), np.repeat(0.5 / 2.0 ** (g.level - 1), 8),
                           np.repeat(0.25 / 2.0 ** (g.level - 1), 64)])
    x, _ = _cells(g)
    for lb in np.random.default_rng(5).choice(nb, 6, replace=False):
        ids = t.block_list(lb)
        cov = np.zeros(512 * nb, np.int64)
        for nid in ids:
            np.add.at(cov, _node_cells(t, g, ex, nid), 1)
        assert (cov == 1).all()
        s = 1.0 / 2.0 ** (g.level[lb] - 1)
        cT = (g.coord[lb] + 0.5) * s
        ext = 3.5 * s / 8
        for i in ids[ids < na + 72 * nb]:
            c = _node_cells(t, g, ex, i)
            gc = (x[c].min(0) + x[c].max(0)) / 2
            ra, h = ex["com"][i], size[i]
            bmax = np.sqrt(((np.abs(ra - gc) + h / 2) ** 2).sum())
            d = np.sqrt((np.maximum(np.abs(cT - ra) - ext, 0.0) ** 2).sum())
            assert d > bmax
            assert _mpe_bound(1.0, d, bmax, B2[i], B3[i]) < a_lim * (1 + 1e-12)
    sel = [0, 5]
    phi, acc, nint = oracle.Tree(g, mac="mpe", a_lim=1e-300).walk_group(sel)
    cells = np.concatenate([512 * b + np.arange(512) for b in sel])
    pd, ad = oracle.Tree(g).direct(cells)
    assert (nint == 512 * nb).all()
    np.testing.assert_allclose(phi, pd, rtol=1e-13)
    assert np.abs(acc - ad).max() <= 1e-13 * np.abs(ad).max()
