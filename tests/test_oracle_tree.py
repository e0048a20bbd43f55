"""Pins of the FP64 oracle's grid, tree build, MACs, walks and direct sums.

Each check ties the oracle to something other than itself: closed forms
(uniform-sphere potential), symmetries, conservation laws, the invariant that a
MAC which opens every node reproduces direct summation, and a geometric
re-derivation of every accept/open decision.
"""
import numpy as np
import pytest

import oracle
import workloads


@pytest.fixture(scope="module")
def sphere():
    g = workloads.c1_sphere(noise=False, rho_bg=0.0)
    t = oracle.Tree(g, theta=0.5)
    pd, ad = t.direct()
    return g, t, pd, ad


def test_morton_bits():
    # x -> bit 0, y -> bit 1, z -> bit 2 of every triple; octant order 0..7
    for o in range(8):
        assert oracle.morton(o & 1, (o >> 1) & 1, (o >> 2) & 1) == o
    rng = np.random.default_rng(0)
    for _ in range(200):
        x, y, z = (int(v) for v in rng.integers(0, 2 ** 21, 3))
        k = oracle.morton(x, y, z)
        back = [0, 0, 0]
        for b in range(21):
            for ax in range(3):
                back[ax] |= ((k >> (3 * b + ax)) & 1) << b
        assert back == [x, y, z]


def test_grid_validation():
    g = workloads.c1_sphere(noise=False)
    lv, cd, rho = g.level, g.coord, g.rho

    def bad(level, coord, r, code):
        gg = workloads.Grid((1, 1, 1), 1.0, (0, 0, 0), level, coord, r)
        with pytest.raises(ValueError, match=code):
            oracle.Tree(gg)

    bad(lv[1:], cd[1:], rho[1:], "hole")
    bad(np.concatenate([lv, lv[:1]]), np.concatenate([cd, cd[:1]]),
        np.concatenate([rho, rho[:1]]), "duplicate")
    # a level-2 block over level-3 blocks
    bad(np.concatenate([lv, [2]]).astype(np.int32), np.concatenate([cd, [[0, 0, 0]]]).astype(np.int32),
        np.concatenate([rho, rho[:1]]), "overlap")
    lv2 = lv.copy()
    lv2[0] = 0
    bad(lv2, cd, rho, "level")
    cd2 = cd.copy()
    cd2[0, 0] = 4
    bad(lv, cd2, rho, "level")
    r2 = rho.copy()
    r2[3, 1, 2, 3] = -1.0
    bad(lv, cd, r2, "density")
    r2[3, 1, 2, 3] = np.nan
    bad(lv, cd, r2, "density")


def test_amr_topology_and_moments():
    g = workloads.small_amr()
    t = oracle.Tree(g)
    ex = t.export()
    na, nb = t.na, g.nb
    # amr nodes sorted by (level, key), keys unique per level
    lev, key = ex["alev"], ex["akey"]
    order = np.lexsort((key, lev))
    assert np.array_equal(order, np.arange(na))
    # every leaf block appears exactly once
    leaves = ex["aleaf"][ex["aleaf"] >= 0]
    assert np.array_equal(np.sort(leaves), np.arange(nb))
    # masses: each tree level partitions the total mass; cells = rho h^3
    h = 1.0 / 2.0 ** (g.level + 2)
    m = g.rho.reshape(nb, -1) * (h ** 3)[:, None]
    base = na + 72 * nb
    assert np.array_equal(ex["M"][base:].reshape(nb, 512), m)
    mtot = m.sum()
    roots = np.nonzero(lev == 1)[0]
    assert abs(ex["M"][roots].sum() - mtot) <= 1e-14 * mtot
    p1 = ex["M"][na:na + 8 * nb].reshape(nb, 8)
    p2 = ex["M"][na + 8 * nb:base].reshape(nb, 64)
    leafM = np.empty(nb)
    leafM[ex["aleaf"][ex["aleaf"] >= 0]] = ex["M"][np.nonzero(ex["aleaf"] >= 0)[0]]
    np.testing.assert_allclose(p1.sum(1), m.sum(1), rtol=1e-14)
    np.testing.assert_allclose(p2.sum(1), m.sum(1), rtol=1e-14)
    np.testing.assert_allclose(leafM, m.sum(1), rtol=1e-14)
    # cell COM is the cell centre; root COM is the global centre of mass
    xc = workloads.cell_centres(1.0, (0, 0, 0), g.level, g.coord).reshape(-1, 3)
    np.testing.assert_allclose(ex["com"][base:], xc, rtol=0, atol=1e-15)
    gcom = (m.reshape(-1)[:, None] * xc).sum(0) / mtot
    np.testing.assert_allclose(ex["com"][roots[0]], gcom, rtol=1e-13)
    # each internal amr node: mass = sum of children, children one level finer
    for i in range(na):
        if ex["aleaf"][i] < 0:
            ch = ex["achild"][i]
            assert (lev[ch] == lev[i] + 1).all()
            for o in range(8):
                assert tuple(ex["acoord"][ch[o]]) == tuple(2 * ex["acoord"][i] + [(o >> k) & 1 for k in range(3)])
            np.testing.assert_allclose(ex["M"][ch].sum(), ex["M"][i], rtol=1e-14)


def _node_cells(t, g, ex, nid):
    """Global cell indices covered by node nid (geometric re-derivation)."""
    na, nb = t.na, g.nb
    if nid >= na + 72 * nb:
        return np.array([nid - na - 72 * nb])
    if nid >= na + 8 * nb:
        r = nid - na - 8 * nb
        lb, q = divmod(r, 64)
        o1, o2 = divmod(q, 8)
        lo = [4 * ((o1 >> k) & 1) + 2 * ((o2 >> k) & 1) for k in range(3)]
        sz = 2
    elif nid >= na:
        lb, o1 = divmod(nid - na, 8)
        lo = [4 * ((o1 >> k) & 1) for k in range(3)]
        sz = 4
    else:
        out = []
        stack = [nid]
        while stack:
            a = stack.pop()
            if ex["aleaf"][a] >= 0:
                out.append(512 * ex["aleaf"][a] + np.arange(512))
            else:
                stack.extend(ex["achild"][a])
        return np.concatenate(out)
    i = np.arange(sz)
    kk, jj, ii = np.meshgrid(i + lo[2], i + lo[1], i + lo[0], indexing="ij")
    return 512 * lb + (ii + 8 * jj + 64 * kk).ravel()


@pytest.mark.parametrize("mac", ["bh", "ape"])
def test_lists_partition_domain_and_respect_mac(mac):
    """Every block's list covers each cell exactly once, and each accepted
    internal node passes the safe box + MAC at the block's closest point while
    each opened ancestor fails it (geometry recomputed here with numpy)."""
    g = workloads.small_amr()
    kw = dict(theta=0.5) if mac == "bh" else dict(mac="ape", a_lim=3e-3)
    t = oracle.Tree(g, **kw)
    ex = t.export()
    na, nb = t.na, g.nb
    size = np.concatenate([1.0 / 2.0 ** (ex["alev"] - 1), np.repeat(0.5 / 2.0 ** (g.level - 1), 8),
                           np.repeat(0.25 / 2.0 ** (g.level - 1), 64)])
    rng = np.random.default_rng(5)
    for lb in rng.choice(nb, 6, replace=False):
        ids = t.block_list(lb)
        cov = np.zeros(512 * nb, np.int64)
        for nid in ids:
            np.add.at(cov, _node_cells(t, g, ex, nid), 1)
        assert (cov == 1).all()
        s = 1.0 / 2.0 ** (g.level[lb] - 1)
        cT = (g.coord[lb] + 0.5) * s
        ext = 3.5 * s / 8
        internal = ids[ids < na + 72 * nb]
        h = size[internal]
        com = ex["com"][internal]
        d = np.maximum(np.abs(cT - com) - ext, 0.0)
        d2 = (d ** 2).sum(1)
        if mac == "bh":
            assert (h * h < 0.25 * d2).all()
        else:
            assert (ex["M"][internal] * h * h < 3e-3 * d2 * d2).all()


def test_open_everything_equals_direct(sphere):
    g, _, pd, ad = sphere
    t = oracle.Tree(g, theta=1e-6)
    sel = [0, 21, 42, 63]
    phi, acc, nint = t.walk_group(sel)
    cells = np.concatenate([512 * b + np.arange(512) for b in sel])
    assert (nint == 512 * g.nb).all()
    np.testing.assert_allclose(phi, pd[cells], rtol=1e-13)
    amax = np.abs(ad).max()
    assert np.abs(acc - ad[:, cells]).max() <= 1e-13 * amax
    # same for the per-cell walk and the APE MAC with a vanishing limit
    p2, a2, _ = oracle.Tree(g, theta=1e-6).walk_percell(cells[::97])
    np.testing.assert_allclose(p2, pd[cells[::97]], rtol=1e-13)
    p3, a3, _ = oracle.Tree(g, mac="ape", a_lim=1e-300).walk_group([7])
    np.testing.assert_allclose(p3, pd[512 * 7:512 * 8], rtol=1e-13)


def test_sphere_potential_closed_form(sphere):
    """Voxel sphere of rho = 1, R = 0.3: outside Phi = -G M / r (cubic
    symmetry leaves no dipole or quadrupole); inside -G M (3R^2 - r^2)/(2R^3)
    up to voxel error."""
    g, _, pd, _ = sphere
    xc = workloads.cell_centres(1.0, (0, 0, 0), g.level, g.coord).reshape(-1, 3)
    r = np.sqrt(((xc - 0.5) ** 2).sum(1))
    M = (g.rho.reshape(-1) * (1 / 32) ** 3).sum()
    out = r > 0.45
    np.testing.assert_allclose(pd[out], -M / r[out], rtol=1e-3)
    ins = r < 0.2
    R = 0.3
    Mc = 4 / 3 * np.pi * R ** 3
    np.testing.assert_allclose(pd[ins], -Mc * (3 * R * R - r[ins] ** 2) / (2 * R ** 3), rtol=2e-2)


def test_direct_sum_symmetry_and_newton3(sphere):
    g, _, pd, ad = sphere
    nb = g.nb
    m = g.rho.reshape(-1) * (1 / 32) ** 3
    f = m[None] * ad
    assert np.abs(f.sum(1)).max() <= 1e-13 * np.abs(f).sum()
    # mirror symmetry x -> 1 - x of the centred sphere: a_x odd, a_y even
    xc = workloads.cell_centres(1.0, (0, 0, 0), g.level, g.coord).reshape(-1, 3)
    key = {tuple(np.round(x * 64).astype(int)): i for i, x in enumerate(xc)}
    mir = np.array([key[(64 - int(round(x[0] * 64)), int(round(x[1] * 64)), int(round(x[2] * 64)))] for x in xc])
    amax = np.abs(ad).max()
    assert np.abs(ad[0] + ad[0][mir]).max() <= 1e-13 * amax
    assert np.abs(ad[1] - ad[1][mir]).max() <= 1e-13 * amax
    np.testing.assert_allclose(pd, pd[mir], rtol=1e-13)
    # acceleration points inwards everywhere outside the sphere
    r = xc - 0.5
    assert ((ad * r.T).sum(0)[np.linalg.norm(r, axis=1) > 0.35] < 0).all()


def test_tree_error_vs_direct(sphere):
    """BH monopole error on the uniform sphere: e_a,max (Eq. e_a, normalised
    by the maximum reference acceleration).  The maximum sits at the sphere
    centre where opposing contributions cancel."""
    g, t, pd, ad = sphere
    phi, acc, nint = t.walk_group()
    amax = np.sqrt((ad ** 2).sum(0)).max()
    ea = np.sqrt(((acc - ad) ** 2).sum(0)) / amax
    assert ea.max() < 3.5e-3
    assert np.quantile(ea, 0.99) < 2e-3
    assert np.abs(phi / pd - 1).max() < 1e-3
    t3 = oracle.Tree(g, theta=0.3)
    _, a3, n3 = t3.walk_group()
    assert (np.sqrt(((a3 - ad) ** 2).sum(0)) / amax).max() < 1e-3
    assert n3.mean() > nint.mean()
    # the paper-literal per-cell walk interacts with fewer nodes per cell
    tg = np.arange(0, 512 * g.nb, 61)
    _, _, npc = t.walk_percell(tg)
    assert npc.mean() < nint.mean()


def test_block_order_independence():
    g = workloads.small_amr()
    gs = workloads.shuffled(g)
    p1, a1, _ = oracle.Tree(g, theta=0.5).walk_group()
    p2, a2, _ = oracle.Tree(gs, theta=0.5).walk_group()
    perm = gs.meta["perm"]
    idx = (512 * perm[:, None] + np.arange(512)).ravel()
    np.testing.assert_allclose(p2, p1[idx], rtol=1e-14)
    np.testing.assert_allclose(a2, a1[:, idx], rtol=1e-12, atol=1e-15 * np.abs(a1).max())
