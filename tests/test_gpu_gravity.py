"""GPU parity of the gravity path against the FP64 oracle (through the C ABI).

Bars: integer work (topology, accepted node sets) and FP64 node moments are
bit-exact; the FP64 walk agrees with the oracle's group walk to 1e-12
(potential per cell, relative; acceleration relative to the largest |a|);
the FP32 walk with Kahan-compensated potential to 1e-6 (potential, per cell
relative) and 1e-5 (acceleration, max-normalised).
"""
import numpy as np
import pytest

import oracle
import paper_1708_06142_amd as ot
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def gpu(grid, fp64=True, **kw):
    phi, acc, st, s = ot.run(grid, fp64=fp64, **kw)
    return phi.cpu().numpy().astype(np.float64), acc.cpu().numpy().astype(np.float64), st, s


def oracle_kw(kw):
    k = dict(kw)
    if "ewald_n" in k:
        k["ew_n"] = k.pop("ewald_n")
        k["ewald"] = "table"
    return k


def check64(p, a, pr, ar, tol=1e-12):
    np.testing.assert_allclose(p, pr, rtol=tol, atol=0)
    amax = np.abs(ar).max()
    assert np.abs(a - ar).max() <= tol * amax, np.abs(a - ar).max() / amax


def check32(p, a, pr, ar):
    rel = np.abs(p - pr) / np.abs(pr)
    assert rel.max() <= 1e-6, rel.max()
    amax = np.sqrt((ar ** 2).sum(0)).max()
    err = np.abs(a - ar).max() / amax
    assert err <= 1e-5, err


GRIDS = {
    "sphere32": lambda: workloads.c1_sphere(),
    "amr": lambda: workloads.small_amr(),
    "amr_shuffled": lambda: workloads.shuffled(workloads.small_amr()),
    "forest_offset": lambda: _forest_offset(),
}


def _forest_offset():
    """Two root blocks, non-dyadic root size and a shifted origin."""
    g = workloads.small_amr(nroot=(2, 1, 1), seed=3)
    return workloads.Grid(g.nroot, 0.3, (0.1, -0.2, 0.05), g.level, g.coord, g.rho, g.bc, "forest")


@pytest.mark.parametrize("name", list(GRIDS))
def test_moments_bit_exact(name):
    g = GRIDS[name]()
    s = ot.Solver.for_grid(g)
    s.build(torch.from_numpy(g.rho.reshape(-1)).cuda())
    M, com = s.export_moments()
    ref = oracle.Tree(g).export()
    assert np.array_equal(M, ref["M"])
    assert np.array_equal(com, ref["com"])


@pytest.mark.parametrize("name", ["sphere32", "amr", "forest_offset"])
@pytest.mark.parametrize("mac", ["bh", "ape", "mpe"])
def test_lists_and_fp64_walk(name, mac):
    g = GRIDS[name]()
    kw = dict(theta=0.5)
    if mac != "bh":
        # a_lim chosen here (from the oracle's own BH walk), passed to both sides
        t0 = oracle.Tree(g, theta=0.5)
        _, a0, _ = t0.walk_group()
        kw = dict(mac=mac, a_lim=1e-3 * np.sqrt((a0 ** 2).sum(0)).max())
    t = oracle.Tree(g, **kw)
    pr, ar, nr = t.walk_group()
    p, a, st, s = gpu(g, fp64=True, **kw)
    for b in range(g.nb):
        mine = np.sort(s.export_list(b).astype(np.int64))
        assert np.array_equal(mine, np.sort(t.block_list(b))), b
    assert st.total_list == nr.sum()
    assert st.n_interactions == 512 * (nr.sum() - g.nb)
    check64(p, a, pr, ar)


@pytest.mark.parametrize("name", ["sphere32", "amr", "forest_offset"])
def test_fp32_kahan_walk(name):
    g = GRIDS[name]()
    t = oracle.Tree(g, theta=0.5)
    pr, ar, _ = t.walk_group()
    p, a, _, _ = gpu(g, fp64=False, theta=0.5)
    check32(p, a, pr, ar)


def test_tree_vs_direct_sphere():
    """The voxel sphere against the direct sum over every cell.  BH at the
    paper's theta = 0.5 leaves e_a,max at 2.9e-3 (the maximum sits at the
    sphere's centre, where opposing contributions cancel); the metric's
    e_a,max <= 1e-3 and e_Phi,max <= 1e-3 are reached at theta = 0.3, the
    setting reported for this configuration."""
    g = workloads.c1_sphere()
    pd, ad = oracle.Tree(g).direct()
    amax = np.sqrt((ad ** 2).sum(0)).max()
    for fp64 in (True, False):
        p, a, _, _ = gpu(g, fp64=fp64, theta=0.5)
        ea = np.sqrt(((a - ad) ** 2).sum(0)) / amax
        assert ea.max() < 3.5e-3 and np.quantile(ea, 0.99) < 2e-3
        assert np.abs(p / pd - 1).max() < 1e-3
        p, a, _, _ = gpu(g, fp64=fp64, theta=0.3)
        ea = np.sqrt(((a - ad) ** 2).sum(0)) / amax
        ep = np.abs(p - pd) / np.abs(pd).max()
        print(f"C1 theta 0.3 {'FP64' if fp64 else 'FP32'}: e_a,max {ea.max():.3e}, e_Phi,max {ep.max():.3e}")
        assert ea.max() <= 1e-3 and ep.max() <= 1e-3


def test_determinism():
    g = workloads.small_amr()
    for fp64 in (True, False):
        p1, a1, _, _ = gpu(g, fp64=fp64)
        p2, a2, _, _ = gpu(g, fp64=fp64)
        assert np.array_equal(p1, p2) and np.array_equal(a1, a2)


def test_single_block_and_zero_density():
    lv, cd = workloads.uniform_blocks(8)
    rng = np.random.default_rng(3)
    g = workloads.Grid((1, 1, 1), 1.0, (0, 0, 0), lv, cd, rng.random((1, 8, 8, 8)))
    pr, ar, _ = oracle.Tree(g).walk_group()
    p, a, st, _ = gpu(g)
    check64(p, a, pr, ar)
    assert st.total_list == 512
    z = workloads.Grid((1, 1, 1), 1.0, (0, 0, 0), *workloads.uniform_blocks(16), np.zeros((8, 8, 8, 8)))
    p, a, _, s = gpu(z)
    assert not p.any() and not a.any()
    M, com = s.export_moments()
    ref = oracle.Tree(z).export()
    assert np.array_equal(com, ref["com"])


def test_bad_density_is_rejected():
    g = workloads.c1_sphere()
    rho = g.rho.reshape(-1).copy()
    rho[1234] = np.nan
    s = ot.Solver.for_grid(g)
    with pytest.raises(ot.OTError, match="NUMERIC"):
        s.build(torch.from_numpy(rho).cuda())
    rho[1234] = -1.0
    with pytest.raises(ot.OTError, match="NUMERIC"):
        s.build(torch.from_numpy(rho).cuda())
    phi = torch.empty(g.nb * 512, device="cuda")
    with pytest.raises(ot.OTError, match="STATE"):
        s.solve(phi, torch.empty(3 * g.nb * 512, device="cuda"))


def test_ape_limit_prepass():
    """a_lim <= 0: the library derives a_lim = eps_lim * max|a| from a BH walk."""
    g = workloads.small_amr()
    _, a0, _ = oracle.Tree(g, theta=0.5).walk_group()
    expect = 1e-3 * np.sqrt((a0 ** 2).sum(0)).max()
    _, _, st, _ = gpu(g, mac="ape", eps_lim=1e-3)
    assert abs(st.a_lim_used - expect) <= 1e-12 * expect


# ------------------------------------------------------------- periodic
PER = {
    "3p": lambda: workloads.Grid((1, 1, 1), 1.0, (0, 0, 0), *workloads.uniform_blocks(16),
                                 np.random.default_rng(5).lognormal(0, 1, (8, 8, 8, 8)), (1, 1, 1)),
    "2p1i": lambda: workloads.small_amr(bc=(1, 1, 0), nroot=(1, 1, 2)),
}


@pytest.mark.parametrize("name", list(PER))
def test_ewald_table_parity(name):
    g = PER[name]()
    s = ot.Solver.for_grid(g, ewald_n=24)
    s.ewald_prepare()
    tab = s.export_ewald_table()
    ref = oracle.ewald_table(g.bc, g.box(), n=24)
    for ch in range(10):
        scale = np.abs(ref[..., ch]).max()
        assert np.abs(tab[..., ch] - ref[..., ch]).max() <= 1e-12 * max(scale, 1e-300), ch


@pytest.mark.parametrize("name", list(PER))
@pytest.mark.parametrize("mac", ["bh", "mpe"])
def test_periodic_walk_parity(name, mac):
    g = PER[name]()
    kw = dict(theta=0.5, ewald_n=32)
    if mac == "mpe":
        # the MPE moments are intrinsic to a node; the MAC distance is the minimum image
        kw.update(mac="mpe", a_lim=1e-2)
    t = oracle.Tree(g, **oracle_kw(kw))
    pr, ar, _ = t.walk_group()
    p, a, _, s = gpu(g, fp64=True, **kw)
    for b in range(0, g.nb, 7):
        assert np.array_equal(np.sort(s.export_list(b).astype(np.int64)), np.sort(t.block_list(b))), b
    check64(p, a, pr, ar)
    p32, a32, _, _ = gpu(g, fp64=False, **kw)
    # the periodic potential changes sign, so its error is judged against max |Phi|
    assert np.abs(p32 - pr).max() <= 1e-6 * np.abs(pr).max()
    assert np.abs(a32 - ar).max() <= 1e-5 * np.sqrt((ar ** 2).sum(0)).max()


# ------------------------------------------------------------- full size
@pytest.fixture(scope="module")
def lognormal128():
    return workloads.c2_lognormal(128)


@pytest.mark.parametrize("mac", ["bh", "ape", "mpe"])
def test_lognormal128_sampled(lognormal128, mac):
    """The 128^3 lognormal workload in the benchmark's launch configuration,
    checked on 24 sampled blocks against the oracle's group walk."""
    g = lognormal128
    kw = dict(theta=0.5) if mac == "bh" else dict(mac=mac, a_lim=2.0e-3)
    sel = np.random.default_rng(1).choice(g.nb, 24, replace=False)
    t = oracle.Tree(g, **kw)
    pr, ar, nr = t.walk_group(sel)
    cells = (512 * sel[:, None] + np.arange(512)).ravel()
    p, a, st, s = gpu(g, fp64=True, **kw)
    check64(p[cells], a[:, cells], pr, ar)
    for q, b in enumerate(sel[:6]):
        assert np.array_equal(np.sort(s.export_list(b).astype(np.int64)), np.sort(t.block_list(b)))
    p32, a32, _, _ = gpu(g, fp64=False, **kw)
    check32(p32[cells], a32[:, cells], pr, ar)


@pytest.mark.parametrize("mac", ["ape", "mpe"])
def test_lognormal128_tree_vs_direct(lognormal128, mac):
    """The benchmark's accuracy claim: the FP32 walk at its MAC (APE with
    a_lim = 1e-3 a_max, plus BH at theta_pix for the 48-pixel columns; and
    the MPE MAC at the same limit) against the oracle's direct sum, on 128
    seeded cells and the 64 cells of largest |a|.  e_a = |a - a_dir| / max
    |a_dir|, e_phi = |Phi / Phi_dir - 1|."""
    g = lognormal128
    phi, acc, st, s, npix, tau = ot.run(g, fp64=False, mac=mac, eps_lim=1e-3, theta=0.5, nside=2)
    p, a = phi.cpu().numpy().astype(np.float64), acc.cpu().numpy().astype(np.float64)
    amag = np.sqrt((a ** 2).sum(0))
    tg = np.unique(np.concatenate([np.random.default_rng(4).choice(g.ncells, 128, replace=False),
                                   np.argsort(amag)[-64:]]))
    pd, ad = oracle.Tree(g).direct(tg)
    amax = np.sqrt((ad ** 2).sum(0)).max()
    ea = np.sqrt(((a[:, tg] - ad) ** 2).sum(0)) / amax
    ep = np.abs(p[tg] / pd - 1)
    print(f"lognormal128 {mac} 1e-3 + columns MAC: e_a max {ea.max():.3e}, e_phi max {ep.max():.3e}, "
          f"a_lim {st.a_lim_used:.4g}")
    assert ea.max() <= 1e-3 and ep.max() <= 1e-3


def test_list_statistics_vs_oracle():
    """ot_stats counts: the list-length histogram covers every block once;
    accepted non-cell entries and opened nodes summed over the blocks equal
    the oracle's lists (opened = the proper ancestors of each list's entries,
    accepted = its entries that are not cells)."""
    from test_oracle_mac import node_geometry, visited
    g = workloads.small_amr()
    kw = dict(mac="ape", a_lim=3e-3)
    t = oracle.Tree(g, **kw)
    _, _, _, parent = node_geometry(t, g)
    ncell0 = t.na + 72 * g.nb
    n_open = n_acc = 0
    lens = []
    for b in range(g.nb):
        ids = t.block_list(b)
        acc, opened = visited(ids, parent)
        n_open += opened.size
        n_acc += int((acc < ncell0).sum())
        lens.append(ids.size)
    _, _, st, _ = ot.run(g, **kw)
    hist = np.array(st.list_hist)
    assert hist.sum() == g.nb
    ref = np.bincount(np.floor(np.log2(lens)).astype(int), minlength=32)
    assert np.array_equal(hist, ref)
    assert st.n_accepted == n_acc and st.n_opened == n_open
    assert st.total_list == sum(lens)
