"""The mixed-boundary AMR workload at full size: four Plummer cores in a
1 x 1 x 4 box (x, y periodic, z isolated), 64^3 base cells per root block,
three refinement levels, 2.5-3.5M cells, generalised Ewald from the 64^3
table, BH theta = 0.5.

* 24 seeded blocks against the oracle's group walk (same MAC, same table):
  lists identical, FP64 walk 1e-12 (Phi and a max-normalised: the periodic
  potential changes sign), FP32-Kahan walk 1e-6 (Phi) and 1e-5 (a).
* Tree against the oracle's direct sum with the same table (exact pair sum)
  on 96 seeded cells: the group walk's error at theta = 0.5.
"""
import numpy as np
import pytest

import oracle
import paper_1708_06142_amd as ot
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def c3():
    g = workloads.c3_amr()
    assert 2.5e6 <= g.ncells <= 3.5e6
    return g


def solve(g, fp64, **kw):
    phi, acc, st, s = ot.run(g, fp64=fp64, **kw)
    return phi.cpu().numpy().astype(np.float64), acc.cpu().numpy().astype(np.float64), st, s


def test_c3_sampled_parity(c3):
    g = c3
    kw = dict(theta=0.5, ewald_n=64)
    sel = np.sort(np.random.default_rng(5).choice(g.nb, 24, replace=False))
    t = oracle.Tree(g, theta=0.5, ewald="table", ew_n=64)
    pr, ar, nr = t.walk_group(sel)
    cells = (512 * sel[:, None] + np.arange(512)).ravel()
    p, a, st, s = solve(g, True, **kw)
    for b in sel[:6]:
        assert np.array_equal(np.sort(s.export_list(b).astype(np.int64)), np.sort(t.block_list(b)))
    pmax, amax = np.abs(pr).max(), np.sqrt((ar ** 2).sum(0)).max()
    assert np.abs(p[cells] - pr).max() <= 1e-12 * pmax
    assert np.abs(a[:, cells] - ar).max() <= 1e-12 * amax
    p32, a32, st32, _ = solve(g, False, **kw)
    assert np.abs(p32[cells] - pr).max() <= 1e-6 * pmax
    assert np.abs(a32[:, cells] - ar).max() <= 1e-5 * amax
    print(f"C3: {g.nb} blocks, {g.ncells} cells, rho_c {g.meta['rho_c']:.4g}; "
          f"{st.n_interactions / g.ncells:.0f} interactions per cell; eval FP64 {st.ms_eval:.1f} ms, "
          f"FP32 {st32.ms_eval:.1f} ms")


def test_c3_tree_vs_direct(c3):
    """FP32 walk (BH theta 0.5, 64^3 table) against the oracle's direct sum
    over all other cells with the same table, on 128 seeded cells and the 32
    of largest |a|: the metric's e_a,max and e_Phi,max <= 1e-3."""
    g = c3
    p, a, st, _ = solve(g, False, theta=0.5, ewald_n=64)
    top = np.argsort((a ** 2).sum(0))[-32:]
    tg = np.unique(np.concatenate([np.random.default_rng(6).choice(g.ncells, 128, replace=False), top]))
    pd, ad = oracle.Tree(g, ewald="table", ew_n=64).direct(tg)
    amax = np.sqrt((ad ** 2).sum(0)).max()
    ea = np.sqrt(((a[:, tg] - ad) ** 2).sum(0)) / amax
    ep = np.abs(p[tg] - pd) / np.abs(pd).max()
    print(f"C3 tree (BH 0.5) vs direct: e_a max {ea.max():.3e}, e_phi max (of max |Phi|) {ep.max():.3e}")
    assert ea.max() <= 1e-3 and ep.max() <= 1e-3
