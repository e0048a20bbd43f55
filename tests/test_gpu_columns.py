"""GPU parity of the column densities (OpticalDepth, Sec. 2.3) against the oracle.

Node-ray table: pixel ids bit-exact, weights to 1e-12.  Walk: direction bins
are decided in FP64 on both sides, so a single differing bin would move a
node's whole contribution between pixels; the FP64 maps agree to 1e-12 of the
largest column, tau to 1e-12; the FP32 walk to 1e-5 (maps, tau) with the
gravity bars of the gravity tests.
"""
import numpy as np
import pytest

import oracle
import paper_1708_06142_amd as ot
import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("nside", [1, 2, 4])
def test_raytable_parity(nside):
    s = ot.Solver(nside=nside)
    off, pix, w = s.export_raytable()
    roff, rpix, rw = oracle.raytable(nside)
    assert np.array_equal(off, roff)
    assert np.array_equal(pix, rpix)
    assert np.abs(w - rw).max() <= 1e-12


def _gpu_cols(g, fp64, **kw):
    phi, acc, st, s, npix, tau = ot.run(g, fp64=fp64, **kw)
    f = lambda t: t.cpu().numpy().astype(np.float64)
    return f(phi), f(acc), f(npix), f(tau), st, s


def _oracle_kw(kw):
    k = dict(kw)
    if "ewald_n" in k:
        k["ew_n"] = k.pop("ewald_n")
        k["ewald"] = "table"
    return k


CASES = {
    "sphere32_n2": (lambda: workloads.c1_sphere(), dict(theta=0.5, nside=2)),
    "amr_ape_n2": (lambda: workloads.small_amr(), dict(mac="ape", a_lim=0.05, nside=2)),
    "amr2p1i_n1": (lambda: workloads.small_amr(bc=(1, 1, 0), nroot=(1, 1, 2)),
                   dict(theta=0.5, nside=1, ewald_n=32)),
    # fully periodic: the 3P table walks (FP32 and FP64) with lattice rows and the wrap margin
    "amr3p_n2": (lambda: workloads.small_amr(bc=(1, 1, 1)), dict(theta=0.5, nside=2, ewald_n=32)),
    "sphere32_n4": (lambda: workloads.c1_sphere(), dict(theta=0.5, nside=4, kappa=3.0)),
    # non-dyadic root size and shifted origin: exact zeros of d must survive
    "forest_offset_n2": (lambda: _forest_offset(), dict(theta=0.5, nside=2)),
}


def _forest_offset():
    g = workloads.small_amr(nroot=(2, 1, 1), seed=3)
    return workloads.Grid(g.nroot, 0.3, (0.1, -0.2, 0.05), g.level, g.coord, g.rho, g.bc, "forest")


@pytest.mark.parametrize("name", list(CASES))
def test_column_walk_parity(name):
    mk, kw = CASES[name]
    g = mk()
    t = oracle.Tree(g, **_oracle_kw(kw))
    sel = np.arange(g.nb) if g.nb <= 72 else np.random.default_rng(2).choice(g.nb, 48, replace=False)
    pr, ar, nr, npr, tr = t.walk_group(sel, columns=True)
    cells = (512 * sel[:, None] + np.arange(512)).ravel()
    p, a, n, tau, st, s = _gpu_cols(g, True, **kw)
    for q, b in enumerate(sel[:8]):
        assert np.array_equal(np.sort(s.export_list(b).astype(np.int64)), np.sort(t.block_list(b)))
    # 3P: Phi changes sign, so it is compared relative to its largest value
    np.testing.assert_allclose(p[cells], pr, rtol=1e-12, atol=1e-12 * np.abs(pr).max() if all(g.bc) else 0.0)
    assert np.abs(a[:, cells] - ar).max() <= 1e-12 * np.abs(ar).max()
    nmax = np.abs(npr).max()
    assert np.abs(n[sel] - npr).max() <= 1e-12 * nmax
    np.testing.assert_allclose(tau[cells], tr, rtol=1e-12, atol=1e-14)
    # FP32 walk
    p, a, n, tau, _, _ = _gpu_cols(g, False, **kw)
    assert np.abs(p[cells] - pr).max() <= 1e-6 * np.abs(pr).max()
    assert np.abs(a[:, cells] - ar).max() <= 1e-5 * np.sqrt((ar ** 2).sum(0)).max()
    assert np.abs(n[sel] - npr).max() <= 1e-5 * nmax
    assert np.abs(tau[cells] - tr).max() <= 1e-5 * max(np.abs(tr).max(), 1.0)


def test_lognormal128_columns_sampled():
    """The benchmark configuration: 128^3 lognormal, APE + 48-pixel columns,
    FP32 walk, checked on sampled blocks against the oracle's FP64 walk."""
    g = workloads.c2_lognormal(128)
    kw = dict(mac="ape", a_lim=0.0195, nside=2)
    sel = np.random.default_rng(4).choice(g.nb, 12, replace=False)
    t = oracle.Tree(g, **kw)
    pr, ar, nr, npr, tr = t.walk_group(sel, columns=True)
    cells = (512 * sel[:, None] + np.arange(512)).ravel()
    p, a, n, tau, st, s = _gpu_cols(g, False, **kw)
    assert np.abs(p[cells] - pr).max() <= 1e-6 * np.abs(pr).max()
    assert np.abs(a[:, cells] - ar).max() <= 1e-5 * np.sqrt((ar ** 2).sum(0)).max()
    assert np.abs(n[sel] - npr).max() <= 1e-5 * np.abs(npr).max()
    assert np.abs(tau[cells] - tr).max() <= 1e-5 * np.abs(tr).max()
    p64, a64, n64, tau64, _, _ = _gpu_cols(g, True, **kw)
    np.testing.assert_allclose(p64[cells], pr, rtol=1e-12)
    assert np.abs(n64[sel] - npr).max() <= 1e-12 * np.abs(npr).max()


def test_columns_need_outputs():
    g = workloads.c1_sphere()
    s = ot.Solver.for_grid(g, nside=2)
    s.build(torch.from_numpy(g.rho.reshape(-1)).cuda())
    phi = torch.empty(g.nb * 512, device="cuda")
    acc = torch.empty(3 * g.nb * 512, device="cuda")
    with pytest.raises(ot.OTError, match="INVALID_ARG"):
        s.solve(phi, acc)
