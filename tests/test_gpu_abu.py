"""GPU parity of the adaptive block update (Sec. 2.2.6) with the oracle's:
the zero-tolerance and unchanged-density limits, and a locally perturbed
field whose previous solution is the oracle's walk on the unperturbed one."""
import numpy as np
import pytest

import oracle
import paper_1708_06142_amd as ot
import workloads
from test_oracle_abu import CORNERS, _perturbed

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _solver(g, **kw):
    s = ot.Solver.for_grid(g, theta=0.5, **kw)
    s.build(torch.from_numpy(g.rho.reshape(-1)).cuda())
    return s


def test_abu_limits():
    g = workloads.small_amr()
    s = _solver(g)
    n = 512 * g.nb
    phi = torch.empty(n, dtype=torch.float64, device="cuda")
    acc = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    s.solve64(phi, acc)
    p_ref, a_ref = phi.cpu().numpy(), acc.cpu().numpy()
    # tol 0: every block evaluated, the same values as the plain solve
    phi.zero_()
    acc.zero_()
    st, upd = s.solve_abu(phi, acc, 0.0, fp64=True)
    assert upd.all() and st.n_interactions > 0
    assert np.array_equal(phi.cpu().numpy(), p_ref) and np.array_equal(acc.cpu().numpy(), a_ref)
    # unchanged density: the corners reproduce the previous values, nothing is evaluated
    st, upd = s.solve_abu(phi, acc, 1e-12, fp64=True)
    assert not upd.any() and st.n_interactions == 0
    assert np.array_equal(phi.cpu().numpy(), p_ref) and np.array_equal(acc.cpu().numpy(), a_ref)
    with pytest.raises(ot.OTError, match="INVALID_ARG"):
        s.solve_abu(phi, acc, -1.0, fp64=True)


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 0, 0)])
@pytest.mark.parametrize("fp64", [True, False])
def test_abu_perturbed_matches_oracle(fp64, bc):
    """Isolated, and 1P2I (x-periodic, 1 x 2 x 2 box) with the 32^3 Ewald table
    on both sides."""
    per = bc != (0, 0, 0)
    g = workloads.small_amr(bc=bc, nroot=(1, 2, 2) if per else (1, 1, 1))
    okw = dict(theta=0.5, ewald="table", ew_n=32) if per else dict(theta=0.5)
    p0, a0, _ = oracle.Tree(g, **okw).walk_group()
    dt = torch.float64 if fp64 else torch.float32
    if not fp64:  # both sides start from the same FP32 previous solution
        p0, a0 = p0.astype(np.float32).astype(np.float64), a0.astype(np.float32).astype(np.float64)
    g1 = _perturbed(g)
    t1 = oracle.Tree(g1, **okw)
    p1, a1, _ = t1.walk_group()
    tol = 1e-3 * np.sqrt((a1 ** 2).sum(0)).max()
    pr, ar, upd_r = t1.walk_abu(p0, a0, tol)
    s = _solver(g1, ewald_n=32) if per else _solver(g1)
    phi = torch.from_numpy(p0.copy()).to(dt).cuda()
    acc = torch.from_numpy(a0.reshape(-1).copy()).to(dt).cuda()
    st, upd = s.solve_abu(phi, acc, tol, fp64=fp64)
    p, a = phi.cpu().numpy().astype(np.float64), acc.cpu().numpy().astype(np.float64).reshape(3, -1)
    assert 0 < upd_r.sum() < g.nb
    # a block may only be decided differently where its corners sit at the tolerance
    da = np.sqrt(((a1 - a0) ** 2).sum(0)).reshape(g.nb, 512)[:, CORNERS].max(1)
    differ = upd != upd_r
    assert np.all(np.abs(da[differ] - tol) <= 1e-9 * tol), (np.nonzero(differ), da[differ] / tol)
    same = ~differ
    pb, ab = p.reshape(g.nb, 512), a.reshape(3, g.nb, 512)
    prb, arb = pr.reshape(g.nb, 512), ar.reshape(3, g.nb, 512)
    keep = same & (upd == 0)
    assert np.array_equal(pb[keep], p0.reshape(g.nb, 512)[keep])
    assert np.array_equal(ab[:, keep], a0.reshape(3, g.nb, 512)[:, keep])
    ev = same & (upd == 1)
    amax = np.sqrt((ar ** 2).sum(0)).max()
    if fp64:
        np.testing.assert_allclose(pb[ev], prb[ev], rtol=1e-12)
        assert np.abs(ab[:, ev] - arb[:, ev]).max() <= 1e-12 * amax
    else:
        if per:  # the periodic potential changes sign: judged against max |Phi|
            assert np.abs(pb[ev] - prb[ev]).max() <= 1e-6 * np.abs(pr).max()
        else:
            assert (np.abs(pb[ev] / prb[ev] - 1)).max() <= 1e-6
        assert np.abs(ab[:, ev] - arb[:, ev]).max() <= 1e-5 * amax


@pytest.mark.parametrize("fp64", [True, False])
def test_abu_columns_matches_oracle(fp64):
    """With 12-pixel columns the corner test also compares the optical depth
    of every pixel.  With the two tolerances at the 60% quantiles of the
    corners' changes (so that each test alone updates some blocks) the
    decisions are the oracle's, up to corners within 1e-9 of a tolerance; kept blocks keep phi, acc, the maps
    and tau bit for bit; updated blocks match the oracle's walk with columns
    at the walk's bar (1e-12 FP64, 1e-6 / 1e-5 FP32; maps relative to the
    largest column)."""
    g = workloads.small_amr()
    kw = dict(theta=0.5, nside=1)
    p0, a0, _, n0, t0 = oracle.Tree(g, **kw).walk_group(columns=True)
    if not fp64:
        p0, a0, n0, t0 = (x.astype(np.float32).astype(np.float64) for x in (p0, a0, n0, t0))
    g1 = _perturbed(g)
    t1 = oracle.Tree(g1, **kw)
    _, a1, _, n1, _ = t1.walk_group(columns=True)
    da = np.sqrt(((a1 - a0) ** 2).sum(0)).reshape(g.nb, 512)[:, CORNERS].max(1)
    dtau = np.abs(n1 - n0).reshape(g.nb, -1, 512)[:, :, CORNERS].max((1, 2))  # kappa = 1
    tol, tol_tau = np.quantile(da, 0.6), np.quantile(dtau, 0.6)
    pr, ar, upd_r, nr, tr = t1.walk_abu(p0, a0, tol, n0, t0, tol_tau=tol_tau)
    s = _solver(g1, nside=1)
    dt = torch.float64 if fp64 else torch.float32
    phi, acc = (torch.from_numpy(x.reshape(-1).copy()).to(dt).cuda() for x in (p0, a0))
    npix, tau = (torch.from_numpy(x.reshape(-1).copy()).to(dt).cuda() for x in (n0, t0))
    with pytest.raises(ot.OTError, match="INVALID_ARG"):
        s.solve_abu(phi, acc, tol, fp64=fp64, npix=npix, tau=tau, tol_tau=-1.0)
    with pytest.raises(TypeError):
        s.solve_abu(phi, acc, tol, fp64=fp64, npix=npix, tau=tau)
    st, upd = s.solve_abu(phi, acc, tol, fp64=fp64, npix=npix, tau=tau, tol_tau=tol_tau)
    assert 0 < upd_r.sum() < g.nb
    assert ((dtau >= tol_tau) & (da < tol) & (upd_r == 1)).any()  # updated for tau alone
    differ = upd != upd_r
    near = (np.abs(da - tol) <= 1e-9 * tol) | (np.abs(dtau - tol_tau) <= 1e-9 * tol_tau)
    assert np.all(near[differ]), np.nonzero(differ)
    keep, ev = ~differ & (upd == 0), ~differ & (upd == 1)
    got = [x.cpu().numpy().astype(np.float64) for x in (phi, acc, npix, tau)]
    shapes = [(g.nb, 512), (3, g.nb, 512), (g.nb, -1, 512), (g.nb, 512)]
    for x, x0, xr, shp in zip(got, (p0, a0, n0, t0), (pr, ar, nr, tr), shapes):
        xb, x0b, xrb = x.reshape(shp), x0.reshape(shp), xr.reshape(shp)
        if xb.ndim == 3 and shp[0] == 3:
            assert np.array_equal(xb[:, keep], x0b[:, keep])
            e = np.abs(xb[:, ev] - xrb[:, ev]).max() / np.abs(xrb).max()
        else:
            assert np.array_equal(xb[keep], x0b[keep])
            e = np.abs(xb[ev] - xrb[ev]).max() / np.abs(xrb).max()
        assert e <= (1e-12 if fp64 else 1e-5), e


@pytest.mark.parametrize("nside", [2, 4])
@pytest.mark.parametrize("fp64", [True, False])
def test_abu_columns_zero_tolerance_is_the_plain_solve(fp64, nside):
    """Tolerances 0 evaluate every block through the update's block-list
    walk (48-pixel maps in LDS, 192-pixel maps in memory): phi, acc, the maps
    and tau equal the plain solve's bit for bit."""
    g = workloads.small_amr()
    s = _solver(g, nside=nside)
    n, npx = 512 * g.nb, 12 * nside * nside
    dt = torch.float64 if fp64 else torch.float32
    outs = [torch.empty(m, dtype=dt, device="cuda") for m in (n, 3 * n, n * npx, n)]
    (s.solve64 if fp64 else s.solve)(*outs)
    ref = [o.cpu().numpy() for o in outs]
    for o in outs:
        o.zero_()
    st, upd = s.solve_abu(outs[0], outs[1], 0.0, fp64=fp64, npix=outs[2], tau=outs[3], tol_tau=0.0)
    assert upd.all()
    for o, r in zip(outs, ref):
        assert np.array_equal(o.cpu().numpy(), r)


def test_abu_after_regrid_to_more_blocks():
    """The update's per-block buffers follow the grid: a first update on a
    small grid, then a larger grid on the same context, where the update with
    tolerance 0 must equal the plain solve bit for bit."""
    small, big = workloads.c1_sphere(n=16), workloads.small_amr()
    assert big.nb > small.nb
    s = _solver(small)
    n = 512 * small.nb
    phi = torch.zeros(n, dtype=torch.float64, device="cuda")
    acc = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    st, upd = s.solve_abu(phi, acc, 0.0, fp64=True)
    assert upd.all()
    s.set_blocks(big.level, big.coord)
    s.build(torch.from_numpy(big.rho.reshape(-1)).cuda())
    n = 512 * big.nb
    for fp64 in (True, False):
        dt = torch.float64 if fp64 else torch.float32
        phi = torch.empty(n, dtype=dt, device="cuda")
        acc = torch.empty(3 * n, dtype=dt, device="cuda")
        (s.solve64 if fp64 else s.solve)(phi, acc)
        p_ref, a_ref = phi.cpu().numpy(), acc.cpu().numpy()
        phi.zero_()
        acc.zero_()
        st, upd = s.solve_abu(phi, acc, 0.0, fp64=fp64)
        assert upd.shape == (big.nb,) and upd.all()
        assert np.array_equal(phi.cpu().numpy(), p_ref) and np.array_equal(acc.cpu().numpy(), a_ref)
