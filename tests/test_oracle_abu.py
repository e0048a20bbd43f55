"""Pins of the oracle's adaptive block update (Sec. 2.2.6): with a zero
tolerance it is the plain group walk; on an unchanged density it keeps every
block; on a locally perturbed density its block decisions are those of the
corner criterion applied to an independent full walk, and each block holds
either the full walk's values or the previous ones."""
import numpy as np

import oracle
import workloads

CORNERS = np.array([7 * (k & 1) + 56 * ((k >> 1) & 1) + 448 * ((k >> 2) & 1) for k in range(8)])


def _perturbed(g, amp=0.5, centre=(0.2, 0.2, 0.2), width=0.08):
    x = workloads.cell_centres(g.root_size, g.origin, g.level, g.coord)
    r2 = ((x - np.array(centre)) ** 2).sum(-1)
    rho = g.rho * (1.0 + amp * np.exp(-r2 / (2 * width ** 2)))
    return workloads.Grid(g.nroot, g.root_size, g.origin, g.level, g.coord, rho, g.bc, g.name)


def test_zero_tolerance_is_the_plain_walk_and_unchanged_density_keeps_all():
    g = workloads.small_amr()
    t = oracle.Tree(g, theta=0.5)
    p0, a0, _ = t.walk_group()
    p, a, upd = t.walk_abu(np.zeros_like(p0), np.zeros_like(a0), 0.0)
    assert upd.all()
    assert np.array_equal(p, p0) and np.array_equal(a, a0)
    p, a, upd = t.walk_abu(p0, a0, 1e-12)
    assert not upd.any()
    assert np.array_equal(p, p0) and np.array_equal(a, a0)


def test_local_perturbation_follows_the_corner_criterion():
    g = workloads.small_amr()
    p0, a0, _ = oracle.Tree(g, theta=0.5).walk_group()
    g1 = _perturbed(g)
    t1 = oracle.Tree(g1, theta=0.5)
    p1, a1, _ = t1.walk_group()
    amax = np.sqrt((a1 ** 2).sum(0)).max()
    tol = 1e-3 * amax
    p, a, upd = t1.walk_abu(p0, a0, tol)
    da = np.sqrt(((a1 - a0) ** 2).sum(0)).reshape(g.nb, 512)[:, CORNERS].max(1)
    assert np.array_equal(upd.astype(bool), ~(da < tol))
    assert 0 < upd.sum() < g.nb
    pb, ab = p.reshape(g.nb, 512), a.reshape(3, g.nb, 512)
    for arr, new, old in ((pb, p1.reshape(g.nb, 512), p0.reshape(g.nb, 512)),
                          (ab, a1.reshape(3, g.nb, 512), a0.reshape(3, g.nb, 512))):
        sel = upd.astype(bool)
        assert np.array_equal(arr[..., sel, :], new[..., sel, :])
        assert np.array_equal(arr[..., ~sel, :], old[..., ~sel, :])


def test_columns_decision_adds_the_corner_tau():
    """With columns the corner test also compares the optical depth kappa N_p
    of every pixel: tolerances 0 give the plain walk's maps and tau bit for
    bit and an unchanged density keeps every block; on the perturbed density
    a block is evaluated exactly when a corner's acceleration moved by tol or
    more or one of its pixels' optical depth by tol_tau or more (both read
    from independent full walks), with the acceleration test switched off
    the pixel test alone decides, and the updated blocks hold the new walk's
    maps, the others the previous ones."""
    g = workloads.small_amr()
    kw = dict(theta=0.5, nside=1)
    t0w = oracle.Tree(g, **kw)
    p0, a0, _, n0, t0 = t0w.walk_group(columns=True)
    _, _, upd, _, _ = t0w.walk_abu(p0, a0, 1e-12, n0, t0, tol_tau=1e-12)
    assert not upd.any()
    g1 = _perturbed(g)
    t1 = oracle.Tree(g1, **kw)
    p1, a1, _, n1, ta1 = t1.walk_group(columns=True)
    p, a, upd, npx, tau = t1.walk_abu(p0, a0, 0.0, n0, t0, tol_tau=0.0)
    assert upd.all() and np.array_equal(npx, n1) and np.array_equal(tau, ta1)
    da = np.sqrt(((a1 - a0) ** 2).sum(0)).reshape(g.nb, 512)[:, CORNERS].max(1)
    dtau = np.abs(n1 - n0).reshape(g.nb, -1, 512)[:, :, CORNERS].max((1, 2))  # kappa = 1
    tol, tol_tau = np.quantile(da, 0.6), np.quantile(dtau, 0.6)
    p, a, upd, npx, tau = t1.walk_abu(p0, a0, tol, n0, t0, tol_tau=tol_tau)
    sel = upd.astype(bool)
    assert np.array_equal(sel, ~(da < tol) | ~(dtau < tol_tau))
    assert (~(dtau < tol_tau) & (da < tol)).any()  # blocks that only the tau test updates
    assert ((dtau < tol_tau) & ~(da < tol)).any()  # and only the acceleration test
    assert 0 < sel.sum() < g.nb
    assert np.array_equal(npx[sel], n1[sel]) and np.array_equal(npx[~sel], n0[~sel])
    tb, t1b, t0b = tau.reshape(g.nb, 512), ta1.reshape(g.nb, 512), t0.reshape(g.nb, 512)
    assert np.array_equal(tb[sel], t1b[sel]) and np.array_equal(tb[~sel], t0b[~sel])
    _, _, upd, _, _ = t1.walk_abu(p0, a0, np.inf, n0, t0, tol_tau=tol_tau)
    assert np.array_equal(upd.astype(bool), ~(dtau < tol_tau))
