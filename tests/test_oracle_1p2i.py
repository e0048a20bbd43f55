"""Pins of the oracle's 1P2I Ewald kernel (periodic along x, isolated in y
and z), Sec. 2.2.4 and App. A.

Checked against mathematics that does not depend on the series as written:
the defining integrals K and M by adaptive quadrature with library Bessel
functions, independence of the splitting parameter alpha, a brute-force sum
over the periodic images, derivatives by central differences, symmetry about
the periodic axis, and the field of an infinite line mass far from the axis.
"""
import numpy as np
import pytest
from scipy import integrate, special

import oracle
import workloads

BC = (1, 0, 0)
BOX = (1.0, 2.0, 2.0)
ZETA = np.pi ** 2 / 4  # alpha = 2 / Lx


def _rand(n, seed, rmax=1.8):
    rng = np.random.default_rng(seed)
    d = np.empty((n, 3))
    d[:, 0] = rng.uniform(-0.5, 0.5, n)
    d[:, 1:] = rng.uniform(-rmax, rmax, (n, 2))
    return d


def _quad(f):
    return integrate.quad(f, 0, 8, limit=500, epsabs=1e-15, epsrel=1e-13)[0]


@pytest.mark.parametrize("l", [0, 1, 2, 3])
@pytest.mark.parametrize("eta", [0.0, 0.3, 2.0, 9.0, 19.0])
def test_integrals_vs_quadrature(l, eta):
    """K(l, eta) (l != 0) and M(l, eta) against their defining integrals;
    M = -dK/deta and dM/deta by central differences (also for the regularised
    l = 0 form of K); M/eta tends to dM/deta at eta = 0."""
    K, M, Mp, Mq = oracle.kfuncs(l, eta, ZETA)
    Mr = _quad(lambda q: special.j1(eta * q) * np.exp(-ZETA * q * q) * q * q / (l * l + q * q))
    assert abs(M - Mr) < 1e-13
    if l > 0:
        Kr = _quad(lambda q: special.j0(eta * q) * np.exp(-ZETA * q * q) * q / (l * l + q * q))
        assert abs(K - Kr) < 1e-13
    else:
        assert K <= 0.0 and (eta > 0 or K == 0.0)
    if eta > 0:
        h = 1e-5
        kp, km = oracle.kfuncs(l, eta + h, ZETA), oracle.kfuncs(l, eta - h, ZETA)
        assert abs(M + (kp[0] - km[0]) / (2 * h)) < 1e-9
        assert abs(Mp - (kp[1] - km[1]) / (2 * h)) < 1e-9
        assert abs(Mq - M / eta) < 1e-15 * max(1.0, abs(Mq))
    else:
        assert M == 0.0 and Mq == Mp
        kp = oracle.kfuncs(l, 1e-4, ZETA)
        assert abs(kp[1] / 1e-4 - Mp) < 1e-7


def test_alpha_independence():
    """A is the same for any splitting parameter; phi shifts by a constant
    (the dropped divergent constant of the l = 0 term depends on alpha)."""
    d = _rand(24, 2)
    f2 = oracle.ewald_eval(BC, BOX, d, alpha=2.0, rcut2=10, fcut2=10)
    f1 = oracle.ewald_eval(BC, BOX, d, alpha=1.0, rcut2=40, fcut2=10)
    f3 = oracle.ewald_eval(BC, BOX, d, alpha=3.0, rcut2=10, fcut2=25)
    amax = np.abs(f2[:, 1:4]).max()
    for f in (f1, f3):
        assert np.abs(f[:, 1:4] - f2[:, 1:4]).max() < 1e-11 * amax
        assert np.ptp(f[:, 0] - f2[:, 0]) < 1e-11 * np.abs(f2[:, 0]).max()
    # the constant is that of -(2 ln alpha)/Lx in the line-mass limit
    np.testing.assert_allclose(f1[:, 0] - f2[:, 0], 2 * np.log(2.0), rtol=0, atol=1e-10)


def test_acceleration_and_potential_vs_image_sum():
    """A against the direct sum over 400,001 images of a unit mass (the tail
    beyond is below 3e-11); differences of phi against the image sum of the
    differences of 1/r (the sum of 1/r itself diverges)."""
    d = _rand(6, 5)
    f = oracle.ewald_eval(BC, BOX, d)
    N = 200000
    i = np.arange(-N, N + 1, dtype=np.float64)
    pots = []
    for k in range(len(d)):
        x = np.stack([d[k, 0] - i, np.full_like(i, d[k, 1]), np.full_like(i, d[k, 2])], 1)
        r = np.sqrt((x * x).sum(1))
        A = (x / r[:, None] ** 3).sum(0)
        assert np.abs(A - f[k, 1:4]).max() < 1e-9 * np.abs(f[:, 1:4]).max()
        pots.append(1 / r)
    for k in range(1, len(d)):
        ref = (pots[k] - pots[0]).sum()
        assert abs((f[k, 0] - f[0, 0]) - ref) < 1e-9 * np.abs(f[:, 0]).max()


@pytest.mark.parametrize("corr", [False, True])
def test_derivatives_by_central_differences(corr):
    """A = -grad phi and H = grad grad phi against differences, including
    offsets on the periodic axis (rho = 0)."""
    d = _rand(12, 3)
    d[np.linalg.norm(d, axis=1) < 0.05] += 0.1
    d[0, 1:] = 0.0  # on the axis
    eps = 1e-5
    f = oracle.ewald_eval(BC, BOX, d, correction=corr)
    hidx = [[4, 7, 8], [7, 5, 9], [8, 9, 6]]
    for j in range(3):
        s = np.zeros(3)
        s[j] = eps
        fp = oracle.ewald_eval(BC, BOX, d + s, correction=corr)
        fm = oracle.ewald_eval(BC, BOX, d - s, correction=corr)
        np.testing.assert_allclose(-(fp[:, 0] - fm[:, 0]) / (2 * eps), f[:, 1 + j], rtol=1e-7, atol=1e-7)
        for k in range(3):
            dA = (fp[:, 1 + k] - fm[:, 1 + k]) / (2 * eps)
            np.testing.assert_allclose(-dA, f[:, hidx[k][j]], rtol=1e-6, atol=1e-6)


def test_periodicity_and_axial_symmetry():
    d = _rand(20, 4)
    f = oracle.ewald_eval(BC, BOX, d)
    fs = oracle.ewald_eval(BC, BOX, d + [1.0, 0, 0])
    np.testing.assert_allclose(fs, f, rtol=1e-11, atol=1e-11)
    # a rotation about the x axis rotates A and leaves phi and A_x unchanged
    c, s = np.cos(0.7), np.sin(0.7)
    R = np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    fr = oracle.ewald_eval(BC, BOX, d @ R.T)
    np.testing.assert_allclose(fr[:, 0], f[:, 0], rtol=1e-12)
    np.testing.assert_allclose(fr[:, 1:4], f[:, 1:4] @ R.T, rtol=1e-10, atol=1e-12)
    # the correction is smooth at the origin: A_c = 0 there
    z = oracle.ewald_eval(BC, BOX, np.zeros((1, 3)), correction=True)
    assert np.abs(z[0, 1:4]).max() < 1e-14 and np.isfinite(z[0]).all()


def test_line_mass_far_field():
    """Far from the axis the images act as a line of mass 1/Lx:
    phi -> -(2 ln(alpha rho) + gamma_E)/Lx, A -> 2 rho_vec/(Lx rho^2); at the
    switch to this limit (rho = 4 Lx) the series agrees with it to 1e-10,
    and the difference falls further out (at 3 Lx it is still 3e-8 in A)."""
    rho = np.array([3.0, 4.0, 5.0])
    ang = np.array([0.3, 1.1, 2.0])
    d = np.stack([np.array([0.1, -0.4, 0.25]), rho * np.cos(ang), rho * np.sin(ang)], 1)
    f = oracle.ewald_eval(BC, (1.0, 12.0, 12.0), d)
    lim = -(2 * np.log(2.0 * rho) + np.euler_gamma)
    err = np.abs(f[:, 0] - lim)
    ea = np.abs(f[:, 1:4] - np.concatenate([np.zeros((3, 1)), 2 * d[:, 1:] / rho[:, None] ** 2], 1)).max(1)
    assert err[1:].max() < 1e-10 and ea[1:].max() < 1e-10
    assert err[2] <= err[1] <= err[0] < 1e-8 and ea[2] <= ea[1] <= ea[0] < 1e-7


def test_table_lookup_accuracy():
    """First-order Taylor look-up vs the series over the folded domain
    [0, Lx/2] x [0, min(Ly, 4 Lx)] x [0, min(Lz, 4 Lx)]: below 1.5e-3 of the
    largest value at 64^3, falling by more than 2.5x from 32^3."""
    rng = np.random.default_rng(11)
    d = (rng.random((400, 3)) - 0.5) * np.array([1.0, 4.0, 4.0])
    d = d[np.linalg.norm(d, axis=1) > 0.02]
    ex = oracle.ewald_eval(BC, BOX, d, correction=True)
    errs = []
    for n in (32, 64):
        tab = oracle.ewald_table(BC, BOX, n=n)
        lk = oracle.ewald_table_lookup(BC, BOX, tab, d)
        errs.append(max(np.abs(lk[:, 1:4] - ex[:, 1:4]).max() / np.abs(ex[:, 1:4]).max(),
                        np.abs(lk[:, 0] - ex[:, 0]).max() / np.abs(ex[:, 0]).max()))
    assert errs[1] < 1.5e-3  # the y and z spacing is 4x the x spacing
    assert errs[0] / errs[1] > 2.5


def test_open_everything_equals_direct_1p2i():
    """Group walk with a MAC that opens every node equals the direct sum on a
    1P2I AMR grid (1 x 2 x 2 roots), both with the 32^3 table per pair."""
    g = workloads.small_amr(bc=BC, nroot=(1, 2, 2))
    t = oracle.Tree(g, theta=1e-6, ewald="table", ew_n=32)
    sel = [0, g.nb // 2, g.nb - 1]
    phi, acc, _ = t.walk_group(sel)
    cells = np.concatenate([512 * b + np.arange(512) for b in sel])[::37]
    pd, ad = t.direct(cells)
    idx = np.concatenate([np.arange(512) + 512 * k for k in range(len(sel))])[::37]
    np.testing.assert_allclose(phi[idx], pd, rtol=1e-12)
    assert np.abs(acc[:, idx] - ad).max() <= 1e-12 * np.abs(ad).max()
