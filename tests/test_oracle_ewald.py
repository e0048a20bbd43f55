"""Pins of the oracle's Ewald kernels (3P and 2P1I), Sec. 2.2.3-2.2.5, App. A.

Checked against mathematics that does not depend on the series as written:
periodicity, independence of the splitting parameter alpha, derivatives by
central differences, quadrature of the 2P1I integrals from their definition
(Eq. I(l1, l2, z - z_a)), the Jeans sine-wave solution and the slab law.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads

BOX3 = (1.0, 1.5, 2.0)     # non-cubic 3P box: b = 1.5, c = 2
BOX2 = (1.0, 1.0, 4.0)     # 2P1I box of the AMR workload


def _rand(n, box, seed, zmax=None):
    rng = np.random.default_rng(seed)
    d = (rng.random((n, 3)) - 0.5) * np.asarray(box)
    if zmax is not None:
        d[:, 2] = (rng.random(n) * 2 - 1) * zmax
    return d


def test_3p_periodicity_and_symmetry():
    # the truncated series is meant for minimum-image offsets: compare a point
    # just inside the +L/2 face with its image just outside the -L/2 face
    d = _rand(40, BOX3, 1)
    f0 = oracle.ewald_eval((1, 1, 1), BOX3, d)
    for k in range(3):
        e = d.copy()
        e[:, k] = 0.5 * BOX3[k] * (0.8 + 0.2 * np.random.default_rng(k).random(40))
        sh = np.zeros(3)
        sh[k] = BOX3[k]
        fa = oracle.ewald_eval((1, 1, 1), BOX3, e)
        fb = oracle.ewald_eval((1, 1, 1), BOX3, e - sh)
        np.testing.assert_allclose(fb[:, :4], fa[:, :4], rtol=1e-12, atol=1e-12)
    # A_x vanishes on the face x = Lx/2 (mirror symmetry of the lattice)
    e = d.copy()
    e[:, 0] = 0.5
    f = oracle.ewald_eval((1, 1, 1), BOX3, e)
    assert np.abs(f[:, 1]).max() < 1e-12
    # phi even, A odd
    fm = oracle.ewald_eval((1, 1, 1), BOX3, -d)
    np.testing.assert_allclose(fm[:, 0], f0[:, 0], rtol=1e-13)
    np.testing.assert_allclose(fm[:, 1:4], -f0[:, 1:4], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("bc,box", [((1, 1, 1), BOX3), ((1, 1, 0), BOX2)])
def test_alpha_independence(bc, box):
    """The Ewald split does not change the physics: A is identical for any
    alpha; the printed 3P potential (no k = 0 term) shifts by pi/(alpha^2 V)."""
    d = _rand(30, box, 2, zmax=1.5 if bc[2] == 0 else None)
    Lx = box[0]
    f2 = oracle.ewald_eval(bc, box, d, alpha=2 / Lx, rcut2=15, fcut2=10)
    f1 = oracle.ewald_eval(bc, box, d, alpha=1 / Lx, rcut2=40, fcut2=10)
    f4 = oracle.ewald_eval(bc, box, d, alpha=4 / Lx, rcut2=9, fcut2=60)
    amax = np.abs(f2[:, 1:4]).max()
    assert np.abs(f1[:, 1:4] - f2[:, 1:4]).max() < 1e-10 * amax
    assert np.abs(f4[:, 1:4] - f2[:, 1:4]).max() < 1e-10 * amax
    if bc == (1, 1, 1):
        V = np.prod(box)
        c12 = np.pi / V * (1 / (1 / Lx) ** 2 - 1 / (2 / Lx) ** 2)
        c42 = np.pi / V * (1 / (4 / Lx) ** 2 - 1 / (2 / Lx) ** 2)
        np.testing.assert_allclose(f1[:, 0] - f2[:, 0], c12, rtol=0, atol=1e-10)
        np.testing.assert_allclose(f4[:, 0] - f2[:, 0], c42, rtol=0, atol=1e-10)
    else:
        # 2P1I potential: defined up to a constant as well
        df = f1[:, 0] - f2[:, 0]
        assert np.ptp(df) < 1e-10 * np.abs(f2[:, 0]).max()


@pytest.mark.parametrize("bc,box", [((1, 1, 1), BOX3), ((1, 1, 0), BOX2)])
@pytest.mark.parametrize("corr", [False, True])
def test_derivatives_by_central_differences(bc, box, corr):
    """A = -grad phi and H = grad grad phi (App. A) against differences."""
    d = _rand(12, box, 3, zmax=1.8 if bc[2] == 0 else None)
    d[np.linalg.norm(d, axis=1) < 0.05] += 0.1
    eps = 1e-5
    f = oracle.ewald_eval(bc, box, d, correction=corr)
    hidx = [[4, 7, 8], [7, 5, 9], [8, 9, 6]]
    for j in range(3):
        s = np.zeros(3)
        s[j] = eps
        fp = oracle.ewald_eval(bc, box, d + s, correction=corr)
        fm = oracle.ewald_eval(bc, box, d - s, correction=corr)
        dphi = (fp[:, 0] - fm[:, 0]) / (2 * eps)
        np.testing.assert_allclose(-dphi, f[:, 1 + j], rtol=1e-7, atol=1e-7)
        for k in range(3):
            dA = (fp[:, 1 + k] - fm[:, 1 + k]) / (2 * eps)
            np.testing.assert_allclose(-dA, f[:, hidx[k][j]], rtol=1e-6, atol=1e-6)


def test_correction_is_total_minus_newton_and_smooth_at_origin():
    for bc, box in [((1, 1, 1), BOX3), ((1, 1, 0), BOX2)]:
        d = _rand(20, box, 4, zmax=1.0 if bc[2] == 0 else None)
        ft = oracle.ewald_eval(bc, box, d)
        fc = oracle.ewald_eval(bc, box, d, correction=True)
        r = np.linalg.norm(d, axis=1)
        np.testing.assert_allclose(fc[:, 0], ft[:, 0] - 1 / r, rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(fc[:, 1:4], ft[:, 1:4] - d / r[:, None] ** 3, rtol=1e-9, atol=1e-10)
        # continuity across the series/closed-form switch of -erf(alpha r)/r
        a = 2 / box[0]
        rs = 0.2 / a
        u = np.array([[rs * (1 - 1e-14), 0, 0], [rs * (1 + 1e-14), 0, 0]])
        g = oracle.ewald_eval(bc, box, u, correction=True)
        assert np.abs(g[0] - g[1]).max() < 1e-12
        # value at d = 0: A_c = 0 (odd), phi_c finite
        z = oracle.ewald_eval(bc, box, np.zeros((1, 3)), correction=True)
        assert np.abs(z[0, 1:4]).max() < 1e-14 and np.isfinite(z[0]).all()


def test_jeans_sine_wave_3p():
    """Sine-wave density rho0 + rho1 cos(k.r) on a periodic lattice (Sec. 3.1.2):
    a_i = V sin(k.r_i) exactly, V -> -4 pi G rho1 k / k^2 with O(h^2) error."""
    kvec = 2 * np.pi * np.array([1.0, 1.0, 0.0])
    vanal = -4 * np.pi * kvec / kvec.dot(kvec)
    errs = []
    for n in (16, 32):
        h = 1.0 / n
        p = np.arange(n) - n // 2
        P = np.stack(np.meshgrid(p, p, p, indexing="ij"), -1).reshape(-1, 3)
        P = P[np.abs(P).sum(1) > 0]
        dl = P * h
        f = oracle.ewald_eval((1, 1, 1), (1, 1, 1), dl)
        V = -(h ** 3) * (np.sin(dl @ kvec)[:, None] * f[:, 1:4]).sum(0)
        errs.append(np.linalg.norm(V - vanal) / np.linalg.norm(vanal))
    assert errs[1] < 0.05
    assert 3.0 < errs[0] / errs[1] < 5.0
    # full direct sum on one 8^3 block: a_i is V sin(k.r_i) to round-off
    lv, cd = workloads.uniform_blocks(8)
    xc = workloads.cell_centres(1.0, (0, 0, 0), lv, cd)
    rho = 1.0 + 0.3 * np.cos(xc @ kvec)
    g = workloads.Grid((1, 1, 1), 1.0, (0, 0, 0), lv, cd, rho, (1, 1, 1))
    t = oracle.Tree(g, bc=(1, 1, 1))
    _, acc = t.direct()
    s = np.sin(xc.reshape(-1, 3) @ kvec)
    Vfit = acc @ s / (s @ s)
    resid = acc - Vfit[:, None] * s[None]
    assert np.abs(resid).max() < 1e-10 * np.abs(acc).max()
    assert np.abs(Vfit[2]) < 1e-10 * np.abs(Vfit).max()


@pytest.mark.parametrize("s", [0.0, 0.5, 1.0, np.sqrt(2.0), 3.0])
@pytest.mark.parametrize("gam", [0.0, 0.3, 2.0, -1.7, 8.0])
def test_2p1i_integrals_vs_quadrature(s, gam):
    zeta = np.pi ** 2 / 4
    I0, I1, I2 = oracle.itilde(s, zeta, gam)
    if s == 0.0:
        q0 = 2 * integrate.quad(lambda u: np.exp(-zeta * u * u) * (np.cos(gam * u) - 1) / max(u * u, 1e-300)
                                if u > 1e-8 else -gam * gam / 2, 0, 20, limit=400, epsabs=1e-14)[0]
        q1 = -2 * integrate.quad(lambda u: np.exp(-zeta * u * u) * (np.sin(gam * u) / u if u > 1e-12 else gam),
                                 0, 20, limit=400, epsabs=1e-14)[0]
        q2 = -2 * integrate.quad(lambda u: np.exp(-zeta * u * u) * np.cos(gam * u), 0, 20, limit=400, epsabs=1e-14)[0]
        scale = 1.0
    else:
        w = lambda u: 2 * np.exp(-zeta * u * u) / (s * s + u * u)
        q0 = integrate.quad(lambda u: w(u) * np.cos(gam * u), 0, 20, limit=400, epsabs=1e-15)[0]
        q1 = integrate.quad(lambda u: -w(u) * u * np.sin(gam * u), 0, 20, limit=400, epsabs=1e-15)[0]
        q2 = integrate.quad(lambda u: -w(u) * u * u * np.cos(gam * u), 0, 20, limit=400, epsabs=1e-15)[0]
        scale = np.exp(-zeta * s * s)
    np.testing.assert_allclose([I0, I1, I2], np.array([q0, q1, q2]) * scale, rtol=1e-9, atol=1e-12)


def test_2p1i_slab_law_and_symmetry():
    """A periodic sheet of point masses pulls with 2 pi sigma toward it, plus
    the exponentially small lattice terms of a square point lattice."""
    n = 8
    h = 1.0 / n
    p = (np.arange(n) - n // 2) * h
    X, Y = np.meshgrid(p, p, indexing="ij")
    for dz in (2 * h, 3 * h, 0.9, 1.9, 3.3):
        d = np.stack([X.ravel(), Y.ravel(), np.full(n * n, dz)], 1)
        f = oracle.ewald_eval((1, 1, 0), BOX2, d)
        S = f[:, 1:4].sum(0)
        # a = -G m A: A_z > 0 for dz > 0 means attraction toward the sheet.
        # Field of a square lattice sheet above a lattice site:
        # 2 pi sigma sum_G exp(-|G| dz), G = (2 pi / h) (m1, m2)
        m = np.arange(-4, 5)
        M1, M2 = np.meshgrid(m, m)
        lat = np.exp(-2 * np.pi * dz / h * np.sqrt(M1 ** 2 + M2 ** 2)).sum()
        np.testing.assert_allclose(S[2], 2 * np.pi * n * n * lat, rtol=1e-10)
        assert np.abs(S[:2]).max() < 1e-9 * S[2]
        fm = oracle.ewald_eval((1, 1, 0), BOX2, d * [1, 1, -1])
        np.testing.assert_allclose(fm[:, 3], -f[:, 3], rtol=1e-12)


def test_2p1i_far_field_limit():
    """For |dz| >= 2 Lx the kernel equals the analytic l = 0 limit
    phi = -2 pi |dz|/(b Lx^2) + sqrt(pi)/(b Lx), A = (0, 0, 2 pi sgn dz/(b Lx^2))."""
    rng = np.random.default_rng(9)
    d = np.stack([rng.uniform(-.5, .5, 20), rng.uniform(-.5, .5, 20), rng.choice([-1, 1], 20) * 2.0], 1)
    f = oracle.ewald_eval((1, 1, 0), BOX2, d)
    phi_a = -2 * np.pi * np.abs(d[:, 2]) + np.sqrt(np.pi)
    np.testing.assert_allclose(f[:, 0], phi_a, rtol=1e-5)
    A = np.stack([0 * d[:, 0], 0 * d[:, 0], 2 * np.pi * np.sign(d[:, 2])], 1)
    assert np.abs(f[:, 1:4] - A).max() < 1e-4 * 2 * np.pi
    # the remainder decays like exp(-2 pi |dz| / Lx)
    d[:, 2] *= 1.5
    f = oracle.ewald_eval((1, 1, 0), BOX2, d)
    assert np.abs(f[:, 0] - (-2 * np.pi * np.abs(d[:, 2]) + np.sqrt(np.pi))).max() < 1e-7


@pytest.mark.parametrize("bc,box", [((1, 1, 1), (1.0, 1.0, 1.0)), ((1, 1, 0), BOX2)])
def test_table_lookup_accuracy(bc, box):
    """First-order Taylor look-up vs the exact series (error normalised by the
    largest |A_c| or |phi_c|): at 64^3 below 2e-4 (3P cube) and 1e-3 (2P1I
    1x1x4 box); it falls by more than 2.5x from 32^3 to 64^3."""
    zext = min(box[2], 2 * box[0]) if bc[2] == 0 else box[2] / 2
    rng = np.random.default_rng(11)
    d = (rng.random((400, 3)) - 0.5) * np.array([box[0], box[1], 2 * zext])
    d = d[np.linalg.norm(d, axis=1) > 0.02]
    ex = oracle.ewald_eval(bc, box, d, correction=True)
    errs = []
    for n in (32, 64):
        tab = oracle.ewald_table(bc, box, n=n)
        lk = oracle.ewald_table_lookup(bc, box, tab, d)
        amax = np.abs(ex[:, 1:4]).max()
        errs.append(max(np.abs(lk[:, 1:4] - ex[:, 1:4]).max() / amax,
                        np.abs(lk[:, 0] - ex[:, 0]).max() / np.abs(ex[:, 0]).max()))
        # at the grid points themselves the look-up returns the table values
        g = np.array([[3, 5, 7], [0, 0, 0], [n - 1, n - 1, n - 1]])
        step = np.array([box[0] / 2, box[1] / 2, zext]) / (n - 1)
        lk0 = oracle.ewald_table_lookup(bc, box, tab, g * step)
        np.testing.assert_array_equal(lk0[:, 0], tab[g[:, 2], g[:, 1], g[:, 0], 0])
    # 2P1I: the z spacing is 4x the x spacing (2 Lx over the same n points)
    assert errs[1] < (2e-4 if bc[2] else 1e-3)
    assert errs[0] / errs[1] > 2.5
