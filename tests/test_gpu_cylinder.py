"""The device's 1P2I walk on the isothermal cylinder at the paper's resolution
(Sec. 3.1.4: 256 x 128 x 128 cells, periodic along the axis x, isolated in
y and z) against the closed-form radial acceleration
g(R) = 2 pi G rho0 R / (1 + R^2 / r0^2) of the infinite cylinder.

The cells between 2h from the axis and 2h inside the cut-off are compared
(h = 1/128).  Representing the profile by point masses at the cell centres
costs a relative error of second order in h: about 9.3e-4 at h = 1/32 in the
oracle (tests/test_oracle_cylinder.py), so about 6e-5 here.  Bars:

* BH theta 0.2 (MAC error far below the bar): relative error <= 3e-4 of g(R)
  per cell, FP64 and FP32: the device's image sums, table and walk reproduce
  the closed form up to the grid's own error.
* APE with a_lim = 1e-3 max g (an absolute limit, as everywhere in this
  library): the MAC keeps each accepted node's estimated error below a_lim
  but does not bound their sum, which on this smooth, symmetric profile adds
  up coherently (measured 1.10e-3 max g; the paper reports 8.2e-4 for its
  version of the test against its direct sum, Table 4).  Bar: the radial
  error and the axial component (zero by symmetry) within 1.5e-3 max g.
"""
import numpy as np
import pytest

import paper_1708_06142_amd as ot
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N = 128
R0 = 1.0


@pytest.fixture(scope="module")
def cyl():
    g = workloads.iso_cylinder(n=N, r0=R0)
    rc = g.meta["rcyl"]
    x = workloads.cell_centres(1.0, g.origin, g.level, g.coord).reshape(-1, 3)
    dy, dz = x[:, 1] - 0.5, x[:, 2] - 0.5
    R = np.hypot(dy, dz)
    gan = 2 * np.pi * R / (1 + R * R / (R0 * R0))
    gmax = gan[R <= rc].max()
    sel = (R >= 2.0 / N) & (R <= rc - 2.0 / N)
    return g, dy[sel], dz[sel], R[sel], gan[sel], gmax, sel


def _radial(cyl, fp64, **kw):
    g, dy, dz, R, gan, gmax, sel = cyl
    phi, acc, _, s = ot.run(g, fp64=fp64, ewald_n=64, **kw)
    a = acc.cpu().numpy().astype(np.float64)
    s.close()
    a_r = (a[1][sel] * dy + a[2][sel] * dz) / R
    return a_r + gan, np.abs(a[0]).max()


@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_cylinder_strict_mac_matches_closed_form(cyl, fp64):
    err, _ = _radial(cyl, fp64, theta=0.2)
    gan = cyl[4]
    rel = np.abs(err) / gan
    assert rel.max() <= 3e-4, rel.max()


@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_cylinder_ape_within_its_limit(cyl, fp64):
    gmax = cyl[5]
    err, ax = _radial(cyl, fp64, mac="ape", a_lim=1e-3 * gmax)
    assert np.abs(err).max() <= 1.5e-3 * gmax, np.abs(err).max() / gmax
    assert ax <= 1.5e-3 * gmax, ax / gmax
