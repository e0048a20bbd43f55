"""Pin of the oracle's 1P2I walk by the isothermal cylinder (Sec. 3.1.4).

An infinite cylinder of density rho0 / (1 + R^2 / r0^2)^2 pulls with the
closed-form radial acceleration g(R) = 2 pi G rho0 R / (1 + R^2 / r0^2)
(its line mass inside R over R, times 2 G), whatever lies outside R as long
as it is cylindrically symmetric.  The workload is a 2 x 1 x 1 box, periodic
along the cylinder's axis x and isolated in y and z, with the cylinder cut
off inside the box; only the periodic images along x make the finite box an
infinite cylinder, so the check covers the 1P2I correction as a whole.

What separates the walk from g(R) on a grid is the representation of the
profile by point masses at the cell centres, an error of second order in the
cell size h.  With a strict opening angle (BH theta 0.2, MAC error well
below it) the largest relative error over the cells between 2h from the axis
and 2h inside the cut-off is about 3.5e-3 at h = 1/16 and 9.3e-4 at h = 1/32:
the test asserts 1.2e-3 at h = 1/32 and a fall by at least 3 when h halves
(4 for exact second order).  With the x axis taken as isolated instead (the
same density, no images) the error is tens of percent: a 1P2I correction
that dropped its images or their sum would fail.  The axial acceleration
vanishes by symmetry, up to the MAC error.
"""
import numpy as np

import oracle
import workloads

R0 = 1.0      # scale radius: the profile falls to 0.69 at the cut-off
EW_N = 32     # 32^3 Ewald table (the look-up error is far below the bars)


def radial_errors(n, bc=None, theta=0.2):
    g = workloads.iso_cylinder(n=n, r0=R0)
    rc = g.meta["rcyl"]
    x = workloads.cell_centres(1.0, g.origin, g.level, g.coord).reshape(-1, 3)
    dy, dz = x[:, 1] - 0.5, x[:, 2] - 0.5
    R = np.hypot(dy, dz)
    gan = 2 * np.pi * R / (1 + R * R / (R0 * R0))
    kw = dict(bc=bc) if bc is not None else {}
    t = oracle.Tree(g, theta=theta, ewald="table", ew_n=EW_N, **kw)
    _, acc, _ = t.walk_group()
    h = 1.0 / n
    sel = (R >= 2 * h) & (R <= rc - 2 * h)
    a_r = (acc[1] * dy + acc[2] * dz)[sel] / R[sel]  # points to the axis: -g
    rel = np.abs(a_r + gan[sel]) / gan[sel]
    return rel.max(), np.abs(acc[0]).max() / gan.max()


def test_cylinder_converges_to_the_closed_form():
    e16, ax16 = radial_errors(16)
    e32, ax32 = radial_errors(32)
    assert e32 <= 1.2e-3, e32
    assert e16 / e32 >= 3.0, (e16, e32)
    assert max(ax16, ax32) <= 1e-4, (ax16, ax32)


def test_cylinder_without_the_periodic_images_fails():
    e, _ = radial_errors(16, bc=(0, 0, 0))
    assert e > 5e-2, e
