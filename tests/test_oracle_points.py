"""Pins of the oracle's walk at arbitrary target points (Sec. 2.1: the tree is
walked for each grid cell or, in general, for any target point such as a sink
particle).

* Every accept/open decision of a point's walk is re-derived in numpy from the
  node geometry alone, with the target box shrunk to the point (half-extent
  0): safe box about the node's geometric centre, the MAC at the point's
  distance to the centre of mass; for BH, APE and MPE, isolated, 3P, 2P1I and
  1P2I, at seeded points including the domain's corners, cell centres and a
  node centre.
* With an opening angle so small that only cells are accepted, the walk at a
  point is the direct sum over all cells, recomputed here in numpy
  (Newtonian, plus the periodic correction from the oracle's separately
  pinned Ewald series for the periodic and mixed cases), to 1e-12.
* At cell centres the point walk is the paper-literal per-cell walk, bit for
  bit, the cell itself skipped.
"""
import numpy as np
import pytest

import oracle
import workloads
from test_oracle_mac import decide, node_geometry, visited
from test_oracle_tree import _node_cells

GRIDS = {
    "iso": dict(),
    "3p": dict(bc=(1, 1, 1)),
    "2p1i": dict(bc=(1, 1, 0), nroot=(1, 1, 2)),
    "1p2i": dict(bc=(1, 0, 0), nroot=(1, 2, 2)),
}
MACS = {
    "bh": dict(theta=0.6),
    "ape": dict(mac="ape", a_lim=3e-3),
    "mpe": dict(mac="mpe", a_lim=3e-3),
}


@pytest.mark.parametrize("grid", sorted(GRIDS))
@pytest.mark.parametrize("mac", sorted(MACS))
def test_point_decisions_rederived(grid, mac):
    g = workloads.small_amr(**GRIDS[grid])
    kw = MACS[mac]
    t = oracle.Tree(g, **kw)
    ex, h, gc, parent = node_geometry(t, g)
    B = t.mpe_moments() if mac == "mpe" else None
    L = np.asarray(g.nroot, np.float64) * g.root_size
    per = np.asarray(g.bc, bool)
    ncell0 = t.na + 72 * g.nb
    roots = np.nonzero(ex["alev"] == 1)[0]
    n = 0
    for x in workloads.target_points(g, 6):
        acc, opened = visited(t.point_list(x), parent)
        inner = acc[acc < ncell0]
        assert decide(kw, ex, h, gc, B, inner, x, 0.0, L, per).all(), (x, "accepted node fails the suite")
        assert not decide(kw, ex, h, gc, B, opened, x, 0.0, L, per).any(), (x, "opened node passes the suite")
        assert np.isin(roots, np.concatenate([acc, opened])).all()
        # every cell of the domain is covered once: the list partitions it
        cov = np.zeros(512 * g.nb, np.int64)
        for a in acc:
            np.add.at(cov, _node_cells(t, g, ex, a), 1)
        assert (cov == 1).all()
        n += inner.size + opened.size
    assert n > 300


def _direct(g, x, bc):
    """Direct sum over all cells at the points x [m, 3] in numpy (Newtonian
    part; plus the Ewald series' periodic correction for bc != isolated)."""
    xc = workloads.cell_centres(g.root_size, g.origin, g.level, g.coord).reshape(-1, 3)
    h = g.root_size / 2.0 ** (np.asarray(g.level, np.float64) + 2)
    m = (g.rho * (h ** 3)[:, None, None, None]).reshape(-1)
    L = np.asarray(g.nroot, np.float64) * g.root_size
    per = np.asarray(bc, bool)
    phi, acc = np.zeros(len(x)), np.zeros((3, len(x)))
    for i, p in enumerate(x):
        d = p - xc
        d = np.where(per, d - L * np.floor(d / L + 0.5), d)
        r2 = (d * d).sum(1)
        k = r2 > 0
        d, r2, mk = d[k], r2[k], m[k]
        inv = 1.0 / np.sqrt(r2)
        ph = inv
        A = d * (inv ** 3)[:, None]
        if per.any():
            c = oracle.ewald_eval(bc, L, d, correction=True)
            ph = ph + c[:, 0]
            A = A + c[:, 1:4]
        phi[i] = -(mk * ph).sum()
        acc[:, i] = -(mk[:, None] * A).sum(0)
    return phi, acc


@pytest.mark.parametrize("grid", ["iso", "2p1i"])
def test_cells_only_is_the_direct_sum(grid):
    g = workloads.small_amr(**GRIDS[grid])
    x = workloads.target_points(g, 3)
    t = oracle.Tree(g, theta=1e-9)
    phi, acc, nint = t.walk_points(x)
    assert (nint == 512 * g.nb).all()
    pd, ad = _direct(g, x, g.bc)
    assert np.abs(phi - pd).max() <= 1e-12 * np.abs(pd).max()
    assert np.abs(acc - ad).max() <= 1e-12 * np.sqrt((ad ** 2).sum(0)).max()


@pytest.mark.parametrize("grid", sorted(GRIDS))
def test_at_cell_centres_is_the_per_cell_walk(grid):
    g = workloads.small_amr(**GRIDS[grid])
    t = oracle.Tree(g, mac="ape", a_lim=3e-3, ewald="table", ew_n=16)
    tg = np.random.default_rng(4).choice(512 * g.nb, 12, replace=False)
    xc = workloads.cell_centres(g.root_size, g.origin, g.level, g.coord).reshape(-1, 3)
    p1, a1, n1 = t.walk_percell(tg)
    p2, a2, n2 = t.walk_points(xc[tg])
    assert np.array_equal(p1, p2) and np.array_equal(a1, a2) and np.array_equal(n1, n2)
