"""C-ABI checks that need no GPU: the library loads, exports every declared
entry point, validates parameters and grids on the host, and its host-built
amr-tree topology matches the oracle bit for bit."""
import ctypes as C

import numpy as np
import pytest

import oracle
import paper_1708_06142_amd as ot
import workloads


def test_library_exports_every_declared_symbol():
    syms = ot.header_symbols()
    assert "ot_solve" in syms and "ot_build" in syms and len(syms) >= 14
    L = ot.lib()
    for s in syms:
        assert hasattr(L, s), s


def test_param_validation():
    with pytest.raises(ot.OTError, match="INVALID_ARG"):
        ot.Solver(theta=-1.0)
    with pytest.raises(ot.OTError, match="INVALID_ARG"):
        ot.Solver(root_size=0.0)
    # x-periodic 1P2I and x, y-periodic 2P1I are the mixed cases; others are not
    for bc in ((0, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1)):
        with pytest.raises(ot.OTError, match="UNSUPPORTED"):
            ot.Solver(bc=bc)
    ot.Solver(bc=(1, 0, 0)).close()
    with pytest.raises(ot.OTError, match="INVALID_ARG"):
        ot.Solver(ewald_n=1)
    s = ot.Solver(bc=(1, 1, 0), nroot=(1, 1, 4))
    s.close()
    # 2P1I with Ly > Lx: the far-field switch at |dz| = 2 Lx would drop Fourier
    # modes that decay only as exp(-2 pi |dz| / Ly)
    with pytest.raises(ot.OTError, match="UNSUPPORTED"):
        ot.Solver(bc=(1, 1, 0), nroot=(1, 2, 4))
    ot.Solver(bc=(1, 1, 0), nroot=(2, 1, 4)).close()
    # targets of the walk: whole blocks (8, or 0) or 4^3 octants (4)
    for bad in (2, 16, -4):
        with pytest.raises(ot.OTError, match="INVALID_ARG"):
            ot.Solver(list_group=bad)
    for good in (0, 4, 8):
        ot.Solver(list_group=good).close()
    # the binding's struct ends where the library's does: its defaults read back
    p = ot.Params()
    ot.lib().ot_params_default(C.byref(p))
    assert p.list_group == 8 and p.mlp_reach == 1.0 and p.psi_max == 0.98


def test_call_order_and_grid_errors():
    g = workloads.c1_sphere(noise=False)
    s = ot.Solver()
    with pytest.raises(ot.OTError, match="STATE"):
        s.export_topology()
    with pytest.raises(ot.OTError, match="BAD_GRID"):
        s.set_blocks(g.level[1:], g.coord[1:])
    with pytest.raises(ot.OTError, match="BAD_GRID"):
        s.set_blocks(np.concatenate([g.level, g.level[:1]]), np.concatenate([g.coord, g.coord[:1]]))
    with pytest.raises(ot.OTError, match="BAD_GRID"):
        s.set_blocks(np.concatenate([g.level, [2]]), np.concatenate([g.coord, [[1, 0, 0]]]))
    bad = g.coord.copy()
    bad[5, 2] = 4
    with pytest.raises(ot.OTError, match="BAD_GRID"):
        s.set_blocks(g.level, bad)
    s.set_blocks(g.level, g.coord)
    # solve before build
    L = ot.lib()
    st = L.ot_solve(s.h, C.c_void_p(1), C.c_void_p(1), None, None, None, None)
    assert st == ot.OT_ERR_STATE
    st = L.ot_export_list(s.h, 0, None, 0, C.byref(C.c_int64()))
    assert st == ot.OT_ERR_STATE


@pytest.mark.parametrize("maker", [lambda: workloads.c1_sphere(noise=False),
                                   lambda: workloads.small_amr(),
                                   lambda: workloads.shuffled(workloads.small_amr()),
                                   lambda: workloads.small_amr(bc=(1, 1, 0), nroot=(1, 1, 2))])
def test_topology_matches_oracle(maker):
    g = maker()
    s = ot.Solver(nroot=g.nroot, bc=g.bc)
    s.set_blocks(g.level, g.coord)
    mine = s.export_topology()
    ref = oracle.Tree(g).export()
    assert s.na == ref["alev"].shape[0]
    for k in ("alev", "acoord", "aleaf", "achild", "akey"):
        assert np.array_equal(mine[k], ref[k]), k


def test_cache_path_errors_before_device_work(tmp_path):
    """An unusable cache path is OT_ERR_IO, found on the host before any
    device work: a file in a missing directory, and a directory."""
    s = ot.Solver(bc=(1, 1, 1), ewald_n=8)
    for bad in (str(tmp_path / "missing" / "ewald.cache"), str(tmp_path)):
        with pytest.raises(ot.OTError, match="IO"):
            s.ewald_prepare(cache_path=bad)
        with pytest.raises(ot.OTError, match="IO"):
            s.mlp_train(cache_path=bad, nsamples=1024, batch=256, epochs=1, nval=64)
    s.close()
