"""Python binding of libocttree (C ABI in include/octtree.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every step of the solver runs in the library's HIP kernels.  There is
no CPU fallback: if the library is missing, importing the binding succeeds but
any solver call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libocttree.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "octtree.h")

OT_OK, OT_ERR_INVALID_ARG, OT_ERR_BAD_GRID, OT_ERR_NUMERIC = 0, -1, -2, -3
OT_ERR_STATE, OT_ERR_OOM, OT_ERR_DEVICE, OT_ERR_UNSUPPORTED, OT_ERR_IO = -4, -5, -6, -7, -8
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "BAD_GRID", -3: "NUMERIC", -4: "STATE", -5: "OOM",
          -6: "DEVICE", -7: "UNSUPPORTED", -8: "IO"}


class OTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("nroot", C.c_int32 * 3), ("bc", C.c_int32 * 3), ("root_size", C.c_double),
                ("origin", C.c_double * 3), ("G", C.c_double), ("theta_lim", C.c_double),
                ("eta_sb", C.c_double), ("mac", C.c_int32), ("ewald", C.c_int32),
                ("a_lim", C.c_double), ("eps_lim", C.c_double), ("ewald_n", C.c_int32),
                ("ewald_rcut2", C.c_int32), ("ewald_fcut2", C.c_int32), ("device", C.c_int32),
                ("ewald_alpha", C.c_double), ("max_device_bytes", C.c_uint64),
                ("nside", C.c_int32), ("il_ntheta", C.c_int32), ("il_nphi", C.c_int32),
                ("il_npsi", C.c_int32), ("il_nr", C.c_int32), ("il_nazi", C.c_int32),
                ("theta_pix", C.c_double), ("kappa", C.c_double), ("max_dist", C.c_double),
                ("psi_max", C.c_double), ("mlp_reach", C.c_double), ("list_group", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_interactions", C.c_int64), ("max_list", C.c_int64), ("total_list", C.c_int64),
                ("a_lim_used", C.c_double), ("ms_build", C.c_double), ("ms_list", C.c_double),
                ("ms_eval", C.c_double), ("ewald_used", C.c_int32), ("eval_wg_per_cu", C.c_int32),
                ("n_opened", C.c_int64), ("n_accepted", C.c_int64), ("list_hist", C.c_int64 * 32),
                ("n_mlp_evals", C.c_int64), ("ms_gravity", C.c_double), ("ms_columns", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}
        d["list_hist"] = list(self.list_hist)
        return d


class MlpConfig(C.Structure):
    _fields_ = [("nsamples", C.c_int64), ("nval", C.c_int64), ("epochs", C.c_int32), ("batch", C.c_int32),
                ("lr_max", C.c_double), ("lr_min", C.c_double), ("seed", C.c_uint64), ("tol", C.c_double)]


class MlpReport(C.Structure):
    _fields_ = [("loss_first", C.c_double), ("loss_last", C.c_double), ("err_mlp", C.c_double * 10),
                ("err_table", C.c_double * 10), ("ms_samples", C.c_double), ("ms_train", C.c_double),
                ("ms_validate", C.c_double), ("ok", C.c_int32), ("from_cache", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["err_mlp"], d["err_table"] = list(self.err_mlp), list(self.err_table)
        return d


MLP_NPARAM, MLP_NNORM, MLP_NOUT = 9226, 23, 10
EWALD = {"table": 0, "exact": 1, "mlp": 2}


_lib = None


def lib():
    """Load libocttree.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        # torch's HIP runtime has the same soname as the system one; loading
        # torch first makes the library bind to it, so that the streams and
        # device memory torch hands over belong to the runtime the library uses
        import torch  # noqa: F401
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIBPATH)
        vp, i64 = C.c_void_p, C.c_int64
        L.ot_params_default.argtypes = [C.POINTER(Params)]
        L.ot_create.argtypes = [C.POINTER(Params), C.POINTER(vp)]
        L.ot_set_blocks.argtypes = [vp, i64, vp, vp]
        L.ot_build.argtypes = [vp, vp, vp]
        L.ot_solve.argtypes = [vp, vp, vp, vp, vp, C.POINTER(Stats), vp]
        L.ot_solve64.argtypes = [vp, vp, vp, vp, vp, C.POINTER(Stats), vp]
        L.ot_solve_abu.argtypes = [vp, vp, vp, vp, vp, C.c_double, C.c_double, vp, C.POINTER(Stats), vp]
        L.ot_solve_abu64.argtypes = [vp, vp, vp, vp, vp, C.c_double, C.c_double, vp, C.POINTER(Stats), vp]
        L.ot_export_raytable.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), vp, vp, vp, vp]
        L.ot_ewald_prepare.argtypes = [vp, C.c_char_p, vp]
        L.ot_num_amr_nodes.restype = i64
        L.ot_num_amr_nodes.argtypes = [vp]
        L.ot_export_topology.argtypes = [vp, vp, vp, vp, vp, vp]
        L.ot_export_moments.argtypes = [vp, vp, vp]
        L.ot_export_list.argtypes = [vp, i64, vp, i64, C.POINTER(i64)]
        L.ot_solve_points.argtypes = [vp, i64, vp, vp, vp, C.POINTER(Stats), vp]
        L.ot_export_point_list.argtypes = [vp, i64, vp, i64, C.POINTER(i64)]
        L.ot_export_ewald_table.argtypes = [vp, vp]
        L.ot_mlp_config_default.argtypes = [C.POINTER(MlpConfig)]
        L.ot_mlp_train.argtypes = [vp, C.POINTER(MlpConfig), C.c_char_p, C.POINTER(MlpReport), vp]
        L.ot_mlp_get.argtypes = [vp, vp, vp]
        L.ot_mlp_set.argtypes = [vp, vp, vp, C.c_int32, vp]
        L.ot_mlp_grad.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
        L.ot_mlp_grad_noalloc.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
        L.ot_mlp_adam_step.argtypes = [vp, vp, vp, vp, i64, vp, vp, C.c_double, i64, vp, vp]
        L.ot_ewald_points.argtypes = [vp, C.c_int32, i64, vp, vp, vp]
        L.ot_column_bins.argtypes = [vp, i64, vp, vp, vp, vp]
        L.ot_last_error.restype = C.c_char_p
        L.ot_last_error.argtypes = [vp]
        L.ot_destroy.argtypes = [vp]
        for name in ("ot_create", "ot_set_blocks", "ot_build", "ot_solve", "ot_solve64", "ot_solve_abu",
                     "ot_solve_abu64",
                     "ot_ewald_prepare", "ot_export_topology", "ot_export_moments",
                     "ot_export_list", "ot_export_ewald_table", "ot_export_raytable", "ot_mlp_train",
                     "ot_solve_points", "ot_export_point_list",
                     "ot_mlp_get", "ot_mlp_set", "ot_mlp_grad", "ot_mlp_grad_noalloc", "ot_mlp_adam_step", "ot_ewald_points",
                     "ot_column_bins"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def header_symbols():
    """Entry points declared in include/octtree.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ot_[a-z0-9_]+)\s*\(", txt)))


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t, dtype):
    import torch
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} device tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None and not torch.cuda.is_available():
        return None  # no device: the call fails on the host or reports the device error
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


MAC = {"bh": 0, "ape": 1, "mpe": 2}


def make_params(nroot=(1, 1, 1), root_size=1.0, origin=(0.0, 0.0, 0.0), bc=(0, 0, 0), G=1.0,
                theta=0.5, eta_sb=1.2, mac="bh", a_lim=0.0, eps_lim=1e-3, ewald="table",
                ewald_n=64, ewald_rcut2=0, ewald_fcut2=0, ewald_alpha=0.0, device=0,
                max_device_bytes=0, nside=0, theta_pix=0.0, kappa=1.0, max_dist=1e99, mlp_reach=1.0,
                list_group=8, **table):
    p = Params()
    lib().ot_params_default(C.byref(p))
    for k in range(3):
        p.nroot[k], p.bc[k], p.origin[k] = int(nroot[k]), int(bc[k]), float(origin[k])
    p.root_size, p.G, p.theta_lim, p.eta_sb = float(root_size), float(G), float(theta), float(eta_sb)
    p.mac = MAC[mac]
    p.ewald = EWALD[ewald]
    p.a_lim, p.eps_lim = float(a_lim), float(eps_lim)
    p.ewald_n, p.ewald_rcut2, p.ewald_fcut2 = int(ewald_n), int(ewald_rcut2), int(ewald_fcut2)
    p.ewald_alpha, p.device, p.max_device_bytes = float(ewald_alpha), int(device), int(max_device_bytes)
    p.nside, p.theta_pix, p.kappa, p.max_dist = int(nside), float(theta_pix), float(kappa), float(max_dist)
    p.mlp_reach = float(mlp_reach)
    p.list_group = int(list_group)
    for k, v in table.items():
        if k not in ("il_ntheta", "il_nphi", "il_npsi", "il_nr", "il_nazi", "psi_max"):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


class Solver:
    """One libocttree context: blocks -> build -> solve."""

    def __init__(self, **kw):
        self.params = make_params(**kw)
        h = C.c_void_p()
        st = lib().ot_create(C.byref(self.params), C.byref(h))
        self.h = h
        if st != OT_OK:
            msg = lib().ot_last_error(h).decode() if h.value else "ot_create failed"
            self.close()
            raise OTError(st, msg)
        self.nb = 0
        self.na = 0

    @classmethod
    def for_grid(cls, grid, **kw):
        s = cls(nroot=grid.nroot, root_size=grid.root_size, origin=grid.origin, bc=grid.bc, **kw)
        s.set_blocks(grid.level, grid.coord)
        return s

    def _check(self, st):
        if st != OT_OK:
            raise OTError(st, lib().ot_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().ot_destroy(self.h)
        self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_blocks(self, level, coord):
        lv = np.ascontiguousarray(level, dtype=np.int32)
        cd = np.ascontiguousarray(coord, dtype=np.int32).reshape(-1, 3)
        self._check(lib().ot_set_blocks(self.h, lv.shape[0], _np_ptr(lv), _np_ptr(cd)))
        self.nb = int(lv.shape[0])
        self.na = int(lib().ot_num_amr_nodes(self.h))

    def build(self, rho, stream=None):
        import torch
        self._check(lib().ot_build(self.h, _dev_ptr(rho, torch.float64), _stream(stream)))

    def solve(self, phi, acc, npix=None, tau=None, stream=None):
        import torch
        st = Stats()
        f = torch.float32
        self._check(lib().ot_solve(self.h, _dev_ptr(phi, f), _dev_ptr(acc, f), _dev_ptr(npix, f),
                                   _dev_ptr(tau, f), C.byref(st), _stream(stream)))
        return st

    def solve64(self, phi, acc, npix=None, tau=None, stream=None):
        import torch
        st = Stats()
        f = torch.float64
        self._check(lib().ot_solve64(self.h, _dev_ptr(phi, f), _dev_ptr(acc, f), _dev_ptr(npix, f),
                                     _dev_ptr(tau, f), C.byref(st), _stream(stream)))
        return st

    def solve_points(self, xyz, phi, acc, stream=None):
        """Potential phi [n] and acceleration acc [3, n] (FP64 device tensors)
        at n target points xyz [n, 3] (FP64, inside the domain), each walked
        with its own list."""
        import torch
        f = torch.float64
        n = xyz.numel() // 3
        if xyz.numel() != 3 * n or phi.numel() != n or acc.numel() != 3 * n:
            raise ValueError("need xyz [n, 3], phi [n] and acc [3, n]")
        st = Stats()
        self._check(lib().ot_solve_points(self.h, n, _dev_ptr(xyz, f), _dev_ptr(phi, f), _dev_ptr(acc, f),
                                          C.byref(st), _stream(stream)))
        return st

    def export_point_list(self, i):
        n = C.c_int64(0)
        self._check(lib().ot_export_point_list(self.h, int(i), None, 0, C.byref(n)))
        ids = np.empty(n.value, np.int32)
        self._check(lib().ot_export_point_list(self.h, int(i), _np_ptr(ids), n.value, C.byref(n)))
        return ids

    def solve_abu(self, phi, acc, tol, fp64=False, npix=None, tau=None, stream=None, tol_tau=None):
        """Adaptive block update: phi, acc (and npix, tau when nside > 0) hold
        the previous step's solution and are updated in place where a block's
        corner cells moved by tol or more in acceleration (or, with columns,
        by tol_tau or more in the optical depth kappa N_p of a pixel).
        Returns (stats, updated [nb] int32)."""
        if self.params.nside and tol_tau is None:
            raise TypeError("solve_abu with columns needs tol_tau")
        import torch
        st = Stats()
        f = torch.float64 if fp64 else torch.float32
        upd = np.empty(self.nb, np.int32)
        fn = lib().ot_solve_abu64 if fp64 else lib().ot_solve_abu
        self._check(fn(self.h, _dev_ptr(phi, f), _dev_ptr(acc, f), _dev_ptr(npix, f), _dev_ptr(tau, f),
                       float(tol), float(tol_tau or 0.0), _np_ptr(upd), C.byref(st), _stream(stream)))
        return st, upd

    def export_raytable(self, stream=None):
        ne, npairs = C.c_int64(0), C.c_int64(0)
        self._check(lib().ot_export_raytable(self.h, C.byref(ne), C.byref(npairs), None, None, None,
                                             _stream(stream)))
        off, pix, w = np.empty(ne.value + 1, np.int64), np.empty(npairs.value, np.int32), np.empty(npairs.value)
        self._check(lib().ot_export_raytable(self.h, C.byref(ne), C.byref(npairs), _np_ptr(off), _np_ptr(pix),
                                             _np_ptr(w), _stream(stream)))
        return off, pix, w

    def ewald_prepare(self, cache_path=None, stream=None):
        """Build the Ewald table now; with cache_path read it from that file
        or write it there."""
        cp = os.fsencode(cache_path) if cache_path is not None else None
        self._check(lib().ot_ewald_prepare(self.h, cp, _stream(stream)))

    # ---- learned Ewald surrogate
    def mlp_train(self, stream=None, cache_path=None, **cfg):
        """Train, validate and accept or reject the surrogate (or read it from
        cache_path when that file matches); returns the report as a dict.
        Keyword arguments override ot_mlp_config_default."""
        c = MlpConfig()
        lib().ot_mlp_config_default(C.byref(c))
        for k, v in cfg.items():
            if k not in dict(MlpConfig._fields_):
                raise TypeError(f"unknown surrogate setting {k}")
            setattr(c, k, v)
        r = MlpReport()
        cp = os.fsencode(cache_path) if cache_path is not None else None
        self._check(lib().ot_mlp_train(self.h, C.byref(c), cp, C.byref(r), _stream(stream)))
        return r.as_dict()

    def mlp_get(self):
        p, n = np.empty(MLP_NPARAM, np.float32), np.empty(MLP_NNORM)
        self._check(lib().ot_mlp_get(self.h, _np_ptr(p), _np_ptr(n)))
        return p, n

    def mlp_set(self, params, norm, accept=True, stream=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        n = np.ascontiguousarray(norm, dtype=np.float64)
        if p.shape != (MLP_NPARAM,) or n.shape != (MLP_NNORM,):
            raise ValueError(f"params [{MLP_NPARAM}] and norm [{MLP_NNORM}] expected")
        self._check(lib().ot_mlp_set(self.h, _np_ptr(p), _np_ptr(n), int(bool(accept)), _stream(stream)))

    def mlp_grad(self, params, x, t, grad, stream=None):
        """Batch loss and gradient on the device; returns the loss."""
        import torch
        f = torch.float32
        loss = C.c_float(0.0)
        self._check(lib().ot_mlp_grad(self.h, _dev_ptr(params, f), int(x.shape[0]), _dev_ptr(x, f),
                                      _dev_ptr(t, f), _dev_ptr(grad, f), C.byref(loss), _stream(stream)))
        return loss.value

    def mlp_adam_step(self, params, m, v, x, t, lr, step, stream=None):
        """One training step in place on device tensors params, m, v (FP32
        [NPARAM]): gradient over x [batch, 3], t [batch, 10], then Adam with
        step size lr and update index step; returns the loss before it."""
        import torch
        f = torch.float32
        loss = C.c_float(0.0)
        self._check(lib().ot_mlp_adam_step(self.h, _dev_ptr(params, f), _dev_ptr(m, f), _dev_ptr(v, f),
                                           int(x.shape[0]), _dev_ptr(x, f), _dev_ptr(t, f), float(lr), int(step),
                                           C.byref(loss), _stream(stream)))
        return loss.value

    def mlp_grad_noalloc(self, params, x, t, grad, loss, stream=None):
        """The same batch gradient with no allocation (fixed library workspace,
        batch <= 1024); the loss goes to the device scalar loss [1].  Enqueues
        only: synchronise the stream before reading the outputs."""
        import torch
        f = torch.float32
        self._check(lib().ot_mlp_grad_noalloc(self.h, _dev_ptr(params, f), int(x.shape[0]), _dev_ptr(x, f),
                                              _dev_ptr(t, f), _dev_ptr(grad, f), _dev_ptr(loss, f),
                                              _stream(stream)))

    def ewald_points(self, method, d, out, stream=None):
        """Correction (phi_c, A_c, second derivatives xx yy zz xy xz yz) at
        device offsets d [n, 3] into out [n, 10]."""
        import torch
        f = torch.float64
        self._check(lib().ot_ewald_points(self.h, EWALD[method], int(d.shape[0]), _dev_ptr(d, f),
                                          _dev_ptr(out, f), _stream(stream)))

    # ---- inspection
    def column_bins(self, d, h, row, stream=None):
        """Node-ray table rows the column walk uses for nodes of size h [n]
        at device offsets d [n, 3] (cell minus node) into row [n] (int32)."""
        import torch
        self._check(lib().ot_column_bins(self.h, int(d.shape[0]), _dev_ptr(d, torch.float64),
                                         _dev_ptr(h, torch.float64), _dev_ptr(row, torch.int32), _stream(stream)))

    def export_topology(self):
        na = self.na
        out = dict(alev=np.empty(na, np.int32), acoord=np.empty((na, 3), np.int32),
                   aleaf=np.empty(na, np.int64), achild=np.empty((na, 8), np.int64),
                   akey=np.empty(na, np.uint64))
        self._check(lib().ot_export_topology(self.h, *(_np_ptr(out[k]) for k in
                                                       ("alev", "acoord", "aleaf", "achild", "akey"))))
        return out

    def export_moments(self):
        nn = self.na + 584 * self.nb
        M, com = np.empty(nn), np.empty((nn, 3))
        self._check(lib().ot_export_moments(self.h, _np_ptr(M), _np_ptr(com)))
        return M, com

    def export_list(self, b):
        n = C.c_int64(0)
        self._check(lib().ot_export_list(self.h, int(b), None, 0, C.byref(n)))
        ids = np.empty(n.value, np.int32)
        self._check(lib().ot_export_list(self.h, int(b), _np_ptr(ids), n.value, C.byref(n)))
        return ids

    def export_ewald_table(self):
        n = self.params.ewald_n
        tab = np.empty((n, n, n, 10))
        self._check(lib().ot_export_ewald_table(self.h, _np_ptr(tab)))
        return tab


def run(grid, fp64=False, stream=None, columns=False, **kw):
    """Convenience: build + solve on cuda:0.  Returns (phi, acc [3, n], stats,
    solver), plus (npix [nb, N_pix, 512], tau) when the solver has nside > 0."""
    import torch
    s = Solver.for_grid(grid, **kw)
    rho = torch.from_numpy(np.ascontiguousarray(grid.rho.reshape(-1))).to("cuda")
    s.build(rho, stream)
    dt = torch.float64 if fp64 else torch.float32
    phi = torch.empty(grid.nb * 512, dtype=dt, device="cuda")
    acc = torch.empty(3 * grid.nb * 512, dtype=dt, device="cuda")
    npix = tau = None
    if s.params.nside:
        npx = 12 * s.params.nside ** 2
        npix = torch.empty(grid.nb * npx * 512, dtype=dt, device="cuda")
        tau = torch.empty(grid.nb * 512, dtype=dt, device="cuda")
    st = (s.solve64 if fp64 else s.solve)(phi, acc, npix, tau, stream)
    if s.params.nside:
        return phi, acc.view(3, -1), st, s, npix.view(grid.nb, -1, 512), tau
    return phi, acc.view(3, -1), st, s
