"""FP64 CPU oracle for the OctTree solver (Wuensch et al. 2018).

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the benchmark's CPU
baseline are the only callers.  The C sources in this directory are plain,
slow and independent of the GPU library (no shared code, headers or tables).
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["octoracle.c", "ewald.c", "columns.c", "mlp.c", "mlpwalk.c"]

ERRORS = {1: "bad level/coord", 2: "duplicate block", 3: "overlapping blocks",
          4: "hole in the block tiling", 5: "bad density", 6: "unsupported BCs",
          7: "list_group must be 0, 4 or 8"}


def build(force=True, src_dir=HERE, out=LIB, extra=()):
    """Compile liboracle.so with gcc (FP64, no FMA contraction, OpenMP).
    src_dir / out / extra flags serve tests that build a copy of the sources."""
    if not force and os.path.exists(out):
        return out
    srcs = [os.path.join(src_dir, s) for s in SOURCES]
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", *extra, "-o", tmp] + srcs + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


class Params(C.Structure):
    _fields_ = [("nroot", C.c_int32 * 3), ("bc", C.c_int32 * 3), ("root_size", C.c_double),
                ("origin", C.c_double * 3), ("G", C.c_double), ("theta", C.c_double),
                ("eta_sb", C.c_double), ("a_lim", C.c_double), ("theta_pix", C.c_double),
                ("mac", C.c_int32), ("ewald", C.c_int32), ("ew_n", C.c_int32),
                ("ew_rcut2", C.c_int32), ("ew_fcut2", C.c_int32), ("pad_", C.c_int32),
                ("ew_alpha", C.c_double), ("nside", C.c_int32), ("il_ntheta", C.c_int32),
                ("il_nphi", C.c_int32), ("il_npsi", C.c_int32), ("il_nr", C.c_int32),
                ("il_nazi", C.c_int32), ("kappa", C.c_double), ("max_dist", C.c_double),
                ("psi_max", C.c_double), ("mlp_reach", C.c_double), ("list_group", C.c_int32)]

# defaults of the column machinery (App. B: tr_ilNTheta 25, tr_ilNPhi 50,
# tr_ilNNS 25, tr_ilNR 50; azimuths and psi_max are this build's readings)
COLUMN_DEFAULTS = dict(il_ntheta=25, il_nphi=50, il_npsi=25, il_nr=50, il_nazi=100, psi_max=0.98)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _load(LIB)
    return _lib


@contextlib.contextmanager
def using_library(path):
    """Run the oracle from another build of its sources (tests that plant a
    mistake in a copy of them and check that a pin catches it)."""
    global _lib
    old = lib()
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = old


def _load(path):
    L = C.CDLL(path)
    vp, i64, dp = C.c_void_p, C.c_int64, C.POINTER(C.c_double)
    L.or_tree_new.restype = vp
    L.or_tree_new.argtypes = [C.POINTER(Params), i64, vp, vp, vp, C.POINTER(C.c_int)]
    L.or_tree_free.argtypes = [vp]
    L.or_tree_na.restype = i64
    L.or_tree_na.argtypes = [vp]
    L.or_tree_nn.restype = i64
    L.or_tree_nn.argtypes = [vp]
    L.or_tree_export.argtypes = [vp] + [vp] * 7
    L.or_tree_mpe_export.argtypes = [vp, vp, vp]
    L.or_walk_group_abu.argtypes = [vp, vp, vp, C.c_double, vp, C.c_double, vp, vp, vp]
    L.or_block_list.restype = i64
    L.or_block_list.argtypes = [vp, i64, vp, i64]
    L.or_group_list.restype = i64
    L.or_group_list.argtypes = [vp, i64, C.c_int, vp, i64]
    L.or_walk_group.argtypes = [vp, vp, vp, vp]
    L.or_walk_group_blocks.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
    L.or_raymarch.argtypes = [vp, vp, i64, i64, i64, vp]
    L.or_healpix_vec2pix.restype = i64
    L.or_healpix_vec2pix.argtypes = [i64, C.c_double, C.c_double, C.c_double]
    L.or_healpix_pix2ang.argtypes = [i64, i64, vp]
    L.or_raytable_entries.argtypes = [C.c_int] * 3 + [C.c_double, i64, vp, vp, vp]
    L.or_raytable_export.restype = i64
    L.or_raytable_export.argtypes = [C.c_int] * 6 + [C.c_double, vp, vp, vp]
    L.or_walk_percell.argtypes = [vp, i64, vp, vp, vp, vp]
    L.or_point_list.restype = i64
    L.or_point_list.argtypes = [vp, vp, vp, i64]
    L.or_walk_points.argtypes = [vp, i64, vp, vp, vp, vp]
    L.or_direct.argtypes = [vp, i64, vp, vp, vp]
    L.or_morton.restype = C.c_uint64
    L.or_morton.argtypes = [C.c_uint64] * 3
    L.or_ewald_eval.argtypes = [C.c_int, vp, C.c_double, C.c_int, C.c_int, C.c_int, i64, vp, vp]
    L.or_ewald_table.argtypes = [C.c_int, vp, C.c_double, C.c_int, C.c_int, C.c_int, vp]
    L.or_ewald_table_lookup.argtypes = [C.c_int, vp, C.c_int, vp, i64, vp, vp]
    L.or_itilde.argtypes = [C.c_double, C.c_double, C.c_double, vp]
    L.or_kfuncs.argtypes = [C.c_int, C.c_double, C.c_double, vp]
    L.or_mlp_nparam.restype = C.c_int
    L.or_mlp_forward.argtypes = [vp, i64, vp, vp]
    L.or_mlp_grad.restype = C.c_double
    L.or_mlp_grad.argtypes = [vp, i64, vp, vp, vp]
    L.or_walk_group_mlp.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
    L.or_mlp_group_level.restype = C.c_int
    L.or_mlp_group_level.argtypes = [vp, i64]
    L.or_adam_update.argtypes = [vp, vp, vp, vp, i64, C.c_double, i64]
    L.or_mlp_adam.restype = C.c_double
    L.or_mlp_adam.argtypes = [vp, vp, vp, i64, vp, vp, C.c_double, i64]
    return L


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


BC_ISO, BC_3P, BC_2P1I, BC_1P2I = 0, 1, 2, 3


def bctype(bc):
    bc = tuple(int(b) for b in bc)
    if bc == (0, 0, 0):
        return BC_ISO
    if bc == (1, 1, 1):
        return BC_3P
    if bc == (1, 1, 0):
        return BC_2P1I
    if bc == (1, 0, 0):
        return BC_1P2I
    raise ValueError("unsupported boundary combination")


def make_params(grid, theta=0.5, eta_sb=1.2, mac="bh", a_lim=0.0, theta_pix=0.0, G=1.0,
                ewald="exact", ew_n=64, ew_alpha=0.0, ew_rcut2=0, ew_fcut2=0, bc=None,
                nside=0, kappa=1.0, max_dist=1e99, mlp_reach=1.0, list_group=8, **cols):
    p = Params()
    for k in range(3):
        p.nroot[k] = int(grid.nroot[k])
        p.bc[k] = int((bc if bc is not None else grid.bc)[k])
        p.origin[k] = float(grid.origin[k])
    p.root_size = float(grid.root_size)
    p.G, p.theta, p.eta_sb, p.a_lim, p.theta_pix = G, theta, eta_sb, a_lim, theta_pix
    p.mac = {"bh": 0, "ape": 1, "mpe": 2}[mac]
    p.ewald = {"exact": 0, "table": 1}[ewald]
    p.ew_n, p.ew_alpha, p.ew_rcut2, p.ew_fcut2 = ew_n, ew_alpha, ew_rcut2, ew_fcut2
    p.nside, p.kappa, p.max_dist = nside, kappa, max_dist
    p.mlp_reach = mlp_reach
    p.list_group = list_group
    c = dict(COLUMN_DEFAULTS, **cols)
    p.il_ntheta, p.il_nphi, p.il_npsi = c["il_ntheta"], c["il_nphi"], c["il_npsi"]
    p.il_nr, p.il_nazi, p.psi_max = c["il_nr"], c["il_nazi"], c["psi_max"]
    if nside and theta_pix <= 0:
        p.theta_pix = 1.0 / nside  # theta_lim ~ sqrt(Omega_pix): 1, 0.5, 0.25 for Nside 1, 2, 4
    return p


class Tree:
    """Oracle tree over a workloads.Grid (FP64 moments, walks, direct sums)."""

    def __init__(self, grid, **kw):
        self.grid = grid
        self.params = make_params(grid, **kw)
        self.level = np.ascontiguousarray(grid.level, dtype=np.int32)
        self.coord = np.ascontiguousarray(grid.coord, dtype=np.int32)
        self.rho = np.ascontiguousarray(grid.rho, dtype=np.float64)
        err = C.c_int(0)
        self.h = lib().or_tree_new(C.byref(self.params), grid.nb, _ptr(self.level),
                                   _ptr(self.coord), _ptr(self.rho), C.byref(err))
        if not self.h:
            raise ValueError(f"oracle rejected the grid: {ERRORS.get(err.value, err.value)}")
        self.nb = grid.nb
        self.na = lib().or_tree_na(self.h)
        self.nn = lib().or_tree_nn(self.h)

    def __del__(self):
        h, self.h = getattr(self, "h", None), None
        # at interpreter exit the module's globals may already be gone (the
        # process frees the memory then)
        if h and callable(lib):
            lib().or_tree_free(h)

    def export(self):
        na, nn = self.na, self.nn
        out = dict(alev=np.empty(na, np.int32), acoord=np.empty((na, 3), np.int32),
                   aleaf=np.empty(na, np.int64), achild=np.empty((na, 8), np.int64),
                   akey=np.empty(na, np.uint64), M=np.empty(nn), com=np.empty((nn, 3)))
        lib().or_tree_export(self.h, *(_ptr(out[k]) for k in
                                       ("alev", "acoord", "aleaf", "achild", "akey", "M", "com")))
        return out

    def mpe_moments(self):
        """B_2, B_3 of the na + 72 nb non-cell nodes (mac="mpe" only)."""
        n = self.na + 72 * self.nb
        B2, B3 = np.empty(n), np.empty(n)
        lib().or_tree_mpe_export(self.h, _ptr(B2), _ptr(B3))
        return B2, B3

    def walk_abu(self, prev_phi, prev_acc, tol, prev_npix=None, prev_tau=None, tol_tau=None):
        """Adaptive block update (Sec. 2.2.6): returns phi [nb*512], acc [3, nb*512]
        and updated [nb] (1 where the block was evaluated).  With prev_npix
        [nb, Npix, 512], prev_tau [nb*512] and tol_tau (trees with nside > 0)
        a block is also evaluated when at a corner the optical depth kappa N_p
        of a direction moved by tol_tau or more, and npix and tau are returned
        too: the group walk's columns for the updated blocks, the previous
        ones for the others."""
        n = 512 * self.nb
        pp = np.ascontiguousarray(prev_phi, dtype=np.float64).reshape(n)
        pa = np.ascontiguousarray(prev_acc, dtype=np.float64).reshape(3, n)
        phi, acc, upd = np.empty(n), np.empty((3, n)), np.empty(self.nb, np.int32)
        pn = None
        if prev_npix is not None:
            if tol_tau is None:
                raise TypeError("walk_abu with columns needs tol_tau")
            pn = np.ascontiguousarray(prev_npix, dtype=np.float64).reshape(-1)
            assert pn.size == n * 12 * self.params.nside ** 2
        lib().or_walk_group_abu(self.h, _ptr(pp), _ptr(pa), float(tol), _ptr(pn),
                                float(tol_tau if tol_tau is not None else 0.0), _ptr(phi), _ptr(acc), _ptr(upd))
        if prev_npix is None:
            return phi, acc, upd
        npix = np.array(prev_npix, dtype=np.float64).reshape(self.nb, -1, 512)
        tau = np.array(prev_tau, dtype=np.float64).reshape(self.nb, 512)
        sel = np.nonzero(upd)[0]
        if sel.size:
            _, _, _, nps, ts = self.walk_group(sel, columns=True)
            npix[sel] = nps
            tau[sel] = ts.reshape(sel.size, 512)
        return phi, acc, upd, npix, tau.reshape(n)

    def block_list(self, lb):
        n = lib().or_block_list(self.h, lb, None, 0)
        ids = np.empty(n, np.int64)
        lib().or_block_list(self.h, lb, _ptr(ids), n)
        return ids

    def octant_list(self, lb, so):
        """Interaction list of octant so (bit a: upper half of axis a) of
        leaf block lb, the walk target of its 4^3 cells with list_group 4."""
        if not 0 <= so < 8:
            raise ValueError("octant must be in [0, 8)")
        n = lib().or_group_list(self.h, lb, so, None, 0)
        ids = np.empty(n, np.int64)
        lib().or_group_list(self.h, lb, so, _ptr(ids), n)
        return ids

    def walk_group(self, blocks=None, columns=False):
        """Group walk over all leaf blocks or a subset.  Returns phi [n*512],
        acc [3, n*512], nint [n] (the lengths of the lists the block's cells
        use: one, or eight with list_group 4); with columns also npix
        [n, Npix, 512] and tau [n*512]."""
        sel = np.arange(self.nb) if blocks is None else np.asarray(blocks)
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        nc = 512 * sel.size
        phi, acc, nint = np.empty(nc), np.empty((3, nc)), np.empty(sel.size, np.int64)
        npix = tau = None
        if columns:
            npx = 12 * self.params.nside ** 2
            npix, tau = np.empty((sel.size, npx, 512)), np.empty(nc)
        lib().or_walk_group_blocks(self.h, sel.size, _ptr(sel), _ptr(phi), _ptr(acc), _ptr(npix),
                                   _ptr(tau), _ptr(nint))
        if columns:
            return phi, acc, nint, npix, tau
        return phi, acc, nint

    def walk_group_mlp(self, params, norm, blocks=None, columns=False):
        """Group walk with the learned surrogate (FP64 network) in place of
        the Ewald table: per (group of cells, listed node) the network's ten
        channels at the group centre, a first-order Taylor step to each cell.
        Returns as walk_group; the column maps (columns=True) are the plain
        walk's."""
        sel = np.arange(self.nb) if blocks is None else np.asarray(blocks)
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        p = np.ascontiguousarray(params, dtype=np.float64)
        nm = np.ascontiguousarray(norm, dtype=np.float64)
        if p.shape != (MLP_NPARAM,) or nm.shape != (3 + 2 * MLP_NOUT,):
            raise ValueError("surrogate parameters or scaling of the wrong size")
        nc = 512 * sel.size
        phi, acc, nint = np.empty(nc), np.empty((3, nc)), np.empty(sel.size, np.int64)
        lib().or_walk_group_mlp(self.h, _ptr(p), _ptr(nm), sel.size, _ptr(sel), _ptr(phi), _ptr(acc), _ptr(nint))
        if columns:
            _, _, _, npix, tau = self.walk_group(sel, columns=True)
            return phi, acc, nint, npix, tau
        return phi, acc, nint

    def mlp_group_level(self, lb):
        """Side 2^gl of the surrogate walk's cell groups in leaf block lb."""
        return int(lib().or_mlp_group_level(self.h, int(lb)))

    def raymarch(self, target, nside, nside_f=16):
        """Reference column map of one cell: mean over the Nside_f pixel-centre
        rays in each coarse pixel of exact integrals of rho through the cells."""
        out = np.empty(12 * nside * nside)
        lib().or_raymarch(self.h, _ptr(self.rho), int(target), int(nside), int(nside_f), _ptr(out))
        return out

    def walk_percell(self, targets):
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        phi, acc, nint = np.empty(tg.size), np.empty((3, tg.size)), np.empty(tg.size, np.int64)
        lib().or_walk_percell(self.h, tg.size, _ptr(tg), _ptr(phi), _ptr(acc), _ptr(nint))
        return phi, acc, nint

    def point_list(self, x):
        """Interaction list of one target point (Sec. 2.1, MAC at the point)."""
        xp = np.ascontiguousarray(x, dtype=np.float64).reshape(3)
        n = lib().or_point_list(self.h, _ptr(xp), None, 0)
        ids = np.empty(n, np.int64)
        lib().or_point_list(self.h, _ptr(xp), _ptr(ids), n)
        return ids

    def walk_points(self, xyz):
        """Potential [n], acceleration [3, n] and list lengths [n] at arbitrary
        target points xyz [n, 3], each walked with its own list."""
        p = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        n = p.shape[0]
        phi, acc, nint = np.empty(n), np.empty((3, n)), np.empty(n, np.int64)
        lib().or_walk_points(self.h, n, _ptr(p), _ptr(phi), _ptr(acc), _ptr(nint))
        return phi, acc, nint

    def direct(self, targets=None):
        if targets is None:
            targets = np.arange(512 * self.nb)
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        phi, acc = np.empty(tg.size), np.empty((3, tg.size))
        lib().or_direct(self.h, tg.size, _ptr(tg), _ptr(phi), _ptr(acc))
        return phi, acc


def morton(x, y, z):
    return int(lib().or_morton(int(x), int(y), int(z)))


def ewald_eval(bc, box, d, alpha=0.0, rcut2=0, fcut2=10, correction=False):
    """phi, A (3), H (6: xx yy zz xy xz yz) of the Ewald series at offsets d [n, 3]."""
    bt = bctype(bc)
    if rcut2 <= 0:
        rcut2 = 15 if bt == BC_3P else 10
    box = np.ascontiguousarray(box, dtype=np.float64)
    d = np.ascontiguousarray(np.atleast_2d(d), dtype=np.float64)
    out = np.empty((d.shape[0], 10))
    a = alpha if alpha > 0 else 2.0 / box[0]
    lib().or_ewald_eval(bt, _ptr(box), a, rcut2, fcut2, int(correction), d.shape[0], _ptr(d), _ptr(out))
    return out


def ewald_table(bc, box, n=64, alpha=0.0, rcut2=0, fcut2=10):
    bt = bctype(bc)
    if rcut2 <= 0:
        rcut2 = 15 if bt == BC_3P else 10
    box = np.ascontiguousarray(box, dtype=np.float64)
    out = np.empty((n, n, n, 10))
    a = alpha if alpha > 0 else 2.0 / box[0]
    lib().or_ewald_table(bt, _ptr(box), a, rcut2, fcut2, n, _ptr(out))
    return out


def ewald_table_lookup(bc, box, table, d):
    bt = bctype(bc)
    box = np.ascontiguousarray(box, dtype=np.float64)
    table = np.ascontiguousarray(table, dtype=np.float64)
    d = np.ascontiguousarray(np.atleast_2d(d), dtype=np.float64)
    out = np.empty((d.shape[0], 4))
    lib().or_ewald_table_lookup(bt, _ptr(box), table.shape[0], _ptr(table), d.shape[0], _ptr(d), _ptr(out))
    return out


def kfuncs(l, eta, zeta):
    """1P2I integrals K(l, eta), M(l, eta) = -dK/deta, dM/deta and M/eta
    (its limit dM/deta at eta = 0); l = 0: the regularised closed forms."""
    out = np.empty(4)
    lib().or_kfuncs(int(l), float(eta), float(zeta), _ptr(out))
    return out


def itilde(s, zeta, gam):
    """2P1I integral Itilde(s, gamma) and its first two gamma-derivatives
    (s = 0: the regularised l = 0 term I(0, 0, gamma))."""
    out = np.empty(3)
    lib().or_itilde(float(s), float(zeta), float(gam), _ptr(out))
    return out


def vec2pix(nside, v):
    v = np.atleast_2d(v)
    return np.array([lib().or_healpix_vec2pix(int(nside), *map(float, x)) for x in v], np.int64)


def pix2ang(nside, p):
    out = np.empty(2)
    lib().or_healpix_pix2ang(int(nside), int(p), _ptr(out))
    return out  # z, phi


def raytable_entries(d, h, il_ntheta=25, il_nphi=50, il_npsi=25, psi_max=0.98):
    """Node-ray table entry (theta, phi, psi bin) the walk uses for nodes of
    size h [n] at offsets d [n, 3] = target cell minus node; -1 for d = 0."""
    d = np.ascontiguousarray(d, np.float64)
    h = np.ascontiguousarray(h, np.float64)
    out = np.empty(d.shape[0], np.int64)
    lib().or_raytable_entries(int(il_ntheta), int(il_nphi), int(il_npsi), float(psi_max), d.shape[0],
                              _ptr(d), _ptr(h), _ptr(out))
    return out


def raytable(nside, il_ntheta=25, il_nphi=50, il_npsi=25, il_nr=50, il_nazi=100, psi_max=0.98):
    """Node-ray intersection table (compressed rows): off [ne+1], pix [n], w [n]."""
    args = [int(nside), il_ntheta, il_nphi, il_npsi, il_nr, il_nazi, float(psi_max)]
    n = lib().or_raytable_export(*args, None, None, None)
    ne = il_ntheta * il_nphi * il_npsi
    off, pix, w = np.empty(ne + 1, np.int64), np.empty(n, np.int32), np.empty(n)
    lib().or_raytable_export(*args, _ptr(off), _ptr(pix), _ptr(w))
    return off, pix, w


# ---------------------------------------------------------------- MLP
MLP_NPARAM, MLP_NOUT = 9226, 10  # 3 -> 64 -> 64 -> 64 -> 10


def mlp_forward(params, x):
    """FP64 forward of the surrogate network: x [B, 3] -> y [B, 10]."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    y = np.empty((x.shape[0], MLP_NOUT))
    lib().or_mlp_forward(_ptr(p), x.shape[0], _ptr(x), _ptr(y))
    return y


def mlp_grad(params, x, t):
    """Batch MSE loss and its gradient (FP64 back-propagation)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    t = np.ascontiguousarray(np.atleast_2d(t), dtype=np.float64)
    g = np.empty(MLP_NPARAM)
    loss = lib().or_mlp_grad(_ptr(p), x.shape[0], _ptr(x), _ptr(t), _ptr(g))
    return loss, g


def adam_update(p, g, m, v, lr, step):
    """One Adam step on copies of p, m, v with gradient g: returns (p, m, v)."""
    p, m, v = (np.array(a, dtype=np.float64) for a in (p, m, v))
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().or_adam_update(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.size, float(lr), int(step))
    return p, m, v


def mlp_adam(params, m, v, x, t, lr, step):
    """Batch gradient + one Adam step (FP64): returns (loss, params, m, v)."""
    p, m, v = (np.array(a, dtype=np.float64) for a in (params, m, v))
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    t = np.ascontiguousarray(np.atleast_2d(t), dtype=np.float64)
    loss = lib().or_mlp_adam(_ptr(p), _ptr(m), _ptr(v), x.shape[0], _ptr(x), _ptr(t), float(lr), int(step))
    return loss, p, m, v
