"""Seeded synthetic AMR workloads (density on 8^3-cell blocks).

This module only produces inputs: block layouts (level, integer coordinate per
leaf block), densities at cell centres, and random numbers. It holds none of
the solver's arithmetic (no tree, no gravity, no columns), so both the oracle
and the GPU library can be fed from it.

Conventions (shared input format, the paper's block-structured grid, Sec. 2):
  * root blocks are cubes of edge ``root_size`` arranged ``nroot[0] x nroot[1] x
    nroot[2]``; a block at level l (root = 1) has edge root_size / 2**(l-1) and
    8 cells per axis;
  * ``coord[b]`` is the integer position of block b at its own level
    (0 <= coord < nroot * 2**(l-1));
  * ``rho[b, k, j, i]`` is the density of cell (i, j, k) of block b, so the
    flat cell index inside a block is i + 8 j + 64 k (x fastest).
"""
from __future__ import annotations

import dataclasses
import numpy as np

BS = 8  # cells per block edge


@dataclasses.dataclass
class Grid:
    nroot: tuple
    root_size: float
    origin: tuple
    level: np.ndarray      # int32 [nb]
    coord: np.ndarray      # int32 [nb, 3]
    rho: np.ndarray        # float64 [nb, 8, 8, 8]
    bc: tuple = (0, 0, 0)  # 0 isolated, 1 periodic, per axis
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nb(self):
        return int(self.level.shape[0])

    @property
    def ncells(self):
        return self.nb * BS ** 3

    def box(self):
        return tuple(self.nroot[k] * self.root_size for k in range(3))


def block_edge(root_size, level):
    return root_size / float(2 ** (int(level) - 1))


def cell_centres(root_size, origin, level, coord):
    """Cell-centre coordinates [nb, 8, 8, 8, 3] (same index order as rho)."""
    level = np.asarray(level)
    coord = np.asarray(coord, dtype=np.float64)
    h = root_size / np.power(2.0, level.astype(np.float64) + 2.0)  # edge / 8
    idx = np.arange(BS, dtype=np.float64) + 0.5
    out = np.empty((level.shape[0], BS, BS, BS, 3))
    for ax in range(3):
        base = origin[ax] + 8.0 * coord[:, ax] * h
        shape = [1, 1, 1]
        shape[2 - ax] = BS  # x varies along the last axis
        off = idx.reshape(shape)
        out[..., ax] = base[:, None, None, None] + off[None] * h[:, None, None, None]
    return out


def uniform_blocks(ncell_axis, nroot=(1, 1, 1)):
    """Leaf blocks of a uniform grid with ``ncell_axis`` cells per root edge."""
    nblk = ncell_axis // BS
    lev = int(round(np.log2(nblk))) + 1
    assert 2 ** (lev - 1) * BS == ncell_axis
    nx, ny, nz = (nroot[k] * nblk for k in range(3))
    cz, cy, cx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coord = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1).astype(np.int32)
    level = np.full(coord.shape[0], lev, dtype=np.int32)
    return level, coord


def scatter_uniform(field, level, coord):
    """Cut a global [Nz, Ny, Nx] array into [nb, 8, 8, 8] blocks."""
    nb = level.shape[0]
    out = np.empty((nb, BS, BS, BS), dtype=np.float64)
    for b in range(nb):
        x0, y0, z0 = (int(c) * BS for c in coord[b])
        out[b] = field[z0:z0 + BS, y0:y0 + BS, x0:x0 + BS]
    return out


# ---------------------------------------------------------------- fields
def gaussian_field_k4(n, seed, box_shape=None):
    """Zero-mean unit-variance Gaussian random field with P(k) ~ k^-4.

    Real white noise -> rfftn -> multiply by |k|^-2 (k in units of 2 pi / L
    over the full grid, k = 0 zeroed) -> irfftn -> standardise.  Array order
    [z, y, x].
    """
    shape = box_shape or (n, n, n)
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    f = np.fft.rfftn(white)
    kz = np.fft.fftfreq(shape[0]) * shape[0]
    ky = np.fft.fftfreq(shape[1]) * shape[1]
    kx = np.fft.rfftfreq(shape[2]) * shape[2]
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = 1.0 / k2[nz]
    f *= amp
    g = np.fft.irfftn(f, s=shape, axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    return g


def c1_sphere(seed=1, noise=True, rho_bg=1e-2, radius=0.3, n=32):
    """Uniform sphere (rho = 1, radius 0.3 about the box centre) in a unit box,
    lognormal background of mean ``rho_bg`` with 10% scatter."""
    level, coord = uniform_blocks(n)
    xc = cell_centres(1.0, (0.0, 0.0, 0.0), level, coord)
    r2 = ((xc - 0.5) ** 2).sum(-1)
    inside = r2 < radius * radius
    if noise:
        rng = np.random.default_rng(seed)
        g = rng.standard_normal(inside.shape)
        bg = rho_bg * np.exp(0.1 * g - 0.005)
    else:
        bg = np.full(inside.shape, rho_bg)
    rho = np.where(inside, 1.0, bg)
    return Grid((1, 1, 1), 1.0, (0.0, 0.0, 0.0), level, coord, rho, (0, 0, 0),
                name=f"sphere{n}", meta={"seed": seed, "noise": noise})


def c2_lognormal(n=128, seed=2, sigma=1.5, bc=(0, 0, 0)):
    """Lognormal density exp(sigma*delta - sigma^2/2) on a uniform n^3 grid,
    delta a P(k) ~ k^-4 Gaussian random field (mean density 1)."""
    level, coord = uniform_blocks(n)
    delta = gaussian_field_k4(n, seed)
    field = np.exp(sigma * delta - 0.5 * sigma * sigma)
    rho = scatter_uniform(field, level, coord)
    return Grid((1, 1, 1), 1.0, (0.0, 0.0, 0.0), level, coord, rho, tuple(bc),
                name=f"lognormal{n}", meta={"seed": seed, "sigma": sigma})


def filament_1p2i(n=64, seed=13, H=0.1, amp=0.3, noise=0.5):
    """A filament along the periodic x axis of a 1 x 2 x 2 box (1P2I): the
    isothermal-cylinder profile rho = 1/(1 + r^2/(8 H^2))^2 about the line
    y = z = 1, modulated by 1 + amp cos(2 pi x) and seeded lognormal cell noise
    (sigma ``noise``), n cells per root edge (n x 2n x 2n cells)."""
    nroot = (1, 2, 2)
    level, coord = uniform_blocks(n, nroot)
    xc = cell_centres(1.0, (0.0, 0.0, 0.0), level, coord)
    r2 = (xc[..., 1] - 1.0) ** 2 + (xc[..., 2] - 1.0) ** 2
    rho = (1.0 + amp * np.cos(2 * np.pi * xc[..., 0])) / (1.0 + r2 / (8 * H * H)) ** 2
    rng = np.random.default_rng(seed)
    rho = rho * rng.lognormal(-0.5 * noise * noise, noise, rho.shape)
    return Grid(nroot, 1.0, (0.0, 0.0, 0.0), level, coord, rho, (1, 0, 0),
                name=f"filament{n}", meta={"seed": seed, "H": H})


def target_points(grid, n, seed=23):
    """Seeded target points [m, 3] inside the domain of ``grid`` (sink
    particles, say): n uniform points, then the domain's lower corner, the
    point one ulp inside its upper corner, the centres of the first cell of
    the first and the last block, and a corner shared by eight cells of the
    first block (a node centre)."""
    rng = np.random.default_rng(seed)
    org = np.asarray(grid.origin, np.float64)
    L = np.asarray(grid.nroot, np.float64) * grid.root_size
    pts = [org + rng.random((n, 3)) * L, org[None], np.nextafter(org + L, org)[None]]
    xc = cell_centres(grid.root_size, grid.origin, grid.level, grid.coord)
    pts += [xc[0, 0, 0, 0][None], xc[-1, 0, 0, 0][None]]
    h = grid.root_size / 2.0 ** (int(grid.level[0]) + 2)
    pts.append((org + 8 * h * np.asarray(grid.coord[0], np.float64) + 4 * h)[None])
    return np.concatenate(pts)


def iso_cylinder(n=32, r0=0.25, rcyl=0.45, amb=1.0 / 2500.0, sub=8):
    """Isothermal cylinder in hydrostatic equilibrium (Sec. 3.1.4): the
    profile rho0 / (1 + R^2 / r0^2)^2 (rho0 = 1) about the line y = z = 0.5 of
    a 2 x 1 x 1 box (roots 2 x 1 x 1, x periodic, y and z isolated), cut off
    at R = rcyl and embedded in an ambient medium of ``amb`` times the edge
    density (the paper's sound-speed ratio 0.2 / 10 squared).  Each cell holds
    the mean of the profile over ``sub`` x ``sub`` points of its (y, z)
    square (the profile does not depend on x), so the cells' masses follow
    the continuous profile across its edge.  n cells per root edge
    (2n x n x n cells)."""
    nroot = (2, 1, 1)
    level, coord = uniform_blocks(n, nroot)
    h = 1.0 / n
    xc = cell_centres(1.0, (0.0, 0.0, 0.0), level, coord)
    off = (np.arange(sub) + 0.5) / sub - 0.5
    edge = 1.0 / (1.0 + rcyl * rcyl / (r0 * r0)) ** 2
    rho = np.zeros(xc.shape[:-1])
    for oy in off:
        for oz in off:
            r2 = (xc[..., 1] + oy * h - 0.5) ** 2 + (xc[..., 2] + oz * h - 0.5) ** 2
            rho += np.where(r2 <= rcyl * rcyl, 1.0 / (1.0 + r2 / (r0 * r0)) ** 2, amb * edge)
    return Grid(nroot, 1.0, (0.0, 0.0, 0.0), level, coord, rho / (sub * sub), (1, 0, 0),
                name=f"iso_cylinder{n}", meta={"r0": r0, "rcyl": rcyl, "amb": amb})


# ---------------------------------------------------------------- AMR
def _key(l, c):
    return (int(l), int(c[0]), int(c[1]), int(c[2]))


def _leaf_covering(leaves, l, c, nroot, bc):
    """Leaf (level, coord) containing level-l block position c, or None if c is
    outside an isolated boundary.  Periodic axes wrap."""
    c = list(c)
    for ax in range(3):
        nmax = nroot[ax] * 2 ** (l - 1)
        if c[ax] < 0 or c[ax] >= nmax:
            if bc[ax]:
                c[ax] %= nmax
            else:
                return None
    for ll in range(l, 0, -1):
        sh = l - ll
        key = (ll, c[0] >> sh, c[1] >> sh, c[2] >> sh)
        if key in leaves:
            return key
    return None


def amr_blocks(density, nroot, root_size, base_level, max_level, thresh, bc=(0, 0, 0)):
    """Block-structured AMR: refine a leaf whose maximum cell-centre density
    exceeds ``thresh`` (up to ``max_level``), then enforce 2:1 balance across
    faces, edges and corners.  ``density(x, y, z)`` is vectorised."""
    origin = (0.0, 0.0, 0.0)
    leaves = set()
    n = [nroot[k] * 2 ** (base_level - 1) for k in range(3)]
    for cz in range(n[2]):
        for cy in range(n[1]):
            for cx in range(n[0]):
                leaves.add((base_level, cx, cy, cz))

    def maxrho(keys):
        lv = np.array([k[0] for k in keys], dtype=np.int32)
        cc = np.array([k[1:] for k in keys], dtype=np.int32)
        xc = cell_centres(root_size, origin, lv, cc)
        r = density(xc[..., 0], xc[..., 1], xc[..., 2])
        return r.reshape(len(keys), -1).max(axis=1)

    for lev in range(base_level, max_level):
        cand = sorted(k for k in leaves if k[0] == lev)
        if not cand:
            break
        mr = np.concatenate([maxrho(cand[i:i + 4096]) for i in range(0, len(cand), 4096)])
        for k, m in zip(cand, mr):
            if m > thresh:
                _refine(leaves, k)
        _balance(leaves, nroot, bc)
    keys = sorted(leaves, key=lambda k: (k[0], k[3], k[2], k[1]))
    level = np.array([k[0] for k in keys], dtype=np.int32)
    coord = np.array([k[1:] for k in keys], dtype=np.int32)
    return level, coord


def _refine(leaves, k):
    leaves.discard(k)
    l, cx, cy, cz = k
    for o in range(8):
        leaves.add((l + 1, 2 * cx + (o & 1), 2 * cy + ((o >> 1) & 1), 2 * cz + ((o >> 2) & 1)))


def _balance(leaves, nroot, bc):
    changed = True
    while changed:
        changed = False
        for k in sorted(leaves, key=lambda t: -t[0]):
            if k not in leaves:
                continue
            l = k[0]
            if l <= 2:
                continue
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        if dx == dy == dz == 0:
                            continue
                        nb = _leaf_covering(leaves, l, (k[1] + dx, k[2] + dy, k[3] + dz), nroot, bc)
                        if nb is not None and nb[0] < l - 1:
                            _refine(leaves, nb)
                            changed = True


def plummer_cores_density(centres, a, rho_c):
    centres = np.asarray(centres, dtype=np.float64)

    def f(x, y, z):
        r = np.ones_like(x)
        for c in centres:
            q = ((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (a * a)
            r = r + rho_c * (1.0 + q) ** -2.5
        return r
    return f


def c3_amr(seed=3, rho_c=None, a=0.02, base_level=4, levels=3, bc=(1, 1, 0), cells=(2.5e6, 3.5e6)):
    """Four Plummer-like cores in a 1 x 1 x 4 box of four unit root blocks;
    64^3-cell base resolution per root (base_level 4), refined up to
    ``levels`` more levels where rho > 8 <rho>; mixed BCs by default.  Unless
    ``rho_c`` is given, the core density is bisected (in log space, 12 steps
    from [1e2, 1e4]) until the grid holds a number of cells inside ``cells``;
    the value used is recorded in ``meta``."""
    rng = np.random.default_rng(seed)
    centres = np.stack([rng.uniform(0.1, 0.9, 4), rng.uniform(0.1, 0.9, 4),
                        rng.uniform(0.5, 3.5, 4)], axis=1)
    nroot = (1, 1, 4)
    vol = 4.0

    def blocks(rc):
        mean = 1.0 + 4 * rc * (4.0 * np.pi / 3.0) * a ** 3 / vol
        dens = plummer_cores_density(centres, a, rc)
        return dens, amr_blocks(dens, nroot, 1.0, base_level, base_level + levels, 8.0 * mean, bc)

    if rho_c is None:
        lo, hi = np.log(1e2), np.log(1e4)
        for _ in range(12):
            rho_c = float(np.exp(0.5 * (lo + hi)))
            dens, (level, coord) = blocks(rho_c)
            n = 512 * len(level)
            if n < cells[0]:
                lo = np.log(rho_c)
            elif n > cells[1]:
                hi = np.log(rho_c)
            else:
                break
    else:
        dens, (level, coord) = blocks(rho_c)
    xc = cell_centres(1.0, (0.0, 0.0, 0.0), level, coord)
    rho = dens(xc[..., 0], xc[..., 1], xc[..., 2])
    return Grid(nroot, 1.0, (0.0, 0.0, 0.0), level, coord, rho, tuple(bc),
                name="plummer_amr", meta={"seed": seed, "rho_c": rho_c, "a": a,
                                          "centres": centres.tolist()})


def small_amr(seed=7, bc=(0, 0, 0), nroot=(1, 1, 1)):
    """Tiny AMR grid (level-2 base, one core refined two levels) for fast tests."""
    rng = np.random.default_rng(seed)
    box = np.array(nroot, dtype=np.float64)
    centre = rng.uniform(0.3, 0.7, 3) * box
    dens = plummer_cores_density([centre], 0.05, 50.0)
    level, coord = amr_blocks(dens, nroot, 1.0, 2, 4, 5.0, bc)
    xc = cell_centres(1.0, (0.0, 0.0, 0.0), level, coord)
    rho = dens(xc[..., 0], xc[..., 1], xc[..., 2])
    noise = rng.lognormal(0.0, 0.3, rho.shape)
    return Grid(tuple(nroot), 1.0, (0.0, 0.0, 0.0), level, coord, rho * noise, tuple(bc),
                name="small_amr", meta={"seed": seed})


def deep_amr(bc=(1, 1, 1), nroot=(1, 1, 1), seed=19):
    """AMR test grid with leaf blocks at five levels, cell sizes 1/32 to 1/512
    of a unit root: a Plummer core (a = 0.01, contrast 1e4) refined from a
    level-3 base up to level 7 where the block's densest cell exceeds 20, with
    2:1 balance, times lognormal cell noise (sigma 0.5)."""
    rng = np.random.default_rng(seed)
    box = np.array(nroot, dtype=np.float64)
    centre = np.array([0.41, 0.57, 0.47]) * box
    dens = plummer_cores_density([centre], 0.01, 1e4)
    level, coord = amr_blocks(dens, nroot, 1.0, 3, 7, 20.0, bc)
    xc = cell_centres(1.0, (0.0, 0.0, 0.0), level, coord)
    rho = dens(xc[..., 0], xc[..., 1], xc[..., 2]) * rng.lognormal(0.0, 0.5, xc.shape[:-1])
    return Grid(tuple(nroot), 1.0, (0.0, 0.0, 0.0), level, coord, rho, tuple(bc), name="deep_amr",
                meta={"seed": seed})


def shuffled(g: Grid, seed=11):
    """Same grid with the leaf blocks listed in a random order."""
    perm = np.random.default_rng(seed).permutation(g.nb)
    return dataclasses.replace(g, level=g.level[perm].copy(), coord=g.coord[perm].copy(),
                               rho=g.rho[perm].copy(), meta=dict(g.meta, perm=perm))


def _pool(a, f):
    """Mean over f^3 cubes of a [z, y, x] array."""
    n = a.shape[0] // f
    return a.reshape(n, f, n, f, n, f).mean(axis=(1, 3, 5))


def _blockmax(a):
    """Maximum over the 8^3 cells of each block of a [z, y, x] field."""
    n = a.shape[0] // BS
    return a.reshape(n, BS, n, BS, n, BS).max(axis=(1, 3, 5))


def _dilate26(m, periodic):
    """Boolean 26-neighbourhood dilation of a [z, y, x] array; periodic per
    axis (x, y, z order in ``periodic``), else clipped."""
    out = m.copy()
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                s = m
                for ax, d, per in ((0, dz, periodic[2]), (1, dy, periodic[1]), (2, dx, periodic[0])):
                    if d == 0:
                        continue
                    s = np.roll(s, d, axis=ax)
                    if not per:
                        sl = [slice(None)] * 3
                        sl[ax] = slice(0, 1) if d > 0 else slice(-1, None)
                        s = s.copy()
                        s[tuple(sl)] = False
                out |= s
    return out


def c5_amr(seed=5, sigma=2.0, n_fine=512, cells=(14e6, 16e6), bc=(1, 1, 0)):
    """Large AMR grid: unit cube, 128^3 base cells (4,096 blocks, level 5),
    refined up to two levels on a lognormal field rho = exp(sigma delta -
    sigma^2/2), delta a P(k) ~ k^-4 Gaussian field on the 512^3 finest grid
    (seed 5); a coarse cell's density is the mean of its fine cells.  A block
    is refined when its maximum cell density exceeds a threshold that is
    bisected (in log space) until the grid holds a number of cells inside
    ``cells``; 2:1 balance across faces, edges and corners (periodic in x, y
    for the default mixed boundaries)."""
    assert n_fine == 512
    delta = gaussian_field_k4(n_fine, seed)
    f7 = np.exp(sigma * delta - 0.5 * sigma * sigma)
    del delta
    f6 = _pool(f7, 2)
    f5 = _pool(f6, 2)
    m5, m6 = _blockmax(f5), _blockmax(f6)          # [16]^3 and [32]^3 blocks
    periodic = tuple(bool(b) for b in bc)

    def layout(t):
        r5 = m5 > t
        r6 = (m6 > t) & np.repeat(np.repeat(np.repeat(r5, 2, 0), 2, 1), 2, 2)
        # 2:1 balance: every neighbour of a refined level-6 block exists at level 6
        need = _dilate26(r6, periodic)
        r5 = r5 | need.reshape(16, 2, 16, 2, 16, 2).any(axis=(1, 3, 5))
        nblk = (r5.size - r5.sum()) + (8 * r5.sum() - r6.sum()) + 8 * r6.sum()
        return r5, r6, int(nblk)

    lo, hi = np.log(f7.mean()), np.log(f7.max())
    for _ in range(40):
        t = float(np.exp(0.5 * (lo + hi)))
        r5, r6, nblk = layout(t)
        if 512 * nblk > cells[1]:
            lo = np.log(t)
        elif 512 * nblk < cells[0]:
            hi = np.log(t)
        else:
            break
    levels, coords, rhos = [], [], []
    for lev, mask, field in ((5, ~r5, f5), (6, None, f6), (7, None, f7)):
        if lev == 6:
            mask = np.repeat(np.repeat(np.repeat(r5, 2, 0), 2, 1), 2, 2) & ~r6
        elif lev == 7:
            mask = np.repeat(np.repeat(np.repeat(r6, 2, 0), 2, 1), 2, 2)
        cz, cy, cx = np.nonzero(mask)
        nb = field.shape[0] // BS
        blocks = field.reshape(nb, BS, nb, BS, nb, BS).transpose(0, 2, 4, 1, 3, 5)  # [bz, by, bx, k, j, i]
        rhos.append(blocks[cz, cy, cx])
        levels.append(np.full(cz.size, lev, np.int32))
        coords.append(np.stack([cx, cy, cz], axis=1).astype(np.int32))
    level = np.concatenate(levels)
    coord = np.concatenate(coords)
    rho = np.ascontiguousarray(np.concatenate(rhos))  # [nb, k, j, i] = [nb][8][8][8], i fastest
    return Grid((1, 1, 1), 1.0, (0.0, 0.0, 0.0), level, coord, rho, tuple(bc), name="lognormal_amr16m",
                meta={"seed": seed, "sigma": sigma, "threshold": t})
