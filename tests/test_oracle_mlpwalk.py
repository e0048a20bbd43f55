"""Pins of the oracle's walk with the learned surrogate (the network's ten
channels per (group of cells, listed node), a first-order Taylor step to each
cell of the group, Sec. 2.2.5's second look-up approach).

A network with every weight and bias zero outputs 0, so its de-standardised
channels are the scaling's means mu: a constant phi_c, A_c and H_c at every
folded offset.  The walk is then a closed form that numpy recomputes here
from the grid geometry, the oracle's interaction lists and node moments:
per group centre c_g and node r, d0 = c_g - r (minimum image), channels
mu with A_c,k times sgn d0_k and H_jk (j != k) times sgn d0_j sgn d0_k; per
cell delta = x - c_g, d = d0 + delta,
  Phi = -G sum M (1/|d| + phi_c - A_c . delta),  a = -G sum M (d/|d|^3 + A_c - H_c delta).
A mistake in the group rule or geometry, the image, a sign, a transposed H
or the far-field switch changes the result far above rounding.
"""
import os
import shutil

import numpy as np
import pytest

import oracle
import workloads

CH = np.array([0.7, 0.3, -0.2, 0.5, 1.1, -0.6, 0.9, 0.25, -0.35, 0.15])  # phi_c, A_c, H xx yy zz xy xz yz
# Ewald table points per axis of the closed-form cases: a coarse 8^3 table
# (half spacing 0.5/7/2 = 0.036) puts the grids' cells (h = 1/16) in 2^3
# groups at reach 1 and 4^3 groups at reach 3, so the Taylor step from the
# group centre (delta up to 1.5 h per axis) is part of what is checked
EW_N = 8


def const_surrogate(ext):
    params = np.zeros(oracle.MLP_NPARAM)
    norm = np.concatenate([ext, CH, np.ones(10)])
    return params, norm


def lognormal16(bc, nroot):
    """16^3 cells per root block (root size 1), lognormal density."""
    level, coord, rho = [], [], []
    rng = np.random.default_rng(23)
    for z in range(nroot[2]):
        l, c = workloads.uniform_blocks(16)
        c = np.array(c).copy()
        c[:, 2] += 2 * z
        level.append(l)
        coord.append(c)
        rho.append(rng.lognormal(0.0, 1.0, (8, 8, 8, 8)))
    return workloads.Grid(tuple(nroot), 1.0, (0.0, 0.0, 0.0), np.concatenate(level), np.concatenate(coord),
                          np.concatenate(rho), tuple(bc), "lognormal16")


def group_level(h, step, reach=1.0):
    tmax = reach * 0.5 * min(step)
    return 2 if 1.5 * h <= tmax else (1 if 0.5 * h <= tmax else 0)


def closed_form(t, g, lb, ext_far, reach=1.0, lists=None):
    """Phi [512], a [3, 512] of block lb by the closed form above; with
    lists (eight octant lists) each cell sums the list of its octant."""
    ex = t.export()
    ids = t.block_list(lb)
    L = np.asarray(g.nroot, float) * g.root_size
    per = np.asarray(g.bc, bool)
    h = g.root_size / 2.0 ** (g.level[lb] - 1) / 8
    n = EW_N
    step = np.array([0.5 * L[0], 0.5 * L[1], 0.5 * L[2] if per[2] else min(L[2], 2 * L[0])]) / (n - 1)
    gl = group_level(h, step, reach)
    gs = 2 ** gl
    phi, acc = np.zeros(512), np.zeros((3, 512))
    ci = np.arange(512)
    ijk = np.stack([ci % 8, (ci // 8) % 8, ci // 64], 1)
    x = np.asarray(g.origin) + (8 * g.coord[lb] + ijk + 0.5) * h
    gidx = ijk // gs
    gc = np.asarray(g.origin) + (8 // gs * g.coord[lb] + gidx + 0.5) * (h * gs)
    H = np.array([[CH[4], CH[7], CH[8]], [CH[7], CH[5], CH[9]], [CH[8], CH[9], CH[6]]])
    bL2 = L[1] / L[0] * L[0] ** 2
    octs = (ijk // 4) @ np.array([1, 2, 4])
    for c in range(512):
        cid = ids if lists is None else lists[octs[c]]
        com, M = ex["com"][cid], ex["M"][cid]
        d0 = gc[c] - com
        d0 = np.where(per, d0 - L * np.floor(d0 / L + 0.5), d0)
        s = np.where(d0 < 0, -1.0, 1.0)
        dl = x[c] - gc[c]
        d = d0 + dl
        r2 = (d ** 2).sum(1)
        ok = r2 != 0
        r = np.sqrt(r2[ok])
        Ac = s[ok] * CH[1:4]
        Hs = H[None] * (s[ok][:, :, None] * s[ok][:, None, :])
        p = 1 / r + CH[0] - (Ac * dl).sum(1)
        A = d[ok] / r[:, None] ** 3 + Ac - Hs @ dl
        if ext_far:
            far = np.abs(d0[ok][:, 2]) > 2 * L[0]
            p = np.where(far, -2 * np.pi * np.abs(d[ok][:, 2]) / bL2 + np.sqrt(np.pi) / (L[1] / L[0] * L[0]), p)
            A = np.where(far[:, None], np.stack([0 * r, 0 * r, np.sign(d[ok][:, 2]) * 2 * np.pi / bL2], 1), A)
        phi[c] = -(M[ok] * p).sum()
        acc[:, c] = -(M[ok][:, None] * A).sum(0)
    return phi, acc, gl


@pytest.mark.parametrize("reach", [1.0, 3.0])
@pytest.mark.parametrize("case", ["3p", "2p1i_far"])
def test_constant_network_closed_form(case, reach):
    if case == "3p":
        g = lognormal16((1, 1, 1), (1, 1, 1))
        ext = np.array([0.5, 0.5, 0.5])
    else:
        g = lognormal16((1, 1, 0), (1, 1, 5))  # box 1 x 1 x 5: pairs beyond |dz| = 2 Lx
        ext = np.array([0.5, 0.5, 2.0])
    t = oracle.Tree(g, theta=0.5, ewald="table", ew_n=EW_N, mlp_reach=reach)
    params, norm = const_surrogate(ext)
    blocks = [0, 5, g.nb - 1]
    phi, acc, _ = t.walk_group_mlp(params, norm, blocks)
    for q, lb in enumerate(blocks):
        pr, ar, gl = closed_form(t, g, lb, case != "3p", reach)
        assert t.mlp_group_level(lb) == gl
        assert gl == (1 if reach == 1.0 else 2)
        sl = slice(512 * q, 512 * (q + 1))
        np.testing.assert_allclose(phi[sl], pr, rtol=1e-12)
        assert np.abs(acc[:, sl] - ar).max() <= 1e-12 * np.abs(ar).max()


def test_group_levels():
    """The group side follows the cell size against half the table's
    smallest spacing: 16^3 per unit root (h = 1/128) groups 2^3 cells, a
    level finer (h = 1/256) 2^3 too (1.5 h > 0.5/63 / 2), two levels finer
    4^3, and 8^3 per root (h = 1/64) single cells."""
    g = workloads.small_amr(bc=(1, 1, 1))
    t = oracle.Tree(g, theta=0.5, ewald="table", ew_n=64)
    step = 0.5 / 63
    for lb in range(g.nb):
        h = 1.0 / 2.0 ** (g.level[lb] - 1) / 8
        assert t.mlp_group_level(lb) == group_level(h, [step] * 3)
    assert group_level(1 / 64, [step] * 3) == 0
    assert group_level(1 / 128, [step] * 3) == 1
    assert group_level(1 / 256, [step] * 3) == 1
    assert group_level(1 / 512, [step] * 3) == 2


def test_group_levels_with_reach():
    """mlp_reach scales the allowed offset: at three times the table's Taylor
    offset 16^3 per unit root (h = 1/128) already takes 4^3 groups (1.5 h =
    0.0117 <= 3 x 0.5 x 0.5/63 = 0.0119), 8^3 per root (h = 1/64) 2^3, and a
    reach <= 0 is the default."""
    step = [0.5 / 63] * 3
    assert group_level(1 / 128, step, 3.0) == 2
    assert group_level(1 / 64, step, 3.0) == 1
    assert group_level(1 / 32, step, 3.0) == 0
    g = workloads.small_amr(bc=(1, 1, 1))
    for reach in (3.0, 0.0):
        t = oracle.Tree(g, theta=0.5, ewald="table", ew_n=64, mlp_reach=reach)
        for lb in range(g.nb):
            h = 1.0 / 2.0 ** (g.level[lb] - 1) / 8
            assert t.mlp_group_level(lb) == group_level(h, step, reach if reach > 0 else 1.0)


# planted mistakes in copies of the oracle's surrogate walk, each of which the
# closed form must catch
MUTANTS = {
    "A_c . delta with the wrong sign": (
        "p = 1.0 / r + (v[0] - (v[1] * dl[0] + v[2] * dl[1] + v[3] * dl[2]));",
        "p = 1.0 / r + (v[0] + (v[1] * dl[0] + v[2] * dl[1] + v[3] * dl[2]));"),
    "H_c with a transposed index": (
        "static const int hidx[3][3] = {{4, 7, 8}, {7, 5, 9}, {8, 9, 6}};",
        "static const int hidx[3][3] = {{4, 8, 7}, {7, 5, 9}, {8, 9, 6}};"),
    "xy second derivative's sign not restored": ("v[7] *= s[0] * s[1];", "v[7] *= s[0];"),
}


@pytest.fixture(scope="module")
def mutant_libs(tmp_path_factory):
    src = open(os.path.join(oracle.HERE, "mlpwalk.c")).read()
    libs = {}
    for name, (old, new) in MUTANTS.items():
        assert src.count(old) == 1, name
        d = tmp_path_factory.mktemp("mutant")
        for f in os.listdir(oracle.HERE):
            if f.endswith((".c", ".h")):
                shutil.copy(os.path.join(oracle.HERE, f), d)
        (d / "mlpwalk.c").write_text(src.replace(old, new))
        libs[name] = oracle.build(src_dir=str(d), out=str(d / "liboracle_mutant.so"))
    return libs


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_closed_form_catches_planted_mistakes(mutant_libs, name):
    with oracle.using_library(mutant_libs[name]):
        with pytest.raises(AssertionError):
            test_constant_network_closed_form("3p", 1.0)

