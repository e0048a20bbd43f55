"""Throughput of the tree-solver hot path on one MI355X.

Workload: 128^3 cells (4,096 blocks of 8^3) of lognormal density
exp(1.5 delta - 1.125), delta a seeded P(k) ~ k^-4 Gaussian random field;
isolated boundaries; APE MAC with a_lim = 1e-3 * max|a| (max|a| from one BH
theta = 0.5 FP64 walk before timing, as the paper derives a_lim from the
initial acceleration field); with 48-direction column densities (HEALPix
Nside 2), so a node is also required to pass BH at theta_pix = 0.5.  A step
is one pass of the whole path: tree build (moments), interaction lists, per-cell
potential + acceleration in FP32 with Kahan-compensated potential, and the
per-cell column map + tau_avg.  Inputs are resident in HBM before timing.

Prints one JSON line, with the roofline of the dominant kernel and the oracle's CPU baseline.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Algorithmic FP32 work of one (cell, node) interaction of the isolated walk:
# 3 sub (d), 5 (r^2: 3 mul + 2 add), rsqrt (1), m/r (1), m/r^3 (2 mul),
# 3 FMA for the acceleration (6), Kahan update of the potential (4).
FLOP_PAIR_ISO = 22
PEAK_FP32_VALU = 157.3  # TFLOP/s, MI355X vector FP32 (256 CU x 2.4 GHz, packed)
PEAK_FP64_VALU = 78.6
# Column walk per (cell, node) pair: the gravity above (its offset and r^2
# serve the bins too) plus the column work: three direction bins, each a
# look-up index (multiply-add and conversion) and one threshold test (product
# and comparison) (12); the N_p weight base m / (Omega r^2) from the gravity's
# m / r^2 (1); the map updates (2 per pixel hit, ~2.4 hits -> 5): 18.
FLOP_PAIR_COLS = FLOP_PAIR_ISO + 18
# Surrogate network per (cell, node) pair: 2 (3*64 + 64*64 + 64*64 + 64*4)
# multiply-adds of the four layers, on FP16 matrix instructions.
FLOP_PAIR_MLP = 2 * (3 * 64 + 64 * 64 + 64 * 64 + 64 * 4)
PEAK_FP16_MFMA = 2500.0  # TFLOP/s, MI355X dense FP16 matrix


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=128, help="cells per axis")
    ap.add_argument("--cpu-blocks", type=int, default=1024, help="oracle sample size (blocks, ~10 s on 16 threads)")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="MiB: one fill + one sum of that size before timing (HBM counter calibration)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--nside", type=int, default=2, help="HEALPix Nside of the column maps (0 = off)")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the learned-Ewald leg (same field, 3P boundaries)")
    ap.add_argument("--surrogate-steps", type=int, default=2)
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the large AMR leg (15.2M cells, 2P1I, 192-pixel columns)")
    ap.add_argument("--no-mpe", action="store_true", help="skip the MPE MAC leg")
    ap.add_argument("--no-abu", action="store_true", help="skip the adaptive block update leg")
    ap.add_argument("--no-p1", action="store_true", help="skip the 1P2I filament leg")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the Plummer AMR leg (2.6M cells, box 1x1x4, 2P1I, 64^3 Ewald table)")
    return ap.parse_args()


def measured_traffic(path, source):
    """HBM bytes of one launch from a committed counter summary, or None when
    the kernel's source has changed since the counters were taken."""
    import hashlib
    try:
        kv = dict(l.split(": ", 1) for l in open(os.path.join(ROOT, path)).read().splitlines()
                  if l and not l.startswith("#") and ": " in l)
        sha = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()
    except OSError:
        return None
    if not sha.startswith(kv.get("source_sha256_prefix", "-")):
        return None
    return {"bytes": float(kv["traffic_bytes"]), "fetch_kib": float(kv["fetch_size_kib"]),
            "write_kib": float(kv["write_size_kib"]), "fetch_factor": float(kv["fetch_factor"]),
            "write_factor": float(kv["write_factor"]), "summary": path}


def timed_steps(solver, rho, outs, fp64, steps, warmup):
    import torch
    solve = solver.solve64 if fp64 else solver.solve
    for _ in range(warmup):
        solver.build(rho)
        solve(*outs)
    torch.cuda.synchronize()
    evals, lists, builds = [], [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        solver.build(rho)
        st = solve(*outs)
        evals.append(st.ms_eval)
        lists.append(st.ms_list)
        builds.append(st.ms_build)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt / steps * 1e3, st, float(np.mean(evals)), float(np.mean(lists)), float(np.mean(builds))


def surrogate_leg(grid, rho, steps, nside=0):
    """Same field with 3P boundaries and the same MAC: the FP32 walk with the
    learned correction beside the FP32 and FP64 table walks.  Training (on the
    device, before timing) is reported, not timed as part of a step."""
    import torch
    import paper_1708_06142_amd as ot
    import workloads
    g = workloads.Grid(grid.nroot, grid.root_size, grid.origin, grid.level, grid.coord, grid.rho, (1, 1, 1),
                       grid.name + "-3p")
    n = g.ncells
    f32 = dict(device="cuda", dtype=torch.float32)
    f64 = dict(device="cuda", dtype=torch.float64)
    sm = ot.Solver.for_grid(g, mac="ape", eps_lim=1e-3, theta=0.5, ewald="mlp")
    t0 = time.perf_counter()
    rep = sm.mlp_train()
    train_s = time.perf_counter() - t0
    sm.build(rho)
    phi_m, acc_m = torch.empty(n, **f32), torch.empty(3 * n, **f32)
    a_lim = sm.solve(phi_m, acc_m).a_lim_used  # APE limit from the BH pre-pass (untimed)
    params, norm = sm.mlp_get()
    sm.close()
    res = {}
    legs = [("mlp_fp32", "mlp", False, 0), ("table_fp32", "table", False, 0), ("table_fp64", "table", True, 0)]
    if nside:
        legs += [("mlp_fp32_cols", "mlp", False, nside), ("table_fp64_cols", "table", True, nside)]
    for label, mode, fp64, ns in legs:
        s = ot.Solver.for_grid(g, mac="ape", a_lim=a_lim, theta=0.5, ewald=mode, nside=ns)
        if mode == "mlp":
            s.mlp_set(params, norm, accept=bool(rep["ok"]))
        kw = f64 if fp64 else f32
        outs = (torch.empty(n, **kw), torch.empty(3 * n, **kw))
        if ns:
            outs += (torch.empty(n * 12 * ns * ns, **kw), torch.empty(n, **kw))
        ms, st, ms_eval, _, _ = timed_steps(s, rho, outs, fp64, steps, 1)
        res[label] = dict(ms=ms, st=st, ms_eval=ms_eval, phi=outs[0].double().cpu().numpy(),
                          acc=outs[1].double().cpu().numpy().reshape(3, -1))
        if ns:
            res[label]["npix"] = outs[2].double().cpu().numpy()
        s.close()
    out = {"workload": f"{grid.name} field with 3P boundaries, APE a_lim=1e-3 a_max ({a_lim:.4g})",
           "training": {"seconds": train_s, "report": rep}, "a_lim": a_lim}
    for label, r in res.items():
        ref = res["table_fp64_cols" if label.endswith("_cols") else "table_fp64"]
        pmax = np.abs(ref["phi"]).max()
        amax = np.sqrt((ref["acc"] ** 2).sum(0)).max()
        st = r["st"]
        e = {"value": n / (r["ms"] * 1e-3), "unit": "cells/s", "ms_per_step": r["ms"], "ms_eval": r["ms_eval"],
             "ewald_used": ["table", "exact", "mlp"][st.ewald_used], "n_int": st.n_interactions}
        if not label.startswith("table_fp64"):
            e["dphi_maxnorm_vs_fp64_table"] = float(np.abs(r["phi"] - ref["phi"]).max() / pmax)
            e["da_maxnorm_vs_fp64_table"] = float(np.abs(r["acc"] - ref["acc"]).max() / amax)
        if "npix" in r and label != "table_fp64_cols":
            e["dnpix_maxnorm_vs_fp64"] = float(np.abs(r["npix"] - ref["npix"]).max() / np.abs(ref["npix"]).max())
        if label == "mlp_fp32":
            ach = st.n_interactions * FLOP_PAIR_MLP / (r["ms_eval"] * 1e-3) / 1e12
            e["roofline"] = {"bound": "mfma", "kernel": "k_eval_mlp<3P>", "achieved": ach,
                             "peak": PEAK_FP16_MFMA, "unit": "TFLOP/s", "frac": ach / PEAK_FP16_MFMA,
                             "flop_per_pair": FLOP_PAIR_MLP}
        out[label] = e
    return out


def c5_leg():
    """Large AMR configuration: 512^3-resolution lognormal field (sigma_ln 2,
    P(k) ~ k^-4, seed 5) on a 128^3 base grid refined up to two levels (15.2M
    cells), x, y periodic and z isolated, APE a_lim = 1e-3 a_max with BH at
    theta_pix = 0.25, 192-pixel columns.  The FP32 walk with the learned
    correction beside the FP32 and FP64 table walks at the same MAC; one
    untimed step, then one timed step each (a step is several seconds)."""
    import torch
    import paper_1708_06142_amd as ot
    import workloads
    t0 = time.perf_counter()
    g = workloads.c5_amr()
    gen_s = time.perf_counter() - t0
    n = g.ncells
    rho = torch.from_numpy(g.rho.reshape(-1)).cuda()
    kw = dict(mac="ape", theta=0.5, theta_pix=0.25, ewald_n=64)
    s = ot.Solver.for_grid(g, eps_lim=1e-3, **kw)
    s.build(rho)
    a_lim = s.solve(torch.empty(n, device="cuda"), torch.empty(3 * n, device="cuda")).a_lim_used
    s.close()
    tr = ot.Solver(bc=g.bc, ewald_n=64, ewald="mlp")
    t0 = time.perf_counter()
    rep = tr.mlp_train()
    train_s = time.perf_counter() - t0
    params, norm = tr.mlp_get()
    tr.close()
    res, out = {}, {"workload": f"AMR lognormal 512^3 effective (sigma_ln 2, seed 5), {g.nb} blocks, {n} cells, "
                                f"2P1I, APE a_lim=1e-3 a_max ({a_lim:.4g}) + BH theta_pix 0.25, 192-pixel columns",
                    "generate_s": gen_s, "training": {"seconds": train_s, "err_mlp": rep["err_mlp"],
                                                     "ok": rep["ok"]}}
    for label, mode, fp64 in (("mlp_fp32_cols", "mlp", False), ("table_fp32_cols", "table", False),
                              ("table_fp64_cols", "table", True)):
        s = ot.Solver.for_grid(g, a_lim=a_lim, ewald=mode, nside=4, **kw)
        if mode == "mlp":
            s.mlp_set(params, norm, accept=bool(rep["ok"]))
        dt = torch.float64 if fp64 else torch.float32
        outs = (torch.empty(n, dtype=dt, device="cuda"), torch.empty(3 * n, dtype=dt, device="cuda"),
                torch.empty(n * 192, dtype=dt, device="cuda"), torch.empty(n, dtype=dt, device="cuda"))
        ms, st, ms_eval, _, _ = timed_steps(s, rho, outs, fp64, 1, 1)
        s.close()
        res[label] = outs
        e = {"value": n / (ms * 1e-3), "unit": "cells/s", "ms_per_step": ms, "ms_eval": ms_eval,
             "ewald_used": ["table", "exact", "mlp"][st.ewald_used], "n_int": st.n_interactions,
             "eval_wg_per_cu": st.eval_wg_per_cu}
        if mode == "mlp":
            ach = st.n_interactions * FLOP_PAIR_MLP / (ms_eval * 1e-3) / 1e12
            e["roofline"] = {"bound": "mfma", "kernel": "k_eval_cols<float, newton> + k_eval_mlp<2P1I, add>",
                             "achieved": ach, "peak": PEAK_FP16_MFMA, "unit": "TFLOP/s",
                             "frac": ach / PEAK_FP16_MFMA, "flop_per_pair": FLOP_PAIR_MLP,
                             "note": "matrix work over the time of both kernels"}
        else:
            fl = st.n_interactions * FLOP_PAIR_COLS / (ms_eval * 1e-3) / 1e12
            peak = PEAK_FP64_VALU if fp64 else PEAK_FP32_VALU
            e["roofline"] = {"bound": "alu", "kernel": f"k_eval_cols<{'double' if fp64 else 'float'}>",
                             "achieved": fl, "peak": peak, "unit": "TFLOP/s", "frac": fl / peak,
                             "flop_per_pair": FLOP_PAIR_COLS}
        out[label] = e
        torch.cuda.synchronize()
    ref = res["table_fp64_cols"]
    names = ("phi", "acc", "npix", "tau")
    for label in ("mlp_fp32_cols", "table_fp32_cols"):
        for nm, a, r in zip(names, res[label], ref):
            out[label][f"d{nm}_maxnorm_vs_fp64_table"] = float((a.double() - r).abs().max() / r.abs().max()) \
                if nm != "npix" else float(max((a[i:i + (1 << 28)].double() - r[i:i + (1 << 28)]).abs().max()
                                               for i in range(0, r.numel(), 1 << 28)) / r.abs().max())
    del res, ref
    torch.cuda.empty_cache()
    return out


def c3_leg(steps):
    """Plummer AMR configuration: box 1 x 1 x 4 (four root blocks), 64^3 base,
    up to three levels around four Plummer cores (5,100 blocks, 2.61M cells),
    x, y periodic and z isolated, BH theta = 0.5, FP64-generated 64^3 Ewald
    table: the FP32-Kahan table walk beside the FP64 table walk."""
    import torch
    import paper_1708_06142_amd as ot
    import workloads
    g = workloads.c3_amr()
    n = g.ncells
    rho = torch.from_numpy(g.rho.reshape(-1)).cuda()
    s = ot.Solver.for_grid(g, mac="bh", theta=0.5, ewald_n=64)
    out = {"workload": f"Plummer AMR, box 1x1x4, {g.nb} blocks, {n} cells, 2P1I, BH theta 0.5, 64^3 Ewald table"}
    res = {}
    for label, fp64 in (("table_fp32", False), ("table_fp64", True)):
        dt = torch.float64 if fp64 else torch.float32
        outs = (torch.empty(n, dtype=dt, device="cuda"), torch.empty(3 * n, dtype=dt, device="cuda"))
        ms, st, ms_eval, ms_list, _ = timed_steps(s, rho, outs, fp64, steps, 1)
        res[label] = outs
        flop = st.n_interactions * (FLOP_PAIR_ISO + 46) / (ms_eval * 1e-3) / 1e12
        peak = PEAK_FP64_VALU if fp64 else PEAK_FP32_VALU
        out[label] = {"value": n / (ms * 1e-3), "unit": "cells/s", "ms_per_step": ms, "ms_eval": ms_eval,
                      "ms_lists": ms_list, "n_int": st.n_interactions,
                      "roofline": {"bound": "alu", "kernel": f"k_eval{'64' if fp64 else '32'}<2P1I>",
                                   "achieved": flop, "peak": peak, "unit": "TFLOP/s", "frac": flop / peak,
                                   "flop_per_pair": FLOP_PAIR_ISO + 46}}
    s.close()
    (p32, a32), (p64, a64) = res["table_fp32"], res["table_fp64"]
    out["table_fp32"]["dphi_rel_vs_fp64"] = float(((p32.double() - p64).abs() / p64.abs()).max())
    a64n = a64.view(3, -1).pow(2).sum(0).sqrt().max()
    out["table_fp32"]["da_maxnorm_vs_fp64"] = float((a32.double() - a64).abs().max() / a64n)
    return out


def p1_leg(steps):
    """1P2I configuration: a filament along the periodic x axis of a 1 x 2 x 2
    box (isothermal-cylinder profile, H = 0.1, modulated along x, lognormal
    noise), 64 x 128 x 128 cells, APE a_lim = 1e-3 a_max, FP64-generated 64^3
    Ewald table: the FP32-Kahan table walk beside the FP64 table walk."""
    import torch
    import paper_1708_06142_amd as ot
    import workloads
    g = workloads.filament_1p2i(64)
    n = g.ncells
    rho = torch.from_numpy(g.rho.reshape(-1)).cuda()
    s0 = ot.Solver.for_grid(g, mac="ape", eps_lim=1e-3, theta=0.5, ewald_n=64)
    s0.build(rho)
    a_lim = s0.solve(torch.empty(n, device="cuda"), torch.empty(3 * n, device="cuda")).a_lim_used
    s0.close()
    s = ot.Solver.for_grid(g, mac="ape", a_lim=a_lim, theta=0.5, ewald_n=64)
    out = {"workload": f"filament 1x2x2 box, 64x128x128 cells ({g.nb} blocks), 1P2I, APE a_lim 1e-3 a_max, "
                       "64^3 Ewald table", "a_lim": a_lim}
    res = {}
    for label, fp64 in (("table_fp32", False), ("table_fp64", True)):
        dt = torch.float64 if fp64 else torch.float32
        outs = (torch.empty(n, dtype=dt, device="cuda"), torch.empty(3 * n, dtype=dt, device="cuda"))
        ms, st, ms_eval, ms_list, _ = timed_steps(s, rho, outs, fp64, steps, 1)
        res[label] = outs
        flop = st.n_interactions * (FLOP_PAIR_ISO + 46) / (ms_eval * 1e-3) / 1e12
        peak = PEAK_FP64_VALU if fp64 else PEAK_FP32_VALU
        out[label] = {"value": n / (ms * 1e-3), "unit": "cells/s", "ms_per_step": ms, "ms_eval": ms_eval,
                      "ms_lists": ms_list, "n_int": st.n_interactions,
                      "roofline": {"bound": "alu", "kernel": f"k_eval{'64' if fp64 else '32'}<1P2I>",
                                   "achieved": flop, "peak": peak, "unit": "TFLOP/s", "frac": flop / peak,
                                   "flop_per_pair": FLOP_PAIR_ISO + 46}}
    s.close()
    (p32, a32), (p64, a64) = res["table_fp32"], res["table_fp64"]
    out["table_fp32"]["dphi_maxnorm_vs_fp64"] = float((p32.double() - p64).abs().max() / p64.abs().max())
    a64n = a64.view(3, -1).pow(2).sum(0).sqrt().max()
    out["table_fp32"]["da_maxnorm_vs_fp64"] = float((a32.double() - a64).abs().max() / a64n)
    return out


def mpe_leg(grid, rho, a_lim, steps, nside):
    """The benchmark field with the MPE MAC (Eq. (2) with p = 1) at the same
    absolute limit: the whole path (tree build with the B_2, B_3 moments,
    lists, FP32-Kahan and FP64 column walks)."""
    import torch
    import paper_1708_06142_amd as ot
    n = grid.ncells
    npx = 12 * nside ** 2
    s = ot.Solver.for_grid(grid, mac="mpe", a_lim=a_lim, theta=0.5, nside=nside)
    out = {"workload": f"lognormal {round(n ** (1 / 3))}^3, isolated, MPE a_lim={a_lim:.5g} (1e-3 a_max), "
                       f"{npx}-pixel columns"}
    res = {}
    for label, fp64 in (("fp32", False), ("fp64", True)):
        dt = torch.float64 if fp64 else torch.float32
        outs = (torch.empty(n, dtype=dt, device="cuda"), torch.empty(3 * n, dtype=dt, device="cuda"))
        if nside:
            outs += (torch.empty(n * npx, dtype=dt, device="cuda"), torch.empty(n, dtype=dt, device="cuda"))
        ms, st, ms_eval, ms_list, ms_build = timed_steps(s, rho, outs, fp64, steps, 1)
        res[label] = outs
        fpair = FLOP_PAIR_COLS if nside else FLOP_PAIR_ISO
        fl = st.n_interactions * fpair / (ms_eval * 1e-3) / 1e12
        peak = PEAK_FP64_VALU if fp64 else PEAK_FP32_VALU
        out[label] = {"value": n / (ms * 1e-3), "unit": "cells/s", "ms_per_step": ms,
                      "phases_ms": {"build": ms_build, "lists": ms_list, "eval": ms_eval},
                      "n_int": st.n_interactions, "per_cell": st.n_interactions / n, "max_list": st.max_list,
                      "roofline": {"bound": "alu", "achieved": fl, "peak": peak, "unit": "TFLOP/s",
                                   "frac": fl / peak, "flop_per_pair": fpair}}
    s.close()
    (p32, a32) = res["fp32"][:2]
    (p64, a64) = res["fp64"][:2]
    out["fp32"]["dphi_rel_vs_fp64"] = float(((p32.double() - p64).abs() / p64.abs()).max())
    out["fp32"]["da_maxnorm_vs_fp64"] = float((a32.double() - a64).abs().max() / a64.view(3, -1).pow(2).sum(0).sqrt().max())
    return out


def abu_leg(grid, a_lim, nsnap=6, seed=12, nside=0):
    """Adaptive block update (gravity only) on a seeded sequence of snapshots of
    the benchmark field: each snapshot multiplies the density by 1 + 0.3 G(x - c),
    G a Gaussian bump of width 0.05 whose centre c moves by 0.02 per snapshot
    from a seeded start.  Per snapshot: the FP32 walk with ABU from the previous
    snapshot's solution (tolerance 1e-3 a_max) beside the plain FP32 walk."""
    import torch
    import paper_1708_06142_amd as ot
    import workloads
    rng = np.random.default_rng(seed)
    x = workloads.cell_centres(grid.root_size, grid.origin, grid.level, grid.coord)
    c = rng.uniform(0.3, 0.7, 3)
    step = rng.normal(size=3)
    step *= 0.02 / np.linalg.norm(step)
    n = grid.ncells
    s = ot.Solver.for_grid(grid, mac="ape", a_lim=a_lim, theta=0.5, nside=nside)
    phi = torch.empty(n, device="cuda")
    acc = torch.empty(3 * n, device="cuda")
    phi_f = torch.empty(n, device="cuda")
    acc_f = torch.empty(3 * n, device="cuda")
    npx = 12 * nside * nside
    npix, tau, npix_f, tau_f = ((torch.empty(m, device="cuda") for m in (n * npx, n, n * npx, n)) if nside
                                else (None,) * 4)
    rows = []
    for k in range(nsnap):
        ck = c + k * step
        r2 = ((x - ck) ** 2).sum(-1)
        rho = torch.from_numpy((grid.rho * (1.0 + 0.3 * np.exp(-r2 / (2 * 0.05 ** 2)))).reshape(-1)).cuda()
        s.build(rho)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stf = s.solve(phi_f, acc_f, npix_f, tau_f)
        torch.cuda.synchronize()
        ms_full = (time.perf_counter() - t0) * 1e3
        if k == 0:
            phi.copy_(phi_f)
            acc.copy_(acc_f)
            if nside:
                npix.copy_(npix_f)
                tau.copy_(tau_f)
            tol = 1e-3 * float(acc_f.view(3, -1).double().pow(2).sum(0).sqrt().max())
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, upd = s.solve_abu(phi, acc, tol, npix=npix, tau=tau)
        torch.cuda.synchronize()
        ms_abu = (time.perf_counter() - t0) * 1e3
        amax = acc_f.view(3, -1).double().pow(2).sum(0).sqrt().max()
        ea = float((acc.double() - acc_f.double()).view(3, -1).pow(2).sum(0).sqrt().max() / amax)
        row = {"updated_frac": float(upd.mean()), "ms_abu": ms_abu, "ms_full": ms_full,
               "ms_eval_abu": st.ms_eval, "ms_eval_full": stf.ms_eval, "e_a_max_vs_full": ea}
        if nside:
            row["e_npix_max_vs_full"] = float((npix - npix_f).abs().max() / npix_f.abs().max())
        rows.append(row)
    s.close()
    return {"workload": f"lognormal 128^3 x {nsnap} snapshots with a moving Gaussian bump (amplitude 0.3, "
                        f"width 0.05, 0.02 per snapshot, seed {seed}), APE a_lim 1e-3 a_max, FP32-Kahan walk, "
                        f"{npx if nside else 'no'} columns, ABU tolerance 1e-3 a_max",
            "snapshots": rows,
            "mean_updated_frac": float(np.mean([r["updated_frac"] for r in rows])),
            "ms_abu_mean": float(np.mean([r["ms_abu"] for r in rows])),
            "ms_full_mean": float(np.mean([r["ms_full"] for r in rows]))}


def cpu_baseline(grid, a_lim, nblk, nside):
    """The FP64 oracle's group walk on a seeded sample of blocks, host cores."""
    import oracle
    threads = os.cpu_count() or 1
    os.environ.setdefault("OMP_NUM_THREADS", str(threads))
    nblk = min(nblk, grid.nb)
    sel = np.sort(np.random.default_rng(7).choice(grid.nb, nblk, replace=False))
    t0 = time.perf_counter()
    t = oracle.Tree(grid, mac="ape", a_lim=a_lim, nside=nside)
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    t.walk_group(sel, columns=nside > 0)
    tw = time.perf_counter() - t0
    cells = 512 * nblk
    # tree build is O(all cells): charge the sample its share
    sec = tw + tb * (nblk / grid.nb)
    return {"value": cells / sec, "unit": "cells/s", "cores": int(os.environ["OMP_NUM_THREADS"]),
            "kind": "oracle",
            "sample": f"{nblk} seeded blocks ({cells} cells) of the same workload, APE same a_lim, "
                      f"Nside {nside} columns; walk {tw:.2f} s + build share {tb * nblk / grid.nb:.3f} s "
                      "(tree build includes the node-ray table)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_1708_06142_amd as ot
    import workloads

    if args.calib_copy:
        n = args.calib_copy * (1 << 20) // 4
        src = torch.ones(n, device="cuda")      # fill kernel: writes exactly n * 4 bytes
        total = src.sum()                        # reduction: reads exactly n * 4 bytes
        torch.cuda.synchronize()
        del src, total
    grid = workloads.c2_lognormal(args.n)
    ncell = grid.ncells
    rho = torch.from_numpy(grid.rho.reshape(-1).copy()).cuda()
    npx = 12 * args.nside ** 2
    s = ot.Solver.for_grid(grid, mac="ape", eps_lim=1e-3, theta=0.5)
    s.build(rho)
    phi = torch.empty(ncell, device="cuda", dtype=torch.float32)
    acc = torch.empty(3 * ncell, device="cuda", dtype=torch.float32)
    st0 = s.solve(phi, acc)  # derives a_lim from the BH pre-pass (untimed)
    a_lim = st0.a_lim_used
    s.close()
    s = ot.Solver.for_grid(grid, mac="ape", a_lim=a_lim, theta=0.5, nside=args.nside)
    outs = (phi, acc)
    if args.nside:
        outs = (phi, acc, torch.empty(ncell * npx, device="cuda"), torch.empty(ncell, device="cuda"))

    ms, st, ms_eval, ms_list, ms_build = timed_steps(s, rho, outs, False, args.steps, args.warmup)
    value = ncell / (ms * 1e-3)
    fpair = FLOP_PAIR_COLS if args.nside else FLOP_PAIR_ISO
    flops = st.n_interactions * fpair
    achieved = flops / (ms_eval * 1e-3) / 1e12
    traffic = measured_traffic("profiles/eval_cols_lognormal128_nside2_hbm_traffic.txt",
                               "paper_1708_06142_amd/csrc/k_columns.hip") \
        if args.nside == 2 and args.n == 128 else None
    out = {
        "metric": "cells/s for potential+accel+N_pix column densities at <=1e-3 rel err",
        "value": value, "unit": "cells/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"lognormal {args.n}^3 (sigma_ln 1.5, P(k)~k^-4, seed 2), isolated, "
                               f"APE a_lim=1e-3 a_max, {npx}-pixel columns, FP32-Kahan walk",
                   "cells": ncell, "blocks": grid.nb, "a_lim": a_lim, "columns": npx},
        "phases_ms": {"build": ms_build, "lists": ms_list, "eval": ms_eval},
        "eval_wg_per_cu": st.eval_wg_per_cu,
        "interactions": {"n_int": st.n_interactions, "per_cell": st.n_interactions / ncell,
                         "max_list": st.max_list},
        "roofline": {"bound": "alu", "kernel": "k_eval_cols<float> (isolated, columns)" if args.nside
                     else "k_eval32 (isolated)", "achieved": achieved,
                     "peak": PEAK_FP32_VALU, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU,
                     "traffic": traffic["bytes"] if traffic else None,
                     "traffic_detail": traffic, "flop_per_pair": fpair,
                     "hbm_gbs_at_traffic": traffic["bytes"] / (ms_eval * 1e-3) / 1e9 if traffic else None},
    }
    if not args.no_fp64:
        f64 = dict(device="cuda", dtype=torch.float64)
        outs64 = (torch.empty(ncell, **f64), torch.empty(3 * ncell, **f64))
        if args.nside:
            outs64 += (torch.empty(ncell * npx, **f64), torch.empty(ncell, **f64))
        ms64, st64, e64, _, _ = timed_steps(s, rho, outs64, True, max(2, args.steps // 2), 1)
        a64 = st64.n_interactions * fpair / (e64 * 1e-3) / 1e12
        out["fp64_walk"] = {"value": ncell / (ms64 * 1e-3), "ms_per_step": ms64, "ms_eval": e64,
                            "achieved_tflops": a64, "frac_fp64_peak": a64 / PEAK_FP64_VALU,
                            "eval_wg_per_cu": st64.eval_wg_per_cu}
    if not args.no_surrogate:
        out["surrogate"] = surrogate_leg(grid, rho, args.surrogate_steps, args.nside)
    if not args.no_abu:
        out["abu"] = abu_leg(grid, a_lim)
        if args.nside:
            out["abu_columns"] = abu_leg(grid, a_lim, nside=args.nside)
    if not args.no_mpe:
        out["mpe"] = mpe_leg(grid, rho, a_lim, max(2, args.steps // 2), args.nside)
    if not args.no_c3:
        out["c3"] = c3_leg(max(2, args.steps // 2))
    if not args.no_p1:
        out["p1"] = p1_leg(max(2, args.steps // 2))
    if not args.no_c5:
        out["c5"] = c5_leg()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(grid, a_lim, args.cpu_blocks, args.nside)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
