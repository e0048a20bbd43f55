"""Throughput of the tree-solver hot path on one MI355X.

Headline workload: the large AMR configuration, the largest that runs on one
GPU.  A 512^3-resolution lognormal density (sigma_ln 2, P(k) ~ k^-4, seed 5)
on a 128^3 base grid refined up to two levels (29,709 blocks of 8^3, 15.2M
cells); x, y periodic and z isolated (generalised Ewald, 64^3 table); APE MAC
with a_lim = 1e-3 max|a| (max|a| from one BH theta = 0.5 FP64 walk before
timing, as the paper derives the limit from the acceleration field) together
with BH at theta_pix = 0.25 for 192-direction column densities (HEALPix
Nside 4).  A step is one pass of the whole path: tree build (moments),
interaction lists, FP32 gravity with Kahan-compensated potential and the
Ewald correction from the learned surrogate (its network evaluated once per
4^3 group of cells and list entry on FP16 matrix instructions, a first-order
Taylor step to each cell reaching up to three times the table's own Taylor
offset), and the per-cell column maps + tau_avg.  The
surrogate is trained on the device before timing.  Inputs are resident in
HBM before timing.  Beside it, on the same lists: the FP64-table walk (the
plain reference) and the FP32-table walk, the accuracy of the headline
against the FP64-table walk over all cells and against the direct sum on
sampled cells, and the other configurations as extra keys.

Prints one JSON line, with the roofline of the dominant kernel and the
oracle's CPU baseline on a sample of the same workload.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Algorithmic work per (cell, node) pair, counted as in the scope's per-unit
# figures: FP32 gravity 21 (3 sub for d, 5 for r^2, 1 m/r, 2 for m/r^3,
# 3 FMA for a = 6, Kahan 4) + the rsqrt; the Ewald table look-up 46 (fold,
# index and offset 12, Taylor of phi_c 6, of A_c 18, unfold and add 10); the
# columns 30 (offset and r^2 8, weight base 2, three direction bins 12, map
# updates of ~2.4 pixels 5, rsqrt 1 and the cut 2).
FLOP_GRAV = 21
FLOP_EWALD_TABLE = 46
FLOP_COLS = 30
FLOP_PAIR_ISO = FLOP_GRAV
FLOP_PAIR_COLS = FLOP_GRAV + FLOP_COLS
FLOP_PAIR_TABLE_COLS = FLOP_GRAV + FLOP_EWALD_TABLE + FLOP_COLS
# Surrogate: per network evaluation 2 (3*64 + 64*64 + 64*64 + 64*10)
# multiply-adds on FP16 matrix instructions; per (cell, node) pair the
# gravity and the Taylor step from the group centre (phi_c 6, A_c 18).
FLOP_MLP_EVAL = 2 * (3 * 64 + 64 * 64 + 64 * 64 + 64 * 10)
FLOP_PAIR_MLP_TAYLOR = FLOP_GRAV + 24
# The headline's surrogate walk lets a cell group reach three times the Ewald
# table's own Taylor offset (4^3 groups on every level of the large grid):
# 13% less time than at the table's offset, and the accuracy against the
# direct sum is unchanged (the MAC's error dominates); the bench line reports
# both comparisons.
C5_MLP_REACH = 3.0
PEAK_FP32_VALU = 157.3  # TFLOP/s, MI355X vector FP32 (published, packed)
PEAK_FP64_VALU = 78.6
PEAK_FP16_MFMA = 2500.0  # TFLOP/s, MI355X dense FP16 matrix


def progress(msg):
    """One line per finished leg on stderr (the JSON line stays alone on stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--side-steps", type=int, default=2,
                    help="timed steps of the FP64- and FP32-table walks beside the headline")
    ap.add_argument("--cpu-blocks", type=int, default=128, help="oracle sample size (blocks of the workload)")
    ap.add_argument("--direct-cells", type=int, default=64,
                    help="seeded cells (plus half as many of largest |a|) for the error against the direct sum")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="MiB: one fill + one sum of that size before timing (HBM counter calibration)")
    ap.add_argument("--mlp-cache", default=None,
                    help="cache file of the trained surrogate (loaded when it matches, else trained and written)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-side", action="store_true", help="skip the table walks beside the headline")
    ap.add_argument("--no-direct", action="store_true", help="skip the error against the direct sum")
    ap.add_argument("--no-c2", action="store_true",
                    help="skip the 128^3 lognormal leg (isolated, 48-pixel columns)")
    ap.add_argument("--c2-steps", type=int, default=10)
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the learned-Ewald leg on the 128^3 field with 3P boundaries")
    ap.add_argument("--surrogate-steps", type=int, default=2)
    ap.add_argument("--no-mpe", action="store_true", help="skip the MPE MAC leg")
    ap.add_argument("--no-abu", action="store_true", help="skip the adaptive block update leg")
    ap.add_argument("--no-p1", action="store_true", help="skip the 1P2I filament leg")
    ap.add_argument("--no-cyl", action="store_true", help="skip the isothermal-cylinder accuracy leg")
    ap.add_argument("--no-points", action="store_true", help="skip the target-point leg")
    ap.add_argument("--no-octant", action="store_true",
                    help="skip the headline walk with one list per 4^3 block octant")
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


def measured_limiter(path, source, prefix=""):
    """Busy fractions of the address units and the vector ALU issue from a
    committed counter summary, or None when the kernel's source has changed
    since the counters were taken."""
    import hashlib
    try:
        kv = dict(l.split(": ", 1) for l in open(os.path.join(ROOT, path)).read().splitlines()
                  if l and not l.startswith("#") and ": " in l)
        sha = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()
    except OSError:
        return None
    if not sha.startswith(kv.get("source_sha256_prefix", "-")):
        return None
    return {"address_units_busy": float(kv[prefix + "ta_busy"]),
            "valu_issue_busy": float(kv[prefix + "valu_issue_busy"]),
            "source": "rocprofv3 counters (TA_TA_BUSY_sum, SQ_INSTS_VALU)", "summary": path}


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
    learned correction (cell groups at the table's Taylor offset, and reaching
    three times as far) beside the FP32 and FP64 table walks.  Training (on the
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
    legs = [("mlp_fp32", "mlp", False, 0, 1.0), ("mlp_fp32_reach3", "mlp", False, 0, 3.0),
            ("table_fp32", "table", False, 0, 1.0), ("table_fp64", "table", True, 0, 1.0)]
    if nside:
        legs += [("mlp_fp32_cols", "mlp", False, nside, 1.0), ("table_fp64_cols", "table", True, nside, 1.0)]
    for label, mode, fp64, ns, reach in legs:
        s = ot.Solver.for_grid(g, mac="ape", a_lim=a_lim, theta=0.5, ewald=mode, nside=ns, mlp_reach=reach)
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
        if label.startswith("mlp_fp32") and not label.endswith("_cols"):
            e["roofline"] = mlp_roofline(st)
            e["n_mlp_evals"] = st.n_mlp_evals
        out[label] = e
    return out


def mlp_roofline(st):
    """The surrogate gravity walk: matrix work of its network evaluations over
    the kernel's time (its vector part: the per-pair Taylor step and the
    activations)."""
    ach = st.n_mlp_evals * FLOP_MLP_EVAL / (st.ms_gravity * 1e-3) / 1e12
    valu = st.n_interactions * FLOP_PAIR_MLP_TAYLOR / (st.ms_gravity * 1e-3) / 1e12
    return {"bound": "mfma", "kernel": "k_eval_mlp_taylor", "achieved": ach, "peak": PEAK_FP16_MFMA,
            "unit": "TFLOP/s", "frac": ach / PEAK_FP16_MFMA, "flop_per_eval": FLOP_MLP_EVAL,
            "n_evals": st.n_mlp_evals, "ms": st.ms_gravity, "valu_tflops_taylor": valu,
            "valu_flop_per_pair": FLOP_PAIR_MLP_TAYLOR}


def fused_roofline(st):
    """The walk that carries the surrogate's gravity and the columns in one
    kernel: its vector work per (cell, node) pair (gravity, Taylor step,
    columns) over the kernel's time; the network's matrix work beside it."""
    ms = st.ms_columns
    fl = st.n_interactions * (FLOP_PAIR_MLP_TAYLOR + FLOP_COLS) / (ms * 1e-3) / 1e12
    mf = st.n_mlp_evals * FLOP_MLP_EVAL / (ms * 1e-3) / 1e12
    return {"bound": "alu", "kernel": "k_eval_cols_mlp", "achieved": fl, "peak": PEAK_FP32_VALU,
            "unit": "TFLOP/s", "frac": fl / PEAK_FP32_VALU, "flop_per_pair": FLOP_PAIR_MLP_TAYLOR + FLOP_COLS,
            "ms": ms, "mfma_tflops_network": mf, "mfma_frac": mf / PEAK_FP16_MFMA,
            "flop_per_eval": FLOP_MLP_EVAL, "n_evals": st.n_mlp_evals}


def cols_roofline(st, flop_pair, fp64, kernel):
    ms = st.ms_columns if st.ms_columns > 0 else st.ms_eval
    fl = st.n_interactions * flop_pair / (ms * 1e-3) / 1e12
    peak = PEAK_FP64_VALU if fp64 else PEAK_FP32_VALU
    return {"bound": "alu", "kernel": kernel, "achieved": fl, "peak": peak, "unit": "TFLOP/s",
            "frac": fl / peak, "flop_per_pair": flop_pair, "ms": ms}


def c5_setup(mlp_cache=None):
    """The headline workload, its APE limit (BH FP64 pre-pass) and the
    surrogate trained for its boundaries (untimed)."""
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
    rep = tr.mlp_train(cache_path=mlp_cache)
    train_s = time.perf_counter() - t0
    mlp = tr.mlp_get()
    tr.close()
    info = {"generate_s": gen_s, "a_lim": a_lim,
            "training": {"seconds": train_s, "ok": rep["ok"], "err_mlp": rep["err_mlp"],
                         "err_table": rep["err_table"], "loss_first": rep["loss_first"],
                         "loss_last": rep["loss_last"], "from_cache": bool(rep["from_cache"])}}
    return g, rho, kw, a_lim, mlp, rep, info


def c5_run(g, rho, kw, a_lim, mode, fp64, steps, warmup, mlp=None, accept=True, list_group=8):
    import torch
    import paper_1708_06142_amd as ot
    s = ot.Solver.for_grid(g, a_lim=a_lim, ewald=mode, nside=4, mlp_reach=C5_MLP_REACH, list_group=list_group,
                           **kw)
    if mlp is not None:
        s.mlp_set(*mlp, accept=accept)
    n = g.ncells
    dt = torch.float64 if fp64 else torch.float32
    outs = (torch.empty(n, dtype=dt, device="cuda"), torch.empty(3 * n, dtype=dt, device="cuda"),
            torch.empty(n * 192, dtype=dt, device="cuda"), torch.empty(n, dtype=dt, device="cuda"))
    ms, st, ms_eval, ms_list, ms_build = timed_steps(s, rho, outs, fp64, steps, warmup)
    s.close()
    e = {"value": n / (ms * 1e-3), "unit": "cells/s", "ms_per_step": ms,
         "phases_ms": {"build": ms_build, "lists": ms_list, "eval": ms_eval, "gravity": st.ms_gravity,
                       "columns": st.ms_columns},
         "ewald_used": ["table", "exact", "mlp"][st.ewald_used], "n_int": st.n_interactions,
         "total_list": st.total_list, "eval_wg_per_cu": st.eval_wg_per_cu}
    return outs, st, e


def maxnorm_diffs(outs, ref):
    """Largest |difference| of phi, acc, npix, tau over all cells, each
    normalised by the reference's largest |value| (|a| as a vector)."""
    res = {}
    for nm, a, r in zip(("phi", "acc", "npix", "tau"), outs, ref):
        d, mx = 0.0, 0.0
        for i in range(0, r.numel(), 1 << 28):
            d = max(d, float((a[i:i + (1 << 28)].double() - r[i:i + (1 << 28)]).abs().max()))
        mx = float(r.view(3, -1).pow(2).sum(0).sqrt().max()) if nm == "acc" else \
            max(float(r[i:i + (1 << 28)].abs().max()) for i in range(0, r.numel(), 1 << 28))
        res[f"d{nm}_maxnorm_vs_fp64_table"] = d / mx
    return res


def oracle_tree(g, kw, a_lim):
    """The oracle's tree of the workload with the same MAC, 64^3 Ewald table
    and 192-pixel column machinery (host FP64)."""
    import oracle
    t0 = time.perf_counter()
    t = oracle.Tree(g, mac="ape", a_lim=a_lim, theta_pix=kw["theta_pix"], nside=4, ewald="table", ew_n=64)
    return t, time.perf_counter() - t0


def direct_errors(t, g, phi, acc, ncells, seed=17):
    """e_a,max and e_Phi,max of the walk against the direct sum (the oracle's
    FP64 sum over all other cells with the same Ewald table) on seeded cells
    and the cells of largest |a|, normalised by the largest reference |a| and
    |Phi| over those cells."""
    import torch
    n = g.ncells
    amag = acc.view(3, -1).double().pow(2).sum(0)
    top = torch.topk(amag, ncells // 2).indices.cpu().numpy()
    rnd = np.random.default_rng(seed).choice(n, ncells, replace=False)
    tg = np.unique(np.concatenate([rnd, top]))
    t0 = time.perf_counter()
    pd, ad = t.direct(tg)
    sec = time.perf_counter() - t0
    idx = torch.from_numpy(tg).cuda()
    pw = phi[idx].double().cpu().numpy()
    aw = acc.view(3, -1)[:, idx].double().cpu().numpy()
    amax = np.sqrt((ad ** 2).sum(0)).max()
    ea = np.sqrt(((aw - ad) ** 2).sum(0)) / amax
    ep = np.abs(pw - pd) / np.abs(pd).max()
    return {"e_a_max": float(ea.max()), "e_phi_max": float(ep.max()), "cells": int(tg.size),
            "sample": f"{ncells} seeded cells and the {ncells // 2} of largest |a|",
            "reference": "oracle direct sum over all other cells, FP64" +
                         (", same 64^3 Ewald table" if any(g.bc) else " (isolated)"),
            "seconds": sec, "seconds_per_target": sec / tg.size}


def raymarch_errors(t, g, maps, ncells=12, seed=19, nside=4):
    """Largest |difference| of the per-cell maps from the oracle's ray-marched
    column densities (exact integrals of rho through the cells along the
    Nside-16 pixel-centre rays, averaged per pixel) on seeded cells and the
    cell of largest reference column, normalised by the largest reference
    value over those cells; one figure per map set."""
    import torch
    rng = np.random.default_rng(seed)
    tg = np.unique(np.concatenate([rng.choice(g.ncells, ncells, replace=False),
                                   [int(np.argmax(g.rho.reshape(-1)))]]))
    t0 = time.perf_counter()
    ref = np.stack([t.raymarch(int(c), nside) for c in tg])
    sec = time.perf_counter() - t0
    rmax = np.abs(ref).max()
    npx = 12 * nside * nside
    res = {}
    for label, npix in maps.items():
        v = npix.view(g.nb, npx, 512)
        got = np.stack([v[c // 512, :, c % 512].double().cpu().numpy() for c in tg])
        res[label] = float(np.abs(got - ref).max() / rmax)
    return {"maxnorm_vs_raymarch": res, "cells": int(tg.size), "seconds": sec,
            "sample": f"{ncells} seeded cells and the densest cell",
            "reference": f"oracle ray-marched columns, Nside 16 rays averaged into the {npx} pixels"}


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return None


def cpu_baseline(t, tree_s, g, nblk, seed=7):
    """The FP64 oracle's group walk with columns on a seeded sample of blocks
    of the same workload, on the host cores."""
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    nblk = min(nblk, g.nb)
    sel = np.sort(np.random.default_rng(seed).choice(g.nb, nblk, replace=False))
    t0 = time.perf_counter()
    t.walk_group(sel, columns=True)
    tw = time.perf_counter() - t0
    cells = 512 * nblk
    sec = tw + tree_s * (nblk / g.nb)  # tree build is O(all cells): the sample's share
    # the paper-literal walk (one depth-first traversal per cell, the MAC suite
    # at the cell itself), gravity only, on seeded cells of the same blocks
    cand = (512 * sel[:, None] + np.arange(512)).ravel()
    tg = np.sort(np.random.default_rng(seed + 1).choice(cand, min(4096, cand.size), replace=False))
    t0 = time.perf_counter()
    _, _, nint = t.walk_percell(tg)
    tp = time.perf_counter() - t0
    return {"value": cells / sec, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{nblk} seeded blocks ({cells} cells) of the same workload: group walk with the same "
                      f"MAC, FP64 64^3 Ewald table and 192-pixel columns; walk {tw:.2f} s + build share "
                      f"{tree_s * nblk / g.nb:.3f} s (tree, Ewald and node-ray tables)",
            "per_cell_walk": {"value": tg.size / tp, "unit": "cells/s", "cells": int(tg.size), "seconds": tp,
                              "entries_per_cell": float(nint.mean()),
                              "note": "the oracle's per-cell depth-first walk (MAC suite at the cell), gravity "
                                      "only, on seeded cells of the same blocks"}}


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
        flop = st.n_interactions * (FLOP_GRAV + FLOP_EWALD_TABLE) / (ms_eval * 1e-3) / 1e12
        peak = PEAK_FP64_VALU if fp64 else PEAK_FP32_VALU
        out[label] = {"value": n / (ms * 1e-3), "unit": "cells/s", "ms_per_step": ms, "ms_eval": ms_eval,
                      "ms_lists": ms_list, "n_int": st.n_interactions,
                      "roofline": {"bound": "alu", "kernel": f"k_eval{'64' if fp64 else '32'}<2P1I>",
                                   "achieved": flop, "peak": peak, "unit": "TFLOP/s", "frac": flop / peak,
                                   "flop_per_pair": FLOP_GRAV + FLOP_EWALD_TABLE}}
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
        flop = st.n_interactions * (FLOP_GRAV + FLOP_EWALD_TABLE) / (ms_eval * 1e-3) / 1e12
        peak = PEAK_FP64_VALU if fp64 else PEAK_FP32_VALU
        out[label] = {"value": n / (ms * 1e-3), "unit": "cells/s", "ms_per_step": ms, "ms_eval": ms_eval,
                      "ms_lists": ms_list, "n_int": st.n_interactions,
                      "roofline": {"bound": "alu", "kernel": f"k_eval{'64' if fp64 else '32'}<1P2I>",
                                   "achieved": flop, "peak": peak, "unit": "TFLOP/s", "frac": flop / peak,
                                   "flop_per_pair": FLOP_GRAV + FLOP_EWALD_TABLE}}
    s.close()
    (p32, a32), (p64, a64) = res["table_fp32"], res["table_fp64"]
    out["table_fp32"]["dphi_maxnorm_vs_fp64"] = float((p32.double() - p64).abs().max() / p64.abs().max())
    a64n = a64.view(3, -1).pow(2).sum(0).sqrt().max()
    out["table_fp32"]["da_maxnorm_vs_fp64"] = float((a32.double() - a64).abs().max() / a64n)
    return out


def points_leg(g, rho, a_lim, npts=20000, steps=3):
    """Gravity at arbitrary target points (sink particles, say; Sec. 2.1) on
    the large AMR grid: 20,000 seeded points inside the domain, each walked
    with its own list under the headline's MAC (APE a_lim; no columns), FP64
    pair kernels with the 64^3 Ewald table."""
    import torch
    import paper_1708_06142_amd as ot
    import workloads
    x = torch.from_numpy(workloads.target_points(g, npts - 5, seed=31)).cuda()
    n = x.shape[0]
    s = ot.Solver.for_grid(g, mac="ape", a_lim=a_lim, theta=0.5, ewald_n=64)
    s.build(rho)
    phi = torch.empty(n, dtype=torch.float64, device="cuda")
    acc = torch.empty((3, n), dtype=torch.float64, device="cuda")
    s.solve_points(x, phi, acc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = [s.solve_points(x, phi, acc) for _ in range(steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    s.close()
    st = sts[-1]
    ms_eval = float(np.mean([q.ms_eval for q in sts]))
    flop = st.n_interactions * (FLOP_GRAV + FLOP_EWALD_TABLE) / (ms_eval * 1e-3) / 1e12
    out = {"workload": f"{n} seeded points in the large AMR grid ({g.nb} blocks), 2P1I, APE a_lim {a_lim:.4g}, "
                       "FP64, 64^3 Ewald table",
           "value": n / (ms * 1e-3), "unit": "points/s", "ms_per_call": ms,
           "phases_ms": {"lists": float(np.mean([q.ms_list for q in sts])), "eval": ms_eval},
           "pairs_per_point": st.n_interactions / n, "max_list": st.max_list,
           "finite": bool(torch.isfinite(phi).all() and torch.isfinite(acc).all()),
           "roofline": {"bound": "alu", "kernel": "k_eval_points64<2P1I>", "achieved": flop,
                        "peak": PEAK_FP64_VALU, "unit": "TFLOP/s", "frac": flop / PEAK_FP64_VALU,
                        "flop_per_pair": FLOP_GRAV + FLOP_EWALD_TABLE}}
    progress("target-point leg done")
    return out


def cylinder_leg():
    """Isothermal cylinder in hydrostatic equilibrium (Sec. 3.1.4) at the
    paper's resolution, 256 x 128 x 128 cells, 1P2I with the 64^3 table: the
    FP32-Kahan walk's radial acceleration against the closed form
    g(R) = 2 pi G rho0 R / (1 + R^2 / r0^2) for the MAC settings of the paper's
    acceleration runs (APE 1e-3 and 1e-2, BH theta 0.5; the APE limits are
    absolute, that fraction of max g).  e_a,max is the largest relative error
    per cell between 2h from the axis and 2h inside the cut-off; e_a,max/gmax
    the largest error over max g."""
    import torch
    import paper_1708_06142_amd as ot
    import workloads
    n, r0 = 128, 1.0
    g = workloads.iso_cylinder(n=n, r0=r0)
    rc = g.meta["rcyl"]
    x = workloads.cell_centres(1.0, g.origin, g.level, g.coord).reshape(-1, 3)
    dy, dz = x[:, 1] - 0.5, x[:, 2] - 0.5
    R = np.hypot(dy, dz)
    gan = 2 * np.pi * R / (1 + R * R / (r0 * r0))
    gmax = float(gan[R <= rc].max())
    sel = (R >= 2.0 / n) & (R <= rc - 2.0 / n)
    rho = torch.from_numpy(g.rho.reshape(-1)).cuda()
    nc = g.ncells
    out = {"workload": f"isothermal cylinder r0 {r0}, cut off at {rc}, box 2x1x1, 256x128x128 cells "
                       f"({g.nb} blocks), 1P2I, 64^3 Ewald table, FP32-Kahan walk", "gmax": gmax}
    for label, kw in (("ape_1e-3", dict(mac="ape", a_lim=1e-3 * gmax)), ("ape_1e-2", dict(mac="ape", a_lim=1e-2 * gmax)),
                      ("bh_0.5", dict(theta=0.5))):
        s = ot.Solver.for_grid(g, ewald_n=64, **kw)
        outs = (torch.empty(nc, device="cuda"), torch.empty(3 * nc, device="cuda"))
        ms, st, ms_eval, _, _ = timed_steps(s, rho, outs, False, 2, 1)
        s.close()
        a = outs[1].view(3, -1).double().cpu().numpy()
        err = (a[1][sel] * dy[sel] + a[2][sel] * dz[sel]) / R[sel] + gan[sel]
        out[label] = {"e_a_max": float((np.abs(err) / gan[sel]).max()),
                      "e_a_median": float(np.median(np.abs(err) / gan[sel])),
                      "e_a_max_over_gmax": float(np.abs(err).max() / gmax),
                      "axial_over_gmax": float(np.abs(a[0]).max() / gmax),
                      "ms_per_step": ms, "pairs_per_cell": st.n_interactions / nc}
    progress("isothermal cylinder leg done")
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


def abu_leg(grid, a_lim, nsnap=6, seed=12, nside=0, tol_a=2.5e-4, tol_tau=1e-3):
    """Adaptive block update on a seeded sequence of snapshots of the
    benchmark field: each snapshot multiplies the density by 1 + 0.3 G(x - c),
    G a Gaussian bump of width 0.05 whose centre c moves by 0.02 per snapshot
    from a seeded start.  Per snapshot: the FP32 walk with ABU from the
    previous snapshot's ABU solution beside the plain FP32 walk; the corner
    tolerances are tol_a max|a| on the acceleration and, with columns,
    tol_tau max(kappa N_p) on every pixel's optical depth (both from the
    first snapshot's full walk).
    Each snapshot reports its time together with the ABU solution's error
    against the full walk (acceleration, maps, tau), so that a speedup is
    never quoted without the accuracy it costs."""
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
            tol = tol_a * float(acc_f.view(3, -1).double().pow(2).sum(0).sqrt().max())
            ttol = tol_tau * s.params.kappa * float(npix_f.abs().max()) if nside else None
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, upd = s.solve_abu(phi, acc, tol, npix=npix, tau=tau, tol_tau=ttol)
        torch.cuda.synchronize()
        ms_abu = (time.perf_counter() - t0) * 1e3
        amax = acc_f.view(3, -1).double().pow(2).sum(0).sqrt().max()
        ea = float((acc.double() - acc_f.double()).view(3, -1).pow(2).sum(0).sqrt().max() / amax)
        ep = float((phi.double() - phi_f.double()).abs().max() / phi_f.double().abs().max())
        row = {"updated_frac": float(upd.mean()), "ms_abu": ms_abu, "ms_full": ms_full,
               "ms_eval_abu": st.ms_eval, "ms_eval_full": stf.ms_eval, "e_a_max_vs_full": ea,
               "e_phi_max_vs_full": ep}
        if nside:
            nmax = npix_f.abs().max()
            dn = (npix - npix_f).abs().view(grid.nb, -1).max(1).values / nmax
            u = torch.from_numpy(upd.astype(bool)).cuda()
            row["e_npix_max_vs_full"] = float(dn.max())
            row["e_npix_max_updated_blocks"] = float(dn[u].max()) if bool(u.any()) else 0.0
            row["e_npix_max_kept_blocks"] = float(dn[~u].max()) if bool((~u).any()) else 0.0
            row["e_tau_max_vs_full"] = float((tau - tau_f).abs().max() / tau_f.abs().max())
        rows.append(row)
    s.close()
    out = {"workload": f"lognormal 128^3 x {nsnap} snapshots with a moving Gaussian bump (amplitude 0.3, "
                       f"width 0.05, 0.02 per snapshot, seed {seed}), APE a_lim 1e-3 a_max, FP32-Kahan walk, "
                       f"{npx if nside else 'no'} columns, corner tolerances {tol_a:g} max|a|"
                       + (f" and {tol_tau:g} max(kappa N_p) per pixel" if nside else ""),
           "snapshots": rows,
           "mean_updated_frac": float(np.mean([r["updated_frac"] for r in rows])),
           "ms_abu_mean": float(np.mean([r["ms_abu"] for r in rows])),
           "ms_full_mean": float(np.mean([r["ms_full"] for r in rows])),
           "e_a_max_vs_full": float(max(r["e_a_max_vs_full"] for r in rows)),
           "e_phi_max_vs_full": float(max(r["e_phi_max_vs_full"] for r in rows))}
    if nside:
        out["e_npix_max_vs_full"] = float(max(r["e_npix_max_vs_full"] for r in rows))
        out["e_tau_max_vs_full"] = float(max(r["e_tau_max_vs_full"] for r in rows))
    out["speedup"] = out["ms_full_mean"] / out["ms_abu_mean"]
    return out


def c2_leg(steps, warmup, nside=2, oracle_checks=True):
    """128^3 lognormal field (sigma_ln 1.5, seed 2), isolated, APE a_lim =
    1e-3 a_max, 48-pixel columns: the FP32-Kahan column walk with its maps in
    LDS, beside the FP64 walk; with its HBM counters when committed.  With
    oracle_checks, the FP32 walk's errors against the oracle's direct sum and
    its maps against the oracle's ray-marched columns."""
    import torch
    import paper_1708_06142_amd as ot
    import workloads
    grid = workloads.c2_lognormal(128)
    n = grid.ncells
    rho = torch.from_numpy(grid.rho.reshape(-1).copy()).cuda()
    npx = 12 * nside ** 2
    s = ot.Solver.for_grid(grid, mac="ape", eps_lim=1e-3, theta=0.5)
    s.build(rho)
    phi = torch.empty(n, device="cuda", dtype=torch.float32)
    acc = torch.empty(3 * n, device="cuda", dtype=torch.float32)
    a_lim = s.solve(phi, acc).a_lim_used  # a_lim from the BH pre-pass (untimed)
    s.close()
    s = ot.Solver.for_grid(grid, mac="ape", a_lim=a_lim, theta=0.5, nside=nside)
    outs = (phi, acc, torch.empty(n * npx, device="cuda"), torch.empty(n, device="cuda"))
    ms, st, ms_eval, ms_list, ms_build = timed_steps(s, rho, outs, False, steps, warmup)
    rl = cols_roofline(st, FLOP_PAIR_COLS, False, "k_eval_cols<float, isolated, maps in LDS>")
    traffic = measured_traffic("profiles/eval_cols_lognormal128_nside2_hbm_traffic.txt",
                               "paper_1708_06142_amd/csrc/k_columns.hip")
    rl["traffic"] = traffic["bytes"] if traffic else None
    rl["traffic_detail"] = traffic
    out = {"workload": f"lognormal 128^3 (sigma_ln 1.5, P(k)~k^-4, seed 2), isolated, APE a_lim=1e-3 a_max "
                       f"({a_lim:.4g}), {npx}-pixel columns, FP32-Kahan walk", "cells": n, "steps": steps,
           "value": n / (ms * 1e-3), "unit": "cells/s", "ms_per_step": ms,
           "phases_ms": {"build": ms_build, "lists": ms_list, "eval": ms_eval},
           "eval_wg_per_cu": st.eval_wg_per_cu, "roofline": rl,
           "interactions": {"n_int": st.n_interactions, "per_cell": st.n_interactions / n,
                            "max_list": st.max_list, "n_opened": st.n_opened, "n_accepted": st.n_accepted}}
    f64 = dict(device="cuda", dtype=torch.float64)
    outs64 = (torch.empty(n, **f64), torch.empty(3 * n, **f64), torch.empty(n * npx, **f64), torch.empty(n, **f64))
    ms64, st64, e64, _, _ = timed_steps(s, rho, outs64, True, max(2, steps // 2), 1)
    out["fp64_walk"] = {"value": n / (ms64 * 1e-3), "ms_per_step": ms64, "ms_eval": e64,
                        "roofline": cols_roofline(st64, FLOP_PAIR_COLS, True, "k_eval_cols<double, isolated>"),
                        "eval_wg_per_cu": st64.eval_wg_per_cu}
    out["fp32_vs_fp64"] = {k.replace("_vs_fp64_table", ""): v for k, v in maxnorm_diffs(outs, outs64).items()}
    s.close()
    del outs64
    if oracle_checks:
        import oracle
        t = oracle.Tree(grid, mac="ape", a_lim=a_lim, nside=nside)
        out["accuracy_vs_direct"] = direct_errors(t, grid, outs[0], outs[1], 256)
        out["columns_vs_raymarch"] = raymarch_errors(t, grid, {"fp32": outs[2]}, nside=nside)
        del t
    return out, grid, rho, a_lim


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    if args.calib_copy:
        nc = args.calib_copy * (1 << 20) // 4
        src = torch.ones(nc, device="cuda")      # fill kernel: writes exactly nc * 4 bytes
        total = src.sum()                         # reduction: reads exactly nc * 4 bytes
        torch.cuda.synchronize()
        del src, total
    g, rho, kw, a_lim, mlp, rep, info = c5_setup(args.mlp_cache)
    progress(f"large AMR set up: {g.nb} blocks, a_lim {a_lim:.4g}, surrogate ok={rep['ok']}")
    n = g.ncells
    outs, st, e = c5_run(g, rho, kw, a_lim, "mlp", False, args.steps, args.warmup, mlp, bool(rep["ok"]))
    progress(f"headline: {e['ms_per_step']:.1f} ms/step")
    if st.ms_gravity > 0:
        # surrogate gravity walk, then a column walk without gravity
        rl_grav = mlp_roofline(st)
        rl_cols = cols_roofline(st, FLOP_COLS, False, "k_eval_cols<float, 2P1I, columns only, maps in memory>")
        if st.ms_gravity >= st.ms_columns:
            dominant = rl_grav
            traffic = measured_traffic("profiles/eval_mlp_taylor_c5amr_hbm_traffic.txt",
                                       "paper_1708_06142_amd/csrc/k_mlp.hip")
        else:
            dominant = rl_cols
            traffic = measured_traffic("profiles/eval_cols_c5amr_nside4_nograv_hbm_traffic.txt",
                                       "paper_1708_06142_amd/csrc/k_columns.hip")
        kernels = {"gravity": rl_grav, "columns": rl_cols}
    else:
        dominant = fused_roofline(st)
        traffic = measured_traffic("profiles/eval_cols_mlp_c5amr_nside4_hbm_traffic.txt",
                                   "paper_1708_06142_amd/csrc/k_columns.hip")
        kernels = {"gravity_and_columns": dominant}
    dominant = dict(dominant, traffic=traffic["bytes"] if traffic else None, traffic_detail=traffic)
    if st.ms_gravity <= 0:
        dominant["busy_units"] = measured_limiter("profiles/eval_cols_mlp_c5amr_nside4_limiter.txt",
                                                  "paper_1708_06142_amd/csrc/k_columns.hip")
    out = {
        "metric": "cells/s for potential+accel+N_pix column densities at <=1e-3 rel err",
        "value": e["value"], "unit": "cells/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": e["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"AMR lognormal 512^3 effective (sigma_ln 2, P(k)~k^-4, seed 5), 128^3 base + 2 "
                               f"levels, {g.nb} blocks, x,y periodic z isolated (unit box), APE a_lim=1e-3 a_max "
                               f"+ BH theta_pix 0.25, 192-pixel columns, FP32-Kahan walk with the learned Ewald "
                               f"correction (FP16 matrix instructions, one evaluation per 4^3 cell group and list "
                               f"entry, Taylor step to each cell, mlp_reach {C5_MLP_REACH:g})",
                   "cells": n, "blocks": g.nb, "a_lim": a_lim, "columns": 192, "ewald": e["ewald_used"]},
        "phases_ms": e["phases_ms"], "eval_wg_per_cu": e["eval_wg_per_cu"],
        "interactions": {"n_int": st.n_interactions, "per_cell": st.n_interactions / n, "max_list": st.max_list,
                         "n_opened": st.n_opened, "n_accepted": st.n_accepted, "n_mlp_evals": st.n_mlp_evals,
                         "list_hist": list(st.list_hist)},
        "roofline": dominant,
        "kernels": kernels,
        "surrogate": info,
    }
    if not args.no_side:
        o64, st64, e64 = c5_run(g, rho, kw, a_lim, "table", True, args.side_steps, 1)
        e64["roofline"] = cols_roofline(st64, FLOP_PAIR_TABLE_COLS, True, "k_eval_cols<double, 2P1I>")
        out["fp64_table"] = e64
        out["accuracy_vs_fp64_table"] = maxnorm_diffs(outs, o64)
        o32, st32, e32 = c5_run(g, rho, kw, a_lim, "table", False, args.side_steps, 1)
        e32["roofline"] = cols_roofline(st32, FLOP_PAIR_TABLE_COLS, False, "k_eval_cols<float, 2P1I>")
        e32.update(maxnorm_diffs(o32, o64))
        out["fp32_table"] = e32
        del o32
        progress("FP64- and FP32-table walks done")
    else:
        o64 = None
    o_oct = None
    if not args.no_octant:
        # the headline walk with one list per 4^3 block octant in place of one
        # per block: the same MAC suite against each octant's box, so shorter
        # lists that still pass it at every cell
        import paper_1708_06142_amd as ot
        try:
            o_oct, st_oct, e_oct = c5_run(g, rho, kw, a_lim, "mlp", False, args.steps, args.warmup, mlp,
                                          bool(rep["ok"]), list_group=4)
        except (ot.OTError, torch.cuda.OutOfMemoryError) as ex:  # no room for eight lists per block
            o_oct, st_oct, e_oct = None, None, {"error": str(ex)}
            torch.cuda.empty_cache()
    if o_oct is not None:
        e_oct["list_group"] = 4
        e_oct["n_mlp_evals"] = st_oct.n_mlp_evals
        tr_oct = measured_traffic("profiles/eval_cols_mlp4_c5amr_nside4_hbm_traffic.txt",
                                  "paper_1708_06142_amd/csrc/k_columns.hip")
        e_oct["roofline"] = dict(fused_roofline(st_oct), kernel="k_eval_cols_mlp4",
                                 traffic=tr_oct["bytes"] if tr_oct else None, traffic_detail=tr_oct,
                                 busy_units=measured_limiter("profiles/eval_cols_mlp_c5amr_nside4_limiter.txt",
                                                             "paper_1708_06142_amd/csrc/k_columns.hip", "octant_"))
        if o64 is not None:
            e_oct.update(maxnorm_diffs(o_oct, o64))
        progress(f"octant lists: {e_oct['ms_per_step']:.1f} ms/step")
    if not args.no_octant:
        out["octant_lists"] = e_oct
    if not args.no_points:
        out["points"] = points_leg(g, rho, a_lim)
    torch.cuda.synchronize()
    if not args.no_direct or not args.no_cpu:
        t, tree_s = oracle_tree(g, kw, a_lim)
        if not args.no_direct:
            out["accuracy_vs_direct"] = direct_errors(t, g, outs[0], outs[1], args.direct_cells)
            if o64 is not None:
                out["fp64_table"]["accuracy_vs_direct"] = direct_errors(t, g, o64[0], o64[1], args.direct_cells)
            if o_oct is not None:
                out["octant_lists"]["accuracy_vs_direct"] = direct_errors(t, g, o_oct[0], o_oct[1],
                                                                          args.direct_cells)
                maps = {"block_lists": outs[2], "octant_lists": o_oct[2]}
                if o64 is not None:
                    maps["fp64_table"] = o64[2]
                out["columns_vs_raymarch"] = raymarch_errors(t, g, maps)
        if not args.no_cpu:
            out["cpu_baseline"] = cpu_baseline(t, tree_s, g, args.cpu_blocks)
        progress("oracle legs done")
        del t
    del outs, o64, o_oct
    torch.cuda.empty_cache()
    if not args.no_c2 or not args.no_surrogate or not args.no_abu or not args.no_mpe:
        c2, grid, rho2, a2 = c2_leg(args.c2_steps, 2, oracle_checks=not args.no_direct and not args.no_c2)
        if not args.no_c2:
            out["c2"] = c2
        progress("128^3 lognormal leg done")
        if not args.no_surrogate:
            out["surrogate_3p"] = surrogate_leg(grid, rho2, args.surrogate_steps, 2)
            progress("3P surrogate leg done")
        if not args.no_abu:
            out["abu"] = abu_leg(grid, a2)
            out["abu_columns"] = abu_leg(grid, a2, nside=2)
            progress("adaptive block update legs done")
        if not args.no_mpe:
            out["mpe"] = mpe_leg(grid, rho2, a2, max(2, args.c2_steps // 2), 2)
        del rho2
    if not args.no_c3:
        out["c3"] = c3_leg(4)
        progress("Plummer AMR leg done")
    if not args.no_p1:
        out["p1"] = p1_leg(4)
        progress("filament leg done")
    if not args.no_cyl:
        out["cylinder"] = cylinder_leg()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
