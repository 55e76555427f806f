#!/usr/bin/env python3
"""Throughput of the randomised primal-dual hot path on one MI355X.

Workload n1024_m4m_d64: a 1024 x 1024 synthetic sky (200 Gaussian blobs + 1000 point
sources), M = 2^22 visibilities with Gaussian u-v density (sigma = pi/4 rad/px) cut into
64 radial blocks of log-normal sizes, complex noise at 20 dB input SNR, l2-ball radii
from the chi-square 0.99 quantile.  All blocks active (p = 1).

One step is one full iteration of Algorithm 1 (steps 3-18: F Z x~, degridding with the
l2-ball projection and FP64 block norms, gridding of the dual change, F^dagger Z^dagger,
Psi^dagger with the dual clip, Psi and the primal update), replayed from a captured HIP
graph; inputs are resident in HBM before the timed region.  Also reported: Phi and
Phi^dagger alone (Gvis/s), the plain per-block form of the step, per-stage HIP-event
timings with the HBM roofline of the dominant kernel, and the FP64 CPU oracle timed on a
bounded sample (one iteration) on the host.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PD iters/s + Φ/Φ† Gvis/s at 1024²; batched FP32 vs plain, SNR within 0.05dB"
HBM_PEAK_GBS = 8000.0
WORKLOAD = "n1024_m4m_d64"


# the kernel each timed stage launches in the batched step
STAGE_KERNEL = {
    "fft_rows": "k_fwd_rows<2048, 1, 256>", "fft_cols": "k_fwd_cols<2048, 8, 512>",
    "degrid": "k_degrid<{T}, 1>", "block_norms": "k_block_stats", "grid": "k_grid_tiles<{T}, 1>",
    "grid_halo": "k_grid_halo<{T}>",
    "ifft_cols": "k_adj_cols<2048, 8, 512>", "ifft_rows": "k_adj_rows<2048, 1, 256, true> (with steps 17-18)",
    "psi_adj": "k_dwt_level (4 launches)", "psi_synth": "k_idwt_level (3 launches) + k_idwt_top",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stage_bytes(n, M_active, wavelets=8):
    """Algorithmic HBM bytes of one launch of each stage (FP32; N = n^2 pixels, 4N grid cells).

    Each operand is counted once at its size: complex grid 32N, half-transformed rows 16N,
    images 4N, coefficients 4N per basis, visibilities 8 B per complex value."""
    N = n * n
    nw = wavelets
    return {
        "fft_rows": 4 * N + 16 * N,                  # read x~, write n x 2n complex rows
        "fft_cols": 16 * N + 32 * N,                 # read the rows, write the 2n x 2n grid
        "degrid": 32 * M_active + 32 * N,            # coords, y, v in; e out; grid read once
        "grid": 32 * M_active + 64 * N,              # coords, e, v in; v out; running grid sum in+out
        "ifft_cols": 32 * N + 16 * N,
        # row pass with steps 17-18: rows, s~ and x in; x and x~ out
        "ifft_rows": 16 * N + 4 * N * 2 + 4 * N * 2,
        # Psi^dagger + clip: x~ in, s in+out (Dirac and details of every level, LL of the last),
        # LL scratch out+in between levels
        "psi_adj": 4 * N + 8 * N + nw * 8 * (3 * N // 4 + 3 * N // 16 + 3 * N // 64 + 4 * N // 256)
                   + nw * 4 * 2 * (N // 4 + N // 16 + N // 64),
        # Psi s: coefficients of levels 2.. in, LL scratch out and in between levels, then the
        # finest level (LL1 scratch, level-1 details, Dirac in; s~ out)
        "psi_synth": nw * 4 * (3 * N // 16 + 3 * N // 64 + 4 * N // 256) + nw * 4 * 2 * (N // 16 + N // 64)
                     + nw * 4 * (N // 4) + nw * 4 * (N // 4 + 3 * N // 4) + 4 * N + 4 * N,
    }


def traffic_from_profile(kernel_stage):
    """HBM bytes per launch from a committed counter summary, if it still matches the source."""
    path = os.path.join(ROOT, "profiles", f"{kernel_stage}_{WORKLOAD}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, rec["source"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--plain-steps", type=int, default=20)
    ap.add_argument("--op-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="grid tile side (0: library default)")
    ap.add_argument("--bin", type=int, default=0, help="max visibilities per work item (0: library default)")
    ap.add_argument("--wgs", type=int, default=0, help="workgroups of the persistent kernels (0: library default)")
    ap.add_argument("--autotune", action="store_true",
                    help="time the autotuner's candidates on this workload and use the fastest")
    ap.add_argument("--slice-vis", type=int, default=0,
                    help="max visibilities per gridding workgroup of one tile (0: default, -1: no split)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also copy a buffer of this many MiB once (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); multi-GPU runs are not part of "
              "this build", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_1610_08895_amd as R
    from paper_1610_08895_amd import _lib
    from paper_1610_08895_amd.solver import Solver, snr

    _lib.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = synth.WORKLOADS[WORKLOAD]
    t0 = time.time()
    inp = synth.make_inputs(w)
    log(f"inputs {time.time() - t0:.1f}s")
    tuned = None
    if args.autotune:
        from paper_1610_08895_amd import autotune

        rng = np.random.default_rng(0)
        y_probe = rng.standard_normal(w.M) + 1j * rng.standard_normal(w.M)
        tuned, _ = autotune.tune(w.n, inp.uv, inp.block_off, y_probe, np.full(w.d, 1.0), log=log)
        args.tile, args.bin, args.slice_vis = tuned["tile"], tuned["bin"], tuned["slice_vis"]
        log(f"autotuned {tuned} ({time.time() - t0:.1f}s)")
    plan = R.Plan(w.n, inp.uv, inp.block_off, tile=args.tile, bin=args.bin, slice_vis=args.slice_vis,
                  persistent_wgs=args.wgs)
    order = plan.order()
    log(f"plan {time.time() - t0:.1f}s items={plan.n_items}")
    x_true = torch.tensor(inp.x_true, dtype=torch.float32, device="cuda")
    y0 = plan.phi(x_true).cpu().numpy()
    y0_user = np.empty_like(y0)
    y0_user[order] = y0
    y_user, sig, eps = synth.add_noise(w, y0_user.astype(np.complex128), inp.block_off)
    y_plan = torch.tensor(y_user[order], dtype=torch.complex64, device="cuda")
    sara = R.Sara(w.n, 4)
    x0 = torch.tensor(synth.power_start(w.n, w.seed(synth.SEED_POWER)), dtype=torch.float32, device="cuda")
    phi_norm, _ = plan.norm(x0, max_it=50, rtol=0.0)
    psi_norm = 3.0
    log(f"setup {time.time() - t0:.1f}s ||Phi|| ~ {phi_norm:.4g}")

    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib * (1 << 18), dtype=torch.float32, device="cuda")
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")

    sol = Solver(plan, sara, y_plan, eps, psi_norm, phi_norm)
    ones = np.ones(plan.d, np.uint8)
    use_graph = not args.no_graph
    for _ in range(args.warmup):
        sol.step(ones)
    if use_graph:
        sol.capture()
        sol.step(ones, graph=True)
    torch.cuda.synchronize()

    # ---- timed region: K iterations ----
    torch.cuda.synchronize()
    t_a = time.perf_counter()
    for _ in range(args.steps):
        sol.step(ones, graph=use_graph)
    torch.cuda.synchronize()
    t_b = time.perf_counter()
    ms_per_step = (t_b - t_a) * 1e3 / args.steps
    iters_s = 1e3 / ms_per_step
    log(f"batched{'+graph' if use_graph else ''}: {ms_per_step:.4f} ms/iter = {iters_s:.1f} iters/s")

    # ---- per-stage HIP-event timings (eager steps, events on each stage's stream) ----
    sol.pd.timing(True)
    for _ in range(args.steps):
        sol.step(ones)
    stages = sol.pd.stage_times()
    sol.pd.timing(False)
    mean_ms = {k: v[0] / v[1] for k, v in stages.items() if v[1]}
    per_iter = {k: v[0] / args.steps for k, v in stages.items() if v[1]}
    sb = stage_bytes(w.n, w.M)
    dom = max((k for k in per_iter if k in sb), key=lambda k: per_iter[k])
    alg = sb[dom]
    achieved = alg / (mean_ms[dom] * 1e-3) / 1e9
    log("stages (mean ms/launch): " + ", ".join(f"{k}={v:.4f}" for k, v in mean_ms.items()))

    # ---- plain per-block form ----
    plain_ms = None
    if args.plain_steps > 0:
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        for _ in range(args.plain_steps):
            sol.step(ones, plain=True)
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - t_a) * 1e3 / args.plain_steps
    snr_db = snr(inp.x_true, sol.x())
    log(f"plain: {plain_ms} ms/iter; SNR after {sol.pd.iteration} iterations {snr_db:.2f} dB")

    # ---- Phi and Phi^dagger alone ----
    yb = torch.empty(plan.M, dtype=torch.complex64, device="cuda")
    xb = torch.empty(w.n, w.n, dtype=torch.float32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(3):
        plan.phi(x_true, yb)
        plan.phi_adj(y_plan, xb)
    ev[0].record()
    for _ in range(args.op_reps):
        plan.phi(x_true, yb)
    ev[1].record()
    for _ in range(args.op_reps):
        plan.phi_adj(y_plan, xb)
    ev[2].record()
    torch.cuda.synchronize()
    phi_ms = ev[0].elapsed_time(ev[1]) / args.op_reps
    phia_ms = ev[1].elapsed_time(ev[2]) / args.op_reps
    log(f"Phi {phi_ms:.4f} ms ({w.M / phi_ms / 1e6:.1f} Gvis/s), Phi^dagger {phia_ms:.4f} ms "
        f"({w.M / phia_ms / 1e6:.1f} Gvis/s)")
    # ---- Eq. 13 at x for every block (the adaptive schedule's exact refresh) ----
    rs = torch.empty(plan.d, 2, dtype=torch.float64, device="cuda")
    sol.pd.residual(rs)
    ev[0].record()
    for _ in range(args.op_reps):
        sol.pd.residual(rs)
    ev[1].record()
    torch.cuda.synchronize()
    resid_ms = ev[0].elapsed_time(ev[1]) / args.op_reps
    log(f"Eq. 13 refresh (all blocks at x) {resid_ms:.4f} ms")

    # ---- CPU oracle baseline: one iteration of Algorithm 1 on the same workload ----
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import pd as opd
        from oracle.measurement import Measurement
        from oracle.wavelets import Sara as OSara

        meas = Measurement(inp.uv, inp.block_off, (w.n, w.n))
        osara = OSara(w.n)
        for i in range(meas.d):
            meas.cells(i)
        prm = opd.default_params(psi_norm, phi_norm)
        yb_o = opd.split_blocks(meas, y_user)
        st = opd.init_state(meas, osara)
        mask = np.ones(meas.d, bool)
        t_a = time.perf_counter()
        opd.iteration(meas, osara, yb_o, eps, prm, st, mask)
        t_cpu = time.perf_counter() - t_a
        cpu = {"value": 1.0 / t_cpu, "unit": "iters/s", "cores": 1, "kind": "oracle",
               "sample": f"1 iteration of Algorithm 1 on the full {WORKLOAD} workload, all 64 blocks "
                         f"active, FP64 numpy/scipy (single-threaded), {t_cpu:.1f} s; host has "
                         f"{len(os.sched_getaffinity(0))} cores available"}
        log(f"cpu oracle: {t_cpu:.2f} s / iteration")

    traffic = traffic_from_profile(dom)
    out = {
        "metric": METRIC,
        "value": round(iters_s, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": w.n, "M": w.M, "d": plan.d, "p": 1.0, "tile": plan.tile,
                   "bin": args.bin or 1024, "slice_vis": args.slice_vis or -1, "autotuned": tuned is not None,
                   "form": "batched persistent kernels" + (" + HIP graph" if use_graph else ""),
                   "kernel": "Kaiser-Bessel 8x8, 2x oversampling", "sara": "Dirac + db1..db8, 4 levels"},
        "phi_gvis_s": round(w.M / phi_ms / 1e6, 2),
        "phi_adj_gvis_s": round(w.M / phia_ms / 1e6, 2),
        "eq13_refresh_ms": round(resid_ms, 4),
        "plain_iters_s": round(1e3 / plain_ms, 3) if plain_ms else None,
        "speedup_vs_plain": round(plain_ms / ms_per_step, 3) if plain_ms else None,
        "stage_algorithmic_bytes": sb,
        "snr_db": round(snr_db, 3),
        "stage_ms_per_launch": {k: round(v, 5) for k, v in mean_ms.items()},
        "roofline": {"kernel": dom, "kernel_symbol": STAGE_KERNEL.get(dom, dom).format(T=args.tile or 32), "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "algorithmic_bytes": alg},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
