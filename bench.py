"""Benchmark: implicit backward-Euler steps per second on one column of 594
species x 150 layers (7720 reactions), the size of the paper's largest
network (Section 2.2) on a 150-layer column.

One step = rates, right-hand side, step-matrix assembly, block-tridiagonal
factorisation (Schur complements inverted by blocked Gauss-Jordan with FP64
MFMA updates), the substitution chain and the state update, i.e. every
stage of the implicit step, on inputs resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line.  The roofline entry is for the dominant kernel (the
Schur-update GEMM of the factorisation); its average launch duration is
measured with HIP events on the column's stream during the timed steps.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
PEAK_HBM_GBS = 8000.0


def schur_update_flops(S, nb=32):
    """Algorithmic flops of the Gauss-Jordan Schur updates of one S x S
    Schur complement, panel by panel: each panel of nb_p real columns updates
    the S x (S - nb_p) remaining columns with a rank-nb_p product."""
    out = []
    for j0 in range(0, S, nb):
        nbp = min(nb, S - j0)
        out.append(2.0 * S * (S - nbp) * nbp)
    return out


def cpu_baseline(net, col, seconds=15.0):
    """The oracle's backward-Euler step on the same column, timed on the host
    cores for a bounded number of steps (about `seconds` of work)."""
    import numpy as np
    from oracle import integrate
    t0 = time.perf_counter()
    prob = integrate.Problem(net, col)
    setup = time.perf_counter() - t0
    n = col.n0.copy()
    steps = 0
    t0 = time.perf_counter()
    while True:
        n, _ = integrate.be_step(prob, n, 1e-6)
        steps += 1
        el = time.perf_counter() - t0
        if el > seconds or steps >= 20:
            break
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    return {"value": steps / el, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} oracle BE steps (dt=1e-6) of the 594x150 column, "
                      f"{el:.1f} s (+{setup:.1f} s grid/rate set-up untimed); "
                      "NumPy/SciPy with their default BLAS threads"}


def bench_mixed(xod, torch, gnet, col, args):
    """The same steps with FP32 Schur complements and FP64 refinement."""
    import numpy as np
    stream = torch.cuda.current_stream().cuda_stream
    gm = xod.Column(gnet, col, precision=xod.XOD_MIXED, stream=stream)
    g64 = xod.Column(gnet, col, precision=xod.XOD_FP64, stream=stream)
    st = xod.xod_step(gm, args.dt)
    xod.xod_step(g64, args.dt)
    a, b = gm.state(), g64.state()
    keep = np.abs(b) > 1e-30 * np.asarray(g64.grid()["ngas"])[:, None]
    err = float(np.max(np.abs(a - b)[keep] / np.abs(b)[keep]))
    for _ in range(max(0, args.warmup - 1)):
        xod.xod_step(gm, args.dt)
    torch.cuda.synchronize()
    iters = fb = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s = xod.xod_step(gm, args.dt)
        iters += s["refine_iters"]
        fb += s["fp64_fallback"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gm.close()
    g64.close()
    return {"value": args.steps / el, "unit": "steps/s", "ms_per_step": 1e3 * el / args.steps,
            "refine_iters_per_step": iters / args.steps, "fp64_fallbacks": fb,
            "first_step_max_rel_err_vs_fp64": err, "first_step_refine_iters": st["refine_iters"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dt", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-every", type=int, default=10)
    ap.add_argument("--skip-mixed", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): columns are "
              "independent, so more GPUs would only shard columns; no multi-GPU run "
              "is part of this benchmark.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2512_06729_amd as xod
    import synth

    torch.cuda.set_device(0)
    net, col = synth.make_config(3)
    stream = torch.cuda.current_stream().cuda_stream
    gnet = xod.Network(net)
    gcol = xod.Column(gnet, col, precision=xod.XOD_FP64, stream=stream)

    for _ in range(args.warmup):
        xod.xod_step(gcol, args.dt)
    torch.cuda.synchronize()

    xod.profile_reset()
    xod.set_option("profile_every", args.profile_every)
    xod.set_option("profile", 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        xod.xod_step(gcol, args.dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    xod.set_option("profile", 0)

    kern = {}
    for name in ("panel", "update", "prologue", "solve", "jacobian", "rates", "rhs"):
        ms, cnt = xod.profile_read(name)
        kern[name] = {"total_ms": ms, "launches": cnt,
                      "avg_us": 1e3 * ms / cnt if cnt else None}

    S, N = net.S, col.N
    fl = schur_update_flops(S)
    upd_launch_flops = float(np.mean(fl[:-1] if len(fl) > 1 else fl))
    # every layer profiled when profile_every == 1: launches = steps * N * npanel
    upd = kern["update"]
    achieved = upd_launch_flops / (upd["avg_us"] * 1e-6) / 1e12 if upd["avg_us"] else None

    steps_per_s = args.steps / el
    line = {
        "metric": "implicit steps/sec at 594 sp x 150 layers (FP64)",
        "value": steps_per_s,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded 594-species / 7720-reaction network, 150-layer column)",
        "config": {"workload": "single column, S=594 species, R=7720 reactions, N=150 layers, "
                               "backward-Euler step (rates+RHS+Jacobian+block Thomas+solve+update)",
                   "S": S, "R": net.R, "N": N, "precision": "fp64", "dt": args.dt},
        "roofline": {"bound": "mfma", "kernel": "k_update (Schur-update GEMM, FP64 MFMA)",
                     "achieved": achieved, "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_MFMA_TFLOPS if achieved else None,
                     "traffic": None,
                     "flops_per_launch": upd_launch_flops,
                     "avg_launch_us": upd["avg_us"]},
        "kernels": kern,
    }
    if not args.skip_mixed:
        line["mixed"] = bench_mixed(xod, torch, gnet, col, args)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(net, col)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
