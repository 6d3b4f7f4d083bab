"""Benchmark: implicit backward-Euler steps per second on one column of 594
species x 150 layers (7720 reactions), the size of the paper's largest
network (Section 2.2) on a 150-layer column.

One step = rates, right-hand side, step-matrix assembly, factorisation of
the block-tridiagonal step system, the substitution and the state update,
i.e. every stage of the implicit step, on inputs resident in HBM.  The
factorisation is block cyclic reduction by default (--solver cr: batched
Gauss-Jordan inversions of the eliminated layers of each level and dense
Schur products on the FP64 matrix cores) or block Thomas (--solver thomas:
one Schur complement inversion per layer, bottom to top).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--solver cr|thomas]
                    [--no-cpu-baseline] [--skip-mixed] [--skip-thomas]

Prints one JSON line.  The roofline entry is for the kernel with the largest
share of the step time; kernel times are measured with HIP events around
every launch on the column's stream during the timed steps.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
PEAK_FP64_VALU_TFLOPS = 78.6  # MI355X FP64 vector peak (256 CUs x 2.4 GHz x 128 flop)
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


def cr_levels(N):
    """Layers eliminated / kept at each level of block cyclic reduction."""
    out, rem, h = [], list(range(N)), 1
    while len(rem) > 1:
        if len(rem) == 3 and h > 1:      # both ends of {0, h, 2h} at once
            elim, kept = [rem[0], rem[2]], [rem[1]]
        else:
            elim = [k for k in rem if (k // h) % 2]
            kept = [k for k in rem if not (k // h) % 2]
        out.append((h, elim, kept))
        rem, h = kept, 2 * h
    return out


def cr_gemm_products(N):
    """Dense S x S block products of one cyclic-reduction factorisation
    (levels >= 1; level 0 has diagonal couplings and no products):
    per kept layer with a left / right neighbour one product A E / C E, one
    per Schur term subtracted from D, and one for each new coupling."""
    n = 0
    for h, elim, kept in cr_levels(N):
        if h == 1:
            continue
        for k in kept:
            hl, hr = k - h >= 0, k + h <= N - 1
            n += 2 * (hl + hr) + (k - 2 * h >= 0) + (k + 2 * h <= N - 1)
    return n


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


def bench_mixed(xod, torch, gnet, col, args, solver):
    """The same steps with FP32 Schur complements / products and FP64
    refinement; error of the first step against the FP64 GPU step."""
    import numpy as np
    stream = torch.cuda.current_stream().cuda_stream
    gm = xod.Column(gnet, col, precision=xod.XOD_MIXED, stream=stream, solver=solver)
    g64 = xod.Column(gnet, col, precision=xod.XOD_FP64, stream=stream, solver=solver)
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


def bench_batch(xod, torch, args, precision):
    """Ragged batch of independent columns (60-200 layers; 90-, 250- and
    594-species networks, three of each; per-column T offset and Kzz scale),
    stepped together: columns with the same padded block size share every
    launch (block Thomas across columns), in FP64 or in mixed precision
    (FP32 Schur complements, FP64 refinement of the group)."""
    import numpy as np
    import synth
    stream = torch.cuda.current_stream().cuda_stream
    t0 = time.perf_counter()
    cols = synth.make_batch(args.batch_cols)
    progress(f"batch: {len(cols)} columns generated")
    gnets, gcols = {}, []
    for i, (net, col) in enumerate(cols):
        if id(net) not in gnets:
            gnets[id(net)] = xod.Network(net)
        gcols.append(xod.Column(gnets[id(net)], col, precision=precision, stream=stream))
        if (i + 1) % 64 == 0:
            progress(f"batch: {i + 1} columns on the device")
    batch = xod.Batch(gcols)
    setup = time.perf_counter() - t0
    dts = np.full(len(gcols), args.dt)
    batch.step(dts)
    torch.cuda.synchronize()
    progress("batch: warm-up step done")
    k = args.batch_steps
    t0 = time.perf_counter()
    refine = fallback = 0
    for _ in range(k):
        st = batch.step(dts)
        refine = max(refine, max(x["refine_iters"] for x in st))
        fallback += sum(x["fp64_fallback"] for x in st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    layers = sum(c.N for c in gcols)
    flops = sum(2.0 * c.S ** 3 * c.N for c in gcols)
    sizes = {}
    for c in gcols:
        sizes[c.S] = sizes.get(c.S, 0) + 1
    out = {"value": k * len(gcols) / el, "unit": "column-steps/s",
           "batched_steps_per_s": k / el, "ms_per_batched_step": 1e3 * el / k,
           "columns": len(gcols), "columns_per_species_count": sizes, "layers": layers,
           "gauss_jordan_tflops": flops * k / el / 1e12, "setup_s": setup, "steps": k,
           "solver": "block Thomas across columns",
           "precision": "fp64" if precision == xod.XOD_FP64 else "mixed"}
    if precision != xod.XOD_FP64:
        out["max_group_refinements"] = refine
        out["column_fp64_fallbacks"] = fallback
    batch.close()
    for c in gcols:
        c.close()
    return out


def bench_photolysis(xod, torch, net, col, dz, calls=20):
    """Spectral photolysis rates of the 594-species network's 772 photolysis
    reactions on the 150-layer column: 10,000 wavelength bins, 463
    absorbers (Section 2.3.3).  Inputs resident on the device; the rate
    product is the MFMA-bound part (2 N L P flop)."""
    import numpy as np
    import synth
    sp = synth.make_spectrum(net)
    dev = torch.device("cuda:0")
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)   # noqa: E731
    n, dzt = d(col.n0), d(dz)
    ab, se, J0, dl, sph = (d(sp["absorbers"]), d(sp["sig_ext"]), d(sp["J0"]), d(sp["dlam"]),
                           d(sp["sig_ph"]))
    N, L, P, A = col.N, len(sp["J0"]), sp["sig_ph"].shape[0], len(sp["absorbers"])
    kph = torch.empty((N, P), dtype=torch.float64, device=dev)
    work = torch.empty(xod.photolysis_workspace(N, A, L, P), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    call = lambda: xod.photolysis_spectral(n, dzt, ab, se, J0, dl, sph, kph, work, 0.5, 1.0,   # noqa: E731
                                           stream)
    call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        call()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / calls
    xod.profile_reset()
    xod.set_option("profile", 1)
    for _ in range(calls):
        call()
    torch.cuda.synchronize()
    xod.set_option("profile", 0)
    ms, cnt = xod.profile_read("photolysis")
    flops = 2.0 * N * L * P
    g_us = 1e3 * ms / cnt if cnt else None
    ach = flops / (g_us * 1e-6) / 1e12 if g_us else None
    return {"us_per_call": 1e6 * el, "N": N, "L": L, "P": P, "A": A,
            "tau_product_flop": 2.0 * N * A * L, "rate_product_flop": flops,
            "roofline_rate_product": {"bound": "mfma", "kernel": "k_ph_gemm (FP64 MFMA, split K)",
                                      "avg_launch_us": g_us, "achieved": ach,
                                      "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                                      "frac": ach / PEAK_FP64_MFMA_TFLOPS if ach else None}}


def bench_serve(xod, torch, args, precision, gnet, net):
    """Poisson arrivals of steady-state solves (594 species x 150 layers,
    per-request T offset / Kzz scale / initial state, t_end 1e12 s,
    max |dn/n| < 1e-4), served by the continuous-batching loop: p50 / p99
    latency (submission to completion) and completed solves per second."""
    import numpy as np
    import synth
    stream = torch.cuda.current_stream().cuda_stream
    n = args.serve_requests
    arrivals = synth.poisson_arrivals(n, args.serve_rate)
    cols = [synth.make_request(j, net) for j in range(n)]
    fp = xod.Server.footprint(gnet, cols[0].N, precision)
    srv = xod.Server(hbm_budget_bytes=args.serve_slots * fp, max_slots=args.serve_slots,
                     precision=precision, stream=stream)
    opts = dict(tol_rel=1e-4, t_end=1e12, max_steps=3000)
    ids, done, lat, steps, states = [], {}, [], [], {}
    t0 = time.perf_counter()
    nsub = 0
    while len(done) < n:
        now = time.perf_counter() - t0
        while nsub < n and arrivals[nsub] <= now:
            ids.append(srv.submit(gnet, cols[nsub], **opts))
            nsub += 1
        if nsub == len(done):             # idle until the next arrival
            time.sleep(max(0.0, min(0.01, arrivals[nsub] - now)))
            continue
        srv.step()
        for j, rid in enumerate(ids):
            if rid in done:
                continue
            o = srv.poll(rid)
            if o["state"] >= xod.Server.DONE:
                progress(f"serve ({'fp64' if precision == xod.XOD_FP64 else 'mixed'}): request "
                         f"{j} done after {o['steps']} steps, latency {o['latency_s']:.2f} s")
                done[rid] = o
                lat.append(o["latency_s"])
                steps.append(o["steps"])
                states[j] = o["n"]
                srv.release(rid)
        if time.perf_counter() - t0 > args.serve_timeout:
            break
    wall = time.perf_counter() - t0
    incomplete = []
    for j, rid in enumerate(ids):
        if rid not in done:
            o = srv.poll(rid)
            incomplete.append({"request": j, "state": o["state"], "steps": o["steps"],
                               "rejects": o["rejects"], "t": o["t"]})
    for j in range(len(ids), n):
        incomplete.append({"request": j, "state": "not submitted"})
    srv.close()
    lat = np.array(lat)
    ok = sum(1 for o in done.values() if o["state"] == xod.Server.DONE)
    return {"requests": n, "completed": len(done), "converged": ok,
            "rate_per_s": args.serve_rate, "slots": args.serve_slots,
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "solves_per_s": len(done) / wall, "wall_s": wall,
            "mean_steps_per_solve": float(np.mean(steps)) if steps else None,
            "unfinished_at_timeout": incomplete,
            "precision": "fp64" if precision == xod.XOD_FP64 else "mixed"}, states


def panel_traffic():
    """HBM bytes per k_panel launch from the committed rocprofv3 counter runs
    (calibrated FETCH_SIZE + WRITE_SIZE), or None if the kernel source has
    changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_panel_594x150_traffic.md")
    src = os.path.join(ROOT, "paper_2512_06729_amd", "csrc", "k_btd.hip")
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    vals = {}
    for ln in text.splitlines():
        if ln.startswith("traffic_bytes_per_launch:"):
            vals["bytes"] = float(ln.split(":")[1])
        if ln.startswith("source_sha256"):
            vals["sha"] = ln.split(":")[-1].strip()
    return vals.get("bytes") if vals.get("sha") == sha else None


def timed_steps(xod, torch, gcol, dt, steps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        xod.xod_step(gcol, dt)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


KERNELS = ("panel", "update", "gemm", "prologue", "solve", "jacobian", "rates", "rhs")
T_START = time.perf_counter()


def progress(msg):
    """One line per finished stage on stderr (the result line is stdout)."""
    print(f"[bench {time.perf_counter() - T_START:7.1f} s] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dt", type=float, default=1e-6)
    ap.add_argument("--solver", choices=("cr", "thomas"), default="cr")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-every", type=int, default=1)
    ap.add_argument("--skip-mixed", action="store_true")
    ap.add_argument("--skip-thomas", action="store_true")
    ap.add_argument("--skip-batch", action="store_true")
    ap.add_argument("--batch-cols", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--skip-serve", action="store_true")
    ap.add_argument("--skip-photolysis", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=4)
    ap.add_argument("--serve-rate", type=float, default=5.0)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-timeout", type=float, default=70.0)
    ap.add_argument("--serve-fp64-only", action="store_true")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="copy 256 MiB device to device three times first (the plain copy "
                         "that scales FETCH_SIZE / WRITE_SIZE counters to bytes)")
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
    if args.pmc_calibrate:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        progress("calibration copies done (3 x 256 MiB)")
    net, col = synth.make_config(3)
    stream = torch.cuda.current_stream().cuda_stream
    gnet = xod.Network(net)
    solver = xod.XOD_SOLVER_CR if args.solver == "cr" else xod.XOD_SOLVER_THOMAS
    gcol = xod.Column(gnet, col, precision=xod.XOD_FP64, stream=stream, solver=solver)

    col_dz = gcol.grid()["dz"]            # layer thicknesses of the library's column grid
    progress("config-3 column on the device")
    for _ in range(args.warmup):
        xod.xod_step(gcol, args.dt)
    torch.cuda.synchronize()

    # timed region: the steps alone
    el = timed_steps(xod, torch, gcol, args.dt, args.steps)
    # kernel breakdown: the same number of steps again with HIP events around
    # every launch (profile_every thins the per-layer block-Thomas events)
    xod.profile_reset()
    xod.set_option("profile_every", args.profile_every)
    xod.set_option("profile", 1)
    el_prof = timed_steps(xod, torch, gcol, args.dt, args.steps)
    xod.set_option("profile", 0)

    kern = {}
    for name in KERNELS:
        ms, cnt = xod.profile_read(name)
        kern[name] = {"total_ms": ms, "launches": cnt,
                      "avg_us": 1e3 * ms / cnt if cnt else None}

    S, N = net.S, col.N
    # algorithmic flops per step of the kernels that carry the factorisation
    npanel = -(-S // 32)
    gj_flops = 2.0 * S ** 3                          # one Gauss-Jordan inversion
    panel_flops = 2.0 * S * 32 * 32 * npanel         # the panels' share of it
    if args.solver == "cr":
        gemm_flops = 2.0 * S ** 3 * cr_gemm_products(N)
    else:
        gemm_flops = 0.0
    upd_flops = N * (gj_flops - panel_flops)
    flops = {"gemm": gemm_flops, "update": upd_flops, "panel": N * panel_flops}
    dominant = max(("panel", "update", "gemm"), key=lambda k: kern[k]["total_ms"])
    dk = kern[dominant]
    steps_prof = args.steps   # events cover every timed step
    frac_prof = 1.0 if args.solver == "cr" else 1.0 / args.profile_every
    per_launch_flops = flops[dominant] * steps_prof * frac_prof / max(dk["launches"], 1)
    achieved = per_launch_flops / (dk["avg_us"] * 1e-6) / 1e12 if dk["avg_us"] else None
    if dominant == "panel":
        rl = {"bound": "alu", "kernel": "k_panel (Gauss-Jordan panel, FP64 VALU, one "
              "work-group per block)", "peak": PEAK_FP64_VALU_TFLOPS}
    else:
        rl = {"bound": "mfma", "kernel": ("k_gemm (cyclic-reduction Schur products, FP64 MFMA)"
                                          if dominant == "gemm" else
                                          "k_update (Gauss-Jordan trailing update, FP64 MFMA)"),
              "peak": PEAK_FP64_MFMA_TFLOPS}
    traffic = panel_traffic() if (dominant == "panel" and args.solver == "cr") else None
    rl.update({"achieved": achieved, "unit": "TFLOP/s",
               "frac": achieved / rl["peak"] if achieved else None, "traffic": traffic,
               "flops_per_launch": per_launch_flops, "avg_launch_us": dk["avg_us"]})
    def gemm_roofline(g, kernel):
        if not g["avg_us"]:
            return None
        g_ach = gemm_flops * args.steps / (g["total_ms"] * 1e-3) / 1e12
        return {"bound": "mfma", "kernel": kernel, "achieved": g_ach,
                "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": g_ach / PEAK_FP64_MFMA_TFLOPS, "flops_per_step": gemm_flops,
                "launches_per_step": g["launches"] / args.steps}

    lib = xod.get_option("gemm_lib")
    names = {0: "k_gemm (hand-written FP64 MFMA, row gathers fused)",
             1: "rocBLAS dgemm_batched (products of row-gathered operands; the gathers are "
                "not included)"}
    gemm_rl = gemm_roofline(kern["gemm"], names[lib])
    gemm_alt = None
    if args.solver == "cr":
        # the other block-product path on the same steps, for comparison
        xod.set_option("gemm_lib", 1 - lib)
        xod.profile_reset()
        xod.set_option("profile", 1)
        el_alt = timed_steps(xod, torch, gcol, args.dt, args.steps)
        xod.set_option("profile", 0)
        xod.set_option("gemm_lib", lib)
        ms, cnt = xod.profile_read("gemm")
        gemm_alt = gemm_roofline({"total_ms": ms, "launches": cnt,
                                  "avg_us": 1e3 * ms / cnt if cnt else None}, names[1 - lib])
        if gemm_alt:
            gemm_alt["ms_per_step_with_kernel_events"] = 1e3 * el_alt / args.steps
        progress("other block-product path profiled for comparison")

    # factor reuse: a step that solves with the factors the step before it
    # left.  Repeated frozen steps diverge on this network at this dt (the
    # oracle does the same), so each one follows a full step; its time is the
    # pair's less a full step's.
    frozen = None
    if args.solver == "cr":
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                xod.xod_step(gcol, args.dt)
                xod.xod_step_frozen(gcol, args.dt)
            torch.cuda.synchronize()
            el_pair = (time.perf_counter() - t0) / args.steps
            el_fr = el_pair - el / args.steps
            frozen = {"value": 1.0 / el_fr, "unit": "steps/s", "ms_per_step": 1e3 * el_fr,
                      "ms_per_full_plus_frozen_pair": 1e3 * el_pair,
                      "what": "xod_step_frozen after each xod_step: rates, F, solve with that "
                              "step's factors, update (no Jacobian, no factorisation)"}
            progress(f"frozen-matrix steps: {1.0 / el_fr:.1f} steps/s")
        except xod.XodError as e:
            frozen = {"error": str(e)}

    # Rosenbrock ROS2: one factorisation, two solves per step
    ros2 = None
    if args.solver == "cr":
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                xod.xod_step_ros2(gcol, args.dt)
            torch.cuda.synchronize()
            el_r = (time.perf_counter() - t0) / args.steps
            ros2 = {"value": 1.0 / el_r, "unit": "steps/s", "ms_per_step": 1e3 * el_r,
                    "what": "xod_step_ros2: two-stage Rosenbrock step (rates, two F, "
                            "Jacobian, one factorisation, two solves, update)"}
            progress(f"ROS2 steps: {1.0 / el_r:.2f} steps/s")
        except xod.XodError as e:
            ros2 = {"error": str(e)}

    # constant-step BDF2 (history: the previous step's starting state)
    bdf2 = None
    if args.solver == "cr":
        try:
            xod.xod_step(gcol, args.dt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                xod.xod_step_bdf2(gcol, args.dt)
            torch.cuda.synchronize()
            el_b = (time.perf_counter() - t0) / args.steps
            bdf2 = {"value": 1.0 / el_b, "unit": "steps/s", "ms_per_step": 1e3 * el_b,
                    "what": "xod_step_bdf2: linearly implicit BDF2 at constant step (rates, F "
                            "with the history term, Jacobian, factorisation, solve, update)"}
            progress(f"BDF2 steps: {1.0 / el_b:.2f} steps/s")
        except xod.XodError as e:
            bdf2 = {"error": str(e)}

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
                               "backward-Euler step (rates+RHS+Jacobian+block-tridiagonal "
                               "factorisation+solve+update)",
                   "S": S, "R": net.R, "N": N, "precision": "fp64", "dt": args.dt,
                   "solver": "block cyclic reduction" if args.solver == "cr" else "block Thomas"},
        "roofline": dict(rl),
        "roofline_schur_gemm": gemm_rl,
        "roofline_schur_gemm_other_path": gemm_alt,
        "frozen_matrix_steps": frozen,
        "ros2_steps": ros2,
        "bdf2_steps": bdf2,
        "kernels": kern,
        "ms_per_step_with_kernel_events": 1e3 * el_prof / args.steps,
    }
    gcol.close()
    progress(f"FP64 steps: {steps_per_s:.2f} steps/s")
    if not args.skip_thomas and args.solver == "cr":
        gt = xod.Column(gnet, col, precision=xod.XOD_FP64, stream=stream)
        xod.xod_step(gt, args.dt)
        k = max(2, args.steps // 5)
        et = timed_steps(xod, torch, gt, args.dt, k)
        line["thomas"] = {"value": k / et, "unit": "steps/s", "ms_per_step": 1e3 * et / k,
                          "steps": k}
        gt.close()
    if not args.skip_mixed:
        line["mixed"] = bench_mixed(xod, torch, gnet, col, args, solver)
        progress(f"mixed steps: {line['mixed']['value']:.2f} steps/s")
    if not args.skip_serve:
        s64, n64 = bench_serve(xod, torch, args, xod.XOD_FP64, gnet, net)
        if args.serve_fp64_only:
            smx, nmx = {}, {}
        else:
            smx, nmx = bench_serve(xod, torch, args, xod.XOD_MIXED, gnet, net)
        diffs = {}
        for floor in (1e-30, 1e-20, 1e-10):
            errs = []
            for j, a in n64.items():
                if j in nmx:
                    keep = np.abs(a) > floor * np.abs(a).sum(axis=1, keepdims=True)
                    errs.append(float(np.max(np.abs(nmx[j] - a)[keep] / np.abs(a)[keep])))
            diffs[f"y>{floor:g}"] = max(errs) if errs else None
        if smx:
            smx["max_rel_diff_vs_fp64_steady_state"] = diffs
        line["serve"] = {"fp64": s64, "mixed": smx or None}
    if not args.skip_photolysis:
        line["photolysis_spectral"] = bench_photolysis(xod, torch, net, col, col_dz)
        progress("spectral photolysis: %.1f us per call" % line["photolysis_spectral"]["us_per_call"])
    if not args.skip_batch:
        b64 = bench_batch(xod, torch, args, xod.XOD_FP64)
        progress(f"batch fp64: {b64['value']:.1f} column-steps/s")
        bmx = bench_batch(xod, torch, args, xod.XOD_MIXED)
        progress(f"batch mixed: {bmx['value']:.1f} column-steps/s")
        line["batch"] = {"fp64": b64, "mixed": bmx}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(net, col)
        progress("oracle timed")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
