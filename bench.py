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


def oracle_steps(seconds, max_steps, keep=0):
    """Backward-Euler steps of the oracle on the 594 x 150 column from its
    initial state at dt = 1e-6, for about `seconds` or `max_steps` steps;
    returns (steps, elapsed s, set-up s, the first `keep` states)."""
    from oracle import integrate
    import synth
    net, col = synth.make_config(3)
    t0 = time.perf_counter()
    prob = integrate.Problem(net, col)
    setup = time.perf_counter() - t0
    n = col.n0.copy()
    states = []
    steps = 0
    t0 = time.perf_counter()
    while True:
        n, _ = integrate.be_step(prob, n, 1e-6)
        steps += 1
        if len(states) < keep:
            states.append(n)
        el = time.perf_counter() - t0
        if (el > seconds and len(states) >= keep) or steps >= max_steps:
            break
    return steps, el, setup, states


def oracle_worker(seconds, max_steps):
    """Entry of the one-thread oracle timing (a child process whose BLAS and
    OpenMP thread counts were set to 1 before NumPy loaded)."""
    steps, el, setup, _ = oracle_steps(seconds, max_steps)
    print(json.dumps({"steps": steps, "elapsed_s": el, "setup_s": setup}), flush=True)


def cpu_baseline(seconds=12.0, keep=3):
    """The oracle's backward-Euler step on the same column, timed on the host
    cores for a bounded number of steps: once with the default BLAS threads
    (all cores) and once in a child process limited to one thread.  The
    first `keep` states of the all-core run are returned for the per-species
    error of the GPU steps."""
    import subprocess
    steps, el, setup, states = oracle_steps(seconds, 20, keep)
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    out = {"value": steps / el, "unit": "steps/s", "cores": cores, "kind": "oracle",
           "sample": f"{steps} oracle BE steps (dt=1e-6) of the 594x150 column from its "
                     f"initial state, {el:.1f} s (+{setup:.1f} s grid/rate set-up untimed); "
                     f"NumPy/SciPy with their default BLAS threads on {cores} cores"}
    env = dict(os.environ)
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS",
              "BLIS_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[v] = "1"
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-worker",
                            str(seconds / 2), "2"], env=env, cwd=ROOT, capture_output=True,
                           text=True, timeout=300)
        w = json.loads(r.stdout.strip().splitlines()[-1])
        out["one_thread"] = {"value": w["steps"] / w["elapsed_s"], "unit": "steps/s",
                             "cores": 1, "sample": f"{w['steps']} oracle BE steps, "
                             f"{w['elapsed_s']:.1f} s, one BLAS/OpenMP thread"}
    except Exception as e:      # reported, not fatal: the all-core figure stands
        out["one_thread"] = {"error": repr(e)[:200]}
    return out, states


def per_species(n, ref, ngas):
    """Largest relative error over layers of each species' densities with
    mixing ratio above 1e-30, summarised: max, median, worst species and the
    number of species per error decade."""
    import numpy as np
    keep = np.abs(ref) > 1e-30 * ngas[:, None]
    rel = np.where(keep, np.abs(n - ref) / np.where(keep, np.abs(ref), 1.0), 0.0)
    e = rel.max(axis=0)
    hist = {}
    for lo in (0, 1e-16, 1e-14, 1e-12, 1e-10, 1e-8, 1e-6, 1e-4):
        hi = lo * 100 if lo else 1e-16
        hist[f"<{hi:g}" if not lo else f"{lo:g}..{hi:g}"] = int(((e >= lo) & (e < hi)).sum())
    hist[">=1e-2"] = int((e >= 1e-2).sum())
    return {"max": float(e.max()), "median": float(np.median(e)),
            "worst_species": int(np.argmax(e)), "species_per_decade": hist}


def time_each(torch, reset, call, reps):
    """Wall time of `reps` calls, each bracketed by device synchronisations
    and each from the state reset() establishes (untimed).  Returns (total
    seconds, list of the calls' results)."""
    total, out = 0.0, []
    for _ in range(reps):
        reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out.append(call())
        torch.cuda.synchronize()
        total += time.perf_counter() - t0
    return total, out


def bench_mixed(xod, torch, gnet, col, args, solver):
    """The same steps with FP32 Schur complements / products and FP64
    refinement, each from the initial state; refinements per step and the
    error of the first step against the FP64 GPU step."""
    import numpy as np
    stream = torch.cuda.current_stream().cuda_stream
    gm = xod.Column(gnet, col, precision=xod.XOD_MIXED, stream=stream, solver=solver)
    g64 = xod.Column(gnet, col, precision=xod.XOD_FP64, stream=stream, solver=solver)
    st = xod.xod_step(gm, args.dt)
    xod.xod_step(g64, args.dt)
    a, b = gm.state(), g64.state()
    keep = np.abs(b) > 1e-30 * np.asarray(g64.grid()["ngas"])[:, None]
    err = float(np.max(np.abs(a - b)[keep] / np.abs(b)[keep]))
    reset = lambda: gm.set_state(col.n0)   # noqa: E731
    time_each(torch, reset, lambda: xod.xod_step(gm, args.dt), args.warmup)
    el, sts = time_each(torch, reset, lambda: xod.xod_step(gm, args.dt), args.steps)
    iters = sum(s["refine_iters"] for s in sts)
    fb = sum(s["fp64_fallback"] for s in sts)
    gm.close()
    g64.close()
    return {"value": args.steps / el, "unit": "steps/s", "ms_per_step": 1e3 * el / args.steps,
            "refine_iters_per_step": iters / args.steps, "fp64_fallbacks": fb,
            "first_step_max_rel_err_vs_fp64": err, "first_step_refine_iters": st["refine_iters"],
            "what": "each step from the initial state at the bench dt"}


def trajectory(xod, gnet, col, precision, solver, dt, steps, stream):
    """States after 1..steps backward-Euler steps from the initial state."""
    g = xod.Column(gnet, col, precision=precision, stream=stream, solver=solver)
    out = []
    for _ in range(steps):
        xod.xod_step(g, dt)
        out.append(g.state())
    g.close()
    return out


def bench_config1(xod, torch, stream, only=None):
    """Latency-bound workload: the 12-species x 20-layer column through the
    200-step fixed schedule dt_j = 1e-8 1.2^j, back to back (every step is
    synchronous: it reads its statistics).  only: one variant ("cr",
    "thomas", "thomas_panels"), for a kernel trace of that variant alone."""
    import synth
    from paper_2512_06729_amd import XOD_SOLVER_CR, XOD_SOLVER_THOMAS
    net, col = synth.make_config(1)
    gnet = xod.Network(net)
    sched = [1e-8 * 1.2 ** j for j in range(200)]
    out = {"workload": "S=12, R=30, N=20: 200 fixed-schedule backward-Euler steps",
           "variants": "thomas: block Thomas in one persistent launch each for the factorisation and "
                     "the solve (blocks up to 64); thomas_panels: the per-layer panel "
                     "kernels of the large blocks"}
    for name, solver, fused in (("cr", XOD_SOLVER_CR, 64), ("thomas", XOD_SOLVER_THOMAS, 64),
                                ("thomas_panels", XOD_SOLVER_THOMAS, 0)):
        if only and name != only:
            continue
        xod.set_option("fused_max_ld", fused)
        g = xod.Column(gnet, col, stream=stream, solver=solver)
        xod.xod_step(g, 1e-8)
        g.set_state(col.n0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for dt in sched:
            xod.xod_step(g, dt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"us_per_step": 1e6 * el / len(sched), "steps_per_s": len(sched) / el}
        g.close()
    xod.set_option("fused_max_ld", 64)
    gnet.close()
    return out


def bench_config2(xod, torch, stream):
    """The 90-species x 120-layer column (1200 reactions) integrated to steady
    state (max |dn/n| < 1e-4 with dt past the mixing time) by the library's
    adaptive driver: wall time, steps and rejections, for both
    factorisations."""
    import synth
    from paper_2512_06729_amd import XOD_SOLVER_CR, XOD_SOLVER_THOMAS
    net, col = synth.make_config(2)
    gnet = xod.Network(net)
    out = {"workload": "S=90, R=1200, N=120: adaptive backward Euler to steady state, "
                       "tol_rel 1e-4"}
    for name, solver in (("cr", XOD_SOLVER_CR), ("thomas", XOD_SOLVER_THOMAS)):
        g = xod.Column(gnet, col, stream=stream, solver=solver)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = xod.xod_integrate_to_steady_state(g, tol_rel=1e-4, check=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"wall_s": el, "steps": r["steps"], "rejects": r["rejects"],
                     "t_end_s": r["t"], "converged": r["converged"],
                     "ms_per_step": 1e3 * el / max(1, r["steps"] + r["rejects"])}
        g.close()
    gnet.close()
    return out


def bench_reuse(xod, torch, stream, gnet3, col3):
    """Factorisations kept across steps (the modified-Newton corrector of the
    DLSODES family): the 90 x 120 column to steady state with method 2
    against method 0 (cyclic reduction), and 20 fixed backward-Euler steps of
    1e-8 s and of 1e-6 s on the 594 x 150 column from its initial state with
    and without reuse.  Reports wall time, steps and factorisations per step."""
    import synth
    from paper_2512_06729_amd import XOD_SOLVER_CR
    net, col = synth.make_config(2)
    gnet = xod.Network(net)
    out = {"workload": "S=90, R=1200, N=120 to steady state (tol_rel 1e-4); S=594, R=7720, "
                       "N=150, 20 steps of 1e-6 s"}
    for method in (0, 2):
        g = xod.Column(gnet, col, stream=stream, solver=XOD_SOLVER_CR)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = xod.xod_integrate_to_steady_state(g, tol_rel=1e-4, method=method, check=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[f"steady_state_method{method}"] = {
            "wall_s": el, "steps": r["steps"], "rejects": r["rejects"],
            "factorizations": r["factorizations"], "newton_iters": r["newton_iters"],
            "factorizations_per_step": r["factorizations"] / max(1, r["steps"]),
            "converged": r["converged"]}
        g.close()
    gnet.close()
    gcol = xod.Column(gnet3, col3, stream=stream, solver=XOD_SOLVER_CR)
    for dt in (1e-8, 1e-6):
        for reuse in (0, 1):
            gcol.set_state(col3.n0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            key = f"fixed_dt_{dt:g}_reuse{reuse}"
            try:
                st = xod.xod_integrate_fixed_dt(gcol, dt, 20, reuse)
            except xod.XodError as e:
                out[key] = {"error": str(e)}
                continue
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            out[key] = {
                "steps_per_s": st["steps"] / el, "steps": st["steps"],
                "factorizations": st["factorizations"], "newton_iters": st["newton_iters"],
                "factorizations_per_step": st["factorizations"] / max(1, st["steps"])}
    gcol.close()
    return out


def hbm_roofline(kern, name, algo_bytes, kernels):
    """Achieved HBM rate of a memory-bound kernel group from its event-timed
    launches and its algorithmic bytes per launch."""
    k = kern.get(name)
    if not k or not k["avg_us"]:
        return None
    ach = algo_bytes / (k["avg_us"] * 1e-6) / 1e9
    return {"bound": "hbm", "kernels": kernels, "achieved": ach, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": ach / PEAK_HBM_GBS, "algorithmic_bytes": algo_bytes,
            "avg_launch_us": k["avg_us"]}


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


def bench_serve_sweep(xod, torch, args):
    """Continuous-batching serving of a two-size request stream (90- and
    250-species networks, 60-120 layers, per-request T offset, Kzz scale
    and initial state; steady state at tol 1e-4, t_end 1e12 s, at most
    3000 steps), Poisson arrivals at each rate of --serve-sweep, FP64 and
    mixed precision: p50 / p99 latency, solves/s, and requests the loop
    left unfinished.  Then the accuracy of the precisions against each
    other on two requests solved to tol 1e-9."""
    import numpy as np
    import synth
    stream = torch.cuda.current_stream().cuda_stream
    nets = {90: synth.make_network("c2", seed=1002), 250: synth.make_network("s250", seed=4250)}
    gnets = {s: xod.Network(n) for s, n in nets.items()}
    rates = [float(r) for r in args.serve_sweep.split(",")]
    n = args.serve_requests
    reqs = [synth.make_mixed_request(j, nets) for j in range(n)]
    fp = max(xod.Server.footprint(gnets[s], c.N, xod.XOD_MIXED) for s, c in reqs)
    out = {"workload": f"{n} requests per rate, networks of 90 and 250 species, 60-120 layers",
           "slots": args.serve_slots}
    for prec, pname in ((xod.XOD_FP64, "fp64"), (xod.XOD_MIXED, "mixed")):
        per = []
        for rate in rates:
            arrivals = synth.poisson_arrivals(n, rate)
            srv = xod.Server(hbm_budget_bytes=args.serve_slots * fp, max_slots=args.serve_slots,
                             precision=prec, stream=stream)
            ids, done, lat = [], {}, []
            t0 = time.perf_counter()
            nsub = 0
            while len(done) < n:
                now = time.perf_counter() - t0
                while nsub < n and arrivals[nsub] <= now:
                    s, c = reqs[nsub]
                    ids.append(srv.submit(gnets[s], c, tol_rel=1e-4, t_end=1e12,
                                          max_steps=3000))
                    nsub += 1
                if nsub == len(done):
                    time.sleep(max(0.0, min(0.01, arrivals[nsub] - now)))
                    continue
                srv.step()
                for rid in ids:
                    if rid in done:
                        continue
                    o = srv.poll(rid)
                    if o["state"] >= xod.Server.DONE:
                        done[rid] = o
                        lat.append(o["latency_s"])
                        srv.release(rid)
                if time.perf_counter() - t0 > args.serve_timeout:
                    break
            wall = time.perf_counter() - t0
            srv.close()
            lat = np.array(lat)
            conv = sum(1 for o in done.values() if o["state"] == xod.Server.DONE)
            per.append({"rate_per_s": rate, "completed": len(done), "converged": conv,
                        "unfinished": n - len(done),
                        "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
                        "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
                        "solves_per_s": len(done) / wall, "wall_s": wall})
            progress(f"serve sweep {pname} rate {rate}: {len(done)}/{n} done in {wall:.1f} s")
        out[pname] = per
    # accuracy: two requests to a tight tolerance in both precisions
    diffs = []
    for j in range(2):
        s, c = reqs[j]
        st = {}
        for prec in (xod.XOD_FP64, xod.XOD_MIXED):
            g = xod.Column(gnets[s], c, precision=prec, stream=stream)
            xod.xod_integrate_to_steady_state(g, tol_rel=1e-9, t_end=1e30, max_steps=6000,
                                              check=False)
            st[prec] = g.state()
            ngas = g.grid()["ngas"][:, None]
            g.close()
        a, b = st[xod.XOD_FP64], st[xod.XOD_MIXED]
        keep = a > 1e-30 * ngas
        diffs.append(float(np.max(np.abs(b - a)[keep] / a[keep])))
    out["mixed_vs_fp64_tight_steady_state_max_rel_diff_y_gt_1e-30"] = diffs
    for g in gnets.values():
        g.close()
    return out


def bench_parcel(xod, torch, gnet, col, stream):
    """One global iteration of the Lagrangian parcel (bottom to top and back
    over the 594-species x 150-layer column, molecular diffusion as a
    pseudo-reaction, adaptive backward Euler within each layer's residence
    time): wall time, visits and steps.  Sequential by construction: every
    step is one S x S block."""
    g = xod.Column(gnet, col, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = xod.xod_parcel_pass(g, 1e-8)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    g.close()
    return {"workload": "one parcel pass over the 594 x 150 column (299 layer visits)",
            "wall_s": el, "visits": st["visits"], "steps": st["steps"],
            "rejects": st["rejects"], "ms_per_step": 1e3 * el / max(1, st["steps"] + st["rejects"])}


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
    ap.add_argument("--skip-small", action="store_true",
                    help="skip the 12-species latency and 90-species steady-state legs")
    ap.add_argument("--skip-integrators", action="store_true",
                    help="skip the frozen, ROS2, BDF2 and Newton legs")
    ap.add_argument("--batch-cols", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--skip-serve", action="store_true")
    ap.add_argument("--skip-photolysis", action="store_true")
    ap.add_argument("--skip-parcel", action="store_true")
    ap.add_argument("--only-config1", choices=("cr", "thomas", "thomas_panels"),
                    help="run only the 12-species latency leg with one factorisation variant "
                         "(201 steps: one warm-up and the 200-step schedule) and print its line")
    ap.add_argument("--skip-reuse", action="store_true",
                    help="skip the kept-factorisation legs (steady state method 2, fixed dt)")
    ap.add_argument("--serve-requests", type=int, default=4)
    ap.add_argument("--serve-rate", type=float, default=5.0)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-timeout", type=float, default=70.0)
    ap.add_argument("--serve-fp64-only", action="store_true")
    ap.add_argument("--serve-sweep", default="",
                    help="comma-separated arrival rates: run the two-size serving sweep "
                         "(not part of the default run)")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="copy 256 MiB device to device three times first (the plain copy "
                         "that scales FETCH_SIZE / WRITE_SIZE counters to bytes)")
    ap.add_argument("--oracle-worker", nargs=2, type=float, metavar=("SECONDS", "STEPS"),
                    help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_worker:
        oracle_worker(args.oracle_worker[0], int(args.oracle_worker[1]))
        return
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
    if args.only_config1:
        stream = torch.cuda.current_stream().cuda_stream
        print(json.dumps({"config1_latency": bench_config1(xod, torch, stream,
                                                           only=args.only_config1)}))
        return
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
    grid = gcol.grid()
    col_dz, ngas = grid["dz"], np.asarray(grid["ngas"])
    progress("config-3 column on the device")

    # Every timed step starts from the column's initial state (reset untimed),
    # so each leg times the same physical step whatever ran before it.
    reset = lambda: gcol.set_state(col.n0)   # noqa: E731
    be = lambda: xod.xod_step(gcol, args.dt)   # noqa: E731
    time_each(torch, reset, be, args.warmup)
    el, _ = time_each(torch, reset, be, args.steps)
    # kernel breakdown: the same steps again with HIP events around every
    # launch (profile_every thins the per-layer block-Thomas events)
    xod.profile_reset()
    xod.set_option("profile_every", args.profile_every)
    xod.set_option("profile", 1)
    el_prof, _ = time_each(torch, reset, be, args.steps)
    xod.set_option("profile", 0)

    kern = {}
    for name in KERNELS:
        ms, cnt = xod.profile_read(name)
        kern[name] = {"total_ms": ms, "launches": cnt,
                      "avg_us": 1e3 * ms / cnt if cnt else None}

    S, N, R = net.S, col.N, net.R
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
    frac_prof = 1.0 if args.solver == "cr" else 1.0 / args.profile_every
    per_launch_flops = flops[dominant] * args.steps * frac_prof / max(dk["launches"], 1)
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
        el_alt, _ = time_each(torch, reset, be, args.steps)
        xod.set_option("profile", 0)
        xod.set_option("gemm_lib", lib)
        ms, cnt = xod.profile_read("gemm")
        gemm_alt = gemm_roofline({"total_ms": ms, "launches": cnt,
                                  "avg_us": 1e3 * ms / cnt if cnt else None}, names[1 - lib])
        if gemm_alt:
            gemm_alt["ms_per_step_with_kernel_events"] = 1e3 * el_alt / args.steps
        progress("other block-product path profiled for comparison")

    # HBM-bound kernel groups: algorithmic bytes per launch (reads of the rate
    # coefficients and the state, writes of the outputs; FP64)
    hbm = {
        "rates": hbm_roofline(kern, "rates", 16.0 * N * R, "k_rates: writes k_f, k_r"),
        "rhs": hbm_roofline(kern, "rhs", 16.0 * N * R + 16.0 * N * S,
                            "k_wrate + k_rhs: reads k_f, k_r, n; writes F"),
        "jacobian": hbm_roofline(kern, "jacobian", 16.0 * N * R + 8.0 * N * S + 8.0 * N * S * S,
                                 "k_dwd + k_jac: reads k_f, k_r, n; writes the S x S blocks "
                                 "(the stored blocks are ld x ld, ld = 608: 4.8 % more)"),
    }

    integ = {}
    if args.solver == "cr" and not args.skip_integrators:
        # factor reuse: a backward-Euler step solving with the factors the full
        # step before it left (both from the initial state; the full step is
        # untimed)
        def after_full():
            reset()
            xod.xod_step(gcol, args.dt)
        for name, call, pre, what in (
                ("frozen_matrix_steps", lambda: xod.xod_step_frozen(gcol, args.dt), after_full,
                 "xod_step_frozen after an untimed xod_step from the initial state: rates, F, "
                 "solve with that step's factors, update (no Jacobian, no factorisation)"),
                ("ros2_steps", lambda: xod.xod_step_ros2(gcol, args.dt), reset,
                 "xod_step_ros2 from the initial state: two-stage Rosenbrock step (rates, two "
                 "F, Jacobian, one factorisation, two solves, update)"),
                ("bdf2_steps", lambda: xod.xod_step_bdf2(gcol, args.dt), after_full,
                 "xod_step_bdf2 after an untimed xod_step from the initial state (its "
                 "history): rates, F with the history term, Jacobian, factorisation, solve, "
                 "update"),
                ("newton3_steps", lambda: xod.xod_step_newton(gcol, args.dt, 3), reset,
                 "xod_step_newton with 3 iterations from the initial state: one Jacobian and "
                 "factorisation, three solves and right-hand sides")):
            try:
                e, _ = time_each(torch, pre, call, max(2, args.steps // 2))
                k = max(2, args.steps // 2)
                integ[name] = {"value": k / e, "unit": "steps/s", "ms_per_step": 1e3 * e / k,
                               "steps": k, "what": what}
                progress(f"{name}: {k / e:.2f} steps/s")
            except xod.XodError as ex:
                integ[name] = {"error": str(ex)}

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
                               "factorisation+solve+update), every timed step from the "
                               "initial state",
                   "S": S, "R": R, "N": N, "precision": "fp64", "dt": args.dt,
                   "solver": "block cyclic reduction" if args.solver == "cr" else "block Thomas"},
        "roofline": dict(rl),
        "roofline_schur_gemm": gemm_rl,
        "roofline_schur_gemm_other_path": gemm_alt,
        "roofline_hbm": hbm,
        "kernels": kern,
        "ms_per_step_with_kernel_events": 1e3 * el_prof / args.steps,
    }
    line.update(integ)
    gcol.close()
    progress(f"FP64 steps: {steps_per_s:.2f} steps/s")
    if not args.skip_thomas and args.solver == "cr":
        gt = xod.Column(gnet, col, precision=xod.XOD_FP64, stream=stream)
        k = max(2, args.steps // 5)
        et, _ = time_each(torch, lambda: gt.set_state(col.n0), lambda: xod.xod_step(gt, args.dt),
                          k)
        line["thomas"] = {"value": k / et, "unit": "steps/s", "ms_per_step": 1e3 * et / k,
                          "steps": k}
        gt.close()
    if not args.skip_mixed:
        line["mixed"] = bench_mixed(xod, torch, gnet, col, args, solver)
        progress(f"mixed steps: {line['mixed']['value']:.2f} steps/s")
    if not args.skip_small:
        line["config1_latency"] = bench_config1(xod, torch, stream)
        progress("config 1: %.1f us/step (cr), %.1f (thomas), %.1f (thomas, panel kernels)" % (
            line["config1_latency"]["cr"]["us_per_step"],
            line["config1_latency"]["thomas"]["us_per_step"],
            line["config1_latency"]["thomas_panels"]["us_per_step"]))
        line["config2_steady_state"] = bench_config2(xod, torch, stream)
        progress("config 2 steady state: %.2f s (cr)" %
                 line["config2_steady_state"]["cr"]["wall_s"])
    if not args.skip_reuse:
        line["factor_reuse"] = bench_reuse(xod, torch, stream, gnet, col)
        fr = line["factor_reuse"]
        progress("factor reuse: steady state %.2f s with kept factorisations (%.2f per step), "
                 "%.2f s without; fixed dt 1e-8: %s vs %s steps/s (%s factorisations per step)" % (
                     fr["steady_state_method2"]["wall_s"],
                     fr["steady_state_method2"]["factorizations_per_step"],
                     fr["steady_state_method0"]["wall_s"],
                     fr["fixed_dt_1e-08_reuse1"].get("steps_per_s"),
                     fr["fixed_dt_1e-08_reuse0"].get("steps_per_s"),
                     fr["fixed_dt_1e-08_reuse1"].get("factorizations_per_step")))
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
    if not args.skip_parcel:
        line["parcel_pass"] = bench_parcel(xod, torch, gnet, col, stream)
        progress("parcel pass: %.2f s" % line["parcel_pass"]["wall_s"])
    if args.serve_sweep:
        line["serve_sweep"] = bench_serve_sweep(xod, torch, args)
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
        base, ref_states = cpu_baseline()
        line["cpu_baseline"] = base
        progress("oracle timed")
        # per-species error of three GPU steps from the initial state against
        # the oracle's three steps (each trajectory on its own)
        err = {}
        k = len(ref_states)
        for name, prec, r64 in (("fp64", xod.XOD_FP64, 0), ("fp64_refined", xod.XOD_FP64, 1),
                                ("mixed", xod.XOD_MIXED, 0)):
            if name == "mixed" and args.skip_mixed:
                continue
            xod.set_option("refine64", r64)
            traj = trajectory(xod, gnet, col, prec, solver, 1e-6, k, stream)
            xod.set_option("refine64", 0)
            err[name] = per_species(traj[-1], ref_states[-1], ngas)
            err[name]["steps"] = k
        line["per_species_error_vs_oracle"] = err
        progress("per-species error vs the oracle done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
