#!/usr/bin/env python3
"""Throughput benchmark of the ms2 force/energy path on one MI355X.

Workload (one "step" = every system advances one MD step through the whole
hot path: Gear predictor, site frames, partner search + site-pair forces /
torques / energy / virial / volume-derivative sums, fixed-order reductions,
corrector, isokinetic thermostat, Lustig moment sums):
  batched state points -- 256 independent rigid two-centre LJ + point
  quadrupole fluids (elongation 0.3, Q^2 = 2), N ~ U{500..4000},
  rho ~ U(0.1, 0.8), T ~ U(1, 3), rc = 0.48 L, reaction field eps = inf,
  FP32 site arithmetic with FP64 accumulation, moments every step, all
  systems resident on the GPU and advanced by one hipGraph per K steps.

Printed JSON line: site-pair interactions/s of the batched form (value; the
median of five timed windows of K steps), MD steps/s, the plain
one-system-per-launch form on the same 256 systems, the same batched
workload in FP64, the ionic-solution system with Ewald (real-space and
reciprocal calls timed apart, and its MD step rate), the serving form at its
configured request size (2e4 steps, 1000-step ACF window) with a second run
at 0.7 x the measured capacity, the pair kernel's roofline (HIP events around
its launches inside the timed graph) and the oracle timed on the host cores
as a CPU baseline.

--case NAME runs one small batch only (a lone system advanced K steps by
graph replay) and prints its step time: the launch-gap traces of the
persistent-kernel decision are taken with it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 operations (a fused multiply-add counts 2, rcp / rsqrt 1)
# of one 2CLJQ molecule pair, counted from the site-pair formulas:
#   LJ site pair   48: separation 6, |r|^2 5, 1/r^2 1, powers and c6, c12
#                      terms 5, u and its sum 2, u'/r 4, force 3, the two
#                      sites' force sums 6 (32); d2U/ds2: r.R 5, u'' 4, the
#                      combination 6, its sum 1 (16)
#   QQ site pair  122: 1/R 1, n 3, three cosines 15, P 16, its three
#                      partial derivatives 19, R^-5 3, prefactor 1, u and its
#                      sum 2, force 24, the two orientation gradients 24,
#                      their sums and the force sums 12, d2U/ds2 and its sum 2
#   molecule pair  21: the pair force summed over its 5 site pairs 15,
#                      dU/ds = -R.F 5 and its sum 1
FLOP_LJ = 48
FLOP_QQ = 122
FLOP_MOL = 21
FLOP_PER_MOL_PAIR = 4 * FLOP_LJ + FLOP_QQ + FLOP_MOL        # 335
PEAK_FP32_VALU = 157.3e12     # MI355X dense FP32 vector FLOP/s (packed FP32)
PEAK_FP32_UNPACKED = 78.6e12  # without packed FP32 instructions (not used by this build)
METRIC = "site-pair interactions/s and MD steps/s (batched vs plain) at 1 GPU; p50/p99 latency"
WINDOWS = 5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_label(tuned):
    """The pair kernel(s) the batched launch used, from the tile shape per size bucket."""
    if not tuned:
        return "pair_kernel<float, 2CLJQ> (heuristic tile shapes)"
    names = sorted({"pair_sym_kernel<float, 2CLJQ> (64 x 64 tile pairs, 4 waves)" if w == 0
                    else f"pair_kernel<float, 2CLJQ, {w} wave(s)> (j chunk {j})" for w, j in tuned.values()})
    return " + ".join(names)


def host_cpu():
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def _oracle_worker(args):
    """One host process: the oracle's Gear NVT with moment sampling on one
    state point (1 initial evaluation + `steps` steps); returns (site pairs,
    seconds)."""
    s_index, steps = args
    import oracle
    from paper_1507_07548_amd import inputs
    s = inputs.batched_state_point(s_index)
    s.md.n_steps = steps
    _, _, sums = oracle.forces(s)
    t0 = time.perf_counter()
    oracle.md(s, want_log=False)
    return sums[11] * (steps + 1), time.perf_counter() - t0


def cpu_baseline(max_procs=16, steps=8):
    """The FP64 oracle as it stands (one thread per process) on the host
    cores: one process per state point of a fixed sample (state points
    0..P-1 of the same workload), all running at once; site pairs of the
    sample / wall time.  The single-process rate is reported beside it."""
    import multiprocessing as mp
    model, avail = host_cpu()
    procs = max(1, min(max_procs, avail))
    jobs = [(k, steps) for k in range(procs)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    sp = sum(r[0] for r in res)
    single = sum(r[0] for r in res) / sum(r[1] for r in res)
    return {"value": sp / wall, "unit": "site-pair interactions/s", "cores": procs, "kind": "oracle",
            "sample": f"state points 0..{procs - 1} of the batched workload (FP64 oracle, Gear NVT with "
                      f"moments, 1 initial evaluation + {steps} steps each), one single-threaded oracle "
                      f"process per state point on {procs} host cores at once, {wall:.1f} s wall",
            "single_thread_value": single, "host_cpu": model, "host_cpus_available": avail}


def serve_run(n_requests, n_steps, rate, window, label, max_inflight):
    """The serving form: Poisson arrivals, models uniform over {one-site LJ,
    2CLJQ, water + 10 % ions with Ewald}, N log-uniform in [256, 8192], each
    request running `n_steps` steps with RDF (400 bins), Lustig moments
    (non-Ewald) and velocity/current ACFs over a `window`-step window on an
    extended step of 10."""
    import torch

    from paper_1507_07548_amd import inputs, ms2
    from paper_1507_07548_amd.serve import GpuBackend, Request, Server, backend_key, percentile
    trace = inputs.serving_trace(n_requests=n_requests, rate=rate, seed=5, n_steps=n_steps,
                                 window=window, acf_every=10, origin_every=100 if window >= 1000 else 50)
    fam = {"lj": [inputs.one_center_lj()], "2cljq": [inputs.two_center_lj_quadrupole()],
           "ionic": [inputs.water_tip4p_like(), inputs.cation(), inputs.anion()]}
    # one batch (context, slots, stream) per model family and size class
    keys = sorted({backend_key(m, s.n) for _, m, s in trace})
    backends = {k: GpuBackend(fam[k.split("/")[0]], max_slots=64) for k in keys}
    reqs = [Request(r, t, backend_key(m, s.n), s, ms2.FP32) for r, (t, m, s) in enumerate(trace)]
    log(f"[bench] serving ({label}): {len(reqs)} requests x {n_steps} steps at {rate:.3g}/s")
    srv = Server(backends, hbm_budget=64 << 30, chunk_steps=50, keep_samples=False, max_inflight=max_inflight)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = srv.run(reqs)
    makespan = time.perf_counter() - t0
    for be in backends.values():
        be.batch.close()
        be.ctx.close()
    lat = [r.latency for r in res]
    steps = sum(r.steps_done for r in res)
    return {"requests": len(res), "steps_per_request": n_steps, "acf_window_steps": window,
            "arrival_rate_per_s": rate, "p50_latency_s": percentile(lat, 50),
            "p99_latency_s": percentile(lat, 99), "md_steps_per_s": steps / makespan,
            "makespan_s": makespan, "all_ok": all(r.status == 0 for r in res), "n_range": [256, 8192],
            "batches": keys, "max_inflight": max_inflight}


def serving(n_requests, n_steps, window, sustained_requests, scaled, max_inflight):
    """Two runs at the configured request size: the workload's own trace at
    50 requests/s (an overload: latency includes queueing), then a run at
    0.7 x the capacity that run measured (system-steps/s / steps per
    request); plus, optionally, the short-request trace of earlier versions."""
    out = {"models": ["1CLJ (VV NVE)", "2CLJQ (Gear NVT, RF)", "water+ions (Gear NVT, Ewald)"]}
    full = serve_run(n_requests, n_steps, 50.0, window, "trace at 50/s", max_inflight)
    capacity = full["md_steps_per_s"] / n_steps
    out["trace_50_per_s"] = full
    out["capacity_requests_per_s"] = capacity
    if sustained_requests > 0:
        out["sustained_0p7_capacity"] = serve_run(sustained_requests, n_steps, 0.7 * capacity, window,
                                                  "0.7 x capacity", max_inflight)
    if scaled:
        sc = serve_run(n_requests, 400, 50.0, 200, "scaled", max_inflight)
        sc["note"] = "scaled requests (400 steps, 200-step window), kept for comparison with earlier lines"
        out["scaled_400_steps"] = sc
    return out


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "pair_sym_kernel_hbm_traffic.md")
SQ_SUMMARY = os.path.join(ROOT, "profiles", "pair_sym_kernel_sq_counters.md")


def _summary_fields(path):
    fields = {}
    if os.path.exists(path):
        for ln in open(path):
            if ln.startswith("- ") and ": " in ln:
                k, v = ln[2:].strip().split(": ", 1)
                fields[k] = v.strip("` ")
    return fields


def recorded(path, key):
    """A figure from a committed counter summary, or None when the pair
    kernel's sources changed since the counters were taken."""
    from paper_1507_07548_amd.rocprof_summary import pair_kernel_source_hash
    f = _summary_fields(path)
    if key not in f or f.get("source_sha256") != pair_kernel_source_hash():
        return None
    return float(f[key])


def plain_form(ms2, torch, ctx, systems, K, W):
    """One system per launch, no graph, plain tile shapes: every state point
    of the batched workload, one after the other."""
    log(f"[bench] plain form on {len(systems)} systems")
    batches = []
    for s in systems:
        b = ms2.Batch(ctx, 1, plain_tiles=True)
        b.admit(s, ms2.FP32)
        b.step(W if W > 0 else 1, graph=False)
        batches.append(b)
    torch.cuda.synchronize()
    pb = [b.sample(0, state=False) for b in batches]
    t0 = time.perf_counter()
    for b in batches:
        b.step(K, graph=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pa = [b.sample(0, state=False) for b in batches]
    sp = sum(a["site_pairs_total"] - b["site_pairs_total"] for a, b in zip(pa, pb))
    for b in batches:
        b.close()
    return {"value": sp / (t1 - t0), "md_steps_per_s": len(systems) * K / (t1 - t0), "systems": len(systems),
            "form": "one system per launch, no graph, plain tile shapes, the same state points"}


def precision_form(ms2, torch, ctx, systems, K, W, graph):
    """The same batched workload with FP64 site arithmetic (symmetric tile
    pairs, the default shape of batched launches)."""
    log(f"[bench] FP64 form on {len(systems)} systems")
    b = ms2.Batch(ctx, len(systems))
    slots = [b.admit(s, ms2.FP64) for s in systems]
    b.step(W if W > 0 else 1, graph=graph)
    torch.cuda.synchronize()
    pb = [b.sample(s, state=False) for s in slots]
    t0 = time.perf_counter()
    b.step(K, graph=graph)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pa = [b.sample(s, state=False) for s in slots]
    assert all(a["status"] == 0 for a in pa)
    sp = sum(a["site_pairs_total"] - p["site_pairs_total"] for a, p in zip(pa, pb))
    b.close()
    return {"value": sp / (t1 - t0), "ms_per_step": (t1 - t0) / K * 1e3, "systems": len(systems),
            "form": "FP64 site arithmetic and sums, same systems, symmetric tile pairs, graph"}


def ionic_form(ms2, torch, inputs, K, W):
    """The ionic-solution configuration (900 water-like molecules + 50 cation/anion
    pairs, Ewald alpha = 5.6 / L with 0 < n^2 <= 64, rc = 0.48 L, tin-foil; FP32 pairs,
    FP64 k-space): one force evaluation timed by its two calls with HIP events, then
    Gear NVT steps of the one system with the 400-bin RDF every 10 steps, graph replay."""
    log("[bench] ionic solution with Ewald")
    s = inputs.ionic_solution()
    s.md.n_steps = max(s.md.n_steps, W + K + 2)
    ctx = ms2.Context(s.species)
    d = ms2.DeviceSystem(s)
    p = ms2.params_struct(s.params, ms2.FP32)
    for _ in range(3):
        ctx.forces(p, d.n, d.species, d.com, d.quat, d.force, d.torque, d.sums)
        ctx.ewald_kspace(p, d.n, d.species, d.com, d.quat, d.force, d.torque, d.sums)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    reps = 20
    ev[0].record()
    for _ in range(reps):
        ctx.forces(p, d.n, d.species, d.com, d.quat, d.force, d.torque, d.sums)
    ev[1].record()
    for _ in range(reps):
        ctx.ewald_kspace(p, d.n, d.species, d.com, d.quat, d.force, d.torque, d.sums)
    ev[2].record()
    torch.cuda.synchronize()
    b = ms2.Batch(ctx, 1)
    slot = b.admit(s, ms2.FP32)
    b.step(W if W > 0 else 1, graph=True)
    torch.cuda.synchronize()
    pb = b.sample(slot, state=False)
    t0 = time.perf_counter()
    b.step(K, graph=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pa = b.sample(slot, state=False)
    assert pa["status"] == 0 and pa["steps_done"] == pb["steps_done"] + K
    sp = pa["site_pairs_total"] - pb["site_pairs_total"]
    b.close()
    ctx.close()
    return {"workload": "ionic_solution_ewald", "molecules": s.n, "k_vectors_half_space": 1054,
            "forces_us": ev[0].elapsed_time(ev[1]) / reps * 1e3,
            "kspace_us": ev[1].elapsed_time(ev[2]) / reps * 1e3,
            "md_ms_per_step": (t1 - t0) / K * 1e3, "site_pairs_per_s": sp / (t1 - t0),
            "form": "one system; forces = ms2_forces (real space, FP32 pairs), kspace = "
                    "ms2_ewald_kspace (FP64); MD step = Gear NVT + RDF every 10 steps, graph"}


CASES = {
    # lone systems of the serving mix, advanced by graph replay (FP32)
    "lone_2cljq_256": lambda I: I.quadrupolar_fluid(n=256, density=0.6),
    "lone_2cljq_1000": lambda I: I.quadrupolar_fluid(n=1000, density=0.6),
    "lone_2cljq_2000": lambda I: I.quadrupolar_fluid(n=2000, density=0.6),
    "lone_2cljq_4000": lambda I: I.quadrupolar_fluid(n=4000, density=0.6),
    "lone_2cljq_8192": lambda I: I.quadrupolar_fluid(n=8192, density=0.6),
    "lone_ionic_500": lambda I: I.ionic_solution(n_water=450, n_pairs=25),
    "lone_ionic_1000": lambda I: I.ionic_solution(),
    "lone_ionic_2000": lambda I: I.ionic_solution(n_water=1800, n_pairs=100),
    "lone_lj_1000": lambda I: I.lj_fluid(n=1000),
}


def run_case(name, K, W, shape=None):
    """One lone system advanced K steps by graph replay; prints its step time
    (with `shape` = (wave_rows, j_chunk): that tile shape for its size)."""
    import torch

    from paper_1507_07548_amd import inputs, ms2
    s = CASES[name](inputs)
    s.md.n_steps = W + 2 * K + 10
    ctx = ms2.Context(s.species)
    if shape:
        ctx.set_tile_config(s.n, ms2.FP32, shape[0], shape[1], mode=1)
    b = ms2.Batch(ctx, 1)
    slot = b.admit(s, ms2.FP32)
    b.step(max(W, 1), graph=True)
    b.step(K, graph=True, prepare=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(K, graph=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out = b.sample(slot, state=False)
    assert out["status"] == 0
    used = list(ctx.tile_config(s.n, ms2.FP32, mode=1))
    b.close()
    ctx.close()
    print(json.dumps({"case": name, "molecules": s.n, "steps": K, "ms_per_step": (t1 - t0) / K * 1e3,
                      "tile_shape": used}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--systems", type=int, default=256)
    ap.add_argument("--plain-systems", type=int, default=-1,
                    help="state points of the plain form (default: all of the batched ones)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 form of the batched workload")
    ap.add_argument("--no-ewald", action="store_true", help="skip the ionic-solution (Ewald) timing")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=20000)
    ap.add_argument("--serve-window", type=int, default=1000)
    ap.add_argument("--serve-sustained-requests", type=int, default=24)
    ap.add_argument("--serve-scaled", action="store_true", help="also run the 400-step request trace")
    ap.add_argument("--serve-inflight", type=int, default=3,
                    help="batches with a chunk on the device at once, launched shortest remaining work "
                         "first (0: no limit, every batch launches)")
    ap.add_argument("--windows", type=int, default=WINDOWS, help="timed windows of K steps (median reported)")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch the batched steps directly instead of through a hipGraph")
    ap.add_argument("--tile-shape", type=str, default=None,
                    help="waves,jchunk for every size bucket instead of autotuning (0,64 = symmetric)")
    ap.add_argument("--heat-flux", action="store_true",
                    help="sample the heat-flux ACF (extended step 10, origins every 100, 100 lags) on every system")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a known-size kernel for HBM counters)")
    ap.add_argument("--case", type=str, default=None, choices=sorted(CASES),
                    help="run only this lone-system batch and print its step time")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: every system runs on a single MI355X and "
              "sharding systems across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    K, W = args.steps, args.warmup
    if args.case:
        run_case(args.case, K, W, tuple(int(x) for x in args.tile_shape.split(",")) if args.tile_shape else None)
        return
    # the host baseline runs first: its worker processes start before this
    # process touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on the host cores)")
        cpu = cpu_baseline()

    import torch

    from paper_1507_07548_amd import inputs, ms2

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    graph = not args.no_graph
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {nbytes} bytes device to device (counter calibration)")
        del src, dst
    systems = [inputs.batched_state_point(s) for s in range(args.systems)]
    if args.heat_flux:
        for s in systems:
            s.md.acf_every, s.md.acf_origin_every, s.md.acf_nlag = 10, 100, 100
            s.md.heat_flux = True
    ctx = ms2.Context(systems[0].species)
    tuned = None
    if args.tile_shape:
        w, j = (int(x) for x in args.tile_shape.split(","))
        for b in range(8, 13):                       # size buckets floor(log2 N) of N in [500, 4000]
            ctx.set_tile_config(1 << b, ms2.FP32, w, j, mode=1)
        tuned = {str(1 << b): [w, j] for b in range(8, 13)}
    elif not args.no_autotune:
        log("[bench] autotuning tile shapes for N in [500, 4000]")
        rows = ctx.autotune(ms2.FP32, 500, 4000)
        for r in rows:
            shape = "symmetric 64x64" if int(r[2]) == 0 else f"{int(r[2])} wave(s), j chunk {int(r[3])}"
            log(f"[autotune] mode {int(r[0])} n {int(r[1])}: {shape}: {r[4]:.2f} us/system")
        tuned = {f"{int(r[1])}": list(ctx.tile_config(int(r[1]), ms2.FP32, mode=1))
                 for r in rows if r[0] == 1}

    # ---------------- batched form: the median of several K-step windows ----------------
    log(f"[bench] admitting {len(systems)} state points")
    batch = ms2.Batch(ctx, len(systems))
    slots = [batch.admit(s, ms2.FP32) for s in systems]
    if W > 0:
        batch.step(W, graph=graph)
    if graph:
        batch.step(K, graph=True, timing=True, prepare=True)    # capture + instantiate, no run
    torch.cuda.synchronize()
    windows = []
    for wi in range(args.windows):
        before = [batch.sample(s, state=False) for s in slots]
        log(f"[bench] timing {K} batched steps (window {wi + 1} of {args.windows})")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.step(K, graph=graph, timing=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        after = [batch.sample(s, state=False) for s in slots]
        pair_ms, timed = batch.pair_time_ms()
        assert all(a["status"] == 0 and a["steps_done"] == b["steps_done"] + K for a, b in zip(after, before))
        windows.append({"dt": t1 - t0, "pair_ms_avg": pair_ms / timed,
                        "site_pairs": sum(a["site_pairs_total"] - b["site_pairs_total"] for a, b in zip(after, before)),
                        "mol_pairs": sum(a["pairs_total"] - b["pairs_total"] for a, b in zip(after, before))})
    batch.close()
    med = sorted(windows, key=lambda w: w["dt"])[len(windows) // 2]
    dt = med["dt"]
    value = med["site_pairs"] / dt
    steps_per_s = len(systems) * K / dt
    mol_pairs_per_launch = med["mol_pairs"] / K
    pair_ms_avg = med["pair_ms_avg"]
    achieved = FLOP_PER_MOL_PAIR * mol_pairs_per_launch / (pair_ms_avg * 1e-3)
    executed = recorded(SQ_SUMMARY, "fp32_flop_per_mol_pair_executed")

    plain_n = len(systems) if args.plain_systems < 0 else args.plain_systems
    plain = plain_form(ms2, torch, ctx, systems[:plain_n], K, W) if plain_n > 0 else None
    fp64 = None if args.no_fp64 else precision_form(ms2, torch, ctx, systems, K, W, graph)
    ewald = None if args.no_ewald else ionic_form(ms2, torch, inputs, K, W)
    ctx.close()
    serve = None if args.no_serve else serving(args.serve_requests, args.serve_steps, args.serve_window,
                                               args.serve_sustained_requests, args.serve_scaled,
                                               args.serve_inflight or None)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "site-pair interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched_state_points_2cljq", "systems": len(systems),
                   "n_range": [500, 4000], "density_range": [0.1, 0.8], "temperature_range": [1.0, 3.0],
                   "molecules": int(sum(s.n for s in systems)), "rc_over_box": 0.48,
                   "precision": "fp32 pairs, fp64 sums", "integrator": "gear-5 quaternion NVT",
                   "moments_every": 1, "graph": graph, "tile_shapes_batched": tuned,
                   "heat_flux_acf": bool(args.heat_flux)},
        "timing": {"windows": len(windows), "window_ms_per_step": [w["dt"] / K * 1e3 for w in windows],
                   "reported": "median window"},
        "md_steps_per_s": steps_per_s,
        "mol_pairs_per_step": mol_pairs_per_launch,
        "site_pairs_per_step": med["site_pairs"] / K,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU,
                     "traffic": recorded(TRAFFIC_SUMMARY, "hbm_bytes_per_launch"),
                     "traffic_source": "profiles/pair_sym_kernel_hbm_traffic.md (rocprofv3 --pmc FETCH_SIZE, "
                                       "WRITE_SIZE, copy-calibrated; null once the kernel sources changed)",
                     "kernel": kernel_label(tuned),
                     "kernel_avg_ms": pair_ms_avg,
                     "flop_per_mol_pair_algorithmic": FLOP_PER_MOL_PAIR,
                     "flop_per_mol_pair_executed": executed,
                     "frac_executed": (executed * mol_pairs_per_launch / (pair_ms_avg * 1e-3) / PEAK_FP32_VALU
                                       if executed else None),
                     "frac_of_unpacked_fp32_peak": achieved / PEAK_FP32_UNPACKED},
    }
    if plain is not None:
        line["plain"] = plain
        line["batched_over_plain"] = value / plain["value"]
    if fp64 is not None:
        line["fp64"] = fp64
    if ewald is not None:
        line["ewald"] = ewald
    if serve is not None:
        line["serving"] = serve
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
