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

Printed JSON line: site-pair interactions/s of the batched form (value), MD
steps/s, the plain one-system-per-launch form on a sample of the same
systems, the same batched workload in FP64, the ionic-solution system with
Ewald (real-space and reciprocal calls timed apart, and its MD step rate), a
serving trace (p50/p99 latency), the pair kernel's roofline (HIP events
around its launches inside the timed graph) and the oracle timed on the host
as a CPU baseline.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 operations per site-pair evaluation (force on both
# molecules via Newton's third law, energy, virial, dU/ds and d2U/ds2), with
# a fused multiply-add counted as 2 and rcp/rsqrt as 1.
FLOP_LJ = 48
FLOP_QQ = 189
PEAK_FP32_VALU = 157.3e12     # MI355X dense FP32 vector (packed) FLOP/s
METRIC = "site-pair interactions/s and MD steps/s (batched vs plain) at 1 GPU; p50/p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_label(tuned):
    """The pair kernel(s) the batched launch used, from the tile shape per size bucket."""
    if not tuned:
        return "pair_kernel<float, 2CLJQ> (heuristic tile shapes)"
    names = sorted({"pair_sym_kernel<float, 2CLJQ> (64 x 64 tile pairs, 4 waves)" if w == 0
                    else f"pair_kernel<float, 2CLJQ, {w} wave(s)> (j chunk {j})" for w, j in tuned.values()})
    return " + ".join(names)


def cpu_baseline(systems, budget_s=12.0):
    """The FP64 oracle (single thread) on a bounded sample of the same state
    points: Gear NVT steps with moment sampling, site pairs per second."""
    import oracle
    t_total, sp_total, used = 0.0, 0.0, []
    for s in systems:
        x = s.copy()
        x.md.n_steps = 2
        _, _, sums = oracle.forces(x)
        t0 = time.perf_counter()
        oracle.md(x, want_log=False)
        dt = time.perf_counter() - t0
        t_total += dt
        sp_total += sums[11] * (x.md.n_steps + 1)   # initial evaluation + one per step
        used.append(s.n)
        if t_total > budget_s:
            break
    return {"value": sp_total / t_total, "unit": "site-pair interactions/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(used)} state points (N={used}) x (1 initial + 2 Gear NVT steps) in FP64, "
                      f"single thread, {t_total:.1f} s"}


def serve_trace(n_requests, n_steps):
    """The serving form on a scaled trace of the mixed-model workload:
    Poisson arrivals at 50/s, models uniform over {one-site LJ, 2CLJQ,
    water + 10 % ions with Ewald}, N log-uniform in [256, 8192], each request
    running `n_steps` steps (the full workload asks 2e4) with RDF (400 bins),
    Lustig moments (non-Ewald) and velocity/current ACFs over a 200-step
    window on an extended step of 10."""
    import torch

    from paper_1507_07548_amd import inputs, ms2
    from paper_1507_07548_amd.serve import GpuBackend, Request, Server, percentile
    trace = inputs.serving_trace(n_requests=n_requests, rate=50.0, seed=5, n_steps=n_steps,
                                 window=200, acf_every=10, origin_every=50)
    fam = {"lj": [inputs.one_center_lj()], "2cljq": [inputs.two_center_lj_quadrupole()],
           "ionic": [inputs.water_tip4p_like(), inputs.cation(), inputs.anion()]}
    backends = {m: GpuBackend(fam[m], max_slots=64) for m in fam}
    reqs = [Request(r, t, m, s, ms2.FP32) for r, (t, m, s) in enumerate(trace)]
    log(f"[bench] serving {len(reqs)} requests x {n_steps} steps")
    srv = Server(backends, hbm_budget=64 << 30, chunk_steps=50, keep_samples=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = srv.run(reqs)
    makespan = time.perf_counter() - t0
    lat = [r.latency for r in res]
    steps = sum(r.steps_done for r in res)
    ok = all(r.status == 0 for r in res)
    return {"requests": len(res), "steps_per_request": n_steps, "arrival_rate_per_s": 50.0,
            "p50_latency_s": percentile(lat, 50), "p99_latency_s": percentile(lat, 99),
            "md_steps_per_s": steps / makespan, "makespan_s": makespan, "all_ok": ok,
            "n_range": [256, 8192], "models": ["1CLJ (VV NVE)", "2CLJQ (Gear NVT, RF)",
                                              "water+ions (Gear NVT, Ewald)"],
            "note": "scaled trace: the full request asks 2e4 steps and a 1000-step ACF window"}


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "pair_sym_kernel_hbm_traffic.md")


def recorded_traffic():
    """HBM bytes per batched pair-kernel launch from the committed counter
    summary, or None when the kernel sources changed since it was taken."""
    from paper_1507_07548_amd.rocprof_summary import pair_kernel_source_hash
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    fields = {}
    for ln in open(TRAFFIC_SUMMARY):
        if ln.startswith("- ") and ": " in ln:
            k, v = ln[2:].strip().split(": ", 1)
            fields[k] = v.strip("` ")
    if fields.get("source_sha256") != pair_kernel_source_hash():
        return None
    return float(fields["hbm_bytes_per_launch"])


def plain_form(ms2, torch, ctx, sample, K, W):
    """One system per launch, no graph, plain tile shapes."""
    log(f"[bench] plain form on {len(sample)} systems")
    batches = []
    for s in sample:
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
    return {"value": sp / (t1 - t0), "md_steps_per_s": len(sample) * K / (t1 - t0), "systems": len(sample),
            "form": "one system per launch, no graph, plain tile shapes"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--systems", type=int, default=256)
    ap.add_argument("--plain-sample", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 form of the batched workload")
    ap.add_argument("--no-ewald", action="store_true", help="skip the ionic-solution (Ewald) timing")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-steps", type=int, default=400)
    ap.add_argument("--no-graph", action="store_true",
                    help="launch the batched steps directly instead of through a hipGraph")
    ap.add_argument("--tile-shape", type=str, default=None,
                    help="waves,jchunk for every size bucket instead of autotuning (0,64 = symmetric)")
    ap.add_argument("--heat-flux", action="store_true",
                    help="sample the heat-flux ACF (extended step 10, origins every 100, 100 lags) on every system")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a known-size kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: every system runs on a single MI355X and "
              "sharding systems across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1507_07548_amd import inputs, ms2

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    K, W = args.steps, args.warmup
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

    # ---------------- batched form ----------------
    log(f"[bench] admitting {len(systems)} state points")
    batch = ms2.Batch(ctx, len(systems))
    slots = [batch.admit(s, ms2.FP32) for s in systems]
    if W > 0:
        batch.step(W, graph=graph)
    if graph:
        batch.step(K, graph=True, timing=True, prepare=True)    # capture + instantiate, no run
    torch.cuda.synchronize()
    before = [batch.sample(s, state=False) for s in slots]
    log(f"[bench] timing {K} batched steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(K, graph=graph, timing=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    after = [batch.sample(s, state=False) for s in slots]
    pair_ms, timed = batch.pair_time_ms()
    dt = t1 - t0
    site_pairs = sum(a["site_pairs_total"] - b["site_pairs_total"] for a, b in zip(after, before))
    mol_pairs = sum(a["pairs_total"] - b["pairs_total"] for a, b in zip(after, before))
    assert all(a["status"] == 0 and a["steps_done"] == b["steps_done"] + K for a, b in zip(after, before))
    value = site_pairs / dt
    steps_per_s = len(systems) * K / dt
    flops_per_launch = (4 * FLOP_LJ + FLOP_QQ) * mol_pairs / K
    pair_ms_avg = pair_ms / timed
    achieved = flops_per_launch / (pair_ms_avg * 1e-3)
    batch.close()

    sample = systems[: args.plain_sample]
    plain = plain_form(ms2, torch, ctx, sample, K, W) if sample else None
    fp64 = None if args.no_fp64 else precision_form(ms2, torch, ctx, systems, K, W, graph)
    ewald = None if args.no_ewald else ionic_form(ms2, torch, inputs, K, W)
    serving = None if args.no_serve else serve_trace(args.serve_requests, args.serve_steps)

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
        "md_steps_per_s": steps_per_s,
        "mol_pairs_per_step": mol_pairs / K,
        "site_pairs_per_step": site_pairs / K,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU, "traffic": recorded_traffic(),
                     "kernel": kernel_label(tuned),
                     "kernel_avg_ms": pair_ms_avg,
                     "flop_per_mol_pair": 4 * FLOP_LJ + FLOP_QQ},
    }
    if plain is not None:
        line["plain"] = plain
        line["batched_over_plain"] = value / plain["value"]
    if fp64 is not None:
        line["fp64"] = fp64
    if ewald is not None:
        line["ewald"] = ewald
    if serving is not None:
        line["serving"] = serving
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(systems)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
