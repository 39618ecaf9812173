#!/usr/bin/env python3
"""Benchmark of the Fourier-convolution Poisson / Biot-Savart solve on one MI355X.

A step is one whole solve (all five passes: first-axis forward, second-axis forward,
fused last-axis forward + Green's-spectrum multiply + inverse, and the two inverse
passes) of one synthetic right-hand side already resident in HBM.  Plans (twiddles and
the Green's spectrum) are built before the timed region, as a user keeps them cached.

Default workload: node-centred 128 x 128 x 256 intervals (arrays 129 x 129 x 257),
x periodic, y even / odd, z unbounded, 8 seeded Gaussian bumps, FP32 (headline value)
and FP64, each result compared with the FP64 oracle.

Prints ONE JSON line.  --gpus above 1 is not supported (single-GPU library).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "mixed_node_128x128x256": dict(
        desc="node-centred 128x128x256 (arrays 129x129x257), x periodic, y even/odd, z unbounded, "
             "Poisson, 8 seeded Gaussian bumps",
        n=[128, 128, 256], h=[1 / 128] * 3, bc=[[2, 2], [0, 1], [3, 3]], layout=1, kind=0),
    "unbounded_cell_32": dict(
        desc="cell-centred 32^3 on [-1,1]^3, fully unbounded, Poisson, Gaussian blob",
        n=[32] * 3, h=[1 / 16] * 3, bc=[[3, 3]] * 3, layout=0, kind=0),
    "biot_savart_ring_256": dict(
        desc="cell-centred 256^3 on [-1,1]^3, fully unbounded, Biot-Savart (spectral curl), "
             "vortex ring R=0.5 core 0.05 with seeded axial perturbation, 3 components",
        n=[256] * 3, h=[2 / 256] * 3, bc=[[3, 3]] * 3, layout=0, kind=1),
    "biot_savart_tubes_512": dict(
        desc="cell-centred 512^3 on [-1,1]^3 (padded to 1024^3), fully unbounded, Biot-Savart, "
             "16 seeded vortex rings, 3 components",
        n=[512] * 3, h=[2 / 512] * 3, bc=[[3, 3]] * 3, layout=0, kind=1),
    "unbounded_cell_512": dict(
        desc="cell-centred 512^3 on [-1,1]^3 (padded to 1024^3), fully unbounded, scalar Poisson, "
             "Gaussian blob",
        n=[512] * 3, h=[2 / 512] * 3, bc=[[3, 3]] * 3, layout=0, kind=0),
}


def make_input(name):
    from paper_2211_07777_amd import workloads as W
    w = WORKLOADS[name]
    if name == "mixed_node_128x128x256":
        coords = [np.arange(w["n"][a] + 1) * w["h"][a] for a in range(3)]
        return W.gaussian_bumps(coords, [1.0, 1.0, 2.0])
    if name == "unbounded_cell_32":
        return W.gaussian_blob(32)[0]
    if name == "biot_savart_ring_256":
        return W.vortex_ring(256)[0]
    if name == "biot_savart_tubes_512":
        return W.vortex_tubes(512)[0]
    if name == "unbounded_cell_512":
        return W.gaussian_blob(512, sigma=0.1)[0]
    raise KeyError(name)


def run_gpu(name, f64, prec, steps, warmup, tune=True):
    import torch
    import paper_2211_07777_amd as F
    w = WORKLOADS[name]
    ncomp = 3 if w["kind"] == 1 else 1
    plan = F.Plan(w["n"], w["h"], w["bc"], w["layout"], F.CHAT2, prec, w["kind"], ncomp)
    info = F.plan_inspect(w["n"], w["h"], w["bc"], w["layout"], F.CHAT2, prec, w["kind"], ncomp)
    tiling = plan.tune() if tune else plan.tiling()
    rhs = torch.from_numpy(f64).to(device="cuda", dtype=plan.dtype).reshape(plan.shape).contiguous()
    out = torch.empty_like(rhs)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.solve(rhs, out, ws)
    # whole solves: the step time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve(rhs, out, ws)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    result = out.double().cpu().numpy()
    # each pass launched `steps` times back to back between two HIP events on the launch
    # stream, after one untimed launch (the in-place fused pass reapplies itself; its
    # values are not used)
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    torch.cuda.synchronize()
    for p in range(5):
        plan.solve_passes(rhs, out, p, p, ws)
        ev0[p].record(stream)
        for _ in range(steps):
            plan.solve_passes(rhs, out, p, p, ws)
        ev1[p].record(stream)
    torch.cuda.synchronize()
    pass_ms = np.array([ev0[p].elapsed_time(ev1[p]) / steps for p in range(5)])
    plan.close()
    return dict(ms_step=ms_step, pass_ms=pass_ms.tolist(), info=info, result=result,
                tiling=tiling)


def calibration_copy(mib):
    """A plain device-to-device copy of known size, profiled beside the solve so that the
    HBM counters (FETCH_SIZE, WRITE_SIZE) can be scaled to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return n * 4


def run_batched(count, reps):
    """Many small solves: a prepared FP32 batch captured in a HIP graph and replayed, the
    FP64 one-launch batch, and plain FP64 solves one at a time (solves/s)."""
    import torch
    import paper_2211_07777_amd as F
    from paper_2211_07777_amd import workloads as W
    reqs = W.serving_stream(count=count, qps=1e4, seed=2300, edges=(32, 48, 64))
    res = {"solves": count, "grid_edges": [32, 48, 64]}
    for prec, tag in ((F.F32, "fp32_graph"), (F.F64, "fp64_batched")):
        dt = torch.float32 if prec == F.F32 else torch.float64
        plans = [F.Plan(r["n"], r["h"], r["bc"], r["layout"], F.CHAT2, prec) for r in reqs]
        rhs = [W.request_rhs_device(r, dt) for r in reqs]
        outs = [torch.empty_like(x) for x in rhs]
        ws = torch.empty(F.batched_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
        batch = F.Batch(plans, rhs, outs, ws)
        batch.run()
        torch.cuda.synchronize()
        if prec == F.F32:
            stream = torch.cuda.Stream()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.stream(stream):
                with torch.cuda.graph(graph, stream=stream):
                    batch.run()
            step = graph.replay
        else:
            step = batch.run
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        res[tag + "_solves_per_s"] = count * reps / (time.perf_counter() - t0)
        if prec == F.F64:
            # plain path: one solve at a time, each waited for
            for p, x, o in zip(plans, rhs, outs):
                p.solve(x, o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for p, x, o in zip(plans, rhs, outs):
                p.solve(x, o)
                torch.cuda.synchronize()
            res["fp64_plain_solves_per_s"] = count / (time.perf_counter() - t0)
        batch.close()
        for p in plans:
            p.close()
    return res


def _percentiles(lat):
    lat = np.sort(np.asarray(lat))
    return float(np.percentile(lat, 50) * 1e3), float(np.percentile(lat, 99) * 1e3)


def run_serving(count, load=0.7):
    """The serving stream: mixed grids (edges 32 ... 192), boundary conditions and layouts,
    FP32 through the serving loop (plans cached on the device), and the same stream on
    the plain FP64 path (one solve at a time).  Inputs are generated on the device
    beforehand; latency = completion - arrival on the host clock."""
    import torch
    import paper_2211_07777_amd as F
    from paper_2211_07777_amd import workloads as W
    reqs = W.serving_stream(count=count, qps=1.0, seed=2211)
    gaps = np.diff([0.0] + [r["t"] for r in reqs])  # unit-rate arrival gaps
    rhs32 = [W.request_rhs_device(r, torch.float32) for r in reqs]
    outs32 = [torch.empty_like(x) for x in rhs32]
    torch.cuda.synchronize()
    server = F.Server(workspace_budget_bytes=24 << 30, plan_budget_bytes=64 << 30, slots=8)
    # cold pass: every plan created (timed separately), results checked below
    t0 = time.perf_counter()
    for r, x, o in zip(reqs, rhs32, outs32):
        server.submit(r["n"], r["h"], r["bc"], r["layout"], x, o)
    server.wait_all()
    server.progress()
    cold_s = time.perf_counter() - t0
    st_cold = server.stats()
    # saturated: the whole stream submitted at once, warm plans
    t0 = time.perf_counter()
    for r, x, o in zip(reqs, rhs32, outs32):
        server.submit(r["n"], r["h"], r["bc"], r["layout"], x, o)
    server.wait_all()
    server.progress()
    sat = count / (time.perf_counter() - t0)
    # open loop at `load` x the saturated rate
    lam = load * sat
    arrive = np.cumsum(gaps) / lam
    lat, done_at, ticket_of = [], {}, {}
    t_start = time.perf_counter()
    i = 0
    while len(done_at) < count:
        now = time.perf_counter() - t_start
        while i < count and arrive[i] <= now:
            r = reqs[i]
            ticket_of[server.submit(r["n"], r["h"], r["bc"], r["layout"], rhs32[i], outs32[i])] = i
            i += 1
        for t in server.progress():
            done_at[ticket_of[t]] = time.perf_counter() - t_start
    lat = [done_at[k] - arrive[k] for k in range(count)]
    p50, p99 = _percentiles(lat)
    st = server.stats()
    server.close()
    # plain FP64 path on the same arrivals: one solve at a time, plans created beforehand
    plans64 = [F.Plan(r["n"], r["h"], r["bc"], r["layout"], F.CHAT2, F.F64) for r in reqs]
    rhs64 = [x.double() for x in rhs32]
    outs64 = [torch.empty_like(x) for x in rhs64]
    for p, x, o in zip(plans64, rhs64, outs64):
        p.solve(x, o)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    lat64 = []
    for k, (p, x, o) in enumerate(zip(plans64, rhs64, outs64)):
        while time.perf_counter() - t_start < arrive[k]:
            pass
        p.solve(x, o)
        torch.cuda.synchronize()
        lat64.append(time.perf_counter() - t_start - arrive[k])
    t64 = time.perf_counter() - t_start
    p50_64, p99_64 = _percentiles(lat64)
    err = max(float((a.double() - b).abs().max() / b.abs().max()) for a, b in zip(outs32, outs64))
    for p in plans64:
        p.close()
    return {"requests": count, "grid_edges": [32, 48, 64, 96, 128, 192], "slots": 8,
            "fp32_saturated_solves_per_s": sat, "arrival_rate_per_s": lam,
            "fp32_p50_ms": p50, "fp32_p99_ms": p99,
            "fp64_plain_solves_per_s": count / t64, "fp64_plain_p50_ms": p50_64, "fp64_plain_p99_ms": p99_64,
            "peak_inflight": st["peak_inflight"], "cold_plan_creation_ms_mean": 1e3 * cold_s / count,
            "cached_plans": st_cold["cached_plans"], "max_rel_linf_fp32_vs_fp64": err}


def oracle_baseline(name, f64, budget_s=15.0):
    """The FP64 oracle on the host cores: whole solves of the same workload, repeated
    until about budget_s seconds of CPU work have been spent."""
    import oracle
    w = WORKLOADS[name]
    t0 = time.perf_counter()
    ref = oracle.solve(f64, w["n"], w["h"], w["bc"], w["layout"], 0, w["kind"])
    first = time.perf_counter() - t0
    reps, total = 1, first
    while total + first < budget_s and reps < 100:
        t0 = time.perf_counter()
        oracle.solve(f64, w["n"], w["h"], w["bc"], w["layout"], 0, w["kind"])
        total += time.perf_counter() - t0
        reps += 1
    return ref, total / reps, reps, oracle.num_threads()


def load_traffic(name, kernel_pass):
    """HBM bytes per launch of the dominant pass from the committed rocprofv3 counter
    summary (profiles/), or None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    return d.get("bytes_per_launch", {}).get(str(kernel_pass))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="mixed_node_128x128x256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-tune", action="store_true", help="time the planner's tiling, not the tuned one")
    ap.add_argument("--serving-requests", type=int, default=500,
                    help="requests of the serving stream (0: skip the serving measurement)")
    ap.add_argument("--batched-solves", type=int, default=64,
                    help="small solves of the batched measurement (0: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this library runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2211_07777_amd as F

    name = args.workload
    w = WORKLOADS[name]
    f64 = make_input(name)
    ncomp = 3 if w["kind"] == 1 else 1
    user_pts = float(np.prod([n + (1 if w["layout"] == 1 else 0) for n in w["n"]]))
    r32 = run_gpu(name, f64, F.F32, args.steps, args.warmup, not args.no_tune)
    r64 = run_gpu(name, f64, F.F64, args.steps, args.warmup, not args.no_tune)

    cpu = None
    err32 = err64 = None
    if not args.no_cpu:
        ref, cpu_s, reps, cores = oracle_baseline(name, f64)
        scale = np.abs(ref).max()
        err32 = float(np.abs(r32["result"] - ref).max() / scale)
        err64 = float(np.abs(r64["result"] - ref).max() / scale)
        cpu = {"value": user_pts * ncomp / cpu_s / 1e6, "unit": "Mpts/s", "cores": int(cores),
               "kind": "oracle",
               "sample": f"{reps} full FP64 oracle solve(s) of the same workload, {cpu_s:.2f} s each"}

    if args.calib_copy_mib:
        calibration_copy(args.calib_copy_mib)
    batched = run_batched(args.batched_solves, 20) if args.batched_solves else None
    serving = run_serving(args.serving_requests) if args.serving_requests else None

    mpts32 = user_pts * ncomp / (r32["ms_step"] * 1e-3) / 1e6
    mpts64 = user_pts * ncomp / (r64["ms_step"] * 1e-3) / 1e6
    dom = int(np.argmax(r32["pass_ms"]))
    algo = r32["info"]["algo_bytes"][dom]
    achieved = algo / (r32["pass_ms"][dom] * 1e-3) / 1e9
    traffic = load_traffic(name, dom)
    step_bytes = sum(r32["info"]["algo_bytes"])
    kinds = ["first-axis forward", "second-axis forward", "fused last axis", "second-axis inverse",
             "first-axis inverse"]
    line = {
        "metric": "unbounded Poisson Mpts/s & solves/s, FP32 vs FP64; serving p50/p99 latency",
        "value": mpts32,
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "description": w["desc"], "points": int(user_pts), "components": ncomp,
                   "precision_of_value": "fp32"},
        "solves_per_s": 1e3 / r32["ms_step"],
        "fp64": {"value": mpts64, "ms_per_step": r64["ms_step"], "solves_per_s": 1e3 / r64["ms_step"],
                 "rel_linf_vs_oracle": err64},
        "fp32_rel_linf_vs_oracle": err32,
        "pass_ms_fp32": r32["pass_ms"],
        "algo_bytes_fp32": r32["info"]["algo_bytes"],
        "tiling_fp32": r32["tiling"],
        "tuned": not args.no_tune,
        "pass_ms_fp64": r64["pass_ms"],
        "effective_GBps_fp32": step_bytes / (sum(r32["pass_ms"]) * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "kernel": f"pass {dom + 1} ({kinds[dom]}, pass_kernel<float>)",
                     "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic},
        "cpu_baseline": cpu,
        "batched": batched,
        "serving": serving,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
