"""Throughput benchmark of the BSS-MPPI hot path on one MI355X.

A step is one receding-horizon control period of the paper-scale workload: one full solve
(rollout + scoring + log-sum-exp update, K=4096 samples x M=64 particles x T=50 steps) from a
device-resident state estimate, followed by the warm-start shift.  The value is rollout-steps per
second (K*M*T per solve) over the timed steps.  Also reported:
  * roofline of the rollout kernel (the dominant kernel): its FP32 operations per launch (175.5
    per rollout-step, counted from the kernel's arithmetic) over its average launch time
    measured by HIP events on the solve stream, against the FP32 vector peak of 157.3 TFLOP/s;
  * the FP64 CPU oracle timed on the host on the same workload (cpu_baseline);
  * plain synchronous solve latency (p50/p99) from host inputs.

    python bench.py [--gpus 1] [--steps 50] [--warmup 10]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# FP32 work of one rollout-step (one particle advanced one step), counted from the operations the
# kernel executes for the method (FMA = 2 FLOP, add / sub / mul = 1, a transcendental rcp / log /
# sqrt / sin / cos = 1; min / max / med3 / rint and integer work excluded):
#   disturbance normals, per particle (a quad's three Philox blocks give six Box-Muller pairs,
#     each 2 sub + 3 mul + log, sqrt, sin, cos): 7.5 + 6 transcendental
#   two vector-field evaluations, each: slip-angle ratios 6, two arctangent polynomials 36,
#     slip angle 1, tire forces 2, heading reduction 1, global velocities 6, accelerations 11,
#     + rcp, sin, cos: 2 x (63 + 3)
#   midpoint combination and update: headings 6, midpoint 6, the three position sums 6 (the
#     compensation terms of the kernel's compensated sums are not counted), velocities with the
#     disturbance 12: 30
# = 163.5 FP32 FLOP + 12 transcendental = 175.5 FP32 operations per rollout-step (the counters
# read 174.9: 64 x (ADD + MUL + 2 FMA + TRANS) per rollout-step).
FP32_FLOP_PER_ROLLOUT_STEP = 175.5
# MI355X FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (packed FP32, two values per lane) x
# 2 FLOP (FMA) x 2.4 GHz = 157.3e12 FLOP/s; without packed FP32 (which this build disables) half.
FP32_PEAK = 157.3e12
FP32_PEAK_NONPACKED = FP32_PEAK / 2

KERNEL_SOURCES = ["paper_2408_00494_amd/csrc/bss_solve.h",
                  "paper_2408_00494_amd/csrc/bss_wave.h",
                  "paper_2408_00494_amd/csrc/bss_device.h",
                  "paper_2408_00494_amd/csrc/bss_internal.h"]

# Counter measurements of the solve kernel on this workload (rocprofv3 --pmc, average per
# dispatch), valid only for the kernel sources (hash) and the launch shape they were taken on:
#   HBM bytes: FETCH_SIZE and WRITE_SIZE (KiB) scaled by what the same counters read for a 1 GiB
#     device copy (FETCH_SIZE x2.0, WRITE_SIZE x1.0);
#   VALU: wave instructions issued (SQ_INSTS_VALU) and the FP32 instruction counts.
MEASURED = {"sources_sha256_16": "a3ddd71f55917378", "lanes": 16, "ppl": 4, "split": True,
            "records_on_chip": True,
            # FETCH_SIZE 287.0 KiB x (1048576 / 524305), WRITE_SIZE 248.0 KiB x 1.0
            "fetch_bytes": 587757, "write_bytes": 253952,
            # SQ_INSTS_VALU; 64 x (ADD + MUL + 2 FMA + TRANS) of the FP32 counters
            "valu_insts": 45369848, "fp32_flop": 2291138560,
            # wave instructions by kind (SQ_INSTS_VALU_*): FP32 arithmetic (ADD, MUL, FMA),
            # FP32 transcendentals, FP64 (ADD, MUL, FMA, TRANS), integer (INT32, INT64),
            # conversions; the rest (moves, DPP, selects, bit operations) has no counter
            "valu_by_kind": {"fp32_arith": 3080192 + 5138432 + 12705792,
                             "fp32_trans": 2168832,
                             "fp64": 3495405 + 518777 + 1155630 + 51901,
                             "int": 1399779 + 2559744, "cvt": 2134016}}


def sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured(lanes, ppl, split, on_chip):
    """Counter measurements of the solve kernel, or None if the kernel, the launch shape or where
    the belief records live changed since they were taken."""
    if MEASURED["sources_sha256_16"] != sources_hash() or \
            (lanes, ppl, split, on_chip) != (MEASURED["lanes"], MEASURED["ppl"], MEASURED["split"],
                                             MEASURED["records_on_chip"]):
        return None
    return MEASURED


def ALG_BYTES_PER_SOLVE(K, M, T, lanes, records_in_hbm):
    """Bytes the solve kernel must move: costs, block partials, the mean sequence read, and, when
    the belief records go through HBM rather than staying on chip, the records written and read
    back by the scoring phase (K (T+1) 9 doubles each way)."""
    groups = 256 // lanes
    blocks = (K + groups - 1) // groups
    rec = 2 * K * (T + 1) * 9 * 8 if records_in_hbm else 0
    return rec + K * 8 + blocks * (2 * T + 5) * 8 + T * 2 * 8


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--ppl", type=int, default=0)
    ap.add_argument("--split", type=int, default=-1,
                    help="noise-producing waves: -1 automatic, 0 off, 1 on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-resampling", action="store_true")
    ap.add_argument("--no-constraints", action="store_true")
    ap.add_argument("--no-shielded", action="store_true")
    ap.add_argument("--no-vehicle8", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the serving trace replayed with batching (0 skips serving)")
    ap.add_argument("--plain-seconds", type=float, default=15.0,
                    help="length of the trace prefix replayed with plain per-request launches")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--latency-solves", type=int, default=50)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration) and exit")
    return ap.parse_args()


def cpu_baseline(prob, x0, v, seconds):
    """The FP64 oracle (as it stands) on the same workload, on the host's cores."""
    import oracle
    nthreads = min(16, os.cpu_count() or 1)
    rs = prob["K"] * prob["M"] * prob["T"]
    n, t0 = 0, time.perf_counter()
    while True:
        oracle.solve(prob, n, x0, v, want_traces=False, nthreads=nthreads)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= 50:
            break
    # the same oracle on one thread, over a quarter of the samples (the rate is per sample)
    one = dict(prob, K=max(1, prob["K"] // 4))
    n1, t1 = 0, time.perf_counter()
    while True:
        oracle.solve(one, n1, x0, v, want_traces=False, nthreads=1)
        n1 += 1
        el1 = time.perf_counter() - t1
        if el1 >= seconds / 2 or n1 >= 10:
            break
    return {"value": rs * n / el, "unit": "rollout-steps/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{n} full solves of the same workload (K={prob['K']}, M={prob['M']}, "
                      f"T={prob['T']}) in {el:.1f} s, split over K across {nthreads} threads",
            "single_thread": {"value": one["K"] * one["M"] * one["T"] * n1 / el1,
                              "sample": f"{n1} solves with K={one['K']} on one thread in "
                                        f"{el1:.1f} s"},
            "host": host_cpu()}


def host_cpu():
    """CPU model and logical core count of the host the oracle ran on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
            else None}


def bench_resampling(bss, W, torch, steps=20, warmup=3):
    """The paper-scale workload with the Gaussian re-sampling reading of Alg. 2 (particles redrawn
    from the mean and full covariance at every step)."""
    prob, x0, _ = W.config_paper_scale()
    return dict(_bench_variant(bss, torch, dict(prob, belief=1), x0, steps, warmup),
                workload="paper-scale solve with Gaussian re-sampling every step (K=4096, M=64, "
                         "T=50)")


def bench_constraints(bss, W, torch, steps=20, warmup=3):
    """The paper-scale workload with four half-space chance constraints on the state (speed
    limit, yaw rate both ways, a lateral-velocity combination), each scored on the variance
    a^T Sigma a of the full covariance."""
    prob, x0, _ = W.config_constrained()
    return dict(_bench_variant(bss, torch, prob, x0, steps, warmup),
                workload="paper-scale solve with four half-space constraints on the state "
                         "(K=4096, M=64, T=50)")


def _bench_variant(bss, torch, prob, x0, steps, warmup):
    """Solves of one variant from a device-resident state, each followed by the shift."""
    rs = prob["K"] * prob["M"] * prob["T"]
    s = bss.Solver(prob)
    s.set_outputs(controls=False)
    x0_dev = torch.as_tensor(x0, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        s.solve_async(x0_dev)
        s.step_shift()
    torch.cuda.synchronize()
    s.timing(True)
    s.timing_read()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.solve_async(x0_dev)
        s.step_shift()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kms, n = s.timing_read()
    info = s.info()
    s.close()
    return {"value": rs * steps / el, "unit": "rollout-steps/s", "ms_per_step": el * 1e3 / steps,
            "kernel_ms": kms / max(n, 1), "lanes": info["lanes"], "ppl": info["ppl"]}


def bench_vehicle8(bss, W, torch, steps=20, warmup=3):
    """The paper's 8-state vehicle (single-track model with wheel speeds, magic-formula tires and
    the friction ellipse, four midpoint substeps per period): the paper's largest BSS-MPPI setting
    of its Table 1 (1000 samples x 20 particles, horizon 20), and a larger one that fills the
    chip (8192 x 64, horizon 20)."""
    out = {}
    for key, sizes in (("table1_size", dict(K=1000, M=20, T=20)),
                       ("large", dict(K=8192, M=64, T=20))):
        prob, x0, _ = W.config_vehicle8()
        prob = dict(prob, **sizes)
        out[key] = dict(_bench_variant(bss, torch, prob, x0, steps, warmup),
                        workload=f"8-state vehicle, K={sizes['K']}, M={sizes['M']}, "
                                 f"T={sizes['T']}")
    return out


def bench_shielded(bss, W, torch, steps=20, warmup=3):
    """The shielded workload of the closed-loop statistics (K=8192, M=128, T=60, two repair
    iterations per sampled control and step), solved from a device-resident state; and the same
    solve followed by the repair of its update (local_repair = 1)."""
    out = {"workload": "shielded solve (K=8192, M=128, T=60, 2 repair iterations, delta=0.05, "
                       "gamma=0.1)"}
    for key, extra in (("shielded", {}), ("with_update_repair", {"local_repair": 1})):
        prob, x0, v = W.config_shielded()
        prob = dict(prob, **extra)
        rs = prob["K"] * prob["M"] * prob["T"]
        s = bss.Solver(prob)
        s.set_outputs(controls=False)
        x0_dev = torch.as_tensor(x0, dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            s.solve_async(x0_dev)
            s.step_shift()
        torch.cuda.synchronize()
        s.timing(True)
        s.timing_read()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.solve_async(x0_dev)
            s.step_shift()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kms, n = s.timing_read()
        info = s.info()
        s.close()
        out[key] = {"value": rs * steps / el, "unit": "rollout-steps/s",
                    "ms_per_step": el * 1e3 / steps, "kernel_ms": kms / max(n, 1),
                    "lanes": info["lanes"], "ppl": info["ppl"]}
    return out


def bench_batched(bss, W, torch, rounds=20, warmup=3):
    """The 64-instance mixed workload (K 512..8192, M 16..256, T 20..80, own track and disturbance
    per instance): one batched solve of every instance per round, replayed from a captured graph
    with the autotuned particles-per-lane, against the plain path (each instance's own solve
    launches, one after another on the same stream)."""
    members = W.config_batch()
    rs = sum(p["K"] * p["M"] * p["T"] for p, _, _ in members)
    stream = torch.cuda.Stream()
    solvers = []
    for p, _, v in members:
        s = bss.Solver(p, stream=stream)
        s.set_outputs(controls=False)
        s.set_controls(v)
        solvers.append(s)
    x0s = np.stack([x0 for _, x0, _ in members])
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    batch = bss.Batch(solvers, ppl=0, shift_after=True)
    ppl = batch.tune()
    layout = batch.layout()
    # the tuned layout's two solve grids side by side, eager launches: the persistent
    # work-queue grid and one workgroup per block-table entry
    grid_ms = {}
    for persistent in (True, False):
        batch.set_grid(persistent)
        batch.set_states(x0s)
        for _ in range(warmup):
            batch.solve()
        ev0.record(stream)
        for _ in range(rounds):
            batch.solve()
        ev1.record(stream)
        ev1.synchronize()
        grid_ms["persistent" if persistent else "one_workgroup_per_block"] = \
            ev0.elapsed_time(ev1) / rounds
    batch.set_grid(layout["persistent"])
    batch.set_states(x0s)
    batch.capture()
    for _ in range(warmup):
        batch.solve()
    stream.synchronize()
    ev0.record(stream)
    t0 = time.perf_counter()
    for _ in range(rounds):
        batch.solve()
    ev1.record(stream)
    ev1.synchronize()
    wall_b = (time.perf_counter() - t0) / rounds
    gpu_b = ev0.elapsed_time(ev1) * 1e-3 / rounds
    st = [s.info() for s in solvers]
    assert all(i["n_finite"] > 0 for i in st)
    batch.close()

    x0_dev = torch.as_tensor(x0s, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            for i, s in enumerate(solvers):
                s.solve_async(x0_dev[i])
                s.step_shift()
        stream.synchronize()
        ev0.record(stream)
        t0 = time.perf_counter()
        for _ in range(rounds):
            for i, s in enumerate(solvers):
                s.solve_async(x0_dev[i])
                s.step_shift()
        ev1.record(stream)
        ev1.synchronize()
    wall_p = (time.perf_counter() - t0) / rounds
    gpu_p = ev0.elapsed_time(ev1) * 1e-3 / rounds
    for s in solvers:
        s.close()
    return {"workload": "64 uneven instances, K 512..8192, M 16..256, T 20..80 (mixed-size "
                        "batch, seed 4)",
            "rollout_steps_per_round": rs,
            "batched": {"value": rs / wall_b, "unit": "rollout-steps/s", "ms_per_round":
                        wall_b * 1e3, "gpu_ms_per_round": gpu_b * 1e3, "ppl": ppl,
                        "ppl_by_M": {str(p["M"]): P for (p, _, _), P in
                                     zip(members, layout["member_ppl"])},
                        "solve_blocks": layout["nblocks"], "noise_split": layout["split"],
                        "persistent_grid": layout["persistent"],
                        "launch": "captured HIP graph",
                        "eager_gpu_ms_per_round_by_grid": grid_ms},
            "plain": {"value": rs / wall_p, "unit": "rollout-steps/s", "ms_per_round":
                      wall_p * 1e3, "gpu_ms_per_round": gpu_p * 1e3,
                      "launch": "two launches per instance, one stream"},
            "speedup": wall_p / wall_b}


def bench_serving(bss, W, seconds, plain_seconds, skip=5.0):
    """256 vehicles issuing solves as Poisson processes at 20 Hz each (K U[1024, 8192], M U[32,
    128], delta U[0.01, 0.1], T = 50), replayed in real time: continuous batching over two
    streams with a 32 GiB scratch budget, against plain per-request launches (one request per
    launch, FIFO, one stream) on the first plain_seconds of the same trace.  Latency = completion
    - arrival, percentiles over requests arriving after `skip` seconds."""
    fleet = W.serving_fleet()
    tr = W.serving_trace(fleet, duration_s=seconds)

    def run(n_streams, max_batch, horizon):
        sel = tr["t"] < horizon
        args = [tr[k][sel] for k in ("t", "vehicle", "K", "M", "delta", "x0")]
        srv = bss.Server(fleet[0], T=50, K_max=8192, M_max=128, ppl=4, n_streams=n_streams,
                         max_batch=max_batch, hbm_budget=32 << 30)
        t0 = time.perf_counter()
        lat, u0, st = srv.replay(*args)
        wall = time.perf_counter() - t0
        srv.close()
        rs = float(np.sum(args[2].astype(np.float64) * args[3] * 50))
        keep = args[0] >= min(skip, horizon / 3)
        return {"requests": int(sel.sum()), "trace_s": horizon, "wall_s": wall,
                "rollout_steps_per_s": rs / wall,
                "offered_rollout_steps_per_s": rs / horizon,
                "p50_ms": float(np.percentile(lat[keep], 50) * 1e3),
                "p99_ms": float(np.percentile(lat[keep], 99) * 1e3),
                "max_ms": float(np.max(lat[keep]) * 1e3),
                "failed": int(np.sum(st != 0)),
                "launch": (f"continuous batching, {n_streams} streams, up to {max_batch} "
                           "requests per launch" if max_batch > 1 else
                           "one request per launch, FIFO, one stream")}

    batched = run(2, 256, seconds)
    progress(f"serving, batched: {batched['requests']} requests, p99 {batched['p99_ms']:.2f} ms")
    plain = run(1, 1, min(plain_seconds, seconds))
    progress(f"serving, plain: {plain['requests']} requests, p99 {plain['p99_ms']:.2f} ms")
    return {"workload": "256 vehicles, Poisson 20 Hz each, K U[1024,8192], M U[32,128], "
                        "delta U[0.01,0.1], T=50, 32 GiB scratch budget (seed 5)",
            "batched": batched, "plain": plain}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solve does not "
              "span GPUs in this build.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2408_00494_amd as bss
    from paper_2408_00494_amd import workloads as W

    if args.calibrate_copy:
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty(n, dtype=torch.uint8, device="cuda")
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": n}))
        return

    prob, x0, v = W.config_paper_scale()
    K, M, T = prob["K"], prob["M"], prob["T"]
    rs_per_solve = K * M * T
    stream = torch.cuda.current_stream()
    solver = bss.Solver(prob, lanes=args.lanes)
    if args.ppl or args.split != -1:
        solver.set_shape(lanes=args.lanes, ppl=args.ppl, split=args.split)
    # a controller needs neither the sampled controls nor the belief records: the records stay on
    # chip where they fit
    solver.set_outputs(controls=False, beliefs=False)
    x0_dev = torch.as_tensor(x0, dtype=torch.float64, device="cuda")

    for _ in range(args.warmup):
        solver.solve_async(x0_dev)
        solver.step_shift()
    torch.cuda.synchronize()
    solver.timing(True)
    solver.timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.solve_async(x0_dev)
        solver.step_shift()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms_total, n_meas = solver.timing_read()
    solver.timing(False)
    info = solver.info()
    stats = solver.buffers()["stats"].cpu().numpy()
    assert stats[4] == 0.0, "solve reported a numeric failure"

    value = rs_per_solve * args.steps / elapsed
    kernel_ms = kernel_ms_total / max(n_meas, 1)
    fp32 = FP32_FLOP_PER_ROLLOUT_STEP * rs_per_solve / (kernel_ms * 1e-3)
    meas = measured(info["lanes"], info["ppl"], info["split"], info["records_on_chip"])

    # plain synchronous solves from host inputs (latency of one control period)
    lat = []
    for i in range(args.latency_solves):
        t1 = time.perf_counter()
        solver.solve(x0)
        lat.append((time.perf_counter() - t1) * 1e3)
    solver.close()

    out = {
        "metric": "rollout-steps/s (K·M·T)",
        "value": value,
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper-scale single solve: K=4096 samples, M=64 particles, "
                               "T=50 steps, disturbance std x2, seeded start on the 30x20 m "
                               "ellipse track",
                   "K": K, "M": M, "T": T, "lanes": info["lanes"], "ppl": info["ppl"],
                   "noise_split": info["split"], "records_on_chip": info["records_on_chip"]},
        "roofline": {"bound": "alu", "achieved": fp32 / 1e12, "peak": FP32_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": fp32 / FP32_PEAK,
                     "traffic": (meas["fetch_bytes"] + meas["write_bytes"]) if meas else None,
                     "kernel": "solve_kernel", "kernel_ms": kernel_ms,
                     "fp32_flop_per_rollout_step": FP32_FLOP_PER_ROLLOUT_STEP,
                     "frac_of_nonpacked_peak": fp32 / FP32_PEAK_NONPACKED,
                     "algorithmic_bytes": ALG_BYTES_PER_SOLVE(K, M, T, info["lanes"],
                                                              not info["records_on_chip"]),
                     "valu_lane_insts_per_rollout_step":
                         meas["valu_insts"] * 64 / rs_per_solve if meas else None,
                     "counter_fp32_flop_per_rollout_step":
                         meas["fp32_flop"] / rs_per_solve if meas else None,
                     # shares of the VALU lane instructions (counters), the transcendental and
                     # integer shares among them
                     "valu_shares": ({kind: n / meas["valu_insts"]
                                      for kind, n in meas["valu_by_kind"].items()}
                                     if meas else None)},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mode": "plain synchronous solve from host inputs"},
    }
    progress(f"single solve: {value:.3e} rollout-steps/s, kernel {kernel_ms:.4f} ms")
    if not args.no_resampling:
        out["resampling"] = bench_resampling(bss, W, torch)
        progress(f"re-sampling variant: {out['resampling']['value']:.3e} rollout-steps/s")
    if not args.no_constraints:
        out["constraints"] = bench_constraints(bss, W, torch)
        progress(f"half-space constraints: {out['constraints']['value']:.3e} rollout-steps/s")
    if not args.no_vehicle8:
        out["vehicle8"] = bench_vehicle8(bss, W, torch)
        progress(f"8-state vehicle: {out['vehicle8']['table1_size']['ms_per_step']:.3f} ms per "
                 f"step at the paper's Table 1 size, {out['vehicle8']['large']['value']:.3e} "
                 "rollout-steps/s large")
    if not args.no_shielded:
        out["shielded"] = bench_shielded(bss, W, torch)
        progress(f"shielded: {out['shielded']['shielded']['value']:.3e} rollout-steps/s, with "
                 f"the repair of the update {out['shielded']['with_update_repair']['value']:.3e}")
    if not args.no_batched:
        out["batched"] = bench_batched(bss, W, torch)
        progress(f"mixed batch: {out['batched']['batched']['value']:.3e} rollout-steps/s")
    if args.serve_seconds > 0:
        out["serving"] = bench_serving(bss, W, args.serve_seconds, args.plain_seconds)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, x0, v, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
