#!/usr/bin/env python3
"""Benchmark: ADMM iterations per second of the multi-scale low-rank decomposition on
the 8192 x 8192, 5-scale workload (blocks 1, 8, 32, 128, 512; 1% active rank-1 blocks
per scale plus N(0, 0.01^2) noise; default lambda; rho = 1; random cycle spinning).

One step is one ADMM iteration over the whole path: consensus update with the fused
1x1 scale, and for every other scale the shifted gather, bound test, block SVDs,
thresholding, rebuild and dual update. The timed region is K iterations of a solve
that starts from Z = U = 0 with Y already resident in HBM. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The solver runs each scale (and a batch each shape class) on a HIP stream of its own;
# streams only run side by side on hardware queues of their own, and HIP's default of
# 4 queues per process puts several of them on one. More queues also make every
# HBM-bound launch about 10% slower here, so the 8192^2 run keeps HIP's 4 (same
# iteration rate, faster stream pass). The batch of 256 instances also runs fastest on 4
# (492 solves/s, against 421 on 2, 321 on 8 and 337 on 16); serving, spinning, video and
# completion take 16 (averaged spinning 308 against 202 iters/s on 4, serving saturates
# at 2.72 against 2.35 solves/s). A batch-mode run with a single queue ended in a host
# segmentation fault during start-up, so at least 2 are required. HIP reads the count
# once, when it initialises, so main() sets it (--hw-queues) before anything imports
# torch.
HW_QUEUES = 4

METRIC = "ADMM iters/s (8192², 5 scales) + served solves/s, p99 lat @ relerr≤1e-3"
LADDER = [(1, 1), (8, 8), (32, 32), (128, 128), (512, 512)]
DENSITY = 0.01
NOISE = 0.01
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


STREAM_BYTES_PER_ELEM = 16     # per decomposed scale: read Z_i and R, write Z_i' and D_i'
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_stream_all__8192x8192_5scales_traffic.md")


def consensus_bytes_per_elem(L, n1x1):
    """k_consensus: read Y and the L planes D_i; write R; for each 1x1 scale read Z_i
    and write Z_i' and D_i'."""
    return 4 * (1 + L + 1 + 3 * n1x1)


STREAM_SRC_BEGIN = b"// ---------------------------------------------------------------- stream pass"
STREAM_SRC_END = b"// ------------------------------------------------------ one-sided Jacobi core"


def stream_source_digest():
    """Digest of the stream pass's source text (its section of kernels.hip, from its
    header comment to the next section's), so that the traffic counters stay valid
    while that code is unchanged."""
    import hashlib
    with open(os.path.join(ROOT, "paper_1507_08751_amd", "csrc", "kernels.hip"), "rb") as f:
        src = f.read()
    a = src.find(STREAM_SRC_BEGIN)
    b = src.find(STREAM_SRC_END)
    if a < 0 or b <= a:
        return None
    return hashlib.sha256(src[a:b]).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per k_stream_all launch from the committed rocprofv3 counter summary:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the stream kernel, each scaled by
    what the same counter reads for a plain copy of known size. None when the summary
    is missing or was taken on a different stream pass source."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            kv = dict(line.strip("- `\n").split(": ", 1) for line in f
                      if line.startswith("- `") and ": " in line)
        if kv.get("stream pass source digest") != stream_source_digest():
            return None
        fr = float(kv["copy bytes read"]) / (1024.0 * float(kv["copy FETCH_SIZE KiB"]))
        fw = float(kv["copy bytes written"]) / (1024.0 * float(kv["copy WRITE_SIZE KiB"]))
        return (1024.0 * float(kv["k_stream_all FETCH_SIZE KiB"]) * fr
                + 1024.0 * float(kv["k_stream_all WRITE_SIZE KiB"]) * fw)
    except (OSError, KeyError, ValueError):
        return None


def stream_roofline(prof, tiers, M, N, K):
    """Roofline of the dominant kernel, k_stream_all, the stream pass: one launch per
    decomposed scale and iteration, each moving 16 B per element of the M x N plane;
    the HIP events bracket the pass, so the average launch time is the pass time over
    the launches. And of the consensus pass."""
    idx = [i for i, t in enumerate(tiers) if t != "1x1"]
    launches = K * len(idx)
    avg_ms = prof["stream_ms"] / max(1, launches)
    nbytes = STREAM_BYTES_PER_ELEM * M * N
    gbs = nbytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": measured_traffic(),
            "kernel": "k_stream_all", "launches": launches, "avg_launch_ms": round(avg_ms, 4),
            "algorithmic_bytes_per_launch": nbytes}
    n1 = sum(1 for t in tiers if t == "1x1")
    cbytes = consensus_bytes_per_elem(len(tiers), n1) * M * N
    cms = prof["consensus_ms"] / K
    cgbs = cbytes / (cms * 1e-3) / 1e9 if cms > 0 else 0.0
    extra = {"bound": "hbm", "achieved": round(cgbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
             "frac": round(cgbs / PEAK_HBM_GBS, 4), "kernel": "k_consensus",
             "avg_launch_ms": round(cms, 4), "algorithmic_bytes_per_launch": cbytes}
    return roof, extra


def completion_bench(args, iters=100, warm=5):
    """Masked data consistency (Sec. 10, collaborative filtering): a 1682 x 943 ratings
    stand-in with 93.7% of the entries missing, users in 23 groups of 41, scales
    {1682 x 41 (group), 1682 x 943 (global)}, default lambda, rho = 1; iterations per
    second over `iters` iterations after `warm`; the oracle times 2 iterations."""
    import numpy as np
    import torch
    import paper_1507_08751_amd as msld
    from synth import completion_instance
    M, N = 1682, 943
    ladder = [(M, 41), (M, N)]
    Y, mask, _ = completion_instance(M, N, groups=23, observed=0.063, seed=0)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    Yd = torch.from_numpy(Y).to(dev)
    Z = torch.empty((len(ladder), M, N), dtype=torch.float32, device=dev)
    solver = msld.Solver(M, N, ladder, rho=1.0, iters=iters, device=dev)
    solver.set_mask(torch.from_numpy(mask.astype(np.uint8)).to(dev))
    solver.reset(Z)
    solver.step(Yd, Z, warm)
    solver.reset(Z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(Yd, Z, iters)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    r = solver.step(Yd, Z, 1, resid=True)
    tiers = [msld.TIERS[solver.tier(i)] for i in range(len(ladder))]
    solver.close()
    out = {"metric": "masked ADMM iters/s (1682 x 943, 93.7% missing)", "value": round(iters / sec, 3),
           "unit": "iters/s", "n_gpus": 1, "steps": iters, "warmup": warm,
           "ms_per_step": round(1e3 * sec / iters, 3), "higher_is_better": True,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "ratings stand-in 1682x943 (items x users, 23 user groups), "
                                  "6.3% observed, scales 1682x41 and 1682x943, rho=1",
                      "tiers": tiers, "resid_after": r}}
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        oracle.admm(Y, ladder, rho=1.0, iters=2, mask=mask)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 2 / dt, "unit": "iters/s", "cores": threads,
                               "kind": "oracle", "sample": f"2 iterations, {dt:.2f} s"}
    out.setdefault("config", {})["hw_queues"] = HW_QUEUES
    print(json.dumps(out), flush=True)


def spin_bench(args, iters=20, warm=2, spins=16):
    """Averaged cycle spinning (Sec. 9): 1024 x 1024, scales {1, 4, 16, 64, 1024}
    squared, default lambda, rho = 1, the Z-step of the 4, 16 and 64 scales averaged
    over 16 shifts (every shift of the 4 x 4 scale, 16 hashed shifts of the others;
    the whole-matrix scale has one distinct shift). Iterations per second over `iters`
    after `warm`; the oracle times one iteration."""
    import numpy as np
    import torch
    import paper_1507_08751_amd as msld
    from synth import make_instance
    M = N = 1024
    ladder = [(1, 1), (4, 4), (16, 16), (64, 64), (M, N)]
    inst = make_instance(M, N, ladder, 0.02, noise=0.01, seed=0, keep_components=False)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    Yd = torch.from_numpy(inst.Y).to(dev)
    Z = torch.empty((len(ladder), M, N), dtype=torch.float32, device=dev)
    solver = msld.Solver(M, N, ladder, rho=1.0, iters=iters, cycle_spin=True, seed=1,
                         spin_count=spins, device=dev)
    solver.reset(Z)
    solver.step(Yd, Z, warm)
    solver.reset(Z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(Yd, Z, iters)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    tiers = [msld.TIERS[solver.tier(i)] for i in range(len(ladder))]
    solver.close()
    # the same ladder with one random shift per iteration, for the cost ratio
    one = msld.Solver(M, N, ladder, rho=1.0, iters=iters, cycle_spin=True, seed=1, device=dev)
    one.reset(Z)
    one.step(Yd, Z, warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    one.step(Yd, Z, iters)
    torch.cuda.synchronize()
    sec1 = time.perf_counter() - t0
    one.close()
    out = {"metric": f"averaged cycle spinning ADMM iters/s (1024 x 1024, {spins} shifts)",
           "value": round(iters / sec, 3), "unit": "iters/s", "n_gpus": 1, "steps": iters,
           "warmup": warm, "ms_per_step": round(1e3 * sec / iters, 3),
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"1024x1024, scales 1,4,16,64,1024 squared, {spins} shifts "
                                  "averaged per scale and iteration, rho=1",
                      "tiers": tiers,
                      "single_shift_iters_per_s": round(iters / sec1, 3)}}
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        oracle.admm(inst.Y, ladder, rho=1.0, iters=1, cycle_spin=True, seed=1,
                    spin_count=spins)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1 / dt, "unit": "iters/s", "cores": threads,
                               "kind": "oracle", "sample": f"1 iteration, {dt:.2f} s"}
    out.setdefault("config", {})["hw_queues"] = HW_QUEUES
    print(json.dumps(out), flush=True)


def video_bench(args, iters=50, warm=5):
    """Space-time blocks (general block reshape of Sec. 2; the surveillance-video
    experiment of Sec. 10): a 144 x 176 pixel x 192 frame stand-in as a 25344 x 192
    matrix, scales 1 x 1 x 1, 4 x 4 x 4, 16 x 16 x 16 and the whole video, default
    lambda, rho = 1, random cycle spinning. Iterations per second over `iters` after
    `warm`; the oracle times one iteration."""
    import torch
    import paper_1507_08751_amd as msld
    from synth import video_instance
    H, W, T = 144, 176, 192
    M, N = H * W, T
    Y = video_instance(H, W, T, seed=0)
    ladder = [(1, 1), (16, 4), (256, 16), (M, N)]
    kinds = [msld.KIND_BLOCK, msld.KIND_SPATIAL, msld.KIND_SPATIAL, msld.KIND_BLOCK]
    pws = [1, 4, 16, 1]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    Yd = torch.from_numpy(Y).to(dev)
    Z = torch.empty((len(ladder), M, N), dtype=torch.float32, device=dev)
    solver = msld.Solver(M, N, ladder, rho=1.0, iters=iters, cycle_spin=True, seed=1,
                         kinds=kinds, image_w=W, patch_w=pws, device=dev)
    solver.reset(Z)
    solver.step(Yd, Z, warm)
    solver.reset(Z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(Yd, Z, iters)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    tiers = [msld.TIERS[solver.tier(i)] for i in range(len(ladder))]
    solver.close()
    out = {"metric": "space-time ADMM iters/s (144 x 176 x 192 video stand-in)",
           "value": round(iters / sec, 3), "unit": "iters/s", "n_gpus": 1, "steps": iters,
           "warmup": warm, "ms_per_step": round(1e3 * sec / iters, 3),
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "video 144x176 pixels x 192 frames as 25344x192, space-time "
                                  "blocks 1x1x1, 4x4x4, 16x16x16 and the whole video, "
                                  "rho=1, random cycle spinning", "tiers": tiers}}
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        oracle.admm(Y, ladder, rho=1.0, iters=1, cycle_spin=True, seed=1, kinds=kinds,
                    image_w=W, patch_w=pws)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1 / dt, "unit": "iters/s", "cores": threads,
                               "kind": "oracle", "sample": f"1 iteration, {dt:.2f} s"}
    out.setdefault("config", {})["hw_queues"] = HW_QUEUES
    print(json.dumps(out), flush=True)


def copy_calibration(nbytes=1 << 30, reps=3):
    """Plain device-to-device copies of nbytes: what FETCH_SIZE / WRITE_SIZE read for
    a kernel that moves a known number of bytes."""
    import torch
    dev = torch.device("cuda", 0)
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_per_copy": nbytes, "copies": reps}), flush=True)


def cpu_baseline(size, threads_env):
    """The FP64 oracle timed on host cores for one ADMM iteration of a size x size
    instance with the same ladder, density and noise; scaled to iterations/s of the
    8192^2 problem by the area ratio (every scale's work is proportional to M N: the
    oracle decomposes every block, there is no skip)."""
    import numpy as np
    import oracle
    from synth import make_instance
    inst = make_instance(size, size, LADDER, DENSITY, noise=NOISE, seed=0, keep_components=False)
    t0 = time.perf_counter()
    oracle.admm(inst.Y, inst.ladder, rho=1.0, iters=1, cycle_spin=True, seed=0)
    dt = time.perf_counter() - t0
    scale = (size * size) / (8192.0 * 8192.0)
    return {"value": scale / dt, "unit": "iters/s", "cores": threads_env, "kind": "oracle",
            "sample": f"1 ADMM iteration of the FP64 oracle on a {size}x{size} instance "
                      f"(same ladder/density/noise), {dt:.2f} s, scaled by {size}^2/8192^2"}


def serving_measure(nreq, nwarm, max_active, hbm_budget_gib, baseline=True, nsat=None,
                    rate=None, server=True, bwarm=None):
    """Serving workload: a Poisson stream of decompositions of mixed sizes
    ({128^2, 512^2, 1024x256, 2048^2}, ratio-4 ladders of 4-6 scales ending in the
    full block, rank-1/rank-2 blocks at 2% + N(0, 0.01^2)), each retired at primal
    residual <= 1e-4 (cap 300 iterations, no cycle spinning). First the saturation
    rate of the continuous-batching server is measured with the first nsat measured
    requests queued at once; then the trace is replayed at 0.7 x that rate, and
    (baseline) again with one request at a time (FIFO) at the same arrivals. Each
    request's final residual and why it retired (tolerance or cap) are recorded. With
    server=False only the baseline runs (after a warm-up on the first bwarm warm-up
    requests, default all), at the given arrival rate. Returns the figures as a dict."""
    import numpy as np
    import torch
    import paper_1507_08751_amd as msld
    from synth import make_instance, serving_trace

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    trace = serving_trace(nreq + nwarm, rate=1.0, seed=0)
    log(f"serving: generating {len(trace)} requests ...")
    reqs = []
    for (t, M, N, lad, rank, dseed) in trace:
        inst = make_instance(M, N, lad, 0.02, rank=rank, noise=0.01, seed=dseed,
                             keep_components=False)
        reqs.append((t, torch.from_numpy(inst.Y).to(dev), lad))

    def run(active, rate, items):
        srv = msld.Server(max_active=active, hbm_budget=hbm_budget_gib << 30, num_streams=8,
                          device=dev)
        t0 = time.perf_counter()
        arrivals = {}
        lat = {}
        iters = {}
        resid = {}
        nxt = 0
        gaps = np.cumsum([0.0] + [items[i + 1][0] - items[i][0] for i in range(len(items) - 1)])
        while len(lat) < len(items):
            now = time.perf_counter() - t0
            while nxt < len(items) and (rate is None or gaps[nxt] / rate <= now):
                _, Y, lad = items[nxt]
                arrivals[nxt] = (time.perf_counter() - t0) if rate is not None else 0.0
                srv.submit(nxt, Y, lad, iters=300, tol=1e-4, check_every=1)
                nxt += 1
            done = srv.step()
            tnow = time.perf_counter() - t0
            for (rid, it, res, st, Z) in done:
                if st != 0:
                    raise RuntimeError(f"request {rid} failed with status {st}")
                lat[rid] = tnow - arrivals[rid]
                iters[rid] = it
                resid[rid] = res
                if len(lat) % 8 == 0:
                    log(f"  serve(active={active}, rate={rate}): {len(lat)}/{len(items)} done "
                        f"at {tnow:.1f} s")
            if not done and srv.active == 0 and srv.queued == 0 and nxt < len(items):
                time.sleep(max(0.0, gaps[nxt] / rate - (time.perf_counter() - t0)))
        span = time.perf_counter() - t0
        srv.close()
        return span, lat, iters, resid

    warm = reqs[:nwarm]
    meas = reqs[nwarm:]
    if not server:
        bwarm = nwarm if bwarm is None else bwarm
        if rate is None:
            raise ValueError("the baseline alone needs the arrival rate")
        run(1, None, warm[:bwarm])
        span1, lat1, _, _ = run(1, rate, meas)
        l1 = np.array([lat1[i] for i in range(len(meas))]) * 1e3
        return {"baseline_one_at_a_time": {"solves_per_s": round(len(meas) / span1, 4),
                                           "p50_ms": round(float(np.percentile(l1, 50)), 2),
                                           "p99_ms": round(float(np.percentile(l1, 99)), 2)}}
    nsat = len(meas) if nsat is None else max(1, min(nsat, len(meas)))
    run(max_active, None, warm)
    span_sat, _, _, _ = run(max_active, None, meas[:nsat])
    sat = nsat / span_sat
    rate = 0.7 * sat
    log(f"serving saturation: {sat:.2f} solves/s ({span_sat:.2f} s for {nsat})")
    span, lat, iters, resid = run(max_active, rate, meas)
    l = np.array([lat[i] for i in range(len(meas))]) * 1e3
    its = np.array([iters[i] for i in range(len(meas))])
    res = np.array([resid[i] for i in range(len(meas))])
    by_tol = float(np.mean(res <= 1e-4))
    out = {"solves_per_s": round(len(meas) / span, 4),
           "saturation_solves_per_s": round(sat, 4), "saturation_requests": nsat,
           "p50_ms": round(float(np.percentile(l, 50)), 2),
           "p99_ms": round(float(np.percentile(l, 99)), 2),
           "mean_iters": round(float(np.mean(its)), 1),
           "retired_by_tolerance_frac": round(by_tol, 4),
           "retired_at_cap_frac": round(float(np.mean((its >= 300) & (res > 1e-4))), 4),
           "final_resid_p50": float(np.percentile(res, 50)),
           "final_resid_max": float(res.max()),
           "label": "cap-bound: every request ran the 300-iteration cap (primal residual "
                    "above 1e-4 at rho = 1)" if by_tol == 0.0 else "tolerance-bound",
           "requests": len(meas), "warmup_requests": nwarm, "arrival_rate": round(rate, 4),
           "max_active": max_active,
           "workload": "Poisson requests, sizes {128^2, 512^2, 1024x256, 2048^2}, ratio-4 "
                       "ladders of 4-6 scales ending in the full block, rank-1/2 blocks at "
                       "2% + N(0,0.01^2), retire at primal residual <= 1e-4, cap 300"}
    if baseline:
        span1, lat1, _, _ = run(1, rate, meas)
        l1 = np.array([lat1[i] for i in range(len(meas))]) * 1e3
        out["baseline_one_at_a_time"] = {"solves_per_s": round(len(meas) / span1, 4),
                                         "p50_ms": round(float(np.percentile(l1, 50)), 2),
                                         "p99_ms": round(float(np.percentile(l1, 99)), 2)}
    return out


def serve_bench(args):
    """The serving workload on its own (serving_measure with the one-at-a-time
    baseline), printed as its own JSON line. A run too long for one session can be
    split: --no-baseline prints the server's line, then --baseline-from FILE runs the
    baseline alone on the same trace at FILE's arrival rate and prints FILE's line with
    the baseline added."""
    if args.baseline_from:
        with open(args.baseline_from) as f:
            out = json.loads(f.read().strip().splitlines()[-1])
        cfg = out["config"]
        if cfg["requests"] != args.requests or cfg["warmup_requests"] != args.warm_requests:
            raise SystemExit("--requests / --warm-requests differ from the server run's")
        bwarm = args.baseline_warm if args.baseline_warm is not None else args.warm_requests
        b = serving_measure(args.requests, args.warm_requests, 1, args.hbm_budget, server=False,
                            rate=cfg["arrival_rate"], bwarm=bwarm)
        out["baseline_one_at_a_time"] = b["baseline_one_at_a_time"]
        out["baseline_run"] = (f"separate process, the same {args.requests} measured requests at "
                               f"the same arrival rate, after {bwarm} warm-up requests")
        print(json.dumps(out), flush=True)
        return
    r = serving_measure(args.requests, args.warm_requests, args.max_active, args.hbm_budget,
                        nsat=args.sat_requests, baseline=not args.no_baseline)
    out = {"metric": "served solves/s, p99 latency @ primal residual <= 1e-4 (cap 300)",
           "value": r["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {k: r[k] for k in ("workload", "requests", "warmup_requests",
                                        "arrival_rate", "max_active")},
           **{k: r[k] for k in ("saturation_solves_per_s", "saturation_requests", "p50_ms",
                                "p99_ms", "mean_iters", "retired_by_tolerance_frac",
                                "retired_at_cap_frac", "final_resid_p50", "final_resid_max",
                                "label", "baseline_one_at_a_time") if k in r}}
    out.setdefault("config", {})["hw_queues"] = HW_QUEUES
    print(json.dumps(out), flush=True)


def batch_bench(args):
    """Batched workload: independent decompositions of sizes drawn from {64^2, 128^2,
    256^2, 128x512} with ladders {1,4,16,full} or {1,8,32,full}, rank-1 blocks at 2%
    + N(0, 0.01^2), 100 iterations with cycle spinning (shift seed = instance id),
    solved in one batch (stacked launches per shape class) and, as the baseline, one
    solve at a time with the same kernels."""
    import numpy as np
    import torch
    import paper_1507_08751_amd as msld
    from synth import batch_instances

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    insts = batch_instances(args.instances, seed=0)
    K = args.steps if args.steps != 50 else 100
    # autotuned launch choice for every block size of the batch (before any plan)
    tuned = {}
    t0 = time.perf_counter()
    for (m, n) in sorted({(m, n) for i in insts for (m, n) in i.ladder if m * n > 1}):
        r = msld.autotune(m, n, device=dev)
        tuned[f"{m}x{n}"] = {"tier": r["tier"], "lds_cap": r["lds_cap"],
                             "lrs_wide": r["lrs_wide"],
                             "us_per_block": round(r["us_per_block"], 4),
                             "us_default": round(r["us_default"], 4)}
    tune_s = time.perf_counter() - t0
    probs = [{"M": i.Y.shape[0], "N": i.Y.shape[1], "ladder": i.ladder, "iters": K,
              "cycle_spin": True, "seed": j} for j, i in enumerate(insts)]
    Ys = [torch.from_numpy(i.Y).to(dev) for i in insts]
    batch = msld.Batch(probs, device=dev)
    outs, _ = batch.solve(Ys)          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs, _ = batch.solve(Ys, outs)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    solvers = [msld.Solver(p["M"], p["N"], p["ladder"], iters=K, cycle_spin=True, seed=p["seed"],
                           device=dev) for p in probs]
    zs = [torch.empty_like(o) for o in outs]
    solvers[0].solve(Ys[0], zs[0], info=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, y, z in zip(solvers, Ys, zs):
        s.solve(y, z, info=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter() - t0
    worst = 0.0
    for o, z in zip(outs, zs):
        d = (o - z).norm().item() / max(z.norm().item(), 1e-12)
        worst = max(worst, d)
    out = {"metric": "batched solves/s (256 mixed instances, 100 iterations each)",
           "value": round(len(insts) / tb, 4), "unit": "solves/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "sizes {64^2,128^2,256^2,128x512}, ladders {1,4,16,full} / "
                                  "{1,8,32,full}, 2% rank-1 + N(0,0.01^2), cycle spinning",
                      "instances": len(insts), "iters": K, "classes": batch.classes,
                      "autotuned": tuned, "autotune_seconds": round(tune_s, 2)},
           "batch_seconds": round(tb, 4), "one_at_a_time_seconds": round(t1, 4),
           "one_at_a_time_solves_per_s": round(len(insts) / t1, 4),
           "speedup": round(t1 / tb, 3), "max_rel_diff_batch_vs_alone": worst}
    out.setdefault("config", {})["hw_queues"] = HW_QUEUES
    print(json.dumps(out), flush=True)
    batch.close()
    for s in solvers:
        s.close()


PEAK_FP32_TFLOPS = 157.3        # MI355X dense FP32, matrix cores and packed vector ALU alike
LR_P = 16                       # subspace width of the low-rank chain (128 wide and up)
LR_PRODUCTS = 8                 # G X products of its subspace iteration (7) and W = G V_r
LRS_P, LRS_PRODUCTS = 4, 7      # the fused 32-wide kernel


def svd_flops(tier, m, n, live, sweeps, rank, gram_certified=0):
    """Algorithmic FP32 flops of one scale's BlockSVT over `live` block-iterations.

    Jacobi tiers (register, LDS): per live m x n block (m >= n) and sweep,
    3 n (n - 1) (2m + n) (the dot products and rotations of n (n - 1) / 2 column pairs,
    with V), plus 2 m n k for the rebuild at output rank k; sweeps and ranks are the
    device counters. Low-rank tiers: the Gram matrix's unique entries m n (n + 1) per
    live block, and for the blocks its bound does not settle (live - gram_certified) the
    subspace products 2 n^2 P each, the projection B X and the rebuild 2 m n P each; the
    certificate's extra products for undecided blocks are not counted. Skipped blocks
    count nothing."""
    m, n = max(m, n), min(m, n)
    if tier in ("register", "lds"):
        return sweeps * 3.0 * n * (n - 1) * (2 * m + n) + 2.0 * m * n * rank
    if tier == "lowrank":
        P, k = LR_P, LR_PRODUCTS
    elif tier == "lowrank_small":
        P, k = LRS_P, LRS_PRODUCTS
    else:
        return 0.0
    chain = live - gram_certified
    return live * m * n * (n + 1.0) + chain * (k * 2.0 * n * n * P + 2 * 2.0 * m * n * P)


def svd_rooflines(prof, stats, tiers, K):
    """The Gram kernel B^T B of the low-rank scales (their dominant matrix-core kernel,
    timed alone with HIP events on the scale's stream), and each scale's BlockSVT
    (SVD and finish phases) against the FP32 peak."""
    gflops, gms, launches = 0.0, 0.0, 0
    per_scale = []
    for i, (m, n) in enumerate(LADDER):
        if tiers[i] == "1x1":
            continue
        live = stats["live"][i]
        if tiers[i] == "lowrank":
            mm, nn = max(m, n), min(m, n)
            gflops += live * mm * nn * (nn + 1.0)
            gms += prof["gram_ms"][i]
            launches += K
        fl = svd_flops(tiers[i], m, n, live, stats["sweeps"][i], stats["rank"][i],
                       stats["gram_certified"][i])
        ms = prof["scale_ms"][i][2] + prof["scale_ms"][i][3]
        tf = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        per_scale.append({"scale": f"{m}x{n}", "tier": tiers[i],
                          "flops_per_iter": round(fl / K), "ms_per_iter": round(ms / K, 4),
                          "achieved_tflops": round(tf, 2),
                          "frac": round(tf / PEAK_FP32_TFLOPS, 4)})
    tf = gflops / (gms * 1e-3) / 1e12 if gms > 0 else 0.0
    gram = {"bound": "mfma", "kernel": "k_mf_gram", "achieved": round(tf, 2),
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / PEAK_FP32_TFLOPS, 4),
            "launches": launches, "avg_launch_ms": round(gms / max(1, launches), 4),
            "algorithmic_flops_per_launch": round(gflops / max(1, launches)),
            "flops_per_block": "m n (n + 1), the Gram matrix's unique entries"}
    return gram, per_scale


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--mode", choices=["iters", "serve", "batch", "copy", "completion", "spin",
                                       "video"],
                    default="iters",
                    help="copy: a plain device copy of known size, the calibration run for "
                         "the HBM byte counters")
    ap.add_argument("--instances", type=int, default=256)
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--warm-requests", type=int, default=8)
    ap.add_argument("--no-baseline", action="store_true",
                    help="--mode serve: skip the one-at-a-time baseline")
    ap.add_argument("--baseline-from", default=None,
                    help="--mode serve: run only the baseline, at the arrival rate of this "
                         "earlier server line (a file), and print that line with it added")
    ap.add_argument("--baseline-warm", type=int, default=None,
                    help="--baseline-from: warm-up requests run before the baseline")
    ap.add_argument("--sat-requests", type=int, default=200,
                    help="measured requests whose all-at-once run sets the saturation rate")
    ap.add_argument("--max-active", type=int, default=32)
    ap.add_argument("--hbm-budget", type=int, default=64, help="GiB")
    ap.add_argument("--hw-queues", type=int, default=None,
                    help="hardware queues per process (GPU_MAX_HW_QUEUES), 2..32; default 4 "
                         "for the 8192^2 run and the batch, 16 for the other modes")
    ap.add_argument("--fork-mode", type=int, default=0, choices=[0, 1, 2, 3],
                    help="where the scales fork from the main stream (msld_params.fork_mode)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the short serving measurement of the default run")
    ap.add_argument("--serve-requests", type=int, default=16,
                    help="requests of the default run's serving measurement")
    args = ap.parse_args()
    if args.hw_queues is None:
        args.hw_queues = 4 if args.mode in ("iters", "batch") else 16
    if not 2 <= args.hw_queues <= 32:
        ap.error("--hw-queues must be in 2..32")
    global HW_QUEUES
    HW_QUEUES = args.hw_queues
    os.environ["GPU_MAX_HW_QUEUES"] = str(HW_QUEUES)
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU (the multi-GPU path is a "
                                   "design only); --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.mode == "serve":
        serve_bench(args)
        return
    if args.mode == "batch":
        batch_bench(args)
        return
    if args.mode == "copy":
        copy_calibration()
        return
    if args.mode == "completion":
        completion_bench(args)
        return
    if args.mode == "spin":
        spin_bench(args)
        return
    if args.mode == "video":
        video_bench(args)
        return

    import numpy as np
    import torch
    import paper_1507_08751_amd as msld
    from synth import make_instance

    M = N = args.size
    K, W = args.steps, args.warmup
    log(f"generating {M}x{N} instance ...")
    inst = make_instance(M, N, LADDER, DENSITY, noise=NOISE, seed=0, keep_components=False)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    Y = torch.from_numpy(inst.Y).to(dev)
    L = len(LADDER)
    Z = torch.empty((L, M, N), dtype=torch.float32, device=dev)
    solver = msld.Solver(M, N, LADDER, rho=1.0, iters=K, cycle_spin=True, seed=0, device=dev,
                         fork_mode=args.fork_mode)
    tiers = [msld.TIERS[solver.tier(i)] for i in range(L)]
    log("tiers:", tiers)
    if W > 0:
        solver.reset(Z)
        solver.step(Y, Z, W)
        torch.cuda.synchronize()
        log(f"warmup {W} iterations done")
    solver.reset(Z)
    torch.cuda.synchronize()
    solver.profile_begin(K)
    t0 = time.perf_counter()
    solver.step(Y, Z, K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = solver.profile_end()
    stats = solver.stats()
    r = solver.step(Y, Z, 1, resid=True)   # untimed: residual after K+1 iterations
    torch.cuda.synchronize()
    sec = t1 - t0
    ips = K / sec
    log(f"timed {K} iterations: {sec:.3f} s -> {ips:.2f} iters/s; resid after K+1: {r:.3e}")
    log(f"consensus ms total {prof['consensus_ms']:.2f}, stream pass (all scales) "
        f"{prof['stream_ms']:.2f}")
    for i, (m, n) in enumerate(LADDER):
        ms = prof["scale_ms"][i]
        nblk = (M // m) * (N // n)
        log(f"scale {i} ({m}x{n}, {tiers[i]}): setup {ms[1]:.2f} "
            f"svd {ms[2]:.2f} finish {ms[3]:.2f} ms; live {stats['live'][i]} of {nblk * K} "
            f"block-iters, sweeps {stats['sweeps'][i]}, rank {stats['rank'][i]}, "
            f"certified {stats['certified'][i]} (fail coupling {stats['fail_coupling'][i]}, "
            f"bound {stats['fail_bound'][i]}, polar {stats['polar'][i]}); undecided by the trace "
            f"bound {stats['undecided'][i]}, certified by Collatz-Wielandt only "
            f"{stats['cw_certified'][i]}, certified zero by the Gram bound "
            f"{stats['gram_certified'][i]}")
    roof, extra = stream_roofline(prof, tiers, M, N, K)
    k50 = None
    if K != 50:
        # the metric's configuration runs 50 iterations: their rate, timed the same way
        solver.reset(Z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.step(Y, Z, 50)
        torch.cuda.synchronize()
        k50 = 50 / (time.perf_counter() - t0)
        log(f"50 iterations from zero: {k50:.2f} iters/s")
    if args.fork_mode == 3:
        sprof, sstats, ssec = prof, stats, sec
    else:
        # the SVD figures come from the same K iterations with the scales run one after
        # another on one stream (fork_mode 3), so that each phase's events time its own
        # kernels rather than kernels sharing the chip with the other scales' chains
        solver.close()
        solver = msld.Solver(M, N, LADDER, rho=1.0, iters=K, cycle_spin=True, seed=0,
                             device=dev, fork_mode=3)
        solver.reset(Z)
        torch.cuda.synchronize()
        solver.profile_begin(K)
        t0 = time.perf_counter()
        solver.step(Y, Z, K)
        torch.cuda.synchronize()
        ssec = time.perf_counter() - t0
        sprof = solver.profile_end()
        sstats = solver.stats()
        log(f"serial-scale run of the same {K} iterations: {K / ssec:.2f} iters/s")
    gram_roof, svd_scales = svd_rooflines(sprof, sstats, tiers, K)
    gram_roof["run"] = "scales one after another on one stream (fork_mode 3)"
    gram_roof["serial_iters_per_s"] = round(K / ssec, 3)
    # the whole iteration against HBM: every Z_i and U_i plane read and written once and
    # Y read once, (4L + 1) 4 M N bytes
    it_bytes = (4 * L + 1) * 4 * M * N
    it_gbs = it_bytes / (sec / K) / 1e9
    it_hbm = {"bound": "hbm", "algorithmic_bytes_per_iter": it_bytes,
              "achieved": round(it_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
              "frac": round(it_gbs / PEAK_HBM_GBS, 4)}
    out = {"metric": METRIC, "value": round(ips, 4), "unit": "iters/s", "n_gpus": 1, "steps": K,
           "warmup": W, "ms_per_step": round(1e3 * sec / K, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"ADMM on {M}x{N} fp32, blocks 1/8/32/128/512, 1% active "
                                  f"rank-1 blocks per scale + N(0,0.01^2) noise, default lambda, "
                                  f"rho=1, random cycle spinning, {K} iterations from zero",
                      "M": M, "N": N, "ladder": [list(b) for b in LADDER], "iters": K,
                      "timed_window": f"iterations 1..{K} of a solve from zero (the warm-up "
                                      f"is a separate {W}-iteration solve)",
                      "hw_queues": HW_QUEUES},
           "value_k50": round(k50 if k50 is not None else ips, 4),
           "roofline": roof, "roofline_consensus": extra, "roofline_svd": gram_roof,
           "blocksvt_fp32": svd_scales, "iteration_hbm": it_hbm,
           "live_fraction": {f"{m}x{n}": round(stats["live"][i] / ((M // m) * (N // n) * K), 4)
                             for i, (m, n) in enumerate(LADDER)},
           "phases_ms_per_iter": {
               "consensus": round(prof["consensus_ms"] / K, 4),
               "stream_all": round(prof["stream_ms"] / K, 4),
               **{f"scale{i}_{m}x{n}_{tiers[i]}": [round(v / K, 4) for v in prof["scale_ms"][i]]
                  for i, (m, n) in enumerate(LADDER) if tiers[i] != "1x1"}}}
    solver.close()
    del Z, Y
    torch.cuda.empty_cache()
    if not args.no_serving:
        # the served half of the metric: a short run of the serving workload (saturation,
        # then Poisson arrivals at 0.7 x saturation); bench.py --mode serve runs it longer
        # with the one-at-a-time baseline
        out["serving"] = serving_measure(args.serve_requests, 4, args.max_active,
                                         args.hbm_budget, baseline=True)
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"cpu baseline: oracle on {args.cpu_sample}^2 with {threads} threads ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample, threads)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
