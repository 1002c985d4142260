#!/usr/bin/env python3
"""Throughput of the whole unwrapping path (residues -> integer cost table ->
edge costs -> exact min-cost flow -> integration) on one MI355X.

Workload: the 74.3-Mpixel synthetic strike-slip scene (6912 x 10752, L = 15,
3 % nodata; see paper_2609_36267_amd/synth.py).  One step is one ww_unwrap
call on device-resident psi / coherence / mask producing device-resident K
and phi; the cost table is cached per L, as the library always does.

Prints one JSON line: Mpixel/s, the roofline of the dominant kernel (the
tile relaxation rounds of the shortest-path search; algorithmic bytes =
tile visits x bytes one visit must move, over the rounds' device time
measured inside the library on the device clock, batch by batch) and the
CPU oracle timed on a bounded sample of the same scene.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel/s unwrapped at 74 Mpix (exact min cost); batched p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# The method's own work (the shortest-path searches of Section II-C), per
# unit: an arc scanned moves its cost (2 B), its flow state (1 B), the
# head's label (8 B) and potential (8 B); a settled node moves about 8 B of
# queue traffic.  The solver counts settled nodes and the residual out-arcs
# of every settled node when WW_MCF_COUNT=1 (an untimed extra solve).
BYTES_PER_ARC_SCAN = 2 + 1 + 8 + 8
BYTES_PER_SETTLED = 8
# Bytes one relaxation visit of a 32 x 32 loop tile stages: per loop node
# its label (8 B read + 8 B write), its potential (4 B) and the two pixel
# edges it owns (2 x (two int16 costs + one int8 flow) = 10 B).
TILE_NODES = 32 * 32
BYTES_PER_NODE_VISIT = 8 + 8 + 4 + 10
BYTES_PER_TILE_VISIT = TILE_NODES * BYTES_PER_NODE_VISIT
GOLDEN = os.path.join(ROOT, "tests", "golden", "fault_6912x10752_L15_cost.json")
# HBM bytes per k_sssp_round launch on the fault scene from rocprofv3
# FETCH_SIZE / WRITE_SIZE runs, scaled by a plain 1 GiB copy's readings
# (fetch x 2.0, write x 1.0), valid for the round-kernel source of that hash
# (see round_kernel_sha) and the solve schedule they were taken with only.
TRAFFIC_SOURCE_SHA = "027a9462dcaf84a4"
TRAFFIC_SCHEDULE = (64, 256, 4, 0, 1024, 6, 32)
TRAFFIC_BYTES_PER_LAUNCH = 14.41e6


def round_kernel_sha() -> str:
    """Hash of the source text of the relaxation-round kernel and the device
    helpers it calls (csrc/mcf.hip, from the staged reduced-cost encoding to
    the end of k_sssp_round) and of the number of rounds launched per host
    check (the share of empty launches in the per-launch average): the
    measured traffic belongs to that code only."""
    import hashlib
    txt = open(os.path.join(ROOT, "paper_2609_36267_amd", "csrc", "mcf.hip")).read()
    a = txt.index("// Reduced costs of the in-arcs are staged as unsigned words")
    b = txt.index("__global__ void k_requeue_pending(")
    c = txt.index("#define WW_ROUNDS_PER_SYNC")
    d = txt.index("\n", c)
    return hashlib.sha256((txt[a:b] + txt[c:d]).encode()).hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c0", "c1", "c2"])
    ap.add_argument("--cpu-rows", type=int, default=384,
                    help="rows of the full-width strip the oracle is timed on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-stack", action="store_true",
                    help="also time the oracle on all 64 stack jobs, one after another (minutes)")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the components, Goldstein and bridging legs (for counter runs)")
    ap.add_argument("--schedule", default=None, metavar="H0,DSTEP[,FULL,FIRSTDEF,REVERSE[,GROWTH[,TILECOLS]]]",
                    help="solve schedule to time (skips tuning), e.g. 64,256,2,0,0")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the library's default solve schedule instead of tuning it on a "
                         "sibling scene first")
    ap.add_argument("--slots", type=int, default=8, help="job-server workers for the stack and serving legs")
    ap.add_argument("--stack-jobs", type=int, default=64, help="interferograms in the stack leg (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="length of the serving leg's Poisson stream (0: skip the leg)")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-pool", type=int, default=128,
                    help="distinct requests, drawn on the GPU and held in pinned host memory")
    ap.add_argument("--serve-sweep", default="", metavar="R1,R2,...",
                    help="arrival rates (requests/s, ascending) at which each path's sustained "
                         "throughput is measured; a path stops at its first rate it cannot sustain")
    ap.add_argument("--serve-sweep-seconds", type=float, default=15.0)
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg and print its record")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes (to scale HBM byte counters) and exit")
    ap.add_argument("--serve-oracle-frac", type=float, default=0.05,
                    help="share of the served requests drawn at random for the oracle check")
    ap.add_argument("--serve-oracle-max-px", type=int, default=1 << 20,
                    help="sampled requests above this many pixels are counted, not checked")
    return ap.parse_args()


def cpu_baseline(sc, rows):
    """The oracle (single thread) on a full-width strip of the same scene
    through the fault: residues + edge costs + SSP + integration, with its
    cost table built beforehand (the GPU path caches its table too)."""
    import numpy as np
    import oracle
    m, n = sc.psi.shape
    r0 = max(0, m // 2 - rows // 2)
    sl = slice(r0, r0 + rows)
    psi = np.ascontiguousarray(sc.psi[sl])
    coh = np.ascontiguousarray(sc.coh[sl])
    valid = np.ascontiguousarray(sc.valid[sl])
    lut = oracle.build_lut(sc.looks)
    t0 = time.perf_counter()
    oracle.unwrap(psi, coh, valid, sc.looks, lut=lut)
    dt = time.perf_counter() - t0
    px = psi.size
    return {"value": round(px / 1e6 / dt, 4), "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
            "sample": f"rows {r0}..{r0 + rows - 1} x all {n} cols of the same scene "
                      f"({px / 1e6:.2f} Mpixel, crosses the fault), {dt:.2f} s single-threaded; "
                      "cost table excluded (cached on both paths)",
            "host": _cpu_model()}


def cpu_baseline_configs(scenes, stack=None):
    """The oracle (single thread, cost table built beforehand) on the
    smaller workloads in full: c0 and c1 (`scenes`, generated before the GPU
    was initialised), and on request every stack job one after another."""
    import oracle
    out = {}
    luts = {}
    for name, sc in scenes.items():
        lut = luts.setdefault(sc.looks, oracle.build_lut(sc.looks))
        t0 = time.perf_counter()
        cost = oracle.unwrap(sc.psi, sc.coh, sc.valid, sc.looks, lut=lut)[2]
        dt = time.perf_counter() - t0
        out[name] = {"mpix_s": round(sc.psi.size / 1e6 / dt, 4), "seconds": round(dt, 2),
                     "pixels": int(sc.psi.size), "cost": int(cost)}
    if stack:
        px, dt, costs = 0, 0.0, []
        for sc in stack:
            lut = luts.setdefault(sc.looks, oracle.build_lut(sc.looks))
            t0 = time.perf_counter()
            costs.append(int(oracle.unwrap(sc.psi, sc.coh, sc.valid, sc.looks, lut=lut)[2]))
            dt += time.perf_counter() - t0
            px += sc.psi.size
        out["stack"] = {"jobs": len(stack), "mpix_s": round(px / 1e6 / dt, 4), "seconds": round(dt, 1),
                        "pixels": int(px), "total_cost_sum": int(sum(costs))}
    return out


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def _sched_dict(sched):
    """A solve schedule (2 to 6 fields, missing ones at their defaults) as a
    dict."""
    from paper_2609_36267_amd import autotune
    full = autotune.pad(sched)
    return {"first_hop_window": full[0], "first_distance_step": full[1], "full_passes": full[2],
            "first_deficit_after": full[3], "reverse_below": full[4], "hop_growth": full[5],
            "tile_cols": full[6]}


def stack_scenes(args, synth):
    t0 = time.time()
    scs = [synth.stack_job(k) for k in range(args.stack_jobs)]
    return scs, time.time() - t0


def serve_pool(args, torch, synth):
    """The request pool: each request drawn on the GPU, then held in pinned
    host memory (inputs and its result buffers)."""
    t0 = time.time()
    pool = []
    for k in range(args.serve_pool):
        arrs = synth.serve_request_device(k)
        pin = []
        for a in arrs:
            h = torch.empty(a.shape, dtype=a.dtype, pin_memory=True)
            h.copy_(a)
            pin.append(h)
        m, n = arrs[0].shape
        del arrs
        pool.append({"psi": pin[0], "coh": pin[1], "valid": pin[2], "m": m, "n": n, "px": m * n,
                     "K": torch.empty((m, n), dtype=torch.int32, pin_memory=True),
                     "phi": torch.empty((m, n), dtype=torch.float32, pin_memory=True)})
        if (k + 1) % 16 == 0:
            print(f"# serve pool: {k + 1} of {args.serve_pool} requests drawn", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return pool, time.time() - t0


def components_leg(ww, torch, psi, coh, valid, looks, m, n, reps=3):
    """Connected components of reliably unwrapped pixels on the scene's own
    solution (Section II-D): device time of ww_connected_components after
    the solve, default threshold and minimum size."""
    res, _, _ = ww.residues(psi, valid)
    costs = ww.edge_costs(psi, coh, valid, ww.build_cost_lut(looks))
    r = ww.mcf_solve(res, costs, m, n)
    del res
    ww.connected_components(r.dk_x, r.dk_y, costs, valid)  # warm workspace
    best, nc = float("inf"), 0
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, nc = ww.connected_components(r.dk_x, r.dk_y, costs, valid)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return {"ms": round(best * 1e3, 3), "mpix_s": round(m * n / 1e6 / best, 1), "components": nc,
            "threshold": 300, "min_size_frac": 0.001}


# FP32 operations of one complex radix-2 N-point transform: (N/2) log2 N
# butterflies of one complex multiply (6) and two complex adds (4).
def _fft_flops(N):
    import math
    return (N // 2) * int(math.log2(N)) * 10


def goldstein_leg(ww, torch, psi, coh, valid, looks, m, n, reps=5):
    """The optional Goldstein preprocessing (Section II-D) on the same scene:
    device time of ww_goldstein_filter (default 32 x 32 patches, 3 x 3
    spectrum smoothing, alpha 0.5), its roofline, and one whole
    ww_unwrap_filtered call."""
    p = ww.default_filter_params()
    N = p.patch
    out = ww.goldstein_filter(psi, valid, p)
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ww.goldstein_filter(psi, valid, p, out=out)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = sorted(ts)[len(ts) // 2]
    S = N // 2
    patches = ((m + S - 1) // S + 1) * ((n + S - 1) // S + 1)
    # forward and inverse 2-D transforms: 2 x 2N one-dimensional transforms
    flops = patches * 4 * N * _fft_flops(N)
    alg_bytes = m * n * (4 + 1 + 4)  # psi + mask in, filtered psi out
    r_raw = int(ww.residues(psi, valid)[0].abs().sum())
    r_f = int(ww.residues(out, valid)[0].abs().sum())
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, _, tot = ww.unwrap_filtered(psi, coh, valid, looks)
    torch.cuda.synchronize()
    uw_ms = (time.perf_counter() - t) * 1e3
    return {"filter_ms": round(ms, 3), "filter_mpix_s": round(m * n / 1e3 / ms, 1),
            "patch": N, "smooth": p.smooth, "alpha": round(p.alpha, 3),
            "fft_gflop": round(flops / 1e9, 2),
            "fp32_tflops": round(flops / (ms * 1e-3) / 1e12, 2),
            "fp32_frac": round(flops / (ms * 1e-3) / 157.3e12, 4),
            "alg_bytes_gbs": round(alg_bytes / (ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "residues_raw": r_raw, "residues_filtered": r_f,
            "unwrap_filtered_ms": round(uw_ms, 1), "unwrap_filtered_cost": tot}


def bridge_leg(ww, torch, synth, psi, coh, valid, looks, m, n, reps=3):
    """Bridging of mask-separated regions (Section II-D) on the same scene
    with a river, a canal and 30 lakes with islands added to its mask
    (synth.river_mask, width 40 px): ww_unwrap on that mask, then the device
    time of ww_bridge on its cycle counts."""
    import numpy as np
    river = synth.river_mask(m, n, np.random.default_rng(7), width=40, lakes=30)
    vr = valid & torch.from_numpy(river).cuda()
    K, _, tot = ww.unwrap(psi, coh, vr, looks)
    Kb = torch.empty_like(K)
    phib = torch.empty((m, n), dtype=torch.float32, device="cuda")
    _, _, R = ww.bridge(psi, vr, K, out=(Kb, phib))
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ww.bridge(psi, vr, K, out=(Kb, phib))
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    moved = int((Kb != K).sum())
    alg = m * n * (4 + 1 + 4 + 4 + 4)  # psi, mask, K in; K, phi out
    return {"ms": round(best * 1e3, 3), "mpix_s": round(m * n / 1e6 / best, 1), "regions": R,
            "pixels_shifted": moved, "unwrap_cost": tot,
            "alg_bytes_gbs": round(alg / best / 1e9, 1),
            "hbm_frac": round(alg / best / 1e9 / HBM_PEAK_GBS, 4),
            "mask": "scene mask + river (40 px) + canal + 30 lakes with islands"}


def streaming_leg(ww, torch, psi, coh, valid, looks, m, n, reps=7):
    """The three streaming steps of the path timed alone on the scene
    (HIP events on the library's stream, median of `reps`), with their
    algorithmic bytes per pixel, beside two measured ceilings: a plain 1 GiB
    device copy, and random 64-bit atomicMin (the SSSP labels' update) by
    torch's scatter_reduce."""
    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return sorted(ts)[len(ts) // 2]
    lut = torch.from_numpy(ww.build_cost_lut(looks)).cuda()
    res = torch.empty((m - 1, n - 1), dtype=torch.int8, device="cuda")
    dkx = torch.zeros((m, n - 1), dtype=torch.int8, device="cuda")
    dky = torch.zeros((m - 1, n), dtype=torch.int8, device="cuda")
    px = m * n
    out = {}
    for name, bpp, fn in (
            ("residues", 6, lambda: ww.load().ww_residues(ww._ptr(psi), ww._ptr(valid), m, n,
                                                          ww._ptr(res), None, None, ww._stream())),
            ("edge_costs", 17, lambda: ww.edge_costs(psi, coh, valid, lut)),
            ("integrate", 15, lambda: ww.integrate(psi, valid, dkx, dky))):
        ms = timed(fn)
        gbs = bpp * px / (ms * 1e-3) / 1e9
        out[name] = {"ms": round(ms, 4), "bytes_per_px": bpp, "gbs": round(gbs, 1),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    del res, dkx, dky
    src = torch.ones(256 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    ms = timed(lambda: dst.copy_(src))
    out["copy_ceiling"] = {"gbs": round(2 * (1 << 30) / (ms * 1e-3) / 1e9, 1),
                           "hbm_frac": round(2 * (1 << 30) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "what": "torch copy of 1 GiB (read + write)"}
    # hand-written ceilings: 16-byte grid sweeps of the library (copy, read
    # only, copy with non-temporal accesses), at 1 GiB and at the size of
    # the scene's phase plane
    hw = {}
    out32k = torch.empty(32 << 10, dtype=torch.uint8, device="cuda")
    for label, nbytes in (("1GiB", 1 << 30), ("psi_plane", px * 4 // 16 * 16)):
        s_ = src.view(torch.uint8)[:nbytes]
        d_ = dst.view(torch.uint8)[:nbytes]
        rec = {}
        for mode, what, moved in ((0, "copy", 2), (1, "read", 1), (2, "copy_nontemporal", 2)):
            ms = ww.stream_probe(s_, out32k if mode == 1 else d_, mode=mode, reps=reps)
            gbs = moved * nbytes / (ms * 1e-3) / 1e9
            rec[what] = {"gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        hw[label] = {"bytes": nbytes, **rec}
    out["hand_written_ceiling"] = hw
    del src, dst, out32k
    # 2^26 random 64-bit atomicMin updates onto as many labels
    nupd = 1 << 26
    g = torch.Generator(device="cuda").manual_seed(7)
    idx = torch.randint(0, nupd, (nupd,), device="cuda", generator=g)
    val = torch.randint(0, 1 << 62, (nupd,), device="cuda", generator=g)
    lab = torch.full((nupd,), (1 << 62), dtype=torch.int64, device="cuda")
    ms = timed(lambda: lab.scatter_reduce_(0, idx, val, reduce="amin"))
    out["atomic_min_ceiling"] = {"gupd_s": round(nupd / (ms * 1e-3) / 1e9, 2),
                                 "what": "torch scatter_reduce amin, 2^26 random int64 updates"}
    return out


def stack_leg(args, ww, torch, scs, gen_s):
    """64 interferograms of mixed size and L, all device resident: one
    ww_unwrap_batch call (every min-cost-flow problem of the stack solved in
    one run of successive shortest paths over the union of the jobs'
    graphs) against 64 sequential plain ww_unwrap calls and against the
    job server with ``--slots`` workers, at identical exact costs."""
    dev = [(torch.from_numpy(sc.psi).cuda(), torch.from_numpy(sc.coh).cuda(),
            torch.from_numpy(sc.valid).cuda(), sc.looks) for sc in scs]
    outs = [(torch.empty(sc.psi.shape, dtype=torch.int32, device="cuda"),
             torch.empty(sc.psi.shape, dtype=torch.float32, device="cuda")) for sc in scs]
    px = sum(sc.psi.size for sc in scs)
    for L in sorted({sc.looks for sc in scs}):
        ww.build_cost_lut(L)
    # solve schedule tuned on a sample of the stack (every 8th job) with the
    # batch call, then used by all three paths
    from paper_2609_36267_amd import autotune
    t = time.perf_counter()
    sched, table = autotune.tune_schedule(dev[::8], batch=True)
    tune_s = time.perf_counter() - t
    # warm every path (workspaces grow to the largest need)
    ww.unwrap(*dev[0][:3], dev[0][3], out=outs[0])
    ww.unwrap_batch(dev, sched=sched)
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain = [ww.unwrap(*d[:3], d[3], out=o)[2] for d, o in zip(dev, outs)]
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t
    best_s, batch = float("inf"), None
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        res, arr = ww.unwrap_batch(dev, sched=sched)
        torch.cuda.synchronize()
        best_s = min(best_s, time.perf_counter() - t)
        batch = [r[2] for r in res]
    st = ww.last_mcf_stats()
    with ww.Server(slots=args.slots) as srv:  # warm the workers
        for d in dev[:args.slots]:
            srv.submit(*d)
        srv.drain()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k, d in enumerate(dev):
            srv.submit(*d, tag=k)
        done = srv.drain()
        torch.cuda.synchronize()
        server_s = time.perf_counter() - t
    server = [0] * len(dev)
    for j, _, _ in done:
        server[j.tag] = int(j.total_cost)
    return {"workload": f"stack of {len(scs)} interferograms, rows logU[512,2048] x cols logU[512,4096], "
                        "L in {5,9,15}, bump 5-80 rad (seeds 1000+k)",
            "pixels": px, "generated_s": round(gen_s, 1),
            "batched_mpix_s": round(px / 1e6 / best_s, 2), "plain_mpix_s": round(px / 1e6 / plain_s, 2),
            "server_mpix_s": round(px / 1e6 / server_s, 2), "server_slots": args.slots,
            "batched_s": round(best_s, 4), "plain_s": round(plain_s, 4), "server_s": round(server_s, 4),
            "speedup_vs_plain": round(plain_s / best_s, 3), "speedup_vs_server": round(server_s / best_s, 3),
            "identical_costs": plain == batch == server, "total_cost_sum": int(sum(batch)),
            "batched_solve": {k: st[k] for k in ("passes", "windows", "rounds", "tile_visits",
                                                 "augmentations", "relax_ms", "solve_ms")},
            "schedule": {**_sched_dict(sched),
                         "tuned_on": f"{len(dev[::8])} of the {len(dev)} jobs, {len(table)} candidates",
                         "tuning_s": round(tune_s, 2)}}


def serve_stream(ww, pool, slots, rate, seconds, seed, alone=None, label=""):
    """One Poisson stream of requests (pool entries drawn uniformly) through
    the job server with ``slots`` workers.  Latency runs from arrival to the
    results back in host memory (copies included).  Returns the record and
    the pool index of every request."""
    import numpy as np
    rng = np.random.default_rng(seed)
    n_req = max(1, int(rate * seconds))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    picks = rng.integers(0, len(pool), n_req)
    lat, done = [], []
    with ww.Server(slots=slots) as srv:
        t_start = ww.clock()
        t_note = t_start

        def collect(jobs):
            for j, _, _ in jobs:
                lat.append(j.t_end - j.t_submit)
                done.append((int(j.tag), int(j.total_cost), int(j.status)))

        for a, k in zip(arrivals, picks):
            while ww.clock() - t_start < a:
                collect(srv.poll(wait_ms=1))
            p = pool[k]
            srv.submit(p["psi"], p["coh"], p["valid"], 9, K=p["K"], phi=p["phi"], tag=int(k))
            if ww.clock() - t_note > 10.0:
                t_note = ww.clock()
                print(f"# serve {label} slots={slots} rate={rate:g}: {len(done)} of {n_req} done "
                      f"at {t_note - t_start:.0f} s", file=sys.stderr, flush=True)
        collect(srv.drain())
        span = ww.clock() - t_start
    px = sum(pool[k]["px"] for k in picks)
    offered = px / 1e6 / float(arrivals[-1])
    rec = {"rate": rate, "requests": len(done), "offered_mpix_s": round(offered, 2),
           "mpix_s": round(px / 1e6 / span, 2), "makespan_s": round(span, 2),
           "arrival_span_s": round(float(arrivals[-1]), 2),
           "p50_ms": round(_pct(lat, 50) * 1e3, 2), "p99_ms": round(_pct(lat, 99) * 1e3, 2),
           "all_ok": all(st == 0 for _, _, st in done)}
    if alone is not None:
        rec["same_cost_as_alone"] = all(st == 0 and c == alone[k] for k, c, st in done)
    # sustained: the stream's pixels were served at >= 95% of the offered rate
    rec["sustained"] = bool(rec["all_ok"] and rec["mpix_s"] >= 0.95 * offered)
    return rec, picks


def serve_leg(args, ww, torch, pool, gen_s):
    """Config-4 serving: a Poisson stream of unwrap requests (c1 recipe,
    rows and columns log-uniform in [256, 8192]) from a pool of distinct
    requests in pinned host memory, through the job server (``--slots``
    workers: continuous batching, admission by device footprint) and through
    the plain path (one request at a time, the same copies), both at the
    same exact costs as each request solved alone; an oracle check on a
    random share of the served requests; optionally the highest rate each
    path sustains."""
    import numpy as np
    ww.build_cost_lut(9)
    from paper_2609_36267_amd import autotune
    # window schedule tuned on four pool requests (plain path, device copies)
    small = sorted(range(len(pool)), key=lambda k: pool[k]["px"])
    tune_on = [small[len(small) // 4], small[len(small) // 2], small[3 * len(small) // 4], small[-1]]
    sample = [tuple(pool[k][a].cuda() for a in ("psi", "coh", "valid")) + (9,) for k in tune_on]
    sched, _ = autotune.tune_schedule(sample)
    del sample
    # every pool entry alone (plain path): the cost each served request must equal
    alone = {}
    t0 = time.time()
    for k, p in enumerate(pool):
        alone[k] = ww.unwrap(p["psi"].cuda(), p["coh"].cuda(), p["valid"].cuda(), 9)[2]
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    alone_s = time.time() - t0
    print(f"# serve: pool solved alone in {alone_s:.1f} s", file=sys.stderr, flush=True)
    served, picks = serve_stream(ww, pool, args.slots, args.serve_rate, args.serve_seconds, 42, alone,
                                 "server")
    print(f"# serve server: {served}", file=sys.stderr, flush=True)
    plain, _ = serve_stream(ww, pool, 1, args.serve_rate, args.serve_seconds, 42, alone, "plain")
    print(f"# serve plain: {plain}", file=sys.stderr, flush=True)
    sweep = None
    if args.serve_sweep:
        rates = [float(r) for r in args.serve_sweep.split(",")]
        sweep = {}
        for name, slots in (("server", args.slots), ("plain", 1)):
            recs, best = [], None
            for r in rates:
                rec, _ = serve_stream(ww, pool, slots, r, args.serve_sweep_seconds, 7, alone, name)
                recs.append(rec)
                print(f"# sweep {name}: {rec}", file=sys.stderr, flush=True)
                if not rec["sustained"]:
                    break
                best = r
            sweep[name] = {"max_sustained_rate": best, "runs": recs}
    # oracle on a random share of the served requests (same seeded draw)
    import oracle
    rng = np.random.default_rng(4242)
    nsamp = max(1, int(round(args.serve_oracle_frac * len(picks))))
    drawn = rng.choice(len(picks), size=min(nsamp, len(picks)), replace=False)
    ks = sorted(set(int(picks[i]) for i in drawn))
    todo = [k for k in ks if pool[k]["px"] <= args.serve_oracle_max_px]
    lut = oracle.build_lut(9)

    def check(k):
        p = pool[k]
        got = oracle.unwrap(p["psi"].numpy(), p["coh"].numpy(), p["valid"].numpy(), 9, lut=lut)[2]
        return k, int(got) == alone[k]

    t0 = time.time()
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        res = list(ex.map(check, todo))
    checked = {"sampled_requests": int(len(drawn)), "distinct_pool_entries": len(ks),
               "checked": len(todo), "over_size_cap": len(ks) - len(todo),
               "size_cap_px": args.serve_oracle_max_px, "all_equal": all(ok for _, ok in res),
               "unequal": [k for k, ok in res if not ok], "oracle_s": round(time.time() - t0, 1)}
    px = np.array([p["px"] for p in pool])
    return {"workload": f"Poisson {args.serve_rate:g} req/s for {args.serve_seconds:g} s, pool of "
                        f"{len(pool)} requests (rows, cols logU[256, 8192], c1 recipe, seeds 2000+k, "
                        "drawn on the GPU), pinned host inputs and outputs",
            "pool_mpix": round(float(px.sum()) / 1e6, 1), "pool_mean_mpix": round(float(px.mean()) / 1e6, 2),
            "generated_s": round(gen_s, 1), "alone_s": round(alone_s, 1), "slots": args.slots,
            "schedule": {**_sched_dict(sched), "tuned_on": "4 pool requests (quartiles of size)"},
            "server": served, "plain": plain,
            "speedup_mpix_s": round(served["mpix_s"] / plain["mpix_s"], 3) if plain["mpix_s"] else None,
            "sweep": sweep, "oracle_check": checked}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip() + f" ({os.cpu_count()} logical CPUs visible)"
    except OSError:
        pass
    return "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the library runs on exactly one GPU (no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2609_36267_amd import binding as ww
    from paper_2609_36267_amd import synth

    if args.copy_calibration > 0:
        # a plain copy of known size: reads and writes exactly MIB MiB each
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nb, "copies": 3}), flush=True)
        return

    ww.load()
    if args.serve_only:
        assert torch.cuda.is_available(), "no GPU visible"
        pool = serve_pool(args, torch, synth)
        out = {"metric": "Mpixel/s served (Poisson stream of unwrap requests)", "n_gpus": 1,
               "higher_is_better": True, "data": "synthetic", "dtype": "i32",
               "serve": serve_leg(args, ww, torch, *pool)}
        out["value"] = out["serve"]["server"]["mpix_s"]
        out["unit"] = "Mpixel/s"
        print(json.dumps(out), flush=True)
        return
    # generate (forked worker processes) before the GPU is initialised
    t0 = time.time()
    sc = synth.config(args.workload)
    m, n = sc.psi.shape
    print(f"# generated {args.workload} {m}x{n} in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    # a sibling of the timed scene (same recipe and size, another seed) on
    # which the solve schedule is tuned: the timed scene is never used for
    # tuning (a half-size sibling picked tile shapes and distance steps that
    # lose on the full size, where fronts cross more tiles)
    sib = None
    if not args.no_tune and args.schedule is None and args.workload == "c2":
        sib = synth.make_fault(m, n, looks=sc.looks, seed=3, mask_frac=0.03)
    stack = stack_scenes(args, synth) if args.stack_jobs > 0 else None
    # the oracle's smaller workloads, also generated before the GPU is used
    # (the generator forks worker processes)
    cpu_scenes = {} if args.no_cpu_baseline else {name: synth.config(name) for name in ("c0", "c1")}
    print(f"# generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    assert torch.cuda.is_available(), "no GPU visible"
    psi = torch.from_numpy(sc.psi).cuda()
    coh = torch.from_numpy(sc.coh).cuda()
    valid = torch.from_numpy(sc.valid).cuda()
    K = torch.empty((m, n), dtype=torch.int32, device="cuda")
    phi = torch.empty((m, n), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()

    tuned_on = "library default (not tuned)"
    tune_top = None  # the five fastest candidates on the sibling scene (schedule, ms)
    if args.schedule:
        ww.set_mcf_params(*[int(x) for x in args.schedule.split(",")])
        tuned_on = "given on the command line"
    if sib is not None:
        from paper_2609_36267_amd import autotune
        sjob = [(torch.from_numpy(sib.psi).cuda(), torch.from_numpy(sib.coh).cuda(),
                 torch.from_numpy(sib.valid).cuda(), sib.looks)]
        t = time.perf_counter()
        choice, table = autotune.tune_schedule(sjob, reps=2)
        tuned_on = (f"fault recipe {sib.psi.shape[0]}x{sib.psi.shape[1]} seed 3 (not the timed "
                    f"scene), {len(table)} candidates, {time.perf_counter() - t:.1f} s")
        tune_top = [[list(autotune.pad(c)), round(1e3 * s, 3)]
                    for c, s in sorted(table.items(), key=lambda kv: kv[1])[:5]]
        del sjob, sib
        print(f"# schedule {choice} tuned on the sibling scene", file=sys.stderr, flush=True)
    sched_main = ww.get_mcf_params()
    totals = []
    for w in range(args.warmup):
        t = time.time()
        _, _, tot = ww.unwrap(psi, coh, valid, sc.looks, out=(K, phi))
        totals.append(tot)
        print(f"# warmup {w}: {time.time() - t:.3f} s cost {tot}", file=sys.stderr, flush=True)

    relax_ms = 0.0
    visits = 0
    stats = []
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    start.record()
    for k in range(args.steps):
        _, _, tot = ww.unwrap(psi, coh, valid, sc.looks, out=(K, phi))
        st = ww.last_mcf_stats()
        relax_ms += st["relax_ms"]
        visits += st["tile_visits"]
        stats.append(st)
        totals.append(tot)
    stop.record()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_wall) * 1e3
    ev_ms = start.elapsed_time(stop)
    ms_per_step = max(ev_ms, wall_ms) / args.steps
    value = m * n / 1e6 / (ms_per_step / 1e3)

    golden = None
    if args.workload == "c2" and os.path.exists(GOLDEN):
        golden = json.load(open(GOLDEN))["total_cost"]
    same_every_step = bool(len(set(totals)) == 1)
    equals_oracle = None if golden is None else bool(same_every_step and totals[0] == golden)

    # the method's work, counted in one more (untimed) solve of the same
    # scene with the same schedule: the counts do not depend on timing
    os.environ["WW_MCF_COUNT"] = "1"
    ww.unwrap(psi, coh, valid, sc.looks, out=(K, phi))
    cnt = ww.last_mcf_stats()
    del os.environ["WW_MCF_COUNT"]
    method_bytes = (BYTES_PER_ARC_SCAN * cnt["arcs_scanned"] + BYTES_PER_SETTLED * cnt["settled_nodes"])
    rps = relax_ms / args.steps  # relaxation device time per solve
    achieved = method_bytes / (rps / 1e3) / 1e9 if rps > 0 else 0.0
    staged = visits * BYTES_PER_TILE_VISIT / (relax_ms / 1e3) / 1e9 if relax_ms > 0 else 0.0
    sha = round_kernel_sha()
    traffic = (TRAFFIC_BYTES_PER_LAUNCH if (sha == TRAFFIC_SOURCE_SHA and args.workload == "c2" and
                                            sched_main.as_tuple() == TRAFFIC_SCHEDULE) else None)
    rounds = sum(st["rounds"] for st in stats)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": {"c2": "strike-slip fault scene 6912x10752 (74.3 Mpixel), L=15, 3% nodata",
                                "c1": "ramp+bump scene 2048x2048, 6 low-coherence disks, 5% nodata, L=9",
                                "c0": "ramp+bump scene 256x256, L=9"}[args.workload],
                   "pixels": m * n, "looks": sc.looks, "seed": {"c0": 0, "c1": 1, "c2": 2}[args.workload]},
        "total_cost": totals[-1],
        "same_cost_every_step": same_every_step,
        "equals_oracle": equals_oracle,
        "oracle_cost": golden,
        "roofline": {"bound": "hbm", "kernel": "k_sssp_round",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 counters, copy-calibrated)",
                     "algorithmic_bytes_per_launch": round(method_bytes * args.steps / max(1, rounds)),
                     "algorithmic_unit": f"{BYTES_PER_ARC_SCAN} B per arc scanned + {BYTES_PER_SETTLED} B "
                                         "per node settled, over the passes' searches",
                     "arcs_scanned_per_step": cnt["arcs_scanned"],
                     "nodes_settled_per_step": cnt["settled_nodes"],
                     "arcs_scanned_per_s": round(cnt["arcs_scanned"] / (rps / 1e3), 1) if rps > 0 else None,
                     "relax_ms_per_step": round(rps, 3),
                     "launches_per_step": rounds // args.steps,
                     "staged_gbs": round(staged, 2),
                     "staged_frac": round(staged / HBM_PEAK_GBS, 5),
                     "staged_bytes_per_launch": round(visits * BYTES_PER_TILE_VISIT / max(1, rounds)),
                     "tile_visits_per_step": visits // args.steps,
                     "bytes_per_tile_visit": BYTES_PER_TILE_VISIT},
        "mcf": stats[-1],
        "schedule": {**_sched_dict(sched_main.as_tuple()), "tuned_on": tuned_on,
                     **({"sibling_top5_ms": tune_top} if tune_top else {})},
        "paper_context": {"whirlwind_74mpix_s": 209, "derived_mpix_s": 0.356,
                          "note": "unstated CPU, real Sentinel-1 scene; context, not the target"},
    }
    if not args.no_legs:
        out["components"] = components_leg(ww, torch, psi, coh, valid, sc.looks, m, n)
        print(f"# components: {out['components']}", file=sys.stderr, flush=True)
        out["goldstein"] = goldstein_leg(ww, torch, psi, coh, valid, sc.looks, m, n)
        print(f"# goldstein: {out['goldstein']}", file=sys.stderr, flush=True)
        out["bridge"] = bridge_leg(ww, torch, synth, psi, coh, valid, sc.looks, m, n)
        print(f"# bridge: {out['bridge']}", file=sys.stderr, flush=True)
        out["streaming"] = streaming_leg(ww, torch, psi, coh, valid, sc.looks, m, n)
        print(f"# streaming: {out['streaming']}", file=sys.stderr, flush=True)
    if args.stack_jobs > 0:
        out["stack"] = stack_leg(args, ww, torch, *stack)
        print(f"# stack: {out['stack']}", file=sys.stderr, flush=True)
    if args.serve_seconds > 0:
        del psi, coh, valid, K, phi
        torch.cuda.empty_cache()
        pool = serve_pool(args, torch, synth)
        out["serve"] = serve_leg(args, ww, torch, *pool)
        print(f"# serve: {out['serve']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, min(args.cpu_rows, m))
        out["cpu_baseline"]["configs"] = cpu_baseline_configs(
            cpu_scenes, stack[0] if (args.cpu_baseline_stack and stack) else None)
        st_o = out["cpu_baseline"]["configs"].get("stack")
        if st_o and "stack" in out:
            st_o["equals_gpu_sum"] = st_o["total_cost_sum"] == out["stack"]["total_cost_sum"]
        if args.workload == "c2" and os.path.exists(GOLDEN):
            # the oracle's one run on the whole scene (context: measured once,
            # on the host that wrote the golden file, not timed here)
            gd = json.load(open(GOLDEN))
            if "oracle_mcf_seconds" in gd:
                out["cpu_baseline"]["whole_scene_once"] = {
                    "mcf_seconds": gd["oracle_mcf_seconds"], "total_cost": gd["total_cost"],
                    "what": "oracle min-cost flow alone on the whole timed scene, single-threaded, "
                            "measured once when tests/golden was written (not on this host)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
