"""Benchmark: decoded blocks/s and queries/s of basic ORBGRAND on one MI355X.

Default workload: narrow-sense BCH(127,113), t = 2, BPSK over AWGN at
Eb/N0 = 4.0, 4.5, ..., 7.0 dB, 10^6 blocks per point, query budget 10^5, plain
ORBGRAND.  One step decodes all 7 x 10^6 blocks (LLRs already resident in HBM)
with one decode call (light pass + heavy pass).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W]
                  [--workload bch127|bch127_1line|rlc32|mixed|learned|stream]

--workload mixed: random linear codes (64,52), (128,116), (256,240) mixed 1:2:1
in one persistent launch per Eb/N0 point (3..6 dB, 4x10^6 blocks, budget
10^6), against the same blocks decoded by one launch per code without the
heavy pass.
--workload learned: the learned batch-order proposal on RLC(128,105), trained
on the GPU, against plain ORBGRAND on the same held-out blocks.
--workload bch127_1line: the default workload decoded by 1-line ORBGRAND (the
one-segment fit of Sec. III-E), with basic ORBGRAND on the same blocks per point.
--workload stream: Poisson request arrivals (single blocks of four codes) served
by a host loop of mixed-code launches; p50/p99 latency and blocks/s at 1e5 and
1e6 requests/s.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "decoded blocks/sec and queries/sec at fixed Eb/N0 and equal BLER, 1 MI355X"

# Peak figures (MI355X): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz one 32-bit integer
# VALU op per lane per clock; HBM3E 8 TB/s.
PEAK_INT32_OPS = 256 * 4 * 16 * 2.4e9
PEAK_HBM = 8.0e12

WORKLOADS = {
    "bch127": dict(code="bch127_113", n=127, k=113, ebn0=[4.0, 4.5, 5.0, 5.5, 6.0, 6.5, 7.0],
                   blocks=10 ** 6, budget=10 ** 5,
                   desc="BCH(127,113) t=2, BPSK/AWGN Eb/N0 4..7 dB step 0.5, 1e6 blocks per point, "
                        "budget 1e5, plain ORBGRAND"),
    "bch127_1line": dict(code="bch127_113", n=127, k=113, ebn0=[4.0, 4.5, 5.0, 5.5, 6.0, 6.5, 7.0],
                         blocks=10 ** 6, budget=10 ** 5, oneline=True,
                         desc="BCH(127,113) t=2, BPSK/AWGN Eb/N0 4..7 dB step 0.5, 1e6 blocks per point, "
                              "budget 1e5, 1-line ORBGRAND (one-segment fit, Sec. III-E) against basic ORBGRAND "
                              "on the same blocks"),
    "bch127_mline": dict(code="bch127_113", n=127, k=113, ebn0=[4.0, 4.5, 5.0, 5.5, 6.0, 6.5, 7.0],
                         blocks=10 ** 6, budget=10 ** 5, mline=True, segments=2,
                         desc="BCH(127,113) t=2, BPSK/AWGN Eb/N0 4..7 dB step 0.5, 1e6 blocks per point, "
                              "budget 1e5, full ORBGRAND with a 2-line fit (Sec. III-D, III-E) against its J/beta variant, "
                              "1-line and basic ORBGRAND on the same blocks"),
    "rlc256_mline": dict(code="rlc256_234", n=256, k=234, ebn0=[5.0, 5.5, 6.0, 6.5],
                         blocks=10 ** 5, budget=65536, mline=True, segments=3,
                         desc="RLC(256,234) H=[P|I22] (the length and redundancy of CA-Polar[256,234]), BPSK/AWGN "
                              "Eb/N0 5..6.5 dB step 0.5, 1e5 blocks per point, budget 2^16, full ORBGRAND with a "
                              "3-line fit (Sec. III-D, III-E) against its J/beta variant and basic ORBGRAND on the same blocks"),
    "rlc32": dict(code="rlc32_26", n=32, k=26, ebn0=[4.0], blocks=10 ** 4, budget=10 ** 4,
                  desc="RLC(32,26) H=[P|I6], BPSK/AWGN Eb/N0 4 dB, 1e4 blocks, budget 1e4, plain ORBGRAND"),
    "learned": dict(code="rlc128_105", n=128, k=105, train_pairs=10 ** 7, train_ebn0=(3.0, 5.0),
                    ebn0=[3.0, 3.5, 4.0, 4.5, 5.0], blocks=10 ** 6, budget=10 ** 6, epochs=2, batch=8192, lr=2e-3,
                    desc="RLC(128,105) H=[P|I23]: BF16 MLP 128-256-256-64 trained on 1e7 decoder-generated pairs "
                         "at Eb/N0 ~ U[3,5] dB (blocks whose first hit lies in batches 1..63), gated decode: batch 0 "
                         "for every block, the network orders batches 1..63 only for blocks batch 0 does not decide, "
                         "ORBGRAND fallback after 64 batches; plain vs learned vs the fixed prior order on 1e6 "
                         "held-out blocks per point at 3..5 dB, budget 1e6"),
    "stream": dict(codes=["rlc64_52", "bch127_113", "rlc128_116", "rlc256_240"], ratio=[1, 1, 1, 1],
                   ebn0_range=(3.0, 6.0), rates=[1e5, 1e6], seconds=1.0, budget=10 ** 5,
                   capacity=1 << 16, max_batch=1 << 13, streams=8,
                   launch=dict(workgroups_per_cu=32, chunk=1, split_steps=16, heavy_waves=16,
                               heavy_workgroups_per_cu=2),
                   desc="request stream: Poisson arrivals of single blocks, codes RLC(64,52), BCH(127,113), "
                        "RLC(128,116), RLC(256,240) uniformly mixed, Eb/N0 ~ U[3,6] dB per request, budget "
                        "1e5, 1 s of arrivals at 1e5 and 1e6 requests/s; LLRs and outputs resident in HBM; "
                        "a host loop launches every arrived request (at most 8192 per launch, at most 65536 "
                        "in flight) as one mixed-code decode, launches dealt round-robin to 8 streams, blocks "
                        "past 16 steps shared by 16 waves"),
    "mixed": dict(codes=["rlc64_52", "rlc128_116", "rlc256_240"], ratio=[1, 2, 1],
                  ebn0=[3.0, 3.5, 4.0, 4.5, 5.0, 5.5, 6.0], blocks=4 * 10 ** 6, budget=10 ** 6, tune_point=4.5,
                  desc="RLC (64,52):(128,116):(256,240) = 1:2:1 in one launch, BPSK/AWGN Eb/N0 3..6 dB "
                       "step 0.5, 4e6 blocks per point, budget 1e6, plain ORBGRAND"),
}


def wilson(k: int, n: int, z: float = 1.96):
    if n == 0:
        return (0.0, 0.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return (max(0.0, c - h), min(1.0, c + h))


_PAIR = []


def warm_events(stream):
    """One reusable pair of timing events, each recorded once already: torch makes
    an event's HIP object at its first record, and a fresh pair around a single
    launch has been measured to add a few hundred microseconds to the interval."""
    import torch
    if not _PAIR:
        pair = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        for e in pair:
            e.record(stream)
        torch.cuda.synchronize()
        _PAIR.extend(pair)
    return _PAIR[0], _PAIR[1]


def time_calls(fn, stream, reps: int = 1) -> float:
    """Milliseconds per call of fn(): `reps` back-to-back calls between the warm
    events (with reps > 1 the host's launch time of all calls but the first hides
    behind the GPU's work)."""
    import torch
    a, b = warm_events(stream)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def algorithmic_ops(q_sum: int, n_sorted: int, n: int) -> float:
    """Integer work the method needs: 4 int32 ops per counted query (one 64-bit
    syndrome XOR and one 64-bit zero test) plus, for each block that needs the
    reliability order (q > 1), n*ceil(log2 n) 64-bit key compares (2 ops each)."""
    return 4.0 * q_sum + 2.0 * n * math.ceil(math.log2(n)) * n_sorted


def query_breakdown(q, ab, err, budget, sweep=(10 ** 2, 10 ** 3, 10 ** 4, 10 ** 5, 10 ** 6)):
    """Counts and mean queries of the blocks decoded correctly, decoded to another
    codeword, and abandoned; and the abandonment sweep: a decode with budget b below
    the run's returns the same result for blocks with q <= b and abandons the others,
    so BLER and mean queries at every smaller budget follow from one decode."""
    q = np.asarray(q, dtype=np.int64)
    ab = np.asarray(ab) != 0
    err = np.asarray(err, dtype=bool)

    def stats(m):
        return {"blocks": int(m.sum()), "mean_queries": float(q[m].mean()) if m.any() else None}
    out = {"correct": stats(~err & ~ab), "incorrect": stats(err & ~ab), "abandoned": stats(ab)}
    sw = {}
    for b in sweep:
        if b > budget:
            continue
        kept = q <= b
        sw[f"{b:.0e}"] = {"bler": float(((err & kept) | ~kept).mean()), "abandoned": float((~kept).mean()),
                          "mean_queries": float(np.minimum(q, b).mean())}
    out["budget_sweep"] = sw
    return out


# Sources the basic and 1-line decode kernels (light and heavy pass, schedules,
# launch) are compiled from, and those of the m-line kernel: committed HBM
# counters stay valid while these are unchanged.
DECODE_SOURCES = ("decode.hip", "decode_impl.h", "decode_nk1.hip", "decode_nk2.hip", "decode_nk4.hip", "decode_nk8.hip",
                  "decode_nk16.hip", "orbg_device.h", "orbg_internal.h", "orbg_kernels.h", "schedule.hip")
MLINE_SOURCES = ("mline.hip", "mline_impl.h", "mline_m1.hip", "mline_m2.hip", "mline_m3.hip", "mline_m4.hip", "orbg_mline.h",
                 "orbg_device.h", "orbg_internal.h")


def kernel_fingerprint(sources=DECODE_SOURCES) -> str:
    """sha256 (first 16 hex digits) over the names and contents of the given kernel sources."""
    import hashlib
    h = hashlib.sha256()
    for name in sources:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2202_13951_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(workload: str, prefix: str = "decode_kernel", sources=DECODE_SOURCES):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary of
    this workload, or None if there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"{prefix}_{WORKLOADS[workload].get('code', workload)}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "source_fingerprint"):
                k, v = line.split(":", 1)
                vals[k] = v.strip()
    if vals.get("source_fingerprint") != kernel_fingerprint(sources) or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(H, rows, npoints: int, per_max: int, budget, target_s=20.0, oneline=False, dec=None):
    """Times the oracle (as it stands) on the first blocks of every Eb/N0 point.
    rows(p, count) -> host float32 [count, n], the first `count` rows of point p.
    A first pass on 2000 blocks per point sizes the sample (that pass overstates the
    per-block cost, so the timed sample lasts about half of target_s).  oneline: the
    oracle's 1-line decoder; dec(H, x, budget, threads) replaces the decoder."""
    from oracle import oracle as O
    if dec is None:
        dec = O.decode_1line if oneline else O.decode
    threads = len(os.sched_getaffinity(0))
    per = min(2000, per_max)
    xs = [rows(p, per) for p in range(npoints)]
    t0 = time.perf_counter()
    for x in xs:
        dec(H, x, budget, threads)
    dt = time.perf_counter() - t0
    per = int(min(per_max, max(per, per * target_s / max(dt, 1e-3))))
    xs = [rows(p, per) for p in range(npoints)]
    t0 = time.perf_counter()
    for x in xs:
        dec(H, x, budget, threads)
    dt = time.perf_counter() - t0
    nb = per * npoints
    # the same oracle on one core, on a sample sized to about a quarter of target_s
    per1 = max(1, int(per * (target_s / 4) / max(dt * threads, 1e-3)))
    t0 = time.perf_counter()
    for p in range(npoints):
        dec(H, xs[p][:per1], budget, 1)
    dt1 = time.perf_counter() - t0
    return {"value": nb / dt, "unit": "blocks/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "one_core_value": per1 * npoints / dt1,
            "sample": f"first {per} blocks of each of the {npoints} Eb/N0 points "
                      f"({nb} blocks, {dt:.1f} s wall); one core: first {per1} of each ({dt1:.1f} s)"}


def single_inputs(wl, dev, points=None):
    """Resident [P * B, n] FP32 LLRs (and sent codewords) of a one-code workload."""
    import torch
    from synth import channel, codes
    H, G = codes.code(wl["code"])
    pts = wl["ebn0"] if points is None else points
    B, n = wl["blocks"], wl["n"]
    llr = torch.empty((len(pts) * B, n), dtype=torch.float32, device=dev)
    sent = torch.empty((len(pts) * B, n), dtype=torch.uint8, device=dev)
    for p, e in enumerate(pts):
        seed = 1000 + point_seed_index(wl, e)
        x, c = channel.awgn_llr_torch(G, B, e, seed=seed, device=dev)
        llr[p * B:(p + 1) * B] = x
        sent[p * B:(p + 1) * B] = c
        del x, c
    return H, llr, sent


def point_seed_index(wl, e):
    """Seed index of an Eb/N0 point: its position in the full grid (0.5 dB steps from 3 dB)."""
    return int(round((e - 3.0) * 2))


def mixed_inputs(wl, e, dev):
    from synth import codes, mixed
    HG = [codes.code(nm) for nm in wl["codes"]]
    llr, sent, bc, ro = mixed.mixed_llr_torch([G for _, G in HG], wl["ratio"], wl["blocks"], e,
                                              seed=2000 + int(round(e * 10)), device=dev)
    return HG, llr, sent, bc, ro


def make_runner(name: str):
    """(run(params), blocks): one decode of the workload's tuning input per call."""
    import torch
    from paper_2202_13951_amd import binding
    dev = torch.device("cuda:0")
    wl = WORKLOADS[name]
    if "codes" in wl:
        HG, llr, sent, bc, ro = mixed_inputs(wl, wl["tune_point"], dev)
        ids = [binding.orbg_code_register(H) for H, _ in HG]
        N = bc.shape[0]
        cw = torch.empty_like(sent)
        q = torch.empty(N, dtype=torch.int64, device=dev)
        ab = torch.empty(N, dtype=torch.uint8, device=dev)
        return (lambda p: binding.orbg_decode_mixed(ids, bc, ro, llr, wl["budget"], cw, q, ab, params=p)), N
    H, llr, sent = single_inputs(wl, dev)
    out = (torch.empty_like(sent), torch.empty(llr.shape[0], dtype=torch.int64, device=dev),
           torch.empty(llr.shape[0], dtype=torch.uint8, device=dev))
    if wl.get("oneline"):
        return (lambda p: binding.orbg_decode_1line(H, llr, wl["budget"], j0=False, params=p, out=out)), \
            llr.shape[0]
    return (lambda p: binding.orbg_decode_ex(H, llr, wl["budget"], params=p, out=out)), llr.shape[0]


def tuned_params(name: str, use_tuned: bool):
    from paper_2202_13951_amd import autotune, binding
    knobs = autotune.load_tuned(name) if use_tuned else None
    return (binding.LaunchParams(**knobs) if knobs else None), knobs


def run_single(args, wl, dev):
    import torch
    from paper_2202_13951_amd import binding
    H, llr, sent = single_inputs(wl, dev)
    n, budget = wl["n"], wl["budget"]
    P, B = len(wl["ebn0"]), wl["blocks"]
    params, knobs = tuned_params(args.workload, not args.no_tuned)
    cw = torch.empty_like(sent)
    q = torch.empty((P * B,), dtype=torch.int64, device=dev)
    ab = torch.empty((P * B,), dtype=torch.uint8, device=dev)
    out = (cw, q, ab)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        binding.orbg_decode_ex(H, llr, budget, params=params, out=out)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a_, b_ in ev:                                 # each event recorded once before the clock
        a_.record(stream)
        b_.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        binding.orbg_decode_ex(H, llr, budget, params=params, out=out)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    blocks = P * B

    q_np = q.cpu().numpy()
    ab_np = ab.cpu().numpy()
    err = (cw != sent).any(dim=1).cpu().numpy()
    q_sum = int(q_np.sum())
    n_sorted = int((q_np > 1).sum())
    per_point = {}
    for p, e in enumerate(wl["ebn0"]):
        sl = slice(p * B, (p + 1) * B)
        ne = int(err[sl].sum())
        lo, hi = wilson(ne, B)
        per_point[f"{e:.1f}"] = {"bler": ne / B, "errors": ne, "bler_ci95": [lo, hi],
                                 "breakdown": query_breakdown(q_np[sl], ab_np[sl], err[sl], budget),
                                 "mean_queries": float(q_np[sl].mean()),
                                 "p99_queries": float(np.percentile(q_np[sl], 99)),
                                 "abandoned": int(ab_np[sl].sum())}
    for p, e in enumerate([] if args.no_per_point else wl["ebn0"]):
        sl = slice(p * B, (p + 1) * B)
        sub_out = (cw[sl], q[sl], ab[sl])
        t = time_calls(lambda: binding.orbg_decode_ex(H, llr[sl], budget, params=params, out=sub_out), stream,
                       reps=3) / 1e3
        per_point[f"{e:.1f}"]["blocks_per_s"] = B / t
        per_point[f"{e:.1f}"]["queries_per_s"] = float(q_np[sl].sum()) / t

    kavg = float(np.mean(kern_ms)) / 1e3
    ops = algorithmic_ops(q_sum, n_sorted, n)
    hbm_bytes = blocks * (4 * n + n + 8 + 1)
    result = {
        "metric": METRIC,
        "value": blocks / (wall / args.steps),
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("u32" if n - wl["k"] <= 32 else "u64") + " syndromes, FP32 LLR",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "code": wl["code"], "n": n, "k": wl["k"], "ebn0_db": wl["ebn0"],
                   "blocks_per_step": blocks, "budget": budget},
        "queries_per_s": q_sum / (wall / args.steps),
        "mean_queries": q_sum / blocks,
        "kernel_ms": float(np.mean(kern_ms)),
        "launch_params": knobs if knobs else "library defaults",
        "per_point": per_point,
        "roofline": {"bound": "alu", "achieved": ops / kavg / 1e12, "peak": PEAK_INT32_OPS / 1e12,
                     "unit": "Tops/s (int32)", "frac": ops / kavg / PEAK_INT32_OPS,
                     "traffic": profiled_traffic(args.workload),
                     "kernel": "light_kernel + heavy_kernel (one decode call)", "ops_per_launch": ops,
                     "hbm": {"achieved_GBps": hbm_bytes / kavg / 1e9, "peak_GBps": PEAK_HBM / 1e9,
                             "frac": hbm_bytes / kavg / PEAK_HBM, "bytes_per_launch": hbm_bytes}},
    }
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)     # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(H, lambda p, c: llr[p * B:p * B + c].cpu().numpy(), P, B, budget)
    return result


def run_oneline(args, wl, dev):
    """1-line ORBGRAND over all points in one call per step (timed), then per point:
    BLER, queries and the fitted offsets of the 1-line decoder, and the basic decoder
    on the same blocks, each timed on its own."""
    import torch
    from paper_2202_13951_amd import binding
    H, llr, sent = single_inputs(wl, dev)
    n, budget = wl["n"], wl["budget"]
    P, B = len(wl["ebn0"]), wl["blocks"]
    params, knobs = tuned_params(args.workload, not args.no_tuned)
    cw = torch.empty_like(sent)
    q = torch.empty((P * B,), dtype=torch.int64, device=dev)
    ab = torch.empty((P * B,), dtype=torch.uint8, device=dev)
    out = (cw, q, ab)
    stream = torch.cuda.current_stream()

    def one():
        binding.orbg_decode_1line(H, llr, budget, j0=False, params=params, out=out)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        one()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a_, b_ in ev:                                 # each event recorded once before the clock
        a_.record(stream)
        b_.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        one()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    blocks = P * B
    # the fitted offsets of every block (an untimed call that also ranks the blocks
    # whose hard decision is a codeword), and the same results
    j0 = torch.empty((P * B,), dtype=torch.int32, device=dev)
    cw2, q2, ab2, _ = binding.orbg_decode_1line(H, llr, budget, j0=j0, params=params)
    torch.cuda.synchronize()
    same = bool((cw2 == cw).all().item() and (q2 == q).all().item() and (ab2 == ab).all().item())
    del cw2, q2, ab2
    q_np = q.cpu().numpy()
    ab_np = ab.cpu().numpy()
    j0_np = j0.cpu().numpy()
    err = (cw != sent).any(dim=1).cpu().numpy()
    _, j0max = binding.orbg_schedule_export_1line(n, budget, 0, 0)

    bcw = torch.empty((B, n), dtype=torch.uint8, device=dev)
    bq = torch.empty((B,), dtype=torch.int64, device=dev)
    bab = torch.empty((B,), dtype=torch.uint8, device=dev)
    binding.orbg_decode_ex(H, llr[:B], budget, params=params, out=(bcw, bq, bab))   # builds its schedule
    torch.cuda.synchronize()
    per_point = {}
    for p, e in enumerate(wl["ebn0"]):
        sl = slice(p * B, (p + 1) * B)
        ne = int(err[sl].sum())
        jp = j0_np[sl]
        vals, cnts = np.unique(np.clip(jp, -1, 9), return_counts=True)
        pt = {"bler": ne / B, "errors": ne, "bler_ci95": list(wilson(ne, B)),
              "mean_queries": float(q_np[sl].mean()), "abandoned": int(ab_np[sl].sum()),
              "breakdown": query_breakdown(q_np[sl], ab_np[sl], err[sl], budget),
              "j0": {"mean": float(jp.mean()), "min": int(jp.min()), "max": int(jp.max()),
                     "share": {("9+" if v == 9 else str(int(v))): float(c / B) for v, c in zip(vals, cnts)},
                     "above_j0max": float((jp > j0max).mean())}}
        t = time_calls(lambda: binding.orbg_decode_1line(H, llr[sl], budget, j0=False, params=params,
                                                          out=(cw[sl], q[sl], ab[sl])), stream, reps=3) / 1e3
        pt["blocks_per_s"] = B / t
        pt["queries_per_s"] = float(q_np[sl].sum()) / t
        tb = time_calls(lambda: binding.orbg_decode_ex(H, llr[sl], budget, params=params, out=(bcw, bq, bab)),
                        stream, reps=3) / 1e3
        berr = (bcw != sent[sl]).any(dim=1).cpu().numpy()
        bq_np = bq.cpu().numpy()
        nb = int(berr.sum())
        pt["basic"] = {"bler": nb / B, "errors": nb, "bler_ci95": list(wilson(nb, B)),
                       "mean_queries": float(bq_np.mean()), "abandoned": int(bab.sum().item()),
                       "blocks_per_s": B / tb}
        # blocks one decoder gets right and the other wrong
        pt["only_1line_correct"] = int((~err[sl] & berr).sum())
        pt["only_basic_correct"] = int((err[sl] & ~berr).sum())
        per_point[f"{e:.1f}"] = pt

    kavg = float(np.mean(kern_ms)) / 1e3
    q_sum = int(q_np.sum())
    n_sorted = int((q_np > 1).sum())
    ops = algorithmic_ops(q_sum, n_sorted, n)
    hbm_bytes = blocks * (4 * n + n + 8 + 1)
    result = {
        "metric": METRIC,
        "value": blocks / (wall / args.steps),
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("u32" if n - wl["k"] <= 32 else "u64") + " syndromes, FP32 LLR",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "code": wl["code"], "n": n, "k": wl["k"], "ebn0_db": wl["ebn0"],
                   "blocks_per_step": blocks, "budget": budget, "j0max": j0max},
        "queries_per_s": q_sum / (wall / args.steps),
        "mean_queries": q_sum / blocks,
        "kernel_ms": float(np.mean(kern_ms)),
        "launch_params": knobs if knobs else "library defaults",
        "offsets_call_identical": same,
        "per_point": per_point,
        "roofline": {"bound": "alu", "achieved": ops / kavg / 1e12, "peak": PEAK_INT32_OPS / 1e12,
                     "unit": "Tops/s (int32)", "frac": ops / kavg / PEAK_INT32_OPS, "traffic": None,
                     "kernel": "light_kernel + heavy_kernel, 1-line (one decode call)", "ops_per_launch": ops,
                     "hbm": {"achieved_GBps": hbm_bytes / kavg / 1e9, "peak_GBps": PEAK_HBM / 1e9,
                             "frac": hbm_bytes / kavg / PEAK_HBM, "bytes_per_launch": hbm_bytes}},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(H, lambda p, c: llr[p * B:p * B + c].cpu().numpy(), P, B, budget,
                                              oneline=True)
    return result


def run_mixed(args, wl, dev):
    """Per Eb/N0 point: the tuned persistent mixed launch against two baselines on
    the same resident buffer, one launch per code over that code's blocks (a
    one-code mixed call with the code's block list, reading the rows in place):
    (a) the naive launch -- one one-wave workgroup per block, no work counter, no
    heavy pass; (b) the persistent light pass without the heavy pass.  Results
    are compared bit for bit."""
    import torch
    from paper_2202_13951_amd import binding
    params, knobs = tuned_params(args.workload, not args.no_tuned)
    shapes = {"one_block_per_workgroup": binding.LaunchParams(one_block_per_workgroup=1),
              "persistent_per_code": binding.LaunchParams(split_steps=0)}
    stream = torch.cuda.current_stream()
    points, tot_blocks, tot_ms, tot_q = {}, 0, 0.0, 0
    tot_base = {k: 0.0 for k in shapes}
    ops_tot, bytes_tot = 0.0, 0.0
    cpu_rows = []                                     # (H, rows) of a bounded sample per point, for the oracle

    def timed(fn):
        return time_calls(fn, stream)

    for e in wl["ebn0"]:
        HG, llr, sent, bc, ro = mixed_inputs(wl, e, dev)
        ids = [binding.orbg_code_register(H) for H, _ in HG]
        N = bc.shape[0]
        cw = torch.empty_like(sent)
        q = torch.empty(N, dtype=torch.int64, device=dev)
        ab = torch.empty(N, dtype=torch.uint8, device=dev)

        def mixed_fn():
            binding.orbg_decode_mixed(ids, bc, ro, llr, wl["budget"], cw, q, ab, params=params)
        for _ in range(args.warmup):
            mixed_fn()
        ms = [timed(mixed_fn) for _ in range(args.steps)]
        print(f"mixed {e} dB: {np.median(ms):.2f} ms", file=sys.stderr, flush=True)
        per_code = []
        for ci, (H, G) in enumerate(HG):
            n = H.shape[1]
            idx = torch.nonzero(bc == ci).flatten()
            per_code.append((H, ids[ci], idx, torch.zeros(idx.numel(), dtype=torch.uint8, device=dev),
                             ro[idx].contiguous(), n))
        base_ms, same = {}, True
        for name, P in shapes.items():
            cwb = torch.empty_like(cw)
            outs = [(torch.empty(idx.numel(), dtype=torch.int64, device=dev),
                     torch.empty(idx.numel(), dtype=torch.uint8, device=dev)) for _, _, idx, _, _, _ in per_code]

            def base_fn():
                for (H, cid, idx, zc, rc, n), o in zip(per_code, outs):
                    binding.orbg_decode_mixed([cid], zc, rc, llr, wl["budget"], cwb, o[0], o[1], params=P)
            base_fn()
            base_ms[name] = float(np.median([timed(base_fn) for _ in range(args.steps)]))
            print(f"{name} {e} dB: {base_ms[name]:.2f} ms", file=sys.stderr, flush=True)
            for (H, cid, idx, zc, rc, n), o in zip(per_code, outs):
                same &= bool((q[idx] == o[0]).all()) and bool((ab[idx] == o[1]).all())
            same &= bool((cwb == cw).all())
            del outs, cwb
        errs = torch.zeros(N, dtype=torch.bool, device=dev)
        ops = 0.0
        for H, cid, idx, zc, rc, n in per_code:
            pos = rc[:, None] + torch.arange(n, device=dev)[None, :]
            errs[idx] = (cw[pos] != sent[pos]).any(dim=1)
            qc = q[idx]
            ops += algorithmic_ops(int(qc.sum()), int((qc > 1).sum()), n)
            bytes_tot += idx.numel() * (5 * n + 9)
            cpu_rows.append((H, llr[pos[:20000]].cpu().numpy()))
        ops_tot += ops
        ne = int(errs.sum())
        qs = int(q.sum())
        m = float(np.median(ms))
        points[f"{e:.1f}"] = {"blocks_per_s": N / (m / 1e3), "ms": m, "mean_queries": qs / N,
                              "baselines_ms": base_ms,
                              "baselines_blocks_per_s": {k: N / (v / 1e3) for k, v in base_ms.items()},
                              "speedup": {k: v / m for k, v in base_ms.items()},
                              "bler": ne / N, "bler_ci95": list(wilson(ne, N)), "abandoned": int(ab.sum()),
                              "identical_to_baselines": same}
        tot_blocks += N
        tot_ms += m
        for k in shapes:
            tot_base[k] += base_ms[k]
        tot_q += qs
        del HG, llr, sent, bc, ro, cw, q, ab, per_code
        torch.cuda.empty_cache()
    ksec = tot_ms / 1e3
    result = {
        "metric": METRIC, "value": tot_blocks / ksec, "unit": "blocks/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": tot_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32 syndromes, FP32 LLR", "data": "synthetic",
        "config": {"workload": wl["desc"], "codes": wl["codes"], "ratio": wl["ratio"], "ebn0_db": wl["ebn0"],
                   "blocks_per_point": wl["blocks"], "budget": wl["budget"]},
        "queries_per_s": tot_q / ksec,
        "baselines_value": {k: tot_blocks / (v / 1e3) for k, v in tot_base.items()},
        "speedup": {k: v / tot_ms for k, v in tot_base.items()},
        "launch_params": knobs if knobs else "library defaults",
        "roofline": {"bound": "alu", "achieved": ops_tot / ksec / 1e12, "peak": PEAK_INT32_OPS / 1e12,
                     "unit": "Tops/s (int32)", "frac": ops_tot / ksec / PEAK_INT32_OPS,
                     "traffic": profiled_traffic(args.workload) if not args.ebn0 else None,
                     "kernel": "light_kernel<4> + heavy_kernel (one mixed decode call per point)",
                     "ops_per_launch": ops_tot / len(wl["ebn0"]),
                     "hbm": {"achieved_GBps": bytes_tot / ksec / 1e9, "peak_GBps": PEAK_HBM / 1e9,
                             "frac": bytes_tot / ksec / PEAK_HBM, "bytes_per_launch": bytes_tot / len(wl["ebn0"])}},
        "per_point": points,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline_mixed(cpu_rows, wl["budget"], len(wl["ebn0"]))
    return result


def cpu_baseline_mixed(samples, budget, npoints, target_s=15.0):
    """The oracle on the first blocks of every code at every point (each code's
    blocks in launch order), sized to about target_s of work."""
    from oracle import oracle as O
    threads = len(os.sched_getaffinity(0))
    per = 20
    t0 = time.perf_counter()
    for H, x in samples:
        O.decode(H, x[:per], budget, threads)
    dt = time.perf_counter() - t0
    per = int(min(min(len(x) for _, x in samples), max(per, per * target_s / max(dt, 1e-3))))
    t0 = time.perf_counter()
    for H, x in samples:
        O.decode(H, x[:per], budget, threads)
    dt = time.perf_counter() - t0
    nb = per * len(samples)
    return {"value": nb / dt, "unit": "blocks/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"first {per} blocks of each code at each of the {npoints} Eb/N0 points "
                      f"({nb} blocks, {dt:.1f} s wall)"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_stream(args, wl, dev):
    """Serving loop over a Poisson request stream.  Arrivals are on the host clock
    (perf_counter from t0); completions on the GPU clock, as the elapsed time from a
    reference event e0 to the event recorded after each launch, moved to the host
    clock by an offset bracketed with record-and-wait round trips before t0.
    Latency = completion - arrival.  Every result is compared with one decode of
    all requests."""
    import collections
    import torch
    from paper_2202_13951_amd import binding
    from synth import codes, mixed
    from synth import stream as arrivals
    HG = [codes.code(nm) for nm in wl["codes"]]
    ids = [binding.orbg_code_register(H) for H, _ in HG]
    params, knobs = binding.LaunchParams(**wl["launch"]), wl["launch"]
    s = torch.cuda.current_stream()
    # launches go round-robin to several streams of default priority, so one long
    # block does not hold up the launches behind it
    streams = [torch.cuda.Stream() for _ in range(wl["streams"])]
    per_rate = {}
    for ri, rate in enumerate(wl["rates"]):
        N = int(round(rate * wl["seconds"]))
        llr, sent, bc, ro, snr = mixed.mixed_llr_torch_snr_range([G for _, G in HG], wl["ratio"], N,
                                                                 *wl["ebn0_range"], seed=3000 + ri, device=dev)
        t_arr = arrivals.poisson_arrivals(N, rate, seed=4000 + ri)
        cw = torch.zeros_like(sent)
        q = torch.zeros(N, dtype=torch.int64, device=dev)
        ab = torch.zeros(N, dtype=torch.uint8, device=dev)
        # schedules of every code and the work spaces of every stream exist before the clock starts
        # (work spaces sized for the largest launch, so none grows on the clock)
        w = min(N, wl["max_batch"])
        for st in streams:
            binding.orbg_decode_mixed(ids, bc[:w], ro[:w], llr, wl["budget"], cw, q[:w], ab[:w],
                                      params=params, stream=st)
        torch.cuda.synchronize()
        inflight, batches = [collections.deque() for _ in streams], []
        n_in, nxt, k = 0, 0, 0
        # completion events come from a pool recorded once before the clock (a
        # fresh event would be made on the clock); an event goes back to the pool
        # once its completion time has been read
        pool = [torch.cuda.Event(enable_timing=True) for _ in range(4096)]
        for ev in pool:
            ev.record(s)
        torch.cuda.synchronize()
        fresh = 0
        gc.collect()
        gc.disable()                                  # no collector pauses on the clock
        # GPU clock (event times since e0) against the host clock: each round trip
        # "host time, record, wait, host time" brackets one GPU stamp, so the
        # offset host(e0) - t0 lies in [off_lo, off_hi], the narrowest bracket
        # setting the width
        e0, ec = pool.pop(), pool.pop()               # both recorded once already
        e0.record(s)
        torch.cuda.synchronize()
        cal = []
        for _ in range(32):
            ta = time.perf_counter()
            ec.record(s)
            ec.synchronize()
            cal.append((ta, time.perf_counter(), e0.elapsed_time(ec) / 1e3))
        t0 = time.perf_counter()
        off_lo = max(ta - t0 - tg for ta, _, tg in cal)
        off_hi = min(tb - t0 - tg for _, tb, tg in cal)
        while nxt < N or any(inflight):
            for fl in inflight:
                while fl and fl[0][0].query():
                    ev, lo, hi = fl.popleft()
                    n_in -= hi - lo
                    batches.append((e0.elapsed_time(ev) / 1e3, lo, hi, time.perf_counter() - t0))
                    pool.append(ev)
            if nxt < N:
                j = int(np.searchsorted(t_arr, time.perf_counter() - t0, side="right"))
                j = min(j, nxt + wl["max_batch"], nxt + wl["capacity"] - n_in)
                if j > nxt:
                    st = streams[k]
                    binding.orbg_decode_mixed(ids, bc[nxt:j], ro[nxt:j], llr, wl["budget"], cw, q[nxt:j],
                                              ab[nxt:j], params=params, stream=st)
                    if pool:
                        ev = pool.pop()
                    else:
                        ev = torch.cuda.Event(enable_timing=True)
                        fresh += 1
                    ev.record(st)
                    inflight[k].append((ev, nxt, j))
                    k = (k + 1) % len(streams)
                    n_in += j - nxt
                    nxt = j
        torch.cuda.synchronize()
        gc.enable()
        # completion on the GPU clock moved to the host clock (between the two ends
        # of the offset bracket; the lower end is reported, the upper end differs
        # by the bracket's width) and as first seen by the host loop (an upper
        # bound: the loop polls)
        done, seen = np.empty(N), np.empty(N)
        for tg, lo, hi, th in batches:
            done[lo:hi] = tg + off_lo
            seen[lo:hi] = th
        lat = (done - t_arr) * 1e6
        lat_host = (seen - t_arr) * 1e6
        sizes = np.array([hi - lo for _, lo, hi, _ in batches])
        # the same requests as one decode
        cw1, q1, ab1 = torch.zeros_like(sent), torch.zeros_like(q), torch.zeros_like(ab)
        binding.orbg_decode_mixed(ids, bc, ro, llr, wl["budget"], cw1, q1, ab1, params=params)
        torch.cuda.synchronize()
        same = bool((q == q1).all()) and bool((ab == ab1).all()) and bool((cw == cw1).all())
        per_code = {}
        bc_np = bc.cpu().numpy()
        for ci, (H, _) in enumerate(HG):
            n = H.shape[1]
            idx = torch.nonzero(bc == ci).flatten()
            pos = ro[idx][:, None] + torch.arange(n, device=dev)[None, :]
            ne = int((cw[pos] != sent[pos]).any(dim=1).sum())
            nb = int(idx.numel())
            per_code[wl["codes"][ci]] = {"requests": nb, "bler": ne / max(nb, 1),
                                         "mean_queries": float(q[idx].double().mean()),
                                         "p99_latency_us": float(np.percentile(lat[bc_np == ci], 99))}
        span = float(done.max() - t_arr[0])
        per_rate[f"{rate:.0e}"] = {
            "requests": N, "blocks_per_s": N / span, "offered_per_s": rate,
            "latency_us": {"p50": float(np.percentile(lat, 50)), "p90": float(np.percentile(lat, 90)),
                           "p99": float(np.percentile(lat, 99)), "max": float(lat.max()),
                           "mean": float(lat.mean())},
            "latency_host_us": {"p50": float(np.percentile(lat_host, 50)),
                                "p99": float(np.percentile(lat_host, 99)), "max": float(lat_host.max())},
            "launches": len(batches), "events_made_on_clock": fresh, "mean_launch_blocks": float(sizes.mean()),
            "max_launch_blocks": int(sizes.max()), "clock_offset_bracket_us": (off_hi - off_lo) * 1e6,
            "queries_per_s": float(q.sum()) / span, "identical_to_one_decode": same, "per_code": per_code}
        print(f"stream {rate:.0e}/s: p50 {np.percentile(lat, 50):.0f} us p99 {np.percentile(lat, 99):.0f} us, "
              f"{N / span:.3g} blocks/s, {len(batches)} launches", file=sys.stderr, flush=True)
        del llr, sent, bc, ro, snr, cw, q, ab, cw1, q1, ab1
        torch.cuda.empty_cache()
    top = per_rate[f"{wl['rates'][-1]:.0e}"]
    return {
        "metric": METRIC, "value": top["blocks_per_s"], "unit": "blocks/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": 1e3 * wl["seconds"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32 syndromes, FP32 LLR", "data": "synthetic",
        "config": {"workload": wl["desc"], "codes": wl["codes"], "rates_per_s": wl["rates"],
                   "ebn0_db_range": list(wl["ebn0_range"]), "budget": wl["budget"],
                   "capacity": wl["capacity"], "max_batch": wl["max_batch"]},
        "launch_params": knobs if knobs else "library defaults", "per_rate": per_rate,
    }


def run_learned(args, wl, dev):
    """Train the proposal on decoder-generated pairs (blocks whose first hit lies
    past batch 0, the ones the gated decode asks the network about), then plain,
    gated learned and the fixed prior order on the same held-out blocks, with a
    cost breakdown of the gated decode's stages."""
    import torch
    from paper_2202_13951_amd import binding, learned
    from synth import channel, codes
    H, G = codes.code(wl["code"])
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    xs, ys, seen, i = [], [], 0, 0
    while sum(int(x.shape[0]) for x in xs) < wl["train_pairs"]:
        x, y = learned.generate_pairs(H, G, 1 << 22, *wl["train_ebn0"], seed=10 + i, device=dev, gated=True)
        xs.append(x)
        ys.append(y)
        seen += 1 << 22
        i += 1
    x = torch.cat(xs)[: wl["train_pairs"]].contiguous()
    y = torch.cat(ys)[: wl["train_pairs"]].contiguous()
    del xs, ys
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    prop = learned.Proposal(dev, seed=0)
    t0 = time.perf_counter()
    losses = learned.train(prop, x, y, epochs=wl["epochs"], batch=wl["batch"], lr=wl["lr"],
                           log=lambda m: print(m, file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    hist = torch.bincount(y.long(), minlength=64)[:64].cpu().numpy().astype(np.float64)
    pl = hist[hist > 0] / hist.sum()
    label_entropy = float(-(pl * np.log(pl)).sum())
    prior = learned.prior_order(y, dev)
    del x, y

    def timed(fn):
        out = [fn()]                                  # untimed: work spaces reach their size here
        torch.cuda.synchronize()
        ms = time_calls(lambda: out.append(fn()), stream, reps=3)
        return out[-1], ms / 1e3

    shapes = {"defaults": None, "no_heavy_pass": binding.LaunchParams(split_steps=0)}
    points = {}
    tot = {k: dict(plain_s=0.0, learned_s=0.0) for k in shapes}
    tot_q = dict(blocks=0, plain=0.0, learned=0.0, prior=0.0)
    flops_fwd = 2.0 * (128 * 256 + 256 * 256 + 256 * 64)
    fwd_t, fwd_rows = 0.0, 0
    for e in wl["ebn0"]:
        llr, sent = channel.awgn_llr_torch(G, wl["blocks"], e, seed=5000 + int(round(e * 10)), device=dev)
        N = wl["blocks"]
        binding.orbg_decode(H, llr[:1024], wl["budget"])                    # warm caches
        learned.decode_learned_gated(prop, H, llr[:1024], wl["budget"])
        pt = {}
        for name, P in shapes.items():
            (pc, pq, pab), pt[name] = timed(lambda: binding.orbg_decode_ex(H, llr, wl["budget"], params=P))
        lt = {}
        for name, P in shapes.items():
            (lc, lq, lab, rest), lt[name] = timed(lambda: learned.decode_learned_gated(prop, H, llr, wl["budget"],
                                                                                      params=P))
        po = prior.unsqueeze(0).expand(N, 64).contiguous()
        rc_, rq, rab = binding.orbg_decode_ordered(H, llr, wl["budget"], po)
        # stages of the gated decode, each timed on its own (default shape)
        _, t_first = timed(lambda: binding.orbg_decode(H, llr, 64))
        idx = torch.nonzero(pq > 64).flatten()
        sub = llr[idx].contiguous()
        ordr = torch.empty((idx.numel(), 64), dtype=torch.uint8, device=dev)
        # the gated decode's network step: features, three layers and order in one launch
        _, t_net = timed(lambda: binding.orbg_mlp_infer(prop.w, prop.wb, llr=llr, ids=idx, order=ordr, pin0=True))
        # the network alone (features given, logits out) for the MFMA roofline
        xf = learned.features(sub)
        lg = torch.empty((idx.numel(), 64), dtype=torch.float32, device=dev)
        _, t_fwd = timed(lambda: binding.orbg_mlp_infer(prop.w, prop.wb, x=xf, logits=lg))
        if idx.numel():
            fwd_t += t_fwd
            fwd_rows += int(idx.numel())
        _, t_rest = timed(lambda: binding.orbg_decode_ordered(H, sub, wl["budget"], ordr))
        pe = (pc != sent).any(dim=1).cpu().numpy()
        le = (lc != sent).any(dim=1).cpu().numpy()
        re_ = (rc_ != sent).any(dim=1).cpu().numpy()
        pqn, lqn, rqn = (t.cpu().numpy().astype(np.float64) for t in (pq, lq, rq))
        mu, ci = learned.paired_ci(lqn - pqn)
        mur, cir = learned.paired_ci(lqn - rqn)
        points[f"{e:.1f}"] = {
            "bler_plain": float(pe.mean()), "bler_plain_ci95": list(wilson(int(pe.sum()), N)),
            "bler_learned": float(le.mean()), "bler_learned_ci95": list(wilson(int(le.sum()), N)),
            "bler_prior": float(re_.mean()),
            "bler_diff_ci95": list(learned.paired_ci(le.astype(np.float64) - pe.astype(np.float64))[1]),
            "mean_queries_plain": float(pqn.mean()), "mean_queries_learned": float(lqn.mean()),
            "mean_queries_prior_order": float(rqn.mean()),
            "queries_diff_vs_plain": mu, "queries_diff_vs_plain_ci95": list(ci),
            "queries_diff_vs_prior": mur, "queries_diff_vs_prior_ci95": list(cir),
            "blocks_network_ran_on": int(rest),
            "blocks_per_s_plain": {k: N / v for k, v in pt.items()},
            "blocks_per_s_learned": {k: N / v for k, v in lt.items()},
            "stage_ms": {"plain_decode": pt["defaults"] * 1e3, "first_batch_pass": t_first * 1e3,
                         "network_fused": t_net * 1e3, "network_forward_only": t_fwd * 1e3,
                         "ordered_search_of_listed": t_rest * 1e3, "gated_total": lt["defaults"] * 1e3},
            "abandoned_plain": int(pab.sum()), "abandoned_learned": int(lab.sum())}
        print(f"learned {e} dB: {points[f'{e:.1f}']}", file=sys.stderr, flush=True)
        tot_q["blocks"] += N
        tot_q["plain"] += float(pqn.sum())
        tot_q["learned"] += float(lqn.sum())
        tot_q["prior"] += float(rqn.sum())
        for k in shapes:
            tot[k]["plain_s"] += pt[k]
            tot[k]["learned_s"] += lt[k]
        del llr, sent, pc, pq, pab, lc, lq, lab, rc_, rq, rab, sub, xf, lg, ordr
        torch.cuda.empty_cache()
    Nt = tot_q["blocks"]
    mfma = (flops_fwd * fwd_rows / fwd_t) if fwd_t > 0 else 0.0
    return {
        "metric": METRIC, "value": Nt / tot["defaults"]["learned_s"], "unit": "blocks/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": tot["defaults"]["learned_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32 syndromes / FP32 LLR (decode), bf16 MFMA with fp32 "
                                                      "accumulation (network)", "data": "synthetic",
        "config": {"workload": wl["desc"], "code": wl["code"], "ebn0_db": wl["ebn0"],
                   "blocks_per_point": wl["blocks"], "budget": wl["budget"], "train_pairs": wl["train_pairs"],
                   "train_ebn0_db": list(wl["train_ebn0"]), "epochs": wl["epochs"], "minibatch": wl["batch"],
                   "lr": wl["lr"], "form": "gated: network only for blocks the first 64 queries do not decide"},
        "plain_value": Nt / tot["defaults"]["plain_s"],
        "by_launch_shape": {k: {"plain_blocks_per_s": Nt / v["plain_s"], "learned_blocks_per_s": Nt / v["learned_s"]}
                            for k, v in tot.items()},
        "mean_queries_plain": tot_q["plain"] / Nt, "mean_queries_learned": tot_q["learned"] / Nt,
        "mean_queries_prior_order": tot_q["prior"] / Nt,
        "roofline": {"bound": "mfma", "achieved": mfma / 1e12, "peak": 2500.0, "unit": "TFLOP/s (bf16)",
                     "frac": mfma / 2.5e15, "traffic": None,
                     "kernel": "mlp_infer_kernel (fused three-layer forward, activations in LDS)",
                     "flop_per_launch": flops_fwd * fwd_rows / max(len(wl["ebn0"]), 1)},
        "pair_generation_s": gen_s, "blocks_decoded_for_pairs": seen, "training_s": train_s,
        "train_loss_per_epoch": losses, "label_entropy_nats": label_entropy, "per_point": points,
    }


def run_mline(args, wl, dev):
    """Full m-line ORBGRAND over all points in one call per step (timed), then per
    point: BLER, queries and the segment counts of the fit, the same with the J/beta
    rounding, and the 1-line (where its schedules reach the budget) and basic
    decoders on the same blocks at the same budget, each timed on its own."""
    import torch
    from paper_2202_13951_amd import binding
    H, llr, sent = single_inputs(wl, dev)
    n, budget = wl["n"], wl["budget"]
    segments = args.segments if args.segments else wl["segments"]
    P, B = len(wl["ebn0"]), wl["blocks"]
    cw = torch.empty_like(sent)
    q = torch.empty((P * B,), dtype=torch.int64, device=dev)
    ab = torch.empty((P * B,), dtype=torch.uint8, device=dev)
    out = (cw, q, ab)
    stream = torch.cuda.current_stream()

    def one():
        binding.orbg_decode_mline(H, llr, budget, segments, segments_out=False, out=out)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        one()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a_, b_ in ev:
        a_.record(stream)
        b_.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        one()
        ev[i][1].record(stream)
        print(f"step {i + 1}/{args.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    blocks = P * B
    q_np = q.cpu().numpy()
    ab_np = ab.cpu().numpy()
    err = (cw != sent).any(dim=1).cpu().numpy()
    per_point = {}
    if not args.no_per_point:
        ms = torch.empty((B,), dtype=torch.int32, device=dev)
        ocw = torch.empty((B, n), dtype=torch.uint8, device=dev)
        oq = torch.empty((B,), dtype=torch.int64, device=dev)
        oab = torch.empty((B,), dtype=torch.uint8, device=dev)

        def other(fn, sl):
            t = time_calls(lambda: fn(sl), stream, reps=1) / 1e3
            e_ = (ocw != sent[sl]).any(dim=1).cpu().numpy()
            qq = oq.cpu().numpy()
            ne_ = int(e_.sum())
            return {"bler": ne_ / B, "errors": ne_, "bler_ci95": list(wilson(ne_, B)),
                    "mean_queries": float(qq.mean()), "abandoned": int(oab.sum().item()), "blocks_per_s": B / t}, e_
        binding.orbg_decode_ex(H, llr[:B], budget, out=(ocw, oq, oab))             # builds the schedules
        one_line_err = None
        try:
            binding.orbg_decode_1line(H, llr[:B], budget, j0=False, out=(ocw, oq, oab))
        except binding.OrbgError as ex:                   # budget beyond the 1-line schedules for this n
            one_line_err = str(ex)
        torch.cuda.synchronize()
        for p, e in enumerate(wl["ebn0"]):
            sl = slice(p * B, (p + 1) * B)
            print(f"point {e} dB", file=sys.stderr, flush=True)
            ne = int(err[sl].sum())
            binding.orbg_decode_mline(H, llr[sl], budget, segments, segments_out=ms, out=(ocw, oq, oab))
            torch.cuda.synchronize()
            same = bool((ocw == cw[sl]).all().item() and (oq == q[sl]).all().item())
            vals, cnts = np.unique(ms.cpu().numpy(), return_counts=True)
            t = time_calls(lambda: binding.orbg_decode_mline(H, llr[sl], budget, segments, segments_out=False,
                                                              out=(ocw, oq, oab)), stream, reps=1) / 1e3
            pt = {"bler": ne / B, "errors": ne, "bler_ci95": list(wilson(ne, B)),
                  "mean_queries": float(q_np[sl].mean()), "abandoned": int(ab_np[sl].sum()),
                  "breakdown": query_breakdown(q_np[sl], ab_np[sl], err[sl], budget,
                                               sweep=tuple(b for b in (10 ** 2, 10 ** 3, 10 ** 4, 10 ** 5)
                                                           if b < budget) + (budget,)),
                  "segments_used": {str(int(v)): float(c / B) for v, c in zip(vals, cnts)},
                  "segments_call_identical": same,
                  "blocks_per_s": B / t, "queries_per_s": float(q_np[sl].sum()) / t}
            pt["jbeta"], _ = other(lambda s_: binding.orbg_decode_mline(H, llr[s_], budget, segments, jdiv=True,
                                                                        segments_out=False, out=(ocw, oq, oab)), sl)
            if one_line_err is None:
                pt["one_line"], _ = other(lambda s_: binding.orbg_decode_1line(H, llr[s_], budget, j0=False,
                                                                               out=(ocw, oq, oab)), sl)
            else:
                pt["one_line"] = {"unsupported": one_line_err}
            pt["basic"], eb = other(lambda s_: binding.orbg_decode_ex(H, llr[s_], budget, out=(ocw, oq, oab)), sl)
            pt["only_mline_correct_vs_basic"] = int((~err[sl] & eb).sum())
            pt["only_basic_correct"] = int((err[sl] & ~eb).sum())
            per_point[f"{e:.1f}"] = pt

    kavg = float(np.mean(kern_ms)) / 1e3
    q_sum = int(q_np.sum())
    n_sorted = int((q_np > 1).sum())
    ops = algorithmic_ops(q_sum, n_sorted, n)
    hbm_bytes = blocks * (4 * n + n + 8 + 1)
    result = {
        "metric": METRIC,
        "value": blocks / (wall / args.steps),
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 syndromes, FP32 LLR and fit",
        "data": "synthetic",
        "config": {"workload": wl["desc"] if segments == wl["segments"] else
                   wl["desc"].replace("a 2-line fit", f"a fit of at most {segments} lines"),
                   "code": wl["code"], "n": n, "k": wl["k"], "ebn0_db": wl["ebn0"],
                   "blocks_per_step": blocks, "budget": budget, "segments": segments},
        "queries_per_s": q_sum / (wall / args.steps),
        "mean_queries": q_sum / blocks,
        "kernel_ms": float(np.mean(kern_ms)),
        "per_point": per_point,
        "roofline": {"bound": "alu", "achieved": ops / kavg / 1e12, "peak": PEAK_INT32_OPS / 1e12,
                     "unit": "Tops/s (int32)", "frac": ops / kavg / PEAK_INT32_OPS,
                     # counters were taken for the workload's own line count
                     "traffic": (profiled_traffic(args.workload, "mline_kernel", MLINE_SOURCES)
                                 if segments == wl["segments"] else None),
                     "kernel": "mline_kernel (one decode call)", "ops_per_launch": ops,
                     "hbm": {"achieved_GBps": hbm_bytes / kavg / 1e9, "peak_GBps": PEAK_HBM / 1e9,
                             "frac": hbm_bytes / kavg / PEAK_HBM, "bytes_per_launch": hbm_bytes}},
    }
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)     # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        result["cpu_baseline"] = cpu_baseline(H, lambda p, c: llr[p * B:p * B + c].cpu().numpy(), P, B, budget,
                                              dec=lambda H_, x, b_, th: O.decode_mline(H_, x, b_, segments, False,
                                                                                       th))
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="bch127", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-point", action="store_true",
                    help="skip the per-Eb/N0 launches (profiling runs: only the timed launches remain)")
    ap.add_argument("--no-tuned", action="store_true", help="library default launch shape")
    ap.add_argument("--segments", type=int, default=0, help="m-line workload: largest number of segments (1..4)")
    ap.add_argument("--ebn0", type=float, nargs="*", default=None,
                    help="decode only these Eb/N0 points of the workload (diagnosis runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(blocks are independent: shard the block range over GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2202_13951_amd import binding
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    binding.load()
    wl = dict(WORKLOADS[args.workload])
    if args.ebn0:
        wl["ebn0"] = [e for e in wl["ebn0"] if any(abs(e - x) < 1e-9 for x in args.ebn0)]
        assert wl["ebn0"], "no such Eb/N0 point in the workload"
        wl["desc"] += f" (only Eb/N0 {wl['ebn0']})"
    if "rates" in wl:
        result = run_stream(args, wl, dev)
    elif "codes" in wl:
        result = run_mixed(args, wl, dev)
    elif "train_pairs" in wl:
        result = run_learned(args, wl, dev)
    elif wl.get("oneline"):
        result = run_oneline(args, wl, dev)
    elif wl.get("mline"):
        result = run_mline(args, wl, dev)
    else:
        result = run_single(args, wl, dev)
    if args.ebn0 and "roofline" in result:
        result["roofline"]["traffic"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
