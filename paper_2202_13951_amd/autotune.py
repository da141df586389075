"""Autotuner of the decode launch shape (orbg_launch_params).

Coordinate descent over the five knobs of the persistent two-pass decode:
light-pass workgroups per CU, blocks per work-counter increment, the step at
which a block moves to the heavy pass, waves per heavy block and heavy
workgroups per CU.  Each candidate is timed with HIP events on the stream the
decode runs on (median of a few launches of the caller's workload).  The
decoded bits do not depend on the launch shape, so tuning never changes
results.  Best shapes are cached in tuned.json next to this file, keyed by
architecture and compute-unit count (e.g. gfx950-256cu) and workload name.

  python -m paper_2202_13951_amd.autotune --workload bch127 --out tuned.json
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")

KNOBS = {
    "split_steps": [0, 16, 32, 64, 128, 256],
    "workgroups_per_cu": [8, 16, 24, 28, 32, 48],
    "chunk": [0, 8, 16, 32, 64],
    "heavy_waves": [4, 8, 16],
    "heavy_workgroups_per_cu": [1, 2, 4, 8],
}
DEFAULT = dict(workgroups_per_cu=32, chunk=0, split_steps=64, heavy_waves=8, heavy_workgroups_per_cu=2)


_EVENTS = []


def time_launch(run, params, reps: int = 3) -> float:
    """Median milliseconds of `run(params)` (one decode on torch's current stream).
    One pair of events serves every measurement, recorded once before the first:
    torch makes an event's HIP object at its first record, which would stretch
    the first interval it bounds."""
    import torch
    stream = torch.cuda.current_stream()
    if not _EVENTS:
        _EVENTS.extend(torch.cuda.Event(enable_timing=True) for _ in range(2))
        for e in _EVENTS:
            e.record(stream)
    a, b = _EVENTS
    run(params)                                       # warm-up (caches, work space)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a.record(stream)
        run(params)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def tune(run, start: dict | None = None, rounds: int = 2, reps: int = 3, log=None):
    """Coordinate descent from `start`; returns (best knob dict, best ms, history)."""
    from .binding import LaunchParams
    cur = dict(DEFAULT if start is None else start)
    best_ms = time_launch(run, LaunchParams(**cur), reps)
    history = [(dict(cur), best_ms)]
    for _ in range(rounds):
        changed = False
        for knob, values in KNOBS.items():
            if knob in ("heavy_waves", "heavy_workgroups_per_cu") and cur["split_steps"] == 0:
                continue                              # no heavy pass: these do not matter
            for v in values:
                if v == cur[knob]:
                    continue
                cand = dict(cur, **{knob: v})
                ms = time_launch(run, LaunchParams(**cand), reps)
                history.append((cand, ms))
                if log:
                    log(f"{cand} {ms:.3f} ms")
                if ms < best_ms * 0.995:
                    best_ms, cur, changed = ms, cand, True
        if not changed:
            break
    return cur, best_ms, history


def device_name() -> str:
    """Architecture and compute-unit count, e.g. gfx950-256cu (marketing names vary
    with the driver's device table)."""
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.gcnArchName.split(':')[0]}-{p.multi_processor_count}cu"


def load_tuned(workload: str, path: str = CACHE):
    """Tuned knob dict for this device and workload, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    entry = table.get(device_name(), {}).get(workload)
    return dict(entry["params"]) if entry else None


def save_tuned(workload: str, params: dict, ms: float, default_ms: float, path: str = CACHE):
    table = {}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    table.setdefault(device_name(), {})[workload] = {"params": params, "ms": ms, "default_ms": default_ms}
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True, help="a workload name of bench.py")
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--rounds", type=int, default=2)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import bench
    from .binding import LaunchParams
    run, blocks = bench.make_runner(args.workload)
    default_ms = time_launch(run, LaunchParams(**DEFAULT))
    best, ms, hist = tune(run, rounds=args.rounds, log=lambda s: print(s, flush=True))
    # single timings differ by a few percent, so the descent can end on a worse
    # shape than one found before: the cached shape, if any, meets the new one
    # in a final comparison with more repetitions, and the faster is kept
    prev = load_tuned(args.workload, args.out) or load_tuned(args.workload)
    if prev and prev != best:
        new_ms = time_launch(run, LaunchParams(**best), 9)
        prev_ms = time_launch(run, LaunchParams(**prev), 9)
        print(f"new {best} {new_ms:.3f} ms, cached {prev} {prev_ms:.3f} ms", flush=True)
        best, ms = (prev, prev_ms) if prev_ms < new_ms else (best, new_ms)
    print(json.dumps({"workload": args.workload, "blocks": blocks, "default_ms": default_ms, "best_ms": ms,
                      "params": best, "evaluations": len(hist)}), flush=True)
    save_tuned(args.workload, best, ms, default_ms, args.out)


if __name__ == "__main__":
    main()
