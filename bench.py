"""Benchmark of the MI355X partition sort (one JSON line on stdout).

Workload: pdq_sort of 2^28 int32 keys (keys only), uniform random, seed 0 --
the plain GPU partition-sort configuration. A step is one full sort (every
pass of the hot path) of a fresh copy of the input already resident in HBM;
the device-to-device reset copy before each step is outside the HIP events
that time the sort. Also reported:
  * roofline: the partition kernel's algorithmic bytes (read + write of every
    key it partitions, 8 B/key for 32-bit keys) divided by its launch
    durations, measured by the library with HIP events on the launch stream
    over the timed steps, against the 8 TB/s HBM peak; the first pass (one
    2^28-key segment) separately;
  * patterns: keys/s for each of the seven input patterns;
  * cpu_baseline: the oracle (single-threaded CPU pdqsort) on a bounded
    sample of the same input, timed on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--log2n 28]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "sorted keys/s and HBM GB/s fraction, uint32 2^28 keys: learned+batched vs plain GPU"


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_sorts(pdq, torch, pristine, work, ws, steps: int, profile: bool, tile: int = 0):
    """Returns (list of sort ms, list of stats dicts)."""
    ms, stats = [], []
    stream = torch.cuda.current_stream()
    for _ in range(steps):
        work.copy_(pristine)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        st = pdq.sort_(work, workspace=ws, profile=profile, tile=tile)
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
        if st is not None:
            stats.append(st)
    return ms, stats


def profiled_traffic():
    """HBM bytes per partition launch measured with rocprofv3 counters (see
    profiles/), or None when the kernel source changed since."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "partition_i32_2p28_traffic.md")
    src = os.path.join(ROOT, "paper_2106_05123_amd", "csrc", "k_partition.hip")
    try:
        fields = {}
        for ln in open(prof):
            if ":" in ln and not ln.startswith(("|", "#", "`")):
                k, v = ln.split(":", 1)
                fields[k.strip()] = v.strip()
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        if fields.get("kernel_source_sha256_16") != h:
            return None
        return int(fields["avg_hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--pattern-steps", type=int, default=3)
    ap.add_argument("--no-patterns", action="store_true")
    ap.add_argument("--cpu-log2n", type=int, default=26)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              f"the sort has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    import gen.workloads as W
    import paper_2106_05123_amd as pdq

    dev = torch.device("cuda:0")
    n = 1 << args.log2n
    log(f"generating {n} int32 keys")
    host = W.pattern_i32("random", n, seed=0)
    pristine = torch.from_numpy(host).to(dev)
    work = torch.empty_like(pristine)
    ws = torch.empty(pdq.workspace_bytes(n, 1, "i32"), dtype=torch.uint8, device=dev)

    # check once that the timed configuration sorts correctly (sortedness + sum)
    work.copy_(pristine)
    pdq.sort_(work, workspace=ws, tile=args.tile)
    torch.cuda.synchronize()
    ok = bool((work[1:] >= work[:-1]).all().item()) and int(work.sum(dtype=torch.int64)) == int(
        pristine.sum(dtype=torch.int64))
    if not ok:
        raise SystemExit("bench: GPU output is not a sorted permutation of the input")

    log(f"warmup {args.warmup}")
    time_sorts(pdq, torch, pristine, work, ws, args.warmup, profile=False, tile=args.tile)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    ms, stats = time_sorts(pdq, torch, pristine, work, ws, args.steps, profile=True, tile=args.tile)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = float(np.mean(ms))
    value = n / (ms_step * 1e-3)

    part_ms = sum(s["partition_ms"] for s in stats)
    part_bytes = sum(s["partition_bytes"] for s in stats)
    launches = sum(s["partition_launches"] for s in stats)
    achieved = part_bytes / (part_ms * 1e-3) / 1e9 if part_ms > 0 else 0.0
    fp_ms = float(np.mean([s["first_pass_ms"] for s in stats]))
    fp_bytes = stats[0]["first_pass_bytes"]
    fp_gbs = fp_bytes / (fp_ms * 1e-3) / 1e9
    s0 = stats[0]
    # achievable ceiling on this machine: a device-to-device copy of the same bytes
    cms = []
    for _ in range(5):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        work.copy_(pristine)
        b.record()
        b.synchronize()
        cms.append(a.elapsed_time(b))
    copy_gbs = 2 * n * 4 / (min(cms) * 1e-3) / 1e9
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": profiled_traffic(),
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "kernel": "k_partition",
        "avg_launch_ms": round(part_ms / max(launches, 1), 4),
        "avg_launch_bytes": int(part_bytes / max(launches, 1)),
        "launches": launches,
        "first_pass": {"ms": round(fp_ms, 4), "bytes": int(fp_bytes), "GB/s": round(fp_gbs, 1),
                       "frac": round(fp_gbs / HBM_PEAK_GBS, 4)},
        "partition_share_of_sort": round(part_ms / sum(ms), 3),
        "copy_ceiling_GBps": round(copy_gbs, 1),
    }

    patterns = {}
    if not args.no_patterns:
        for p in W.C2_PATTERNS:
            if p == "random":
                patterns[p] = {"keys/s": round(value, 0), "ms": round(ms_step, 3), "passes": s0["passes"]}
                continue
            log(f"pattern {p}")
            hp = W.pattern_i32(p, n, seed=0)
            pp = torch.from_numpy(hp).to(dev)
            pms, pst = time_sorts(pdq, torch, pp, work, ws, args.pattern_steps, profile=True, tile=args.tile)
            patterns[p] = {"keys/s": round(n / (np.mean(pms) * 1e-3), 0), "ms": round(float(np.mean(pms)), 3),
                           "passes": pst[0]["passes"], "sorted_elements": pst[0]["sorted_elements"],
                           "heapsort_elements": pst[0]["heapsort_elements"]}
            del pp

    cpu = None
    if not args.no_cpu:
        import oracle
        m = 1 << min(args.cpu_log2n, args.log2n)
        sample = host[:m].copy()
        log(f"cpu oracle on {m} keys")
        t1 = time.perf_counter()
        oracle.sort(sample)
        dt = time.perf_counter() - t1
        cpu = {"value": round(m / dt, 0), "unit": "keys/s", "cores": 1, "kind": "oracle",
               "sample": f"first 2^{int(np.log2(m))} keys of the same int32 input, one single-threaded "
                         f"oracle sort ({dt:.2f} s)",
               "host_cpu": _cpu_model(), "host_nproc": os.cpu_count()}

    line = {
        "metric": METRIC,
        "value": round(value, 0),
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_wall_incl_reset": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": f"pdq_sort of 2^{args.log2n} int32 keys, uniform random (seed 0), keys only",
                   "n": n, "key_type": "i32", "pattern": "random", "tile": args.tile or 32768,
                   "passes": s0["passes"], "element_visits": s0["element_visits"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "patterns": patterns,
    }
    print(json.dumps(line), flush=True)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
