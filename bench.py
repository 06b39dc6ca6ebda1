"""Benchmark of the MI355X partition sort (one JSON line on stdout).

Workload: pdq_sort of 2^28 uint32 keys drawn uniformly from [0, 2^32), seed
0, keys only, in two forms on the same input: the plain partition sort, and
the sort with the learned multiway first pass (PDQ_LEARNED: sample, fused MLP
training, splitters, histogram, scatter into up to 511 bins, then partition
passes inside the bins). `value` is the learned form; the plain form is
reported beside it. A step is one full sort of a fresh copy of the input
already resident in HBM; the device-to-device reset copy before each step is
outside the HIP events that time the sort, and both forms' outputs are
checked (sorted, same sum) before timing.

Also reported:
  * roofline: the partition kernel's algorithmic bytes (read + write of every
    key it partitions: 8 B/key for 32-bit keys) over its launch durations,
    timed by the library with HIP events on the launch stream during the
    timed steps of the learned form, against the 8 TB/s HBM peak; the
    histogram and scatter kernels of the learned pass, and the plain form's
    partition kernel and first pass, beside it;
  * patterns: keys/s of both forms on 2^28 int32 keys in the seven input
    patterns;
  * equal_keys_u64_pairs: 2^27 uint64 keys with k in {2, 16, 1024, 65536}
    distinct values and a 90%-one-value mix, with payloads: passes and keys
    partitioned per key against Theorem 1's 2k + 2;
  * learned_mixtures_u64: learned against plain on 2^29 uint64 lognormal,
    Zipf and Gaussian-mixture keys, with the learned judge's decision;
  * cpu_baseline: the oracle (single-threaded CPU pdqsort) on the whole
    headline input, median of three runs pinned to one core, plus the
    segmented batch over every usable core.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--log2n 28]
"""
from __future__ import annotations

import argparse
import ctypes
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


def time_sorts(pdq, torch, pristine, work, ws, steps: int, profile: bool, **kw):
    """Returns (list of sort ms, list of stats dicts)."""
    ms, stats = [], []
    stream = torch.cuda.current_stream()
    for _ in range(steps):
        work.copy_(pristine)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        st = pdq.sort_(work, workspace=ws, profile=profile, **kw)
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
        if st is not None:
            stats.append(st)
    return ms, stats


def check_sorted(torch, work, pristine, what):
    w = work.to(torch.int64)  # torch has no device comparison for uint32
    ok = bool((w[1:] >= w[:-1]).all().item()) and int(w.sum()) == int(pristine.to(torch.int64).sum())
    del w
    if not ok:
        raise SystemExit(f"bench: {what} output is not a sorted permutation of the input")


def profiled_traffic():
    """HBM bytes per partition launch measured with rocprofv3 counters (see
    profiles/), or None when the kernel source changed since."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "partition_u32_2p28_learned_traffic.md")
    src = os.path.join(ROOT, "paper_2106_05123_amd", "csrc", "partition_kernel.h")
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


def summarize(ms, stats, n):
    s0 = stats[0]
    part_ms = sum(s["partition_ms"] for s in stats)
    part_bytes = sum(s["partition_bytes"] for s in stats)
    launches = sum(s["partition_launches"] for s in stats)
    out = {
        "keys/s": round(n / (float(np.mean(ms)) * 1e-3), 0),
        "ms": round(float(np.mean(ms)), 4),
        "ms_min": round(float(np.min(ms)), 4),
        "passes": s0["passes"],
        "element_visits": s0["element_visits"],
        "partition_ms": round(part_ms / len(stats), 4),
        "partition_GBps": round(part_bytes / (part_ms * 1e-3) / 1e9, 1) if part_ms > 0 else None,
        "partition_launches_per_sort": launches // len(stats),
        "partition_bytes_per_sort": part_bytes // len(stats),
    }
    if s0.get("learned", 0):
        out["learned_state"] = s0["learned"]
    if s0.get("learned", 0) == 1:
        fit = float(np.mean([s["learned_fit_ms"] for s in stats]))
        hist = float(np.mean([s["learned_hist_ms"] for s in stats]))
        scat = float(np.mean([s["learned_scatter_ms"] for s in stats]))
        out.update({
            "fit_ms": round(fit, 4),
            "hist_ms": round(hist, 4),
            "hist_GBps": round(s0["learned_hist_bytes"] / (hist * 1e-3) / 1e9, 1),
            "scatter_ms": round(scat, 4),
            "scatter_GBps": round(s0["learned_scatter_bytes"] / (scat * 1e-3) / 1e9, 1),
            "splitters": s0["learned_splitters"],
            "max_range_bin_over_fair": round(s0["learned_max_range_bin"] / (n / 256), 3),
            "final_loss": s0["learned_final_loss"],
            "train_steps": s0["learned_steps"],
        })
    return out, part_ms, part_bytes, launches


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--pattern-steps", type=int, default=3)
    ap.add_argument("--no-patterns", action="store_true")
    ap.add_argument("--paper-log2n", type=int, default=26,
                    help="size of the uint64 inputs in the paper's remaining distributions (0 = skip)")
    ap.add_argument("--equal-log2n", type=int, default=27,
                    help="size of the uint64 equal-key inputs with payloads (0 = skip)")
    ap.add_argument("--mix-log2n", type=int, default=29,
                    help="size of the uint64 skewed mixtures of the learned form (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-segmented", action="store_true")
    ap.add_argument("--seg-count", type=int, default=65536)
    ap.add_argument("--forms", default="plain,learned",
                    help="comma list of the 2^n forms to time (the learned one is the headline value)")
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
    log(f"generating {n} uint32 keys")
    host = W.uniform_u32(n, seed=0)
    pristine = torch.from_numpy(host).to(dev)
    work = torch.empty_like(pristine)
    lopt = pdq.Options(ctypes.sizeof(pdq.Options), pdq.FLAG_LEARNED, -1, args.tile, 0, 0.0, 0, 0, 0)
    ws = torch.empty(pdq.workspace_bytes(n, 1, "u32", options=lopt), dtype=torch.uint8, device=dev)

    wanted = [f for f in args.forms.split(",") if f]
    if "learned" not in wanted or any(f not in ("plain", "learned") for f in wanted):
        raise SystemExit("bench: --forms must list 'learned' (the headline form), optionally with 'plain'")
    forms = {k: v for k, v in (("plain", dict(tile=args.tile)), ("learned", dict(tile=args.tile, learned=True)))
             if k in wanted}
    results = {}
    for name, kw in forms.items():
        work.copy_(pristine)
        pdq.sort_(work, workspace=ws, **kw)
        torch.cuda.synchronize()
        check_sorted(torch, work, pristine, name)
        log(f"{name}: warmup {args.warmup}")
        time_sorts(pdq, torch, pristine, work, ws, args.warmup, profile=False, **kw)
        torch.cuda.synchronize()
        log(f"{name}: timing {args.steps} steps")
        t0 = time.perf_counter()
        ms, stats = time_sorts(pdq, torch, pristine, work, ws, args.steps, profile=True, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        results[name] = (ms, stats, wall)

    ms, stats, wall = results["learned"]
    learned, part_ms, part_bytes, launches = summarize(ms, stats, n)
    plain = None
    if "plain" in results:
        plain, p_part_ms, p_part_bytes, p_launches = summarize(*results["plain"][:2], n)
        p_stats = results["plain"][1]
        fp_ms = float(np.mean([s["first_pass_ms"] for s in p_stats]))
        fp_bytes = p_stats[0]["first_pass_bytes"]
        fp_gbs = fp_bytes / (fp_ms * 1e-3) / 1e9
    ms_step = float(np.mean(ms))
    value = n / (ms_step * 1e-3)
    achieved = part_bytes / (part_ms * 1e-3) / 1e9 if part_ms > 0 else 0.0

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
        "partition_share_of_sort": round(part_ms / sum(ms), 3),
        "learned_hist": {"GB/s": learned.get("hist_GBps"),
                         "frac": round(learned["hist_GBps"] / HBM_PEAK_GBS, 4) if "hist_GBps" in learned else None},
        "learned_scatter": {"GB/s": learned.get("scatter_GBps"),
                            "frac": round(learned["scatter_GBps"] / HBM_PEAK_GBS, 4)
                            if "scatter_GBps" in learned else None},
        "plain_partition": {"GB/s": plain["partition_GBps"],
                            "frac": round(plain["partition_GBps"] / HBM_PEAK_GBS, 4),
                            "avg_launch_ms": round(p_part_ms / max(p_launches, 1), 4)} if plain else None,
        "plain_first_pass": {"ms": round(fp_ms, 4), "bytes": int(fp_bytes), "GB/s": round(fp_gbs, 1),
                             "frac": round(fp_gbs / HBM_PEAK_GBS, 4)} if plain else None,
        "copy_ceiling_GBps": round(copy_gbs, 1),
    }

    patterns = {}
    if not args.no_patterns:
        for p in W.C2_PATTERNS:
            log(f"pattern {p}")
            hp = W.pattern_i32(p, n, seed=0)
            pp = torch.from_numpy(hp).to(dev)
            wi = torch.empty_like(pp)  # int32 work buffer: the pattern keys are signed
            row = {}
            for name, kw in forms.items():
                pms, pst = time_sorts(pdq, torch, pp, wi, ws, args.pattern_steps, profile=True, **kw)
                row[name] = {"keys/s": round(n / (np.mean(pms) * 1e-3), 0), "ms": round(float(np.mean(pms)), 3),
                             "passes": pst[0]["passes"], "learned_state": pst[0]["learned"]}
            patterns[p] = row
            del pp, wi

    # the paper's remaining distributions (Section 6.1), uint64 keys like the
    # paper's 64-bit int, in both forms
    paper = {}
    if not args.no_patterns and args.paper_log2n > 0:
        m = 1 << args.paper_log2n
        for p in W.PAPER_PATTERNS:
            log(f"paper distribution {p}")
            hp = W.paper_pattern_u64(p, m, seed=0)
            pp = torch.from_numpy(hp).to(dev)
            wu = torch.empty_like(pp)
            row = {}
            for name, kw in forms.items():
                pms, pst = time_sorts(pdq, torch, pp, wu, None, args.pattern_steps, profile=True, **kw)
                row[name] = {"keys/s": round(m / (np.mean(pms) * 1e-3), 0), "ms": round(float(np.mean(pms)), 3),
                             "passes": pst[0]["passes"], "learned_state": pst[0]["learned"]}
            paper[p] = row
            del pp, wu

    segmented = None
    if not args.no_segmented:
        segmented = bench_segmented(pdq, torch, W, dev, args)

    equal_keys = None
    if not args.no_patterns and args.equal_log2n > 0:
        equal_keys = bench_equal_keys(pdq, torch, W, dev, args)

    learned_mix = None
    if not args.no_patterns and args.mix_log2n > 0:
        learned_mix = bench_learned_mixtures(pdq, torch, W, dev, args)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(host, keys_seg=None if args.no_segmented else args.seg_count, W=W)

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
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"pdq_sort with the learned first pass of 2^{args.log2n} uint32 keys, "
                               f"uniform random (seed 0), keys only",
                   "n": n, "key_type": "u32",
                   "tile": args.tile or "per pass: 8192 once no segment holds over 1/10 of the keys, else 16384 (segments >= 2^18 keys)"},
        "forms": {"learned": learned, "plain": plain,
                  "learned_over_plain": round(plain["ms"] / learned["ms"], 3) if plain else None},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "patterns_i32": patterns,
        "paper_distributions_u64": {"n": 1 << args.paper_log2n, "rows": paper} if paper else None,
        "segmented_f32_pairs": segmented,
        "equal_keys_u64_pairs": equal_keys,
        "learned_mixtures_u64": learned_mix,
    }
    print(json.dumps(line), flush=True)


def bench_segmented(pdq, torch, W, dev, args):
    """65,536 segments with log-uniform sizes 1 ... 2^16, float32 N(0, 1) keys
    with 5% in-segment duplicates and 2^10 each of -0.0 / +0.0, uint32
    payloads; host-driven segmented sort timed like the main workload."""
    log(f"generating {args.seg_count} segments")
    keys, off, vals = W.segmented_f32(args.seg_count, max_log2=16, seed=0)
    n = keys.size
    pk = torch.from_numpy(keys).to(dev)
    pv = torch.from_numpy(vals).to(dev)
    po = torch.from_numpy(off).to(dev)
    wk = torch.empty_like(pk)
    wv = torch.empty_like(pv)
    topt = pdq.Options(ctypes.sizeof(pdq.Options), pdq.FLAG_BATCHED | pdq.FLAG_AUTOTUNE, -1, 0, 0, 0.0, 0, 0, 0, 0)
    ws = torch.empty(pdq.workspace_bytes(n, args.seg_count, "f32", has_vals=True, options=topt),
                     dtype=torch.uint8, device=dev)
    steps = max(3, args.steps)

    def timed(fn, reps, profile):
        ms, stats = [], []
        for _ in range(reps):
            wk.copy_(pk)
            wv.copy_(pv)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            st = fn(profile)
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
            if st:
                stats.append(st)
        return ms, stats

    def check(what):
        kk = wk.view(torch.int32).to(torch.int64)
        img = torch.where(kk < 0, ~kk & 0xFFFFFFFF, kk | 0x80000000)
        starts = po[:-1].to(torch.int64)
        seg_start = torch.zeros(n, dtype=torch.bool, device=dev)
        seg_start[starts[starts < n]] = True
        bad = bool(((img[1:] < img[:-1]) & ~seg_start[1:]).any().item())
        same = int(wv.to(torch.int64).sum()) == n * (n - 1) // 2
        del kk, img
        if bad or not same:
            raise SystemExit(f"bench: segmented output ({what}) not sorted within segments")

    plain = lambda prof: pdq.segmented_sort_(wk, po, wv, workspace=ws, profile=prof, stats=prof)
    timed(plain, 1, False)
    check("plain")
    ms_p, st_p = timed(plain, steps, True)
    log("segmented: autotuning the batched plan")
    wk.copy_(pk)
    wv.copy_(pv)
    plan = pdq.Plan(wk, po, wv, autotune=True, workspace=ws)
    shape, tune_ms = plan.info()
    class_threads, class_ms = plan.classes()
    # the eager call takes the configuration the plan tuned (kept in process)
    eager = lambda prof: pdq.segmented_sort_(wk, po, wv, workspace=ws, batched=True, profile=prof, stats=prof)
    timed(eager, 1, False)
    check("batched")
    ms_b, st_b = timed(eager, steps, True)
    graph = lambda prof: plan.launch()
    timed(graph, 1, False)
    check("graph")
    ms_g, _ = timed(graph, steps, False)
    plan.destroy()
    s0 = st_p[0]
    mp, mb, mg = float(np.mean(ms_p)), float(np.mean(ms_b)), float(np.mean(ms_g))
    return {"workload": f"{args.seg_count} segments, log-uniform sizes 1..2^16, float32 N(0,1) keys with 5% "
                        f"duplicates and signed zeros, uint32 payloads (seed 0)",
            "n": n,
            "plain": {"keys/s": round(n / (mp * 1e-3), 0), "ms": round(mp, 3), "passes": s0["passes"],
                      "partition_ms": round(s0["partition_ms"], 3),
                      "partition_GBps": round(s0["partition_bytes"] / (s0["partition_ms"] * 1e-3) / 1e9, 1)
                      if s0["partition_ms"] else None},
            "batched_eager": {"keys/s": round(n / (mb * 1e-3), 0), "ms": round(mb, 3),
                              "queue_items": st_b[0]["batch_items"], "passes": st_b[0]["passes"],
                              "partition_tile": pdq.BATCH_SHAPES[shape][0]},
            "batched_graph": {"keys/s": round(n / (mg * 1e-3), 0), "ms": round(mg, 3),
                              "partition_tile": pdq.BATCH_SHAPES[shape][0],
                              "autotune_ms_per_tile": [round(x, 3) for x in tune_ms[:3]],
                              "base_class_threads": class_threads,
                              "autotune_ms_per_class_shape": [[round(x, 3) for x in row] for row in class_ms]},
            "batched_over_plain": round(mp / mg, 3)}


def bench_equal_keys(pdq, torch, W, dev, args):
    """The equal-key stress of the Dutch-flag scheme (Section 3, Theorem 1):
    2^27 uint64 keys taking k distinct values (and a 90%-one-value mix) with
    a uint32 index payload; passes and keys partitioned per key against the
    2k + 2 bound, and the oracle's comparisons per key on a 2^22-key input of
    the same generator (comparisons / n depends on k, not on n)."""
    import oracle
    n = 1 << args.equal_log2n
    rows = {}
    wk = torch.empty(n, dtype=torch.uint64, device=dev)
    wv = torch.empty(n, dtype=torch.uint32, device=dev)
    pv = torch.from_numpy(W.index_payload(n)).to(dev)
    for k in (2, 16, 1024, 65536, "mix"):
        log(f"equal keys k={k}")
        h = W.one_value_mix_u64(n, seed=0) if k == "mix" else W.k_distinct_u64(n, k, seed=0)
        pk = torch.from_numpy(h).to(dev)
        ms, sts = [], []
        for _ in range(args.pattern_steps + 1):
            wk.copy_(pk)
            wv.copy_(pv)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            st = pdq.sort_pairs_(wk, wv, stats=True)
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
            sts.append(st)
        ms = ms[1:]
        st = sts[-1]
        m = 1 << 22
        small = W.one_value_mix_u64(m, seed=0) if k == "mix" else W.k_distinct_u64(m, k, seed=0)
        _, _, c, _ = oracle.sort(small, count=True)
        rows[str(k)] = {"keys/s": round(n / (np.mean(ms) * 1e-3), 0), "ms": round(float(np.mean(ms)), 3),
                        "passes": st["passes"], "element_visits_per_key": round(st["element_visits"] / n, 3),
                        "pass_bound_2k_plus_2": (2 * k + 2) if k != "mix" else None,
                        "partitions_right": st["partitions_right"], "partitions_left": st["partitions_left"],
                        "equal_elements": st["equal_elements"], "heapsort_segments": st["heapsort_segments"],
                        "oracle_comparisons_per_key_2p22": round(c["comparisons"] / m, 3)}
        del pk
    del wk, wv, pv
    torch.cuda.empty_cache()
    return {"workload": f"2^{args.equal_log2n} uint64 keys with k distinct values (uniform over them) or 90% one "
                        f"value + 10% uniform, uint32 index payload (seed 0)", "n": n, "rows": rows}


def bench_learned_mixtures(pdq, torch, W, dev, args):
    """The learned form against the plain one on 2^29 uint64 keys from three
    skewed mixtures; reports whether the learned pass ran or its judge sent
    the call back to the plain path, and the largest range bin over the fair
    share n/256."""
    n = 1 << args.mix_log2n
    rows = {}
    wk = torch.empty(n, dtype=torch.uint64, device=dev)
    lopt = pdq.Options(ctypes.sizeof(pdq.Options), pdq.FLAG_LEARNED, -1, 0, 0, 0.0, 0, 0, 0)
    ws = torch.empty(pdq.workspace_bytes(n, 1, "u64", options=lopt), dtype=torch.uint8, device=dev)
    for dist in ("lognormal", "zipf", "gmm"):
        log(f"learned mixture {dist}: generating 2^{args.mix_log2n} keys")
        if dist == "zipf":
            # inverse-CDF lookup of the same uniforms on the device (same keys as zipf_u64)
            cdf = torch.from_numpy(W.zipf_cdf()).to(dev)
            u = torch.from_numpy(W.zipf_uniforms(n, 0)).to(dev)
            pk = torch.clamp(torch.searchsorted(cdf, u, right=True) + 1, max=cdf.numel()).to(torch.int64)
            pk = pk.view(torch.uint64)
            del cdf, u
        else:
            h = W.lognormal_u64(n, seed=0) if dist == "lognormal" else W.gmm_u64(n, seed=0)
            pk = torch.from_numpy(h).to(dev)
            del h
        row = {}
        for name, kw in (("plain", {}), ("learned", {"learned": True})):
            ms, st = time_sorts(pdq, torch, pk, wk, ws, args.pattern_steps + 1, profile=True, **kw)
            ms = ms[1:]
            s0 = st[-1]
            row[name] = {"keys/s": round(n / (np.mean(ms) * 1e-3), 0), "ms": round(float(np.mean(ms)), 3),
                         "passes": s0["passes"], "element_visits_per_key": round(s0["element_visits"] / n, 3)}
            if kw:
                row[name].update({"learned_state": s0["learned"], "splitters": s0["learned_splitters"],
                                  "max_range_bin_over_fair": round(s0["learned_max_range_bin"] / (n / 256), 3),
                                  "fit_ms": round(float(np.mean([x["learned_fit_ms"] for x in st[1:]])), 3),
                                  "train_steps": s0["learned_steps"],
                                  "equal_bin_keys": s0["learned_equal_elements"]})
        row["learned_over_plain"] = round(row["plain"]["ms"] / row["learned"]["ms"], 3)
        rows[dist] = row
        del pk
        torch.cuda.empty_cache()
    del wk, ws
    torch.cuda.empty_cache()
    return {"workload": f"2^{args.mix_log2n} uint64 keys: lognormal(20, 3) rounded, Zipf(1.1) over 2^24 ranks, "
                        f"8-component Gaussian mixture on a 2^40 grid (seed 0); learned state 1 = learned pass "
                        f"used, 2 = judged and sent back to the plain path", "n": n, "rows": rows}


def cpu_baseline(host, keys_seg, W):
    """The oracle (single-threaded CPU pdqsort, generic -O2 build, counters
    compiled out) timed on this host: the full 2^28 headline input, three
    runs pinned to one core, median; plus the 65,536-segment batch sorted
    with the segments spread over every core this process may use."""
    import concurrent.futures as cf
    import oracle
    n = host.size
    cpus = sorted(os.sched_getaffinity(0))
    old = set(cpus)
    runs = []
    try:
        os.sched_setaffinity(0, {cpus[0]})
        for r in range(3):
            log(f"cpu oracle on {n} keys, run {r + 1} of 3 (one core)")
            t1 = time.perf_counter()
            oracle.sort(host)
            runs.append(time.perf_counter() - t1)
    finally:
        os.sched_setaffinity(0, old)
    dt = float(np.median(runs))
    out = {"value": round(n / dt, 0), "unit": "keys/s", "cores": 1, "kind": "oracle",
           "sample": f"the whole 2^{int(np.log2(n))}-key uint32 headline input, median of 3 single-threaded oracle "
                     f"sorts pinned to one core ({', '.join(f'{x:.2f}' for x in runs)} s)",
           "ns_per_n_log2_n": round(float(dt * 1e9 / (n * np.log2(n))), 4),
           "host_cpu": _cpu_model(), "host_nproc": os.cpu_count(), "usable_cores": len(cpus)}
    if keys_seg:
        keys, off, vals = W.segmented_f32(keys_seg, max_log2=16, seed=0)
        nseg = off.size - 1
        threads = len(cpus)
        # contiguous groups of segments with about equal key counts
        cuts = np.searchsorted(off, np.linspace(0, off[-1], threads + 1).astype(np.uint64))
        cuts[0], cuts[-1] = 0, nseg
        groups = [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]

        def one(g):
            a, b = g
            lo, hi = int(off[a]), int(off[b])
            oracle.segmented_sort(keys[lo:hi], (off[a:b + 1] - off[a]).astype(np.uint64), vals[lo:hi])

        truns = []
        with cf.ThreadPoolExecutor(threads) as ex:
            for r in range(3):
                log(f"cpu oracle, segmented batch on {threads} threads, run {r + 1} of 3")
                t1 = time.perf_counter()
                list(ex.map(one, groups))
                truns.append(time.perf_counter() - t1)
        ts = float(np.median(truns))
        out["segmented_all_cores"] = {
            "value": round(keys.size / ts, 0), "unit": "keys/s", "cores": threads, "kind": "oracle",
            "sample": f"the {nseg}-segment float32 + uint32 batch ({keys.size} keys), segments split into "
                      f"{len(groups)} contiguous groups of about equal key counts, one oracle segmented sort per "
                      f"thread, median of 3 ({', '.join(f'{x:.2f}' for x in truns)} s)"}
    return out


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
