"""Seeded synthetic inputs in the paper's input patterns (Section 6.1, the list of
distributions) and in the shapes of the partition-sort workloads.

This module only draws inputs. It holds none of the sorting arithmetic: no
comparison, pivot choice or partition logic lives here, so that the oracle and
the GPU path can both take their inputs from it without sharing any of the
method. Every generator is deterministic in (sizes, seed) and uses numpy's
PCG64 (`numpy.random.default_rng`).

Patterns (Section 6.1 defines uniform, organ, asc, desc, dupsq, dup8, mod8,
ones, sort50/90/99 and merge; sawtooth and the "1% swapped" and "random tail"
variants are extra stress shapes of the same kind):

* random                 uniform over the full value range of the type
* ascending              i - n/2                  (already sorted)
* descending             reverse of ascending
* organ_pipe             first half ascending, second half descending
* sawtooth               i mod period
* random_1pct_sorted     random A; n/100 random positions P get S[P],
                         S = sorted(A)
* ascending_random_tail  ascending, last `tail` entries uniform random
"""
from __future__ import annotations

import numpy as np

C2_PATTERNS = (
    "random",
    "ascending",
    "descending",
    "organ_pipe",
    "sawtooth",
    "random_1pct_sorted",
    "ascending_random_tail",
)

PAPER_PATTERNS = ("dupsq", "dup8", "mod8", "ones", "sort50", "sort90", "sort99", "merge")


def uniform_u32(n: int, seed: int = 0) -> np.ndarray:
    """n uint32 keys drawn uniformly from [0, 2^32)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2**32, n, dtype=np.uint32)


def uniform_u64(n: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2**64, n, dtype=np.uint64, endpoint=False)


def pattern_i32(pattern: str, n: int, seed: int = 0, period: int = 1 << 16,
                tail: int = 1 << 10, sorter=None) -> np.ndarray:
    """int32 keys in one of `C2_PATTERNS` (sign bit exercised: values are
    centred on zero). `sorter`, if given, replaces np.sort for the one
    pattern that needs a sorted copy of its input (any correct sort gives
    the same array)."""
    rng = np.random.default_rng(seed)
    half = n // 2
    if pattern == "random":
        return rng.integers(-(2**31), 2**31, n, dtype=np.int32)
    if pattern == "ascending":
        return (np.arange(n, dtype=np.int64) - half).astype(np.int32)
    if pattern == "descending":
        return (np.arange(n, dtype=np.int64) - half).astype(np.int32)[::-1].copy()
    if pattern == "organ_pipe":
        i = np.arange(n, dtype=np.int64)
        v = np.where(i < half, i, n - 1 - i) - (n // 4)
        return v.astype(np.int32)
    if pattern == "sawtooth":
        return (np.arange(n, dtype=np.int64) % period).astype(np.int32)
    if pattern == "random_1pct_sorted":
        a = rng.integers(-(2**31), 2**31, n, dtype=np.int32)
        s = np.sort(a) if sorter is None else sorter(a)
        pos = rng.choice(n, size=max(1, n // 100), replace=False) if n > 0 else np.zeros(0, np.int64)
        a[pos] = s[pos]
        return a
    if pattern == "ascending_random_tail":
        a = (np.arange(n, dtype=np.int64) - half).astype(np.int32)
        t = min(tail, n)
        if t:
            a[n - t:] = rng.integers(-(n // 2) - 1, n // 2 + 1, t, dtype=np.int32)
        return a
    raise ValueError(f"unknown pattern {pattern!r}")


def paper_pattern_u64(pattern: str, n: int, seed: int = 0) -> np.ndarray:
    """The remaining distributions of Section 6.1, shuffled where the paper
    shuffles, as uint64 keys."""
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.uint64)
    if pattern == "dupsq":
        r = max(1, int(np.floor(np.sqrt(n))))
        a = i % np.uint64(r)
        rng.shuffle(a)
        return a
    if pattern == "dup8":
        with np.errstate(over="ignore"):
            nn = np.uint64(max(n, 1))
            x = i % nn
            p2 = (x * x) % nn
            p4 = (p2 * p2) % nn
            p8 = (p4 * p4) % nn
            a = (p8 + np.uint64(n // 2)) % nn
        rng.shuffle(a)
        return a
    if pattern == "mod8":
        a = i % np.uint64(8)
        rng.shuffle(a)
        return a
    if pattern == "ones":
        return np.ones(n, dtype=np.uint64)
    if pattern in ("sort50", "sort90", "sort99"):
        frac = {"sort50": 0.5, "sort90": 0.9, "sort99": 0.99}[pattern]
        a = i.copy()
        k = int(n * frac)
        rest = a[k:].copy()
        rng.shuffle(rest)
        a[k:] = rest
        return a
    if pattern == "merge":
        h = n // 2
        return np.concatenate([np.arange(h, dtype=np.uint64), np.arange(n - h, dtype=np.uint64)])
    raise ValueError(f"unknown pattern {pattern!r}")


def k_distinct_u64(n: int, k: int, seed: int = 0) -> np.ndarray:
    """n uint64 keys, each uniform over k distinct values drawn uniformly
    from [0, 2^64) (redrawn until distinct)."""
    rng = np.random.default_rng(seed)
    while True:
        vals = rng.integers(0, 2**64, k, dtype=np.uint64, endpoint=False)
        if np.unique(vals).size == k:
            break
    return vals[rng.integers(0, k, n)]


def one_value_mix_u64(n: int, frac_one: float = 0.9, seed: int = 0) -> np.ndarray:
    """`frac_one` of the positions (chosen at random) hold one value V0, the
    rest are uniform over [0, 2^64)."""
    rng = np.random.default_rng(seed)
    v0 = rng.integers(0, 2**64, dtype=np.uint64, endpoint=False)
    a = rng.integers(0, 2**64, n, dtype=np.uint64, endpoint=False)
    m = rng.random(n) < frac_one
    a[m] = v0
    return a


def index_payload(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.uint32)


def segment_sizes_loguniform(nseg: int, max_log2: int = 16, seed: int = 0) -> np.ndarray:
    """Segment sizes max(1, floor(2^(max_log2 * u))), u ~ U[0, 1)."""
    rng = np.random.default_rng(seed)
    u = rng.random(nseg)
    return np.maximum(1, np.floor(np.exp2(max_log2 * u))).astype(np.int64)


def offsets_from_sizes(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(sizes.size + 1, dtype=np.uint64)
    np.cumsum(sizes, out=off[1:])
    return off


def segmented_f32(nseg: int, max_log2: int = 16, dup_frac: float = 0.05,
                  signed_zeros: int = 1 << 10, seed: int = 0):
    """Segmented float32 workload: log-uniform segment sizes, N(0, 1) keys,
    `dup_frac` of the positions of each segment copy another key of the same
    segment, `signed_zeros` positions are set to -0.0 and as many to +0.0.
    Returns (keys f32, offsets u64 of length nseg+1, payload u32)."""
    rng = np.random.default_rng(seed)
    sizes = segment_sizes_loguniform(nseg, max_log2, seed)
    off = offsets_from_sizes(sizes)
    total = int(off[-1])
    keys = rng.standard_normal(total, dtype=np.float32)
    # duplicates: position j takes the key of a random position of its segment
    ndup = int(total * dup_frac)
    if ndup and total:
        pos = rng.integers(0, total, ndup)
        seg = np.searchsorted(off, pos, side="right") - 1
        lo = off[seg].astype(np.int64)
        sz = (off[seg + 1] - off[seg]).astype(np.int64)
        src = lo + (rng.random(ndup) * sz).astype(np.int64)
        keys[pos] = keys[src]
    if signed_zeros and total:
        z = rng.choice(total, size=min(total, 2 * signed_zeros), replace=False)
        keys[z[: z.size // 2]] = np.float32(-0.0)
        keys[z[z.size // 2:]] = np.float32(0.0)
    return keys, off, index_payload(total)


def lognormal_u64(n: int, mu: float = 20.0, sigma: float = 3.0, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = np.rint(rng.lognormal(mu, sigma, n))
    x = np.clip(x, 0.0, float(2**64 - 2**11))
    return x.astype(np.uint64)


def zipf_cdf(s: float = 1.1, ranks: int = 1 << 24) -> np.ndarray:
    """Cumulative probabilities of Zipf(s) over ranks 1..`ranks` (float64)."""
    w = np.arange(1, ranks + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return cdf


def zipf_uniforms(n: int, seed: int = 0) -> np.ndarray:
    """The uniform draws behind zipf_u64 (same seed, same stream)."""
    return np.random.default_rng(seed).random(n)


def zipf_u64(n: int, s: float = 1.1, ranks: int = 1 << 24, seed: int = 0) -> np.ndarray:
    """Zipf(s) over ranks 1..`ranks`, drawn by inverse CDF; key = rank."""
    cdf = zipf_cdf(s, ranks)
    u = zipf_uniforms(n, seed)
    r = np.searchsorted(cdf, u, side="right") + 1
    return np.minimum(r, ranks).astype(np.uint64)


def gmm_u64(n: int, comps: int = 8, grid_log2: int = 40, seed: int = 0) -> np.ndarray:
    """Mixture of `comps` Gaussians on [0, 1) quantised to a 2^grid_log2 grid."""
    rng = np.random.default_rng(seed)
    w = rng.dirichlet(np.ones(comps))
    mu = rng.uniform(0.05, 0.95, comps)
    sd = np.exp(rng.uniform(np.log(1e-4), np.log(1e-2), comps))
    c = rng.choice(comps, size=n, p=w)
    x = rng.standard_normal(n) * sd[c] + mu[c]
    x = np.clip(x, 0.0, 1.0 - 2.0 ** (-grid_log2))
    return np.floor(x * float(2**grid_log2)).astype(np.uint64)


def key_dtype(key_type: str):
    return {"u32": np.uint32, "i32": np.int32, "f32": np.float32, "u64": np.uint64, "i64": np.int64,
            "f64": np.float64}[key_type]


def random_keys(key_type: str, n: int, seed: int = 0) -> np.ndarray:
    """Uniform random keys of a given type; float keys are N(0, 1) with a few
    signed zeros and infinities mixed in (never NaN)."""
    rng = np.random.default_rng(seed)
    if key_type == "u32":
        return rng.integers(0, 2**32, n, dtype=np.uint32)
    if key_type == "i32":
        return rng.integers(-(2**31), 2**31, n, dtype=np.int32)
    if key_type == "u64":
        return rng.integers(0, 2**64, n, dtype=np.uint64, endpoint=False)
    if key_type == "f32":
        a = rng.standard_normal(n, dtype=np.float32)
        if n >= 8:
            idx = rng.choice(n, size=8, replace=False)
            a[idx] = np.array([0.0, -0.0, np.inf, -np.inf, 0.0, -0.0, 1e-45, -1e-45], dtype=np.float32)
        return a
    if key_type == "i64":
        return rng.integers(-(2**63), 2**63, n, dtype=np.int64, endpoint=False)
    if key_type == "f64":
        a = rng.standard_normal(n)
        if n >= 8:
            idx = rng.choice(n, size=8, replace=False)
            a[idx] = np.array([0.0, -0.0, np.inf, -np.inf, 0.0, -0.0, 5e-324, -5e-324])
        return a
    raise ValueError(key_type)
