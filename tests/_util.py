"""Helpers shared by the GPU tests (no sorting arithmetic here)."""
import numpy as np

M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def bits64(a: np.ndarray) -> np.ndarray:
    """Raw key bits widened to uint64 (so every key type hashes alike)."""
    if a.dtype.itemsize == 4:
        return a.view(np.uint32).astype(np.uint64)
    return a.view(np.uint64)


def multiset_hash(keys: np.ndarray, vals: np.ndarray | None = None, chunk: int = 1 << 24):
    """Order-independent (sum, xor) of splitmix64 over keys (and payloads)."""
    s = np.uint64(0)
    x = np.uint64(0)
    for i in range(0, keys.size, chunk):
        k = bits64(keys[i:i + chunk])
        if vals is not None:
            v = vals[i:i + chunk].astype(np.uint64)
            k = k ^ ((v << np.uint64(17)) | (v >> np.uint64(47)))
        h = splitmix64(k)
        with np.errstate(over="ignore"):
            s = np.uint64(s + np.add.reduce(h, dtype=np.uint64))
        x = np.uint64(x ^ np.bitwise_xor.reduce(h))
    return int(s), int(x)


def as_bytes(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a).view(np.uint8)
