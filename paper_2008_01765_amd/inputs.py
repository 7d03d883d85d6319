"""Seeded synthetic inputs (record arrays) shared by the tests, the benchmark
and the smoke check.

This module holds no part of the sorting or permutation method: it only draws
records.  Values come from the splitmix64 generator (Steele, Lea, Flood,
OOPSLA 2014) evaluated at the record index, so any slice of a workload can be
regenerated on its own.

A record array has shape (n, 2): column 0 is the key, column 1 the payload.
dtype uint32 gives 8-byte records, uint64 gives 16-byte records.
"""
import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed, start, count):
    """splitmix64 outputs for indices start .. start+count-1 of stream `seed`."""
    with np.errstate(over="ignore"):
        z = (np.arange(start + 1, start + count + 1, dtype=np.uint64) * GOLDEN
             + np.uint64(seed & 0xFFFFFFFFFFFFFFFF))
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def records(n, rec_bytes, data_seed, key_bits=None, chunk=1 << 24):
    """n records {key, payload = index}; key uniform on [0, 2^key_bits).

    rec_bytes 8 -> uint32 columns (key_bits <= 32, default 32);
    rec_bytes 16 -> uint64 columns (key_bits <= 64, default 64).
    """
    if rec_bytes == 8:
        dt, width = np.uint32, 32
    elif rec_bytes == 16:
        dt, width = np.uint64, 64
    else:
        raise ValueError("rec_bytes must be 8 or 16")
    kb = width if key_bits is None else key_bits
    if not 0 < kb <= width:
        raise ValueError("bad key_bits")
    out = np.empty((n, 2), dtype=dt)
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        x = splitmix64(data_seed, s, c) >> np.uint64(64 - kb)
        out[s:s + c, 0] = x.astype(dt)
        out[s:s + c, 1] = np.arange(s, s + c, dtype=dt)
    return out


# The five workloads (shapes and value distributions of the paper's setting:
# the paper's only concrete sizes are n = 2^30 records and Z = 512).
def workload_small(data_seed=42):
    """n = 2^16 records of 8 bytes, uniform u32 key, payload = index."""
    return records(1 << 16, 8, data_seed)


def workload_dup(data_seed=42):
    """n = 2^24 records of 16 bytes, key uniform on [0, 2^20) (~16 copies of each
    key value), payload = index."""
    return records(1 << 24, 16, data_seed, key_bits=20)


def workload_large(data_seed=42, n=1 << 28):
    """n = 2^28 records of 8 bytes, uniform u32 key, payload = index."""
    return records(n, 8, data_seed)


def batched_sizes(count=4096, lo_log2=10, hi_log2=20, cap=1 << 28, seed=4242):
    """Instance sizes log-uniform on [2^lo, 2^hi], rescaled until the total is at
    most `cap` (every size clamped to >= 2^lo)."""
    u = splitmix64(seed, 0, count).astype(np.float64) / 2.0 ** 64
    n = np.floor(2.0 ** (lo_log2 + u * (hi_log2 - lo_log2))).astype(np.int64)
    while n.sum() > cap:
        n = np.maximum(np.floor(n * (cap / n.sum())).astype(np.int64), 1 << lo_log2)
    return n


def request_sizes(count, lo_log2=12, hi_log2=24, seed=7):
    """Request sizes log-uniform on [2^lo, 2^hi]."""
    u = splitmix64(seed, 0, count).astype(np.float64) / 2.0 ** 64
    return np.floor(2.0 ** (lo_log2 + u * (hi_log2 - lo_log2))).astype(np.int64)
