"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np


def bucket_sets_equal(rec_a, tag_a, rec_b, tag_b):
    """True when every bucket of two slot arrays (B, Z, 2) / (B, Z) holds the same
    multiset of real (record, tag) slots and the same number of dummies, and all
    dummies are canonical (zero record)."""
    def canon(rec, tag):
        B, Z = tag.shape
        real = tag != 0xFFFFFFFF
        bidx = np.broadcast_to(np.arange(B)[:, None], (B, Z))[real]
        t = tag[real].astype(np.uint64)
        k = rec[..., 0][real].astype(np.uint64)
        p = rec[..., 1][real].astype(np.uint64)
        o = np.lexsort((p, k, t, bidx))
        dummies_ok = bool(np.all(rec[~real] == 0))
        return bidx[o], t[o], k[o], p[o], real.sum(axis=1), dummies_ok
    a, b = canon(rec_a, tag_a), canon(rec_b, tag_b)
    return all(np.array_equal(x, y) for x, y in zip(a[:5], b[:5])) and a[5] and b[5]


def record_checksum(a):
    """Order-independent 64-bit checksum of a record array (sum and xor of a mix)."""
    with np.errstate(over="ignore"):
        k = a[:, 0].astype(np.uint64)
        p = a[:, 1].astype(np.uint64)
        z = k * np.uint64(0x9E3779B97F4A7C15) ^ (p + np.uint64(0x632BE59BD9B4E019))
        z ^= z >> np.uint64(29)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(32)
        return int(z.sum(dtype=np.uint64)), int(np.bitwise_xor.reduce(z)) if z.size else 0


def _unsigned_order_i64(col):
    """int32 / int64 record column (bits taken as unsigned) as int64 values
    with the unsigned order (torch has no 64-bit unsigned sort)."""
    import torch
    if col.dtype == torch.int32:
        return col.to(torch.int64) & 0xFFFFFFFF
    return col ^ torch.iinfo(torch.int64).min


def torch_sorted_records(t):
    """Records of a CUDA tensor sorted by (key, payload), unsigned, with torch's
    library sort."""
    import torch
    k = _unsigned_order_i64(t[:, 0])
    p = _unsigned_order_i64(t[:, 1])
    idx = torch.argsort(p, stable=True)
    idx = idx[torch.argsort(k[idx], stable=True)]
    return t[idx]


def torch_is_sorted(t):
    """True when the records of a CUDA tensor are in (key, payload) order."""
    k = _unsigned_order_i64(t[:, 0])
    p = _unsigned_order_i64(t[:, 1])
    if t.shape[0] < 2:
        return True
    ok = (k[1:] > k[:-1]) | ((k[1:] == k[:-1]) & (p[1:] >= p[:-1]))
    return bool(ok.all())
