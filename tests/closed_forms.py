"""Closed forms and library routes that pin the oracle (and, through it, the GPU
path) to the paper rather than to itself.

Everything here is derived from the paper's statements, not from the oracle's
code:
  * random numbers come from numpy.random.Philox (an independent Philox4x64-10),
  * bucket membership at every level comes from the closed form implied by the
    index formula of Algorithm 3.1 and the invariant stated under Figure 1
    (after i levels, each aligned run of 2^i buckets is partitioned by the top
    i label bits): element x with initial group s and label l sits, at level
    i, in bucket 2^i * floor(s / 2^i) + floor(l / 2^(L-i)),
  * the access sequence comes from the simulator of Lemma 3.3 (a fixed routing
    pattern plus the loads of the final bins).
"""
import numpy as np
from numpy.random import Philox

M64 = (1 << 64) - 1


def philox_blocks(key0, key1, ctr1, first, count):
    """Philox4x64-10 blocks for counters (first .. first+count-1, ctr1, 0, 0) as an
    array of shape (count, 4) of uint64, computed by numpy."""
    c = first | (ctr1 << 64)
    c = (c - 1) % (1 << 256)  # numpy advances the counter before each block
    ctr = np.array([(c >> (64 * t)) & M64 for t in range(4)], dtype=np.uint64)
    g = Philox(key=np.array([key0 & M64, key1 & M64], dtype=np.uint64), counter=ctr)
    return g.random_raw(4 * count).reshape(count, 4)


def labels(seed, attempt, n, L):
    """Label of each element 0..n-1: the top L bits of 32-bit word (i mod 8) of
    the block with counter (i // 8, attempt)."""
    if n == 0:
        return np.zeros(0, dtype=np.uint32)
    if L == 0:
        return np.zeros(n, dtype=np.uint32)
    nb = (n + 7) // 8
    w = philox_blocks(seed, 0, attempt, 0, nb).reshape(-1)  # 4 u64 per block
    words32 = np.empty(8 * nb, dtype=np.uint32)
    words32[0::2] = (w & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    words32[1::2] = (w >> np.uint64(32)).astype(np.uint32)
    return (words32[:n] >> np.uint32(32 - L)).astype(np.uint32)


def shuffle_keys(seed, attempt, first_g, count):
    """64-bit keys r(g) for g = first_g .. first_g+count-1."""
    if count == 0:
        return np.zeros(0, dtype=np.uint64)
    b0 = first_g // 4
    b1 = (first_g + count - 1) // 4
    w = philox_blocks(seed, 1, attempt, b0, b1 - b0 + 1).reshape(-1)
    off = first_g - 4 * b0
    return w[off:off + count]


def is_pow2(x):
    return x >= 1 and (x & (x - 1)) == 0


def group_of(n, B):
    """Initial group s(x) of every element under the balanced floor split."""
    starts = (np.arange(B, dtype=object) * n // B).astype(np.int64)
    return np.searchsorted(starts, np.arange(n), side="right") - 1


def bucket_at_level(s, lab, L, i):
    """Closed-form bucket index at level i."""
    s = s.astype(np.int64)
    t = (lab.astype(np.int64) >> (L - i)) if i > 0 else np.zeros_like(s)
    return ((s >> i) << i) + t


def expected_level(recs, lab, B, L, Z, i):
    """Level-i array by the closed form: each bucket holds its elements in
    increasing original index, then dummies (record 0, tag 0xFFFFFFFF).
    Returns (recs (B, Z, 2), tags (B, Z), overflow flag)."""
    n = recs.shape[0]
    s = group_of(n, B)
    b = bucket_at_level(s, lab, L, i)
    order = np.lexsort((np.arange(n), b))  # by bucket, then index
    bs = b[order]
    counts = np.bincount(bs, minlength=B) if n else np.zeros(B, dtype=np.int64)
    if counts.max(initial=0) > Z:
        return None, None, True
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    slot = np.arange(n) - starts[bs] if n else np.zeros(0, dtype=np.int64)
    R = np.zeros((B, Z, 2), dtype=recs.dtype)
    T = np.full((B, Z), 0xFFFFFFFF, dtype=np.uint32)
    R[bs, slot] = recs[order]
    T[bs, slot] = lab[order]
    return R, T, False


def first_overflow(n, lab, B, L, Z):
    """First overflowing MergeSplit (level i, pair j) by the closed form, i.e. the
    smallest (i, j) such that an output bucket 2j or 2j+1 of level i+1 holds more
    than Z elements; (-1, -1) if none."""
    if n == 0:
        return (-1, -1)
    s = group_of(n, B)
    for lev in range(1, L + 1):
        b = bucket_at_level(s, lab, L, lev)
        counts = np.bincount(b, minlength=B)
        over = np.nonzero(counts > Z)[0]
        if over.size:
            return (lev - 1, int(over.min()) // 2)
    return (-1, -1)


def expected_orp(recs, seed, attempt, lab, B, Z):
    """ORP output: bins 0..B-1 (bin = label) concatenated; each bin's elements are
    put in record order and then ordered by (r(b*Z + p), p)."""
    out = []
    key = recs[:, 0].astype(np.uint64)
    pay = recs[:, 1].astype(np.uint64)
    for b in range(B):
        idx = np.nonzero(lab == b)[0]
        if idx.size == 0:
            continue
        o = idx[np.lexsort((pay[idx], key[idx]))]
        r = shuffle_keys(seed, attempt, b * Z, idx.size)
        perm = np.lexsort((np.arange(idx.size), r))
        out.append(recs[o[perm]])
    if not out:
        return np.zeros((0, 2), dtype=recs.dtype)
    return np.concatenate(out)


def _ordered_i64(col):
    """A uint32 or uint64 numpy column as int64 values with the same order."""
    if col.dtype == np.uint32:
        return col.astype(np.int64)
    return (col.view(np.int64) ^ np.int64(-(1 << 63)))


def expected_orp_vec(recs, seed, attempt, lab, B, Z, device="cpu"):
    """expected_orp by whole-array library sorts (torch's stable sort), for
    sizes where the per-bin loop is too slow: group the elements by bin (=
    label) in record order, give the p-th element of bin b the key
    r(b*Z + p), and order each bin by (r, p).  Returns a numpy array."""
    import torch

    n = recs.shape[0]
    if n == 0:
        return np.zeros((0, 2), dtype=recs.dtype)
    dev = torch.device(device)
    key = torch.from_numpy(_ordered_i64(recs[:, 0])).to(dev)
    pay = torch.from_numpy(_ordered_i64(recs[:, 1])).to(dev)
    lb = torch.from_numpy(lab.astype(np.int64)).to(dev)
    idx = torch.argsort(pay, stable=True)
    idx = idx[torch.argsort(key[idx], stable=True)]
    idx = idx[torch.argsort(lb[idx], stable=True)]
    del key, pay
    lab_s = lb[idx]
    del lb
    counts = torch.bincount(lab_s, minlength=B)
    off = torch.cumsum(counts, 0) - counts
    p = torch.arange(n, device=dev) - off[lab_s]
    g = lab_s * Z + p
    nblk = (int(B) * int(Z) + 3) // 4
    rk = philox_blocks(seed, 1, attempt, 0, nblk).reshape(-1)
    r_all = torch.from_numpy(_ordered_i64(rk)).to(dev)
    del rk
    r = r_all[g]
    del r_all, g, p
    idx2 = torch.argsort(r, stable=True)
    idx2 = idx2[torch.argsort(lab_s[idx2], stable=True)]
    order = idx[idx2].cpu().numpy()
    return recs[order]


def sorted_records(recs):
    """Library sort by (key, payload), unsigned."""
    o = np.lexsort((recs[:, 1], recs[:, 0]))
    return recs[o]


def loads(lab, B):
    return np.bincount(lab.astype(np.int64), minlength=B)


def sim_orp_trace(n, Z, B, L, bin_loads):
    """Lemma 3.3's simulator for one successful attempt: the fixed routing
    pattern of Algorithm 3.1 followed by the strip, whose writes depend on the
    loads alone.  Returns (write flags, array ids, indices)."""
    W, A, I = [], [], []

    def acc(w, a, idx):
        W.append(np.full(len(idx), w, dtype=bool))
        A.append(np.full(len(idx), a, dtype=np.int64))
        I.append(np.asarray(idx, dtype=np.int64))

    zs = np.arange(Z)
    for j in range(B):
        lo, hi = j * n // B, (j + 1) * n // B
        acc(False, 0, np.arange(lo, hi))
        acc(True, 1, j * Z + zs)
    for i in range(L):
        for j in range(B // 2):
            jp = (j >> i) << i
            b0, b1 = jp + j, jp + j + (1 << i)
            acc(False, 1 + i, b0 * Z + zs)
            acc(False, 1 + i, b1 * Z + zs)
            acc(True, 2 + i, 2 * j * Z + zs)
            acc(True, 2 + i, (2 * j + 1) * Z + zs)
    off = 0
    for b in range(B):
        acc(False, 1 + L, b * Z + zs)
        acc(True, 100, np.arange(off, off + bin_loads[b]))
        off += bin_loads[b]
    return np.concatenate(W), np.concatenate(A), np.concatenate(I)
