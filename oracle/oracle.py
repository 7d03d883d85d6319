"""ctypes wrapper of the single-threaded C++ oracle (test infrastructure only).

Functions mirror ``bos_oracle.h``; arrays are numpy arrays of shape (n, 2) with
dtype uint32 (8-byte records) or uint64 (16-byte records), column 0 the key and
column 1 the payload.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "bos_oracle.cpp")

OK, INVALID, OVERFLOW = 0, 1, 2
ARR_X, ARR_LEVEL0, ARR_Y, ARR_T = 0, 1, 100, 101


def build(force=True):
    """Compile liboracle.so with g++ (plain -O2, single-threaded code)."""
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-Wall", "-Wextra",
                           "-o", tmp, SRC])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Cfg(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("z", C.c_uint32), ("max_retries", C.c_uint32),
                ("b_override", C.c_uint64), ("label_override", C.POINTER(C.c_uint32)),
                ("trace", C.POINTER(C.c_uint64)), ("trace_cap", C.c_uint64)]


class Report(C.Structure):
    _fields_ = [("buckets", C.c_uint64), ("levels", C.c_uint32), ("attempts", C.c_uint32),
                ("first_overflow_level", C.c_int32), ("pad_", C.c_int32),
                ("first_overflow_pair", C.c_int64), ("accesses_orp", C.c_uint64),
                ("accesses_sort", C.c_uint64), ("digest_orp", C.c_uint64),
                ("digest_sort", C.c_uint64), ("trace_len", C.c_uint64),
                ("sec_labels", C.c_double), ("sec_route", C.c_double),
                ("sec_finish", C.c_double), ("sec_sort", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad_"}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        u64p = C.POINTER(C.c_uint64)
        L.bos_oracle_plan.argtypes = [C.c_uint64, C.c_uint32, u64p, C.POINTER(C.c_uint32)]
        L.bos_oracle_plan.restype = C.c_int
        L.bos_oracle_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.bos_oracle_philox4x64_10.restype = None
        L.bos_oracle_label.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32]
        L.bos_oracle_label.restype = C.c_uint32
        L.bos_oracle_shuffle_key.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64]
        L.bos_oracle_shuffle_key.restype = C.c_uint64
        for fn in (L.bos_oracle_orp, L.bos_oracle_sort):
            fn.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32, C.POINTER(Cfg),
                           C.POINTER(Report)]
            fn.restype = C.c_int
        L.bos_oracle_levels.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.POINTER(Cfg),
                                        C.c_uint32, C.c_void_p, C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.bos_oracle_levels.restype = C.c_int
        L.bos_oracle_merge_sort.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32]
        L.bos_oracle_merge_sort.restype = C.c_int
        _lib = L
    return _lib


def _rec_bytes(a):
    a = np.ascontiguousarray(a)
    if a.ndim != 2 or a.shape[1] != 2 or a.dtype not in (np.uint32, np.uint64):
        raise ValueError("records must be an (n, 2) uint32 or uint64 array")
    return a, 8 if a.dtype == np.uint32 else 16


def plan(n, z):
    b, l = C.c_uint64(), C.c_uint32()
    rc = lib().bos_oracle_plan(n, z, C.byref(b), C.byref(l))
    if rc != OK:
        raise ValueError("invalid plan")
    return b.value, l.value


def philox4x64_10(ctr, key):
    c = (C.c_uint64 * 4)(*ctr)
    k = (C.c_uint64 * 2)(*key)
    o = (C.c_uint64 * 4)()
    lib().bos_oracle_philox4x64_10(c, k, o)
    return list(o)


def label(seed, attempt, i, levels):
    return lib().bos_oracle_label(seed, attempt, i, levels)


def shuffle_key(seed, attempt, g):
    return lib().bos_oracle_shuffle_key(seed, attempt, g)


def _cfg(seed, z, max_retries, b_override, labels, trace_cap):
    cfg = Cfg(seed=seed, z=z, max_retries=max_retries, b_override=b_override)
    keep = []
    if labels is not None:
        lab = np.ascontiguousarray(labels, dtype=np.uint32)
        keep.append(lab)
        cfg.label_override = lab.ctypes.data_as(C.POINTER(C.c_uint32))
    trace = None
    if trace_cap:
        trace = np.zeros(trace_cap, dtype=np.uint64)
        keep.append(trace)
        cfg.trace = trace.ctypes.data_as(C.POINTER(C.c_uint64))
        cfg.trace_cap = trace_cap
    return cfg, trace, keep


def _run(fn, recs, seed, z, max_retries, b_override, labels, trace_cap):
    a, rec = _rec_bytes(recs)
    out = np.zeros_like(a)
    cfg, trace, _keep = _cfg(seed, z, max_retries, b_override, labels, trace_cap)
    rep = Report()
    rc = fn(a.ctypes.data, out.ctypes.data, a.shape[0], rec, C.byref(cfg), C.byref(rep))
    if rc == INVALID:
        raise ValueError("oracle rejected the arguments")
    res = {"rc": rc, "out": out if rc == OK else None, "report": rep.as_dict()}
    if trace is not None:
        res["trace"] = trace[:min(rep.trace_len, trace_cap)]
    return res


def orp(recs, seed, z=512, max_retries=3, b_override=0, labels=None, trace_cap=0):
    """Bucket ORP (Section 3.2).  Returns dict(rc, out, report[, trace])."""
    return _run(lib().bos_oracle_orp, recs, seed, z, max_retries, b_override, labels, trace_cap)


def sort(recs, seed, z=512, max_retries=3, b_override=0, labels=None, trace_cap=0):
    """Bucket oblivious sort (Section 3.3).  Returns dict(rc, out, report[, trace])."""
    return _run(lib().bos_oracle_sort, recs, seed, z, max_retries, b_override, labels, trace_cap)


def levels(recs, seed, z=512, attempt=0, b_override=0, labels=None):
    """All level arrays of one attempt of Algorithm 3.1.

    Returns dict(rc, recs=(L+1, B, Z, 2) array, tags=(L+1, B, Z) uint32,
    overflow=(level, pair)).
    """
    a, rec = _rec_bytes(recs)
    B, L = plan(a.shape[0], z)
    if b_override:
        B, L = b_override, int(b_override).bit_length() - 1
    rbuf = np.zeros((L + 1, B, z, 2), dtype=a.dtype)
    tbuf = np.zeros((L + 1, B, z), dtype=np.uint32)
    cfg, _, _keep = _cfg(seed, z, 0, b_override, labels, 0)
    ol, op = C.c_int32(), C.c_int64()
    rc = lib().bos_oracle_levels(a.ctypes.data, a.shape[0], rec, C.byref(cfg), attempt,
                                 rbuf.ctypes.data, tbuf.ctypes.data_as(C.POINTER(C.c_uint32)),
                                 C.byref(ol), C.byref(op))
    if rc == INVALID:
        raise ValueError("oracle rejected the arguments")
    return {"rc": rc, "recs": rbuf, "tags": tbuf, "overflow": (ol.value, op.value)}


def merge_sort(recs):
    a, rec = _rec_bytes(recs)
    out = np.zeros_like(a)
    rc = lib().bos_oracle_merge_sort(a.ctypes.data, out.ctypes.data, a.shape[0], rec)
    if rc != OK:
        raise ValueError("oracle rejected the arguments")
    return out


def decode_trace(codes):
    """Split access codes into (write flag, array id, index) numpy arrays."""
    codes = np.asarray(codes, dtype=np.uint64)
    write = (codes >> np.uint64(63)).astype(bool)
    arr = ((codes >> np.uint64(56)) & np.uint64(0x7F)).astype(np.int64)
    idx = (codes & np.uint64((1 << 56) - 1)).astype(np.int64)
    return write, arr, idx
