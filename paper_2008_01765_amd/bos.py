"""Python binding of libbos (include/bos.h): argument marshalling only.

Every step of the method runs in the gfx950 kernels of libbos.so; this module
turns torch CUDA tensors into device pointers, sizes workspaces and maps status
codes to exceptions.  There is no CPU fallback: if libbos.so is missing or no
GPU is present the calls raise.

Record tensors have shape (n, 2) on a CUDA device: int32 columns for 8-byte
records {u32 key, u32 payload}, int64 columns for 16-byte records
{u64 key, u64 payload}; the bits are taken as unsigned.
"""
import contextlib
import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbos.so")
# the same library built with BOS_TRACE_DIGEST (address digests; tests only)
TRACE_LIB_PATH = os.path.join(HERE, "libbos_trace.so")

OK, INVALID_ARG, OVERFLOW, WORKSPACE, HIP_ERR, INSECURE_Z, UNSUPPORTED, INTERNAL = range(8)
SYNC = 1
GENERIC_ROUTING = 2
EXACT_FINISH = 4
STRICT = 8


class BosError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


class Params(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("z", C.c_uint32), ("k", C.c_uint32), ("tile", C.c_uint32),
                ("max_retries", C.c_uint32), ("min_security_bits", C.c_uint32), ("flags", C.c_uint32),
                ("attempt", C.c_uint32)]


class Report(C.Structure):
    _fields_ = [("attempts", C.c_uint32), ("z", C.c_uint32), ("k", C.c_uint32), ("tile", C.c_uint32),
                ("levels", C.c_uint32), ("passes", C.c_uint32), ("first_overflow_level", C.c_int32),
                ("reserved", C.c_int32), ("first_overflow_pair", C.c_int64), ("buckets", C.c_uint64),
                ("algorithmic_bytes", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class Instance(C.Structure):
    _fields_ = [("in_", C.c_void_p), ("out", C.c_void_p), ("n", C.c_uint64), ("seed", C.c_uint64)]


class Job(C.Structure):
    _fields_ = [("in_", C.c_void_p), ("out", C.c_void_p), ("n", C.c_uint64), ("seed", C.c_uint64),
                ("ws", C.c_void_p), ("ws_bytes", C.c_size_t), ("phase", C.c_uint32), ("attempt", C.c_uint32),
                ("status", C.c_uint32), ("reserved", C.c_uint32)]


PHASE_DONE = 0xFFFFFFFF


class TuneEntry(C.Structure):
    _fields_ = [("rec", C.c_uint32), ("log2n", C.c_uint32), ("z", C.c_uint32), ("k", C.c_uint32),
                ("tile", C.c_uint32), ("reserved", C.c_uint32)]


class LaunchTime(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("index", C.c_uint32), ("ms", C.c_float), ("reserved", C.c_uint32),
                ("bytes", C.c_uint64)]


KERNEL_KINDS = {1: "route_first", 2: "route_mid", 3: "route_last", 4: "route_single", 5: "sort_tile",
                6: "sort_merge", 7: "bitonic_tile", 8: "bitonic_global", 9: "bitonic_tail", 10: "other",
                11: "strip", 12: "orp_finish"}

EXPORTS = ["bos_default_params", "bos_workspace_bytes", "bos_orp", "bos_sort", "bos_batched_workspace_bytes",
           "bos_sort_batched", "bos_bitonic_workspace_bytes", "bos_bitonic_sort", "bos_release_cache",
           "bos_status_string", "bos_debug_levels", "bos_debug_labels", "bos_plan", "bos_profile_enable",
           "bos_profile_read", "bos_step_workspace_bytes", "bos_sort_step", "bos_set_tuning", "bos_get_tuning",
           "bos_stepper_create", "bos_stepper_destroy", "bos_sort_step_async", "bos_sort_noalloc",
           "bos_status_offset", "bos_trace_bind", "bos_host_workspace_bytes", "bos_host_device_bytes",
           "bos_orp_host", "bos_sort_host"]

_lib = None
_loaded = {}


def lib():
    """Load libbos.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        _lib = _load(LIB_PATH)
    return _lib


@contextlib.contextmanager
def using_library(path):
    """Run the calls of this module through another build of the library
    (e.g. TRACE_LIB_PATH) inside the block."""
    global _lib
    prev = _lib
    _lib = _load(path)
    try:
        yield _lib
    finally:
        _lib = prev


def _load(path):
    if path in _loaded:
        return _loaded[path]
    if not os.path.exists(path):
        raise RuntimeError("%s is not built; run python -m paper_2008_01765_amd.build" % os.path.basename(path))
    L = C.CDLL(path)
    P, R = C.POINTER(Params), C.POINTER(Report)
    vp, u64, u32 = C.c_void_p, C.c_uint64, C.c_uint32
    L.bos_default_params.argtypes = [P]
    L.bos_default_params.restype = None
    L.bos_workspace_bytes.argtypes = [u64, C.c_int, P]
    L.bos_workspace_bytes.restype = C.c_size_t
    L.bos_status_offset.argtypes = [u64, C.c_int, P]
    L.bos_status_offset.restype = C.c_size_t
    L.bos_trace_bind.argtypes = [vp, vp, u64]
    L.bos_trace_bind.restype = C.c_int
    for fn in (L.bos_orp, L.bos_sort):
        fn.argtypes = [vp, vp, u64, C.c_int, P, vp, C.c_size_t, vp, R]
        fn.restype = C.c_int
    for fn in (L.bos_orp_host, L.bos_sort_host):
        fn.argtypes = [vp, vp, u64, C.c_int, P, vp, C.c_size_t, vp, C.c_size_t, vp, R]
        fn.restype = C.c_int
    for fn in (L.bos_host_workspace_bytes, L.bos_host_device_bytes):
        fn.argtypes = [u64, C.c_int, P]
        fn.restype = C.c_size_t
    L.bos_sort_noalloc.argtypes = [vp, vp, u64, C.c_int, P, vp, R]
    L.bos_sort_noalloc.restype = C.c_int
    L.bos_batched_workspace_bytes.argtypes = [C.POINTER(u64), u32, C.c_int, P]
    L.bos_batched_workspace_bytes.restype = C.c_size_t
    L.bos_sort_batched.argtypes = [C.POINTER(Instance), u32, C.c_int, P, vp, C.c_size_t, vp, vp, R]
    L.bos_sort_batched.restype = C.c_int
    L.bos_step_workspace_bytes.argtypes = [u32]
    L.bos_step_workspace_bytes.restype = C.c_size_t
    L.bos_sort_step.argtypes = [C.POINTER(Job), u32, C.c_int, P, vp, C.c_size_t, vp]
    L.bos_sort_step.restype = C.c_int
    L.bos_stepper_create.argtypes = []
    L.bos_stepper_create.restype = vp
    L.bos_stepper_destroy.argtypes = [vp]
    L.bos_stepper_destroy.restype = None
    L.bos_sort_step_async.argtypes = [vp, C.POINTER(Job), u32, C.c_int, P, vp, C.c_size_t, vp]
    L.bos_sort_step_async.restype = C.c_int
    L.bos_set_tuning.argtypes = [C.POINTER(TuneEntry), u32]
    L.bos_set_tuning.restype = C.c_int
    L.bos_get_tuning.argtypes = [C.POINTER(TuneEntry), u32]
    L.bos_get_tuning.restype = u32
    L.bos_bitonic_workspace_bytes.argtypes = [u64, C.c_int]
    L.bos_bitonic_workspace_bytes.restype = C.c_size_t
    L.bos_bitonic_sort.argtypes = [vp, vp, u64, C.c_int, vp, C.c_size_t, vp]
    L.bos_bitonic_sort.restype = C.c_int
    L.bos_release_cache.argtypes = []
    L.bos_release_cache.restype = None
    L.bos_status_string.argtypes = [C.c_int]
    L.bos_status_string.restype = C.c_char_p
    L.bos_debug_levels.argtypes = [vp, u64, C.c_int, P, u32, vp, C.c_size_t, vp, vp, vp, vp,
                                   C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
    L.bos_debug_levels.restype = C.c_int
    L.bos_debug_labels.argtypes = [u64, u32, u64, u32, vp, vp]
    L.bos_debug_labels.restype = C.c_int
    L.bos_plan.argtypes = [u64, C.c_int, P, C.POINTER(u64), C.POINTER(u32), C.POINTER(u32)]
    L.bos_plan.restype = C.c_int
    L.bos_profile_enable.argtypes = [C.c_int]
    L.bos_profile_enable.restype = None
    L.bos_profile_read.argtypes = [C.POINTER(LaunchTime), u32]
    L.bos_profile_read.restype = u32
    _loaded[path] = L
    return L


def _check(st):
    if st != OK:
        raise BosError(st, "libbos: " + lib().bos_status_string(st).decode())


def params(seed=0, z=0, k=0, tile=0, max_retries=3, min_security_bits=80, sync=True, generic=False,
           exact_finish=False, attempt=0, strict=False):
    p = Params()
    lib().bos_default_params(C.byref(p))
    p.attempt = attempt
    p.seed = seed & 0xFFFFFFFFFFFFFFFF
    p.z, p.k, p.tile = z, k, tile
    p.max_retries = max_retries
    p.min_security_bits = min_security_bits
    p.flags = (SYNC if sync else 0) | (GENERIC_ROUTING if generic else 0) | (EXACT_FINISH if exact_finish else 0) | \
        (STRICT if strict else 0)
    return p


def rec_bytes(t):
    if t.dim() != 2 or t.shape[1] != 2 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("records must be a contiguous (n, 2) CUDA tensor")
    if t.dtype == torch.int32:
        return 8
    if t.dtype == torch.int64:
        return 16
    raise ValueError("records must be int32 (8-byte) or int64 (16-byte) pairs")


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


_ws_cache = {}


def workspace(nbytes, device=None):
    """A cached device byte buffer of at least nbytes."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    buf = _ws_cache.get(dev)
    if buf is None or buf.numel() < nbytes:
        _ws_cache.pop(dev, None)
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
        _ws_cache[dev] = buf
    return buf


def release_workspaces():
    _ws_cache.clear()
    lib().bos_release_cache()


def workspace_bytes(n, rec, p):
    nb = lib().bos_workspace_bytes(n, rec, C.byref(p))
    if nb == 0:
        # the planner's own status says why (bos_plan runs the same planner)
        b, l = C.c_uint64(), C.c_uint32()
        passes = (C.c_uint32 * 33)()
        _check(lib().bos_plan(n, rec, C.byref(p), C.byref(b), C.byref(l), passes))
        raise BosError(INVALID_ARG, "libbos: no workspace size for these arguments")
    return nb


def _run(fn, t, p, out, stream):
    rec = rec_bytes(t)
    n = t.shape[0]
    if out is None:
        out = torch.empty_like(t)
    ws = workspace(workspace_bytes(n, rec, p), t.device)
    rep = Report()
    st = fn(C.c_void_p(t.data_ptr()), C.c_void_p(out.data_ptr()), n, rec, C.byref(p),
            C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream), C.byref(rep))
    _check(st)
    return out, rep.as_dict()


def orp(t, seed=0, z=0, k=0, max_retries=3, min_security_bits=80, out=None, stream=None, report=False,
        generic=False, exact_finish=False, sync=True, attempt=0, strict=False):
    """Bucket ORP of the records in t (Section 3.2).  With sync=False the call
    enqueues attempt `attempt` alone and leaves its overflow status on the
    device (status_word)."""
    p = params(seed, z, k, 0, max_retries, min_security_bits, sync=sync, generic=generic,
               exact_finish=exact_finish, attempt=attempt, strict=strict)
    o, rep = _run(lib().bos_orp, t, p, out, stream)
    return (o, rep) if report else o


def sort(t, seed=0, z=0, k=0, tile=0, max_retries=3, min_security_bits=80, out=None, stream=None,
         report=False, generic=False, sync=True, attempt=0, strict=False):
    """Bucket oblivious sort of the records in t (Section 3.3).  With
    sync=False the call does not wait for the overflow check (attempt
    `attempt` alone, stream-ordered); status_word reads its outcome."""
    p = params(seed, z, k, tile, max_retries, min_security_bits, sync=sync, generic=generic, attempt=attempt,
               strict=strict)
    o, rep = _run(lib().bos_sort, t, p, out, stream)
    return (o, rep) if report else o


def status_word(t, z=0, k=0, tile=0, min_security_bits=80):
    """The overflow status word (Algorithm 3.1's abort) that the last
    bos_orp / bos_sort call on t's shape left in the cached workspace: None if
    the attempt did not overflow, else (level, pair).  Synchronizes."""
    rec = rec_bytes(t)
    n = t.shape[0]
    p = params(0, z, k, tile, 3, min_security_bits)
    off = lib().bos_status_offset(n, rec, C.byref(p))
    if off == 2 ** 64 - 1 or off == C.c_size_t(-1).value:
        raise BosError(INVALID_ARG, "libbos: no status word for these arguments")
    ws = workspace(workspace_bytes(n, rec, p), t.device)
    w = int(ws[off:off + 8].cpu().view(torch.int64).item()) & 0xFFFFFFFFFFFFFFFF
    if w == 0xFFFFFFFFFFFFFFFF:
        return None
    return (w >> 32, w & 0xFFFFFFFF)


def host_rec_bytes(t):
    if t.dim() != 2 or t.shape[1] != 2 or t.is_cuda or not t.is_contiguous():
        raise ValueError("records must be a contiguous (n, 2) host tensor")
    if t.dtype == torch.int32:
        return 8
    if t.dtype == torch.int64:
        return 16
    raise ValueError("records must be int32 (8-byte) or int64 (16-byte) pairs")


def pinned_empty(shape, dtype):
    """A host tensor in pinned memory (copied at full DMA rate)."""
    return torch.empty(shape, dtype=dtype, pin_memory=True)


def _run_host(fn, t, p, out, host_ws, dev_ws_bytes, stream):
    rec = host_rec_bytes(t)
    n = t.shape[0]
    if out is None:
        out = pinned_empty(t.shape, t.dtype)
    hb = lib().bos_host_workspace_bytes(n, rec, C.byref(p))
    db = lib().bos_host_device_bytes(n, rec, C.byref(p))
    if hb == 0 or db == 0:
        raise BosError(INVALID_ARG, "libbos: no out-of-core workspace size for these arguments")
    if host_ws is None or host_ws.numel() < hb:
        host_ws = pinned_empty((hb,), torch.uint8)
    db = max(db, dev_ws_bytes or 0)
    dws = workspace(db)  # (the cached buffer may be larger; the call gets db bytes of it)
    rep = Report()
    _check(fn(C.c_void_p(t.data_ptr()), C.c_void_p(out.data_ptr()), n, rec, C.byref(p),
              C.c_void_p(host_ws.data_ptr()), host_ws.numel(), C.c_void_p(dws.data_ptr()), db,
              _stream(stream), C.byref(rep)))
    return out, rep.as_dict()


def orp_host(t, seed=0, z=0, k=0, max_retries=3, min_security_bits=80, out=None, host_ws=None, dev_ws_bytes=0,
             stream=None, report=False, exact_finish=False):
    """Out-of-core bucket ORP (Section 4.3) of the host records in t: the slot
    arrays stay in host memory (host_ws, pinned if None) and stream through a
    device workspace of dev_ws_bytes (at least the library's minimum).  Equals
    orp() on the same records, seed and Z."""
    p = params(seed, z, k, 0, max_retries, min_security_bits, exact_finish=exact_finish)
    o, rep = _run_host(lib().bos_orp_host, t, p, out, host_ws, dev_ws_bytes, stream)
    return (o, rep) if report else o


def sort_host(t, seed=0, z=0, k=0, tile=0, max_retries=3, min_security_bits=80, out=None, host_ws=None,
              dev_ws_bytes=0, stream=None, report=False):
    """Out-of-core bucket oblivious sort (Section 4.3) of the host records in t."""
    p = params(seed, z, k, tile, max_retries, min_security_bits)
    o, rep = _run_host(lib().bos_sort_host, t, p, out, host_ws, dev_ws_bytes, stream)
    return (o, rep) if report else o


def sort_noalloc(t, seed=0, z=0, k=0, tile=0, max_retries=3, min_security_bits=80, out=None, stream=None,
                 report=False):
    """bos_sort with the library's own workspace (bos_sort_noalloc): no
    workspace is allocated; n is limited by that workspace's 64 MiB."""
    rec = rec_bytes(t)
    n = t.shape[0]
    if out is None:
        out = torch.empty_like(t)
    p = params(seed, z, k, tile, max_retries, min_security_bits)
    rep = Report()
    _check(lib().bos_sort_noalloc(C.c_void_p(t.data_ptr()), C.c_void_p(out.data_ptr()), n, rec, C.byref(p),
                                  _stream(stream), C.byref(rep)))
    return (out, rep.as_dict()) if report else out


def sort_batched(tensors, seeds, z=0, k=0, tile=0, max_retries=3, min_security_bits=80, outs=None,
                 stream=None, report=False, sync=True, status=False):
    """Bucket oblivious sort of every tensor in `tensors` (same record type).
    With sync=False the call enqueues the first attempts and returns at once;
    status=True also returns the per-instance device status array."""
    if not tensors:
        return []
    rec = rec_bytes(tensors[0])
    for t in tensors:
        if rec_bytes(t) != rec:
            raise ValueError("all instances must use the same record type")
    if outs is None:
        outs = [torch.empty_like(t) for t in tensors]
    p = params(0, z, k, tile, max_retries, min_security_bits, sync=sync)
    cnt = len(tensors)
    arr = (Instance * cnt)()
    ns = (C.c_uint64 * cnt)()
    for i, (t, o, s) in enumerate(zip(tensors, outs, seeds)):
        arr[i].in_ = t.data_ptr()
        arr[i].out = o.data_ptr()
        arr[i].n = t.shape[0]
        arr[i].seed = s & 0xFFFFFFFFFFFFFFFF
        ns[i] = t.shape[0]
    nb = lib().bos_batched_workspace_bytes(ns, cnt, rec, C.byref(p))
    ws = workspace(nb, tensors[0].device)
    dstat = torch.zeros(cnt, dtype=torch.int32, device=tensors[0].device)
    rep = Report()
    st = lib().bos_sort_batched(arr, cnt, rec, C.byref(p), C.c_void_p(ws.data_ptr()), ws.numel(),
                                _stream(stream), C.c_void_p(dstat.data_ptr()), C.byref(rep))
    _check(st)
    res = (outs, rep.as_dict()) if report else outs
    return (res, dstat) if status else res


def sort_step(jobs, rec, p, step_ws, stream=None, count_left=True):
    """Advance the unfinished Jobs in the ctypes array `jobs` by one step
    (bos_sort_step); returns the number of jobs still unfinished (None with
    count_left=False)."""
    count = len(jobs)
    _check(lib().bos_sort_step(jobs, count, rec, C.byref(p), C.c_void_p(step_ws.data_ptr()), step_ws.numel(),
                               _stream(stream)))
    if not count_left:
        return None
    return sum(1 for j in jobs if j.phase != PHASE_DONE)


def step_workspace_bytes(count):
    return lib().bos_step_workspace_bytes(count)


class Stepper:
    """A pipelined sequence of steps (bos_stepper): each step() call enqueues
    one step and collects the previous one (bos_sort_step_async)."""

    def __init__(self):
        self._h = lib().bos_stepper_create()
        if not self._h:
            raise BosError(UNSUPPORTED, "libbos: bos_stepper_create failed")

    def step(self, jobs, rec, p, step_ws, stream=None):
        """One call of bos_sort_step_async over the ctypes Job array `jobs`;
        step_ws must hold 2 * step_workspace_bytes(len(jobs)) bytes."""
        _check(lib().bos_sort_step_async(self._h, jobs, len(jobs), rec, C.byref(p),
                                         C.c_void_p(step_ws.data_ptr() if step_ws is not None else 0),
                                         step_ws.numel() if step_ws is not None else 0, _stream(stream)))

    def close(self):
        if self._h:
            lib().bos_stepper_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_tuning(entries):
    """Install the tuning table: dicts {rec, log2n, z, k, tile} (bos_set_tuning)."""
    arr = (TuneEntry * max(1, len(entries)))()
    for i, e in enumerate(entries):
        arr[i].rec, arr[i].log2n = int(e["rec"]), int(e["log2n"])
        arr[i].z, arr[i].k, arr[i].tile = int(e.get("z", 0)), int(e.get("k", 0)), int(e.get("tile", 0))
    _check(lib().bos_set_tuning(arr, len(entries)))


def get_tuning():
    cnt = lib().bos_get_tuning(None, 0)
    arr = (TuneEntry * max(1, cnt))()
    lib().bos_get_tuning(arr, cnt)
    return [{"rec": e.rec, "log2n": e.log2n, "z": e.z, "k": e.k, "tile": e.tile} for e in arr[:cnt]]


def bitonic_sort(t, out=None, stream=None):
    """Oblivious bitonic sort of the records in t (the GPU baseline)."""
    rec = rec_bytes(t)
    n = t.shape[0]
    if out is None:
        out = torch.empty_like(t)
    nb = lib().bos_bitonic_workspace_bytes(n, rec)
    ws = workspace(nb, t.device)
    _check(lib().bos_bitonic_sort(C.c_void_p(t.data_ptr()), C.c_void_p(out.data_ptr()), n, rec,
                                  C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))
    return out


def profile_enable(on=True):
    """Bracket every kernel launch with HIP events (see profile_read)."""
    lib().bos_profile_enable(1 if on else 0)


def profile_read():
    """Per-launch records logged since the last read: list of dicts with kind,
    index, ms and algorithmic bytes."""
    cap = 1 << 16
    buf = (LaunchTime * cap)()
    cnt = lib().bos_profile_read(buf, cap)
    return [{"kind": KERNEL_KINDS.get(buf[i].kind, str(buf[i].kind)), "index": buf[i].index,
             "ms": buf[i].ms, "bytes": buf[i].bytes} for i in range(min(cnt, cap))]


def plan(n, rec, z=0, k=0, tile=0, min_security_bits=80, strict=False):
    p = params(0, z, k, tile, 3, min_security_bits, strict=strict)
    b, l = C.c_uint64(), C.c_uint32()
    passes = (C.c_uint32 * 33)()
    _check(lib().bos_plan(n, rec, C.byref(p), C.byref(b), C.byref(l), passes))
    return {"buckets": b.value, "levels": l.value, "passes": list(passes[1:1 + passes[0]])}


def debug_labels(n, levels, seed, attempt=0, device="cuda"):
    out = torch.empty(max(n, 1), dtype=torch.int32, device=device)
    _check(lib().bos_debug_labels(n, levels, seed & 0xFFFFFFFFFFFFFFFF, attempt, C.c_void_p(out.data_ptr()),
                                  _stream(None)))
    torch.cuda.synchronize()
    return out[:n]


def debug_levels(t, seed=0, z=512, k=0, attempt=0, min_security_bits=0, generic=False):
    """Slot arrays at every pass boundary of one attempt (host numpy arrays)."""
    import numpy as np
    if not z:
        raise ValueError("debug_levels needs an explicit z")
    rec = rec_bytes(t)
    n = t.shape[0]
    p = params(seed, z, k, 0, 0, min_security_bits, generic=generic)
    pl = plan(n, rec, z=z, k=k, min_security_bits=min_security_bits)
    B, Z = pl["buckets"], z
    P = len(pl["passes"])
    dt = np.uint32 if rec == 8 else np.uint64
    recs = np.zeros((P + 1, B, Z, 2), dtype=dt)
    tags = np.zeros((P + 1, B, Z), dtype=np.uint32)
    lv = np.zeros(P + 1, dtype=np.uint32)
    ws = workspace(workspace_bytes(n, rec, p), t.device)
    ol, op = C.c_int32(), C.c_int64()
    st = lib().bos_debug_levels(C.c_void_p(t.data_ptr()), n, rec, C.byref(p), attempt, C.c_void_p(ws.data_ptr()),
                                ws.numel(), _stream(None), recs.ctypes.data, tags.ctypes.data, lv.ctypes.data,
                                C.byref(ol), C.byref(op))
    if st not in (OK, OVERFLOW):
        _check(st)
    # boundaries 1..P-1 follow passes 0..P-2 (the last pass strips instead)
    return {"rc": st, "recs": recs[:P], "tags": tags[:P], "levels": lv[:P], "overflow": (ol.value, op.value)}


def to_numpy(t):
    """Records of a CUDA tensor as an unsigned numpy array (n, 2)."""
    import numpy as np
    a = t.cpu().numpy()
    return a.view(np.uint32) if a.dtype == np.int32 else a.view(np.uint64)


def from_numpy(a, device="cuda"):
    """An unsigned numpy record array (n, 2) as a CUDA tensor."""
    import numpy as np
    a = np.ascontiguousarray(a)
    v = a.view(np.int32) if a.dtype == np.uint32 else a.view(np.int64)
    return torch.from_numpy(v).to(device)
