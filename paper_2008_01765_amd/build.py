"""Build libbos.so (gfx950) in-tree with hipcc.

    python -m paper_2008_01765_amd.build
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libbos.so")
TRACE_LIB = os.path.join(PKG, "libbos_trace.so")  # BOS_TRACE_DIGEST build (address digests, tests)
SOURCES = (["orp_kernels.hip", "route_kernels.hip", "sort_kernels.hip", "strip_kernels.hip", "bos_api.hip"]
           + ["route_r%d_z%d.hip" % (r, z) for r in (8, 16) for z in range(4, 12)])
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            # no packed FP32 instructions in device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _headers_mtime():
    t = 0.0
    for d in (CSRC, os.path.join(ROOT, "include")):
        for f in os.listdir(d):
            if f.endswith(".h"):
                t = max(t, os.path.getmtime(os.path.join(d, f)))
    return t


def build(verbose=False, jobs=None, force=True, trace=True):
    """Compile every HIP source and link libbos.so, then (trace=True) the
    same sources with BOS_TRACE_DIGEST into libbos_trace.so.  force=False
    recompiles only objects older than their source or any header."""
    out = _build_one(LIB, "_build", [], verbose, jobs, force)
    if trace:
        _build_one(TRACE_LIB, "_build_trace", ["-DBOS_TRACE_DIGEST"], verbose, jobs, force)
    return out


def _build_one(lib, objdir, extra, verbose, jobs, force):
    if jobs is None:
        jobs = max(1, min(16, os.cpu_count() or 4))
    objs = []
    procs = []
    hdr = _headers_mtime()
    for src in SOURCES:
        obj = os.path.join(CSRC, objdir, src.replace(".hip", ".o"))
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        objs.append(obj)
        if not force and os.path.exists(obj) and \
                os.path.getmtime(obj) >= max(hdr, os.path.getmtime(os.path.join(CSRC, src))):
            continue
        cmd = [HIPCC] + flags() + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    while procs:
        _wait(procs.pop(0))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    if p.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, text))
    lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if lines:
        print("\n".join(lines), file=sys.stderr)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, force="--changed" not in sys.argv, trace="--no-trace" not in sys.argv))
