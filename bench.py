#!/usr/bin/env python3
"""Benchmark of bucket oblivious sort on one MI355X.

A step is one bucket oblivious sort (Section 3.3 of Asharov et al.) of the
whole workload: the bucket ORP's routing passes (labels, butterfly levels with
overflow check, per-bin oblivious sort, strip) followed by the comparison sort,
on n = 2^28 synthetic 8-byte records {u32 key uniform, u32 payload = index},
Z = 512.  Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  Besides the contract fields it carries:
  roofline     the dominant kernel's algorithmic bytes per launch over its
               average launch time (HIP events around every launch of the
               timed steps, on the launch stream), against 8 TB/s HBM;
  cpu_baseline the single-threaded CPU oracle on a bounded sample;
  bitonic      the project's oblivious bitonic sort of the same records;
  kernels      per-kernel-kind averages.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
PROFILES = os.path.join(ROOT, "profiles")


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--rec", type=int, default=8, choices=(8, 16))
    ap.add_argument("--z", type=int, default=512)
    ap.add_argument("--k", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--data-seed", type=int, default=42)
    ap.add_argument("--bitonic-steps", type=int, default=2, help="0 skips the bitonic baseline")
    ap.add_argument("--cpu-log2n", type=int, default=24, help="oracle sample size; 0 skips it")
    ap.add_argument("--mode", default="sort", choices=("sort", "orp", "copy"),
                    help="copy: a plain device copy of the input (counter calibration)")
    return ap.parse_args()


def kernel_source_digest():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2008_01765_amd", "csrc"))):
        if not f.endswith((".h", ".hip")):
            continue
        with open(os.path.join(ROOT, "paper_2008_01765_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kind, config_tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this
    kernel, or None when absent or taken on different kernel sources."""
    path = os.path.join(PROFILES, "%s_%s_pmc.md" % (kind, config_tag))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"kernel_sources:\s*([0-9a-f]+)", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_src or not m_b or m_src.group(1) != kernel_source_digest():
        return None
    return float(m_b.group(1))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    from paper_2008_01765_amd import bos, inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda", 0)
    n = 1 << args.log2n

    # ---- synthetic input, resident in HBM -----------------------------------
    host = inputs.records(n, args.rec, args.data_seed)
    x = bos.from_numpy(host, dev)
    out = torch.empty_like(x)
    del host
    stream = torch.cuda.current_stream()

    if args.mode == "copy":
        for _ in range(args.warmup + args.steps):
            out.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_per_copy": 2 * n * args.rec, "copies": args.warmup + args.steps}))
        return

    def step():
        if args.mode == "sort":
            return bos.sort(x, seed=args.seed, z=args.z, k=args.k, tile=args.tile, out=out, report=True)
        return bos.orp(x, seed=args.seed, z=args.z, k=args.k, out=out, report=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    bos.profile_enable(True)
    bos.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    reps = []
    for _ in range(args.steps):
        _, rep = step()
        reps.append(rep)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches = bos.profile_read()
    bos.profile_enable(False)
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    wall_ms_per_step = wall * 1e3 / args.steps

    # ---- result check (sorted + same multiset) -------------------------------
    ok = True
    if args.mode == "sort":
        k64 = out[:, 0].to(torch.int64) & 0xFFFFFFFF if args.rec == 8 else out[:, 0]
        p64 = out[:, 1].to(torch.int64) & 0xFFFFFFFF if args.rec == 8 else out[:, 1]
        if args.rec == 8:
            comp = ((k64 << 32) | p64) ^ (-(2 ** 63))  # unsigned order as signed
            ok = bool((comp[1:] >= comp[:-1]).all().item()) if n > 1 else True
            del comp
        else:
            ku = k64 ^ (-(2 ** 63))
            pu = p64 ^ (-(2 ** 63))
            ok = bool(((ku[1:] > ku[:-1]) | ((ku[1:] == ku[:-1]) & (pu[1:] >= pu[:-1]))).all().item())
    s_in = int((x.to(torch.int64) * 0x9E3779B1).sum().item())
    s_out = int((out.to(torch.int64) * 0x9E3779B1).sum().item())
    ok = ok and s_in == s_out

    # ---- per-kernel averages and the dominant kernel --------------------------
    kinds = {}
    for l in launches:
        d = kinds.setdefault(l["kind"], {"launches": 0, "ms": 0.0, "bytes": 0})
        d["launches"] += 1
        d["ms"] += l["ms"]
        d["bytes"] += l["bytes"]
    kern = {}
    for kname, d in kinds.items():
        avg_ms = d["ms"] / d["launches"]
        per_launch = d["bytes"] / d["launches"]
        kern[kname] = {"launches_per_step": d["launches"] / args.steps, "avg_ms": round(avg_ms, 4),
                       "bytes_per_launch": int(per_launch), "GB/s": round(per_launch / avg_ms / 1e6, 1),
                       "ms_per_step": round(d["ms"] / args.steps, 3)}
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"]) if kern else None
    cfg_tag = "n2p%d_r%d_z%d" % (args.log2n, args.rec, args.z)
    roof = None
    if dom:
        achieved = kern[dom]["GB/s"]
        traffic = traffic_from_profile(dom, cfg_tag)
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "bytes_per_launch": kern[dom]["bytes_per_launch"]}

    # ---- bitonic baseline on the same records ---------------------------------
    bit = None
    if args.bitonic_steps > 0 and args.mode == "sort":
        bout = torch.empty_like(x)
        bos.bitonic_sort(x, out=bout)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.bitonic_steps):
            bos.bitonic_sort(x, out=bout)
        e1.record(stream)
        torch.cuda.synchronize()
        bms = e0.elapsed_time(e1) / args.bitonic_steps
        same = bool(torch.equal(bout, out))
        bit = {"ms_per_step": round(bms, 3), "Melem/s": round(n / bms / 1e3, 1), "equal_output": same,
               "speedup_of_bucket_sort": round(bms / ms_per_step, 3)}
        del bout

    del x, out
    bos.release_workspaces()
    torch.cuda.empty_cache()

    # ---- CPU oracle on a bounded sample ---------------------------------------
    cpu = None
    if args.cpu_log2n > 0:
        import oracle
        oracle.build(force=False)
        cn = 1 << args.cpu_log2n
        sample = inputs.records(cn, args.rec, args.data_seed)
        t0 = time.perf_counter()
        r = (oracle.sort if args.mode == "sort" else oracle.orp)(sample, args.seed, z=args.z)
        dt = time.perf_counter() - t0
        cpu = {"value": round(cn / dt / 1e6, 3), "unit": "Melem/s", "cores": 1, "kind": "oracle",
               "sample": "first 2^%d records of the same workload (same generator, seed, Z), one %s "
                         "call, %.1f s" % (args.cpu_log2n, args.mode, dt),
               "phases_s": {k: round(r["report"][k], 3) for k in ("sec_labels", "sec_route", "sec_finish",
                                                                  "sec_sort")},
               "host": os.uname().nodename, "nproc": os.cpu_count()}

    rep = reps[-1]
    value = n / ms_per_step / 1e3  # Melem/s
    line = {
        "metric": "Melem/s & HBM GB/s (%peak) at n=2^28 vs GPU bitonic; batched/plain; p99 ms",
        "value": round(value, 2), "unit": "Melem/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "wall_ms_per_step": round(wall_ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32" if args.rec == 8 else "u64",
        "data": "synthetic: splitmix64 keys, payload = index",
        "config": {"workload": "bucket oblivious %s of n=2^%d records of %d B (uniform key, payload=index), Z=%d"
                               % (args.mode, args.log2n, args.rec, args.z),
                   "n": n, "rec_bytes": args.rec, "z": rep["z"], "k": rep["k"], "levels": rep["levels"],
                   "passes": rep["passes"], "tile": rep["tile"], "parallelism": "1 GPU"},
        "attempts": rep["attempts"], "correct": ok,
        "roofline": roof, "cpu_baseline": cpu, "bitonic": bit, "kernels": kern,
        "kernel_sources": kernel_source_digest(),
    }
    print(json.dumps(line), flush=True)
    if not ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
