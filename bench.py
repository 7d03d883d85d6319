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
    ap.add_argument("--cpu-log2n", type=int, default=25, help="oracle sample size; 0 skips it")
    ap.add_argument("--mode", default="sort", choices=("sort", "orp", "copy"),
                    help="copy: a plain device copy of the input (counter calibration)")
    ap.add_argument("--batched-count", type=int, default=4096,
                    help="instances of the batched workload (log-uniform 2^10..2^20, 16 B, total <= 2^28); 0 skips")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="measured requests of the serving workload (log-uniform 2^12..2^24, 16 B, Poisson); 0 skips")
    ap.add_argument("--serving-warmup", type=int, default=200,
                    help="requests before the measured ones in every serving trace (not counted)")
    ap.add_argument("--serving-loads", default="0.5,0.7,0.9",
                    help="offered load as a fraction of the sequential server's capacity")
    ap.add_argument("--sweep-steps", type=int, default=2,
                    help="steps per (Z, k) point of the n=2^28 sweep; 0 skips the sweep")
    ap.add_argument("--sweep-seeds", type=int, default=100,
                    help="ORP seeds per Z for the overflow-retry count")
    ap.add_argument("--dup-steps", type=int, default=10,
                    help="steps of the duplicate-heavy 2^24 x 16 B leg (bucket and bitonic sort); 0 skips it")
    ap.add_argument("--ooc-steps", type=int, default=1,
                    help="timed calls of the out-of-core ORP and sort (headline workload in host memory); 0 skips")
    ap.add_argument("--ooc-dev-gib", type=float, default=2.0,
                    help="device workspace of the out-of-core calls, GiB")
    ap.add_argument("--tuning", default="",
                    help="tuning table for the batched and serving legs (default: the stored table)")
    return ap.parse_args()


def cpu_model():
    """The host CPU's model name (/proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


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


def per_kind(launches, steps):
    kinds = {}
    for l in launches:
        d = kinds.setdefault(l["kind"], [0, 0.0, 0])
        d[0] += 1
        d[1] += l["ms"]
        d[2] += l["bytes"]
    return {k: {"ms_per_step": round(v[1] / steps, 3), "avg_ms": round(v[1] / v[0], 4),
                "GB/s": round(v[2] / v[1] / 1e6, 1), "frac_of_peak": round(v[2] / v[1] / 1e6 / HBM_PEAK_GBS, 4)}
            for k, v in kinds.items()}


def bench_sweep(args, torch, bos, x, out):
    """Z in {256, 512, 1024} x k in {2, 3, 4} at the resident input: ms per
    bos_sort and per bos_orp, per-pass GB/s; then bos_orp over seeds 1..S per Z
    with the retries they needed.  Z = 256 is below the 80-bit floor at this n
    (Lemma 3.2 gives about 2^-36), so the sweep runs with the floor off."""
    from paper_2008_01765_amd import autotune

    stream = torch.cuda.current_stream()
    res = {"points": [], "overflow": []}
    n = x.shape[0]
    for z in (256, 512, 1024):
        for k in (2, 3, 4):
            pt = {"z": z, "k": k}
            for mode, fn in (("sort", bos.sort), ("orp", bos.orp)):
                try:
                    fn(x, seed=args.seed, z=z, k=k, out=out, min_security_bits=0)
                except bos.BosError as e:
                    pt[mode] = {"error": str(e)}
                    continue
                torch.cuda.synchronize()
                bos.profile_enable(True)
                bos.profile_read()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                reps = []
                for _ in range(args.sweep_steps):
                    reps.append(fn(x, seed=args.seed, z=z, k=k, out=out, min_security_bits=0, report=True)[1])
                e1.record(stream)
                torch.cuda.synchronize()
                kinds = per_kind(bos.profile_read(), args.sweep_steps)
                bos.profile_enable(False)
                ms = e0.elapsed_time(e1) / args.sweep_steps
                pt[mode] = {"ms": round(ms, 3), "Melem/s": round(n / ms / 1e3, 1), "passes": reps[-1]["passes"],
                            "k_used": reps[-1]["k"], "kernels": kinds}
            res["points"].append(pt)
            print("sweep: %s" % json.dumps({"z": z, "k": k, "sort_ms": pt.get("sort", {}).get("ms"),
                                            "orp_ms": pt.get("orp", {}).get("ms")}), file=sys.stderr, flush=True)
    for z in (256, 512, 1024):
        retries = failed = 0
        t0 = time.perf_counter()
        for sd in range(1, args.sweep_seeds + 1):
            try:
                _, rep = bos.orp(x, seed=sd, z=z, out=out, min_security_bits=0, max_retries=3, report=True)
                retries += rep["attempts"] - 1
            except bos.BosError:
                failed += 1
        res["overflow"].append({"z": z, "seeds": args.sweep_seeds, "retries": retries, "failed": failed,
                                "log2_eps_bound": round(autotune.log2_eps(n, z), 1),
                                "s": round(time.perf_counter() - t0, 1)})
    return res


def bench_dup(args, torch, bos, inputs):
    """The duplicate-heavy workload: n = 2^24 records of 16 B, keys uniform on
    [0, 2^20) (ties broken by the payload), Z = 512, data seed 42.  bos_sort
    and the bitonic sort of the same resident records, each timed with HIP
    events over `dup_steps` calls after one warm call; outputs compared."""
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    x = bos.from_numpy(inputs.workload_dup(args.data_seed), dev)
    n = x.shape[0]
    out = torch.empty_like(x)
    bout = torch.empty_like(x)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.dup_steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.dup_steps

    res = {"workload": "n=2^24 records of 16 B, key uniform on [0, 2^20), payload=index, Z=512", "n": n,
           "tuning": args.tuning_used}
    for label, kw in (("tuned", {}), ("k3_tile4096", {"k": 3, "tile": 4096})):
        ms = timed(lambda: bos.sort(x, seed=args.seed, z=512, out=out, **kw))
        res["bucket_" + label] = {"ms": round(ms, 3), "Melem/s": round(n / ms / 1e3, 1)}
    bms = timed(lambda: bos.bitonic_sort(x, out=bout))
    best = min(res["bucket_tuned"]["ms"], res["bucket_k3_tile4096"]["ms"])
    res["bitonic"] = {"ms": round(bms, 3), "Melem/s": round(n / bms / 1e3, 1)}
    res["speedup_of_bucket_sort"] = round(bms / best, 3)
    res["equal_output"] = bool(torch.equal(out, bout))
    del x, out, bout
    bos.release_workspaces()
    torch.cuda.empty_cache()
    return res


def bench_ooc(args, torch, bos, inputs):
    """Out-of-core bucket ORP and sort (Section 4.3) of the headline workload
    held in pinned host memory, streamed through a device workspace of
    `ooc_dev_gib` GiB; beside them the pinned host<->device copy rates."""
    import numpy as np

    n = 1 << args.log2n
    rec = args.rec
    dt = torch.int32 if rec == 8 else torch.int64
    a = inputs.records(n, rec, args.data_seed)
    host_in = bos.pinned_empty((n, 2), dt)
    host_in.numpy()[:] = a.view(np.int32 if rec == 8 else np.int64)
    del a
    host_out = bos.pinned_empty((n, 2), dt)
    p = bos.params(args.seed, args.z, args.k, args.tile)
    import ctypes as C
    hws = bos.pinned_empty((bos.lib().bos_host_workspace_bytes(n, rec, C.byref(p)),), torch.uint8)
    dev_bytes = int(args.ooc_dev_gib * (1 << 30))
    stream = torch.cuda.current_stream()
    # copy rates of the host link (pinned, 1 GiB each way)
    blk = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    hblk = bos.pinned_empty((1 << 30,), torch.uint8)
    rates = {}
    for name, fn in (("h2d", lambda: blk.copy_(hblk, non_blocking=True)),
                     ("d2h", lambda: hblk.copy_(blk, non_blocking=True))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        rates[name + "_GB/s"] = round(3 * (1 << 30) / (time.perf_counter() - t0) / 1e9, 1)
    # both directions at once (two streams), the ceiling of a pass that
    # streams its slot arrays in and out together
    blk2 = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    hblk2 = bos.pinned_empty((1 << 30,), torch.uint8)
    s_in, s_out = torch.cuda.Stream(), torch.cuda.Stream()

    def both():
        with torch.cuda.stream(s_in):
            blk.copy_(hblk, non_blocking=True)
        with torch.cuda.stream(s_out):
            hblk2.copy_(blk2, non_blocking=True)

    both()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        both()
    torch.cuda.synchronize()
    rates["both_directions_GB/s"] = round(3 * 2 * (1 << 30) / (time.perf_counter() - t0) / 1e9, 1)
    del blk, hblk, blk2, hblk2
    res = {"workload": "n=2^%d records of %d B in pinned host memory, Z=%d" % (args.log2n, rec, args.z),
           "device_workspace_GiB": args.ooc_dev_gib, "host_link": rates}
    bz = None
    for mode, fn in (("orp", bos.orp_host), ("sort", bos.sort_host)):
        kw = {"z": args.z, "k": args.k, "out": host_out, "host_ws": hws, "dev_ws_bytes": dev_bytes}
        if mode == "sort":
            kw["tile"] = args.tile
        _, rep = fn(host_in, seed=args.seed, report=True, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.ooc_steps):
            fn(host_in, seed=args.seed, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.ooc_steps
        bz = rep["buckets"] * rep["z"]
        # bytes over the host link per call: every routing pass reads and writes
        # the slot arrays (the first reads the n records, the last writes the
        # bins' records), then the finish or strip reads the bins and writes n
        # records; the sort's comparison phase reads and writes them twice more
        link = (n * rec + 2 * (rep["passes"] - 1) * bz * (rec + 4) + bz * (rec + 4) + bz * rec
                + bz * rec + n * rec)
        if mode == "sort":
            link += 4 * n * rec
        res[mode] = {"ms": round(ms, 1), "Melem/s": round(n / ms / 1e3, 1), "passes": rep["passes"],
                     "attempts": rep["attempts"], "host_link_bytes": int(link),
                     "host_link_GB/s": round(link / ms / 1e6, 1)}
    res["sorted"] = bool(np.all(np.diff(host_out.numpy()[:, 0].view(np.uint32 if rec == 8 else np.uint64)
                                        .astype(np.float64)) >= 0))
    del host_in, host_out, hws
    bos.release_workspaces()
    torch.cuda.empty_cache()
    return res


def install_tuning(args, bos):
    """Install the autotuner's table (z, k, tile = 0 then resolve per size class)."""
    from paper_2008_01765_amd import autotune

    path = args.tuning or autotune.DEFAULT_TABLE
    if not os.path.exists(path):
        bos.set_tuning([])
        return None
    autotune.install(path=path)
    return os.path.relpath(path, ROOT)


def bench_batched(args, torch, bos, inputs):
    """4096 independent sorts of log-uniform sizes in one bos_sort_batched call
    (graph replay) against the same instances sorted one call each, all with
    Z, k and tile from the tuning table per size class."""
    import numpy as np

    dev = torch.device("cuda", 0)
    sizes = inputs.batched_sizes(args.batched_count, 10, 20, 1 << 28, seed=4242)
    total = int(sizes.sum())
    master = bos.from_numpy(inputs.records(total, 16, args.data_seed + 1), dev)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    ins = [master[int(o):int(o) + int(n)] for o, n in zip(offs, sizes)]
    outm = torch.empty_like(master)
    outs = [outm[int(o):int(o) + int(n)] for o, n in zip(offs, sizes)]
    seeds = list(range(len(ins)))
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, (time.perf_counter() - t0) * 1e3 / reps

    batched_ms, batched_wall = timed(lambda: bos.sort_batched(ins, seeds, outs=outs), args.batched_steps)
    sorted_ok = True
    chk = bos.to_numpy(outm)
    for o, n in zip(offs, sizes):
        seg = chk[int(o):int(o) + int(n)]
        if n > 1:
            k = seg[:, 0]
            p = seg[:, 1]
            if not bool(np.all((k[1:] > k[:-1]) | ((k[1:] == k[:-1]) & (p[1:] >= p[:-1])))):
                sorted_ok = False
                break
    del chk

    def plain(sync):
        for t, o, sd in zip(ins, outs, seeds):
            bos.sort(t, seed=sd, out=o, sync=sync)

    _, sync_wall = timed(lambda: plain(True), 1)
    _, async_wall = timed(lambda: plain(False), 1)
    res = {"instances": len(ins), "total_records": total, "rec_bytes": 16, "tuning": args.tuning_used,
           "sizes": "log-uniform 2^10..2^20, rescaled to total <= 2^28",
           "batched_ms": round(batched_wall, 3), "batched_gpu_ms": round(batched_ms, 3),
           "batched_Melem/s": round(total / batched_wall / 1e3, 1),
           "plain_sync_ms": round(sync_wall, 3), "plain_async_ms": round(async_wall, 3),
           "speedup_vs_plain_sync": round(sync_wall / batched_wall, 2),
           "speedup_vs_plain_async": round(async_wall / batched_wall, 2), "correct": sorted_ok}
    del ins, outs, master, outm
    bos.release_workspaces()
    torch.cuda.empty_cache()
    return res


def bench_serving(args, torch, bos, inputs):
    """Poisson arrivals of sort requests (log-uniform 2^12..2^24 records of
    16 B) served by the continuous-batching server and by a first-come
    first-served loop of single sorts, on the same arrival trace, at each
    offered load (a fraction of the sequential capacity).  Every trace has
    `serving_warmup` requests before the `serving_requests` measured ones."""
    import numpy as np

    from paper_2008_01765_amd import serving

    dev = torch.device("cuda", 0)
    total_req = args.serving_warmup + args.serving_requests
    sizes = inputs.request_sizes(total_req, 12, 24, seed=7)
    master_n = 1 << 25
    master = bos.from_numpy(inputs.records(master_n, 16, args.data_seed + 2), dev)
    starts = (inputs.splitmix64(99, 0, len(sizes)) % np.uint64(master_n - (1 << 24) + 1)).astype(np.int64)
    reqs = [master[int(s0):int(s0) + int(n)] for s0, n in zip(starts, sizes)]
    # sequential capacity: every request sorted alone, back to back (warm)
    big = int(np.argmax(sizes))
    bos.sort(reqs[big], seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, r in enumerate(reqs):
        bos.sort(r, seed=i)
    torch.cuda.synchronize()
    busy = time.perf_counter() - t0
    # closed loop: every request submitted at once (this also warms the
    # allocator for the server's outputs and workspaces)
    srv = serving.Server(hbm_budget_bytes=64 << 30)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    futs = [srv.submit(r, seed=i) for i, r in enumerate(reqs)]
    srv.run_until_idle()
    torch.cuda.synchronize()
    closed = time.perf_counter() - t0
    ok = all(f.status == bos.OK for f in futs)
    closed_steps = srv.steps
    del futs, srv
    meas = slice(args.serving_warmup, total_req)
    measured_records = int(sizes[meas].sum())

    def summary(lat, fin, arr):
        span = max(fin[meas]) - min(arr[meas])
        return {"p50_ms": round(serving.percentile(lat[meas], 50) * 1e3, 3),
                "p99_ms": round(serving.percentile(lat[meas], 99) * 1e3, 3),
                "Melem/s": round(measured_records / span / 1e6, 1)}

    loads = {}
    for rho in [float(v) for v in args.serving_loads.split(",") if v]:
        rate = rho * len(reqs) / busy
        arr = serving.poisson_arrivals(len(reqs), rate, seed=11)
        srv = serving.Server(hbm_budget_bytes=64 << 30)
        futs = serving.run_trace(srv, reqs, arr)
        t_b = futs[0].arrival - arr[0]  # the trace's clock origin
        lat_b = [f.latency for f in futs]
        fin_b = [f.finished - t_b for f in futs]
        ok = ok and all(f.status == bos.OK for f in futs)
        steps, peak = srv.steps, srv.peak_used
        del futs, srv  # the outputs
        lat_s, _ = serving.run_trace_sequential(reqs, arr, keep_outputs=False)
        fin_s = [a + l for a, l in zip(arr, lat_s)]
        loads["%.2g" % rho] = {"rate_req_s": round(rate, 1), "steps": steps,
                               "peak_resident_GiB": round(peak / 2 ** 30, 2),
                               "batching": summary(lat_b, fin_b, arr), "sequential": summary(lat_s, fin_s, arr)}
        bos.release_workspaces()
    res = {"requests": args.serving_requests, "warmup_requests": args.serving_warmup, "rec_bytes": 16,
           "sizes": "log-uniform 2^12..2^24", "tuning": args.tuning_used,
           "arrivals": "Poisson at rho x the sequential capacity (%.1f req/s at rho = 1)" % (len(reqs) / busy),
           "hbm_budget_GiB": 64,
           "closed_loop": {"sequential_ms": round(busy * 1e3, 1), "batching_ms": round(closed * 1e3, 1),
                           "batching_steps": closed_steps},
           "loads": loads, "correct": ok}
    del reqs, master
    bos.release_workspaces()
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
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
        # per-kernel times in a separate profiled call (events around every launch)
        bos.profile_enable(True)
        bos.profile_read()
        bos.bitonic_sort(x, out=bout)
        torch.cuda.synchronize()
        bkinds = per_kind(bos.profile_read(), 1)
        bos.profile_enable(False)
        bit = {"ms_per_step": round(bms, 3), "Melem/s": round(n / bms / 1e3, 1), "equal_output": same,
               "speedup_of_bucket_sort": round(bms / ms_per_step, 3),
               "kernels": bkinds}
        del bout

    sweep = None
    if args.sweep_steps > 0 and args.mode == "sort" and args.log2n == 28 and args.rec == 8:
        sweep = bench_sweep(args, torch, bos, x, out)

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
               "host": os.uname().nodename, "nproc": os.cpu_count(), "cpu_model": cpu_model()}

    batched = None
    args.tuning_used = None
    if (args.batched_count > 0 or args.serving_requests > 0 or args.dup_steps > 0) and args.mode == "sort":
        args.tuning_used = install_tuning(args, bos)
    ooc = None
    if args.ooc_steps > 0 and args.mode == "sort":
        ooc = bench_ooc(args, torch, bos, inputs)
        print("ooc: %s" % json.dumps(ooc), file=sys.stderr, flush=True)
    dup = None
    if args.dup_steps > 0 and args.mode == "sort":
        dup = bench_dup(args, torch, bos, inputs)
        print("dup: %s" % json.dumps(dup), file=sys.stderr, flush=True)
    if args.batched_count > 0 and args.mode == "sort":
        batched = bench_batched(args, torch, bos, inputs)
        print("batched: %s" % json.dumps(batched), file=sys.stderr, flush=True)
    served = None
    if args.serving_requests > 0 and args.mode == "sort":
        served = bench_serving(args, torch, bos, inputs)
        print("serving: %s" % json.dumps(served), file=sys.stderr, flush=True)

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
        "roofline": roof, "cpu_baseline": cpu, "bitonic": bit, "dup_workload": dup, "out_of_core": ooc, "batched": batched, "serving": served, "sweep": sweep,
        "kernels": kern,
        "kernel_sources": kernel_source_digest(),
    }
    print(json.dumps(line), flush=True)
    if not ok or (batched and not batched["correct"]) or (served and not served["correct"]):
        sys.exit(1)


if __name__ == "__main__":
    main()
