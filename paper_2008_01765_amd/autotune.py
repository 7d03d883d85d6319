"""Autotuner of the bucket oblivious sort's parameters per size class.

For each record size and size class (n = 2^c) it times the candidates on the
GPU and keeps the fastest:

  Z     bucket capacity (Algorithm 3.1); only values whose overflow bound of
        Lemma 3.2 meets the security floor at that n are tried;
  k     butterfly levels fused per HBM pass;
  tile  records per tile of the comparison sort's first phase (1024 .. 16384).

Small classes are timed as batches of equal-size instances through
bos_sort_batched (the way many small sorts run), large ones as single
bos_sort calls.  The search is factored: (Z, k) with the default tile, then
the tile with the best (Z, k).  The table is stored as JSON and installed into
the library with bos_set_tuning; calls that leave z, k or tile at 0 then take
them from it.  bos_sort's output does not depend on the table; bos_orp's does
through Z, so callers that need a fixed permutation pass an explicit z.
"""
import json
import math
import os
import time

from . import bos, inputs

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning", "mi355x.json")

Z_CANDIDATES = (256, 512, 1024)
K_CANDIDATES = (2, 3, 4)
TILE_CANDIDATES = (1024, 2048, 4096, 8192, 16384)


def tile_candidates(rec):
    """Tile sizes of the comparison sort for this record size (a workgroup's LDS
    holds 16384 records of 8 bytes but only 8192 of 16)."""
    return tuple(t for t in TILE_CANDIDATES if not (rec == 16 and t == 16384))


def log2_eps(n, z):
    """log2 of the overflow bound B log2 B e^(-Z/6) of Lemma 3.2 (B = 2^L)."""
    L = 0
    while (1 << L) * z < 2 * n:
        L += 1
    if L == 0:
        return -math.inf
    return L + math.log2(L) - z / (6.0 * math.log(2.0))


def admissible_z(n, min_security_bits=80, candidates=Z_CANDIDATES):
    return [z for z in candidates if log2_eps(n, z) <= -min_security_bits]


def best(timings):
    """The candidate with the smallest time; ties go to the earlier one."""
    return min(timings, key=lambda kv: kv[1])[0]


def _time(fn, reps):
    import torch

    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


class Workload:
    """Device-resident inputs of one size class: one array of n records, or a
    batch of equal-size instances (slices of one array) for small n."""

    def __init__(self, rec, log2n, batch_records=1 << 22, device="cuda"):
        n = 1 << log2n
        self.n, self.rec = n, rec
        count = 1 if n >= batch_records else batch_records // n
        self.master = bos.from_numpy(inputs.records(count * n, rec, 4242 + log2n), device)
        self.outm = self.master.clone()
        self.count = count
        self.ins = [self.master[i * n:(i + 1) * n] for i in range(count)]
        self.outs = [self.outm[i * n:(i + 1) * n] for i in range(count)]

    def seconds_per_record(self, z, k, tile, reps=3):
        if self.count == 1:
            dt = _time(lambda: bos.sort(self.ins[0], seed=1, z=z, k=k, tile=tile, out=self.outs[0],
                                        min_security_bits=0), reps)
        else:
            seeds = list(range(self.count))
            dt = _time(lambda: bos.sort_batched(self.ins, seeds, z=z, k=k, tile=tile, outs=self.outs,
                                                min_security_bits=0), reps)
            bos.release_workspaces()
        return dt / (self.count * self.n)

    def seconds_or_inf(self, z, k, tile, reps=3):
        """seconds_per_record, or infinity for a combination the kernels do not
        cover (e.g. a block of 2^k Z slots beyond a workgroup's LDS)."""
        try:
            return self.seconds_per_record(z, k, tile, reps)
        except bos.BosError as e:
            if e.status != bos.UNSUPPORTED:
                raise
            return math.inf


def tune(classes_by_rec=None, min_security_bits=80, reps=3, log=print):
    """Run the search; returns the table (a list of entries)."""
    if classes_by_rec is None:
        classes_by_rec = {8: range(10, 29, 2), 16: range(10, 25, 2)}
    table = []
    for rec, classes in classes_by_rec.items():
        for c in classes:
            zs = admissible_z(1 << c, min_security_bits)
            if not zs:
                continue
            t0 = time.perf_counter()
            w = Workload(rec, c)
            zk = [((z, k), w.seconds_or_inf(z, k, 4096, reps)) for z in zs for k in K_CANDIDATES]
            z, k = best(zk)
            tl = [(t, w.seconds_or_inf(z, k, t, reps)) for t in tile_candidates(rec)]
            tile = best(tl)
            ns = min(v for _, v in tl) * 1e9
            entry = {"rec": rec, "log2n": c, "z": z, "k": k, "tile": tile, "ns_per_record": round(ns, 4),
                     "instances": w.count}
            table.append(entry)
            del w
            if log:
                log("tune rec=%d n=2^%d -> Z=%d k=%d tile=%d (%.3f ns/record, %.1f s)"
                    % (rec, c, z, k, tile, ns, time.perf_counter() - t0))
    return table


def save(table, path=DEFAULT_TABLE, device_name=None):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump({"device": device_name, "entries": table}, f, indent=1)
        f.write("\n")


def load(path=DEFAULT_TABLE):
    with open(path) as f:
        return json.load(f)["entries"]


def install(table=None, path=DEFAULT_TABLE):
    """Install a table (or the stored one) into the library; returns it."""
    if table is None:
        table = load(path)
    bos.set_tuning([{k: e[k] for k in ("rec", "log2n", "z", "k", "tile")} for e in table])
    return table


if __name__ == "__main__":
    import argparse

    import torch

    ap = argparse.ArgumentParser(description="tune Z, k and tile per size class on this GPU")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--hi8", type=int, default=28, help="largest size class for 8-byte records")
    ap.add_argument("--hi16", type=int, default=24, help="largest size class for 16-byte records")
    ap.add_argument("--lo", type=int, default=10)
    ap.add_argument("--step", type=int, default=2)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    tab = tune({8: range(args.lo, args.hi8 + 1, args.step), 16: range(args.lo, args.hi16 + 1, args.step)},
               reps=args.reps, log=lambda s: print(s, flush=True))
    save(tab, args.out, torch.cuda.get_device_name(0))
    print("wrote", args.out)
