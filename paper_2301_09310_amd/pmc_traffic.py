"""Record the DP kernel's HBM traffic from rocprofv3 counter runs.

Inputs are four `*_counter_collection.csv` files written by rocprofv3:
(the DP kernel, or with --kernel pack_forward --dispatches 2 the packing
kernel over both character streams of one `bench.py --pack` pass)
  --fetch / --write   FETCH_SIZE and WRITE_SIZE runs of
                      `bench.py --steps 1 --warmup 0 --no-cpu-baseline`
  --cfetch / --cwrite the same counters for `bench.py --calibrate-copy BYTES`
                      (a device-to-device copy of a known size)
Each counter is scaled by the factor that makes the copy kernel's reading
equal the bytes it actually moves, and the result (bytes per launch of the
DP kernel) is stored in traffic.json under the kernel-source hash and the
workload, where bench.py looks it up.
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def per_dispatch(path, counter):
    out = collections.OrderedDict()
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
            out[key] = out.get(key, 0.0) + float(r["Counter_Value"])
    return out


def factor(path, counter, nbytes):
    vals = [v for (d, k), v in per_dispatch(path, counter).items() if "copyBuffer" in k]
    if not vals:
        raise SystemExit("no copy kernel in %s" % path)
    kib = sorted(vals)[len(vals) // 2]
    return nbytes / (kib * 1024.0), kib


def kernel_kib(path, counter, name, dispatches=1):
    vals = [v for (d, k), v in per_dispatch(path, counter).items() if name in k]
    if len(vals) < dispatches:
        raise SystemExit("fewer than %d %s dispatches in %s" % (dispatches, name, path))
    return sum(vals[-dispatches:])   # the last (timed) launches of one step


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--cfetch", required=True)
    ap.add_argument("--cwrite", required=True)
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--kernel", default="persistent_kernel")
    ap.add_argument("--workload", default="short_reads")
    ap.add_argument("--source-hash", required=True)
    ap.add_argument("--dispatches", type=int, default=1,
                    help="launches of the kernel that make up one step (summed)")
    ap.add_argument("--out", default=os.path.join(HERE, "traffic.json"))
    args = ap.parse_args(argv)
    ff, fk = factor(args.cfetch, "FETCH_SIZE", args.copy_bytes)
    fw, wk = factor(args.cwrite, "WRITE_SIZE", args.copy_bytes)
    fetch = kernel_kib(args.fetch, "FETCH_SIZE", args.kernel, args.dispatches) * 1024.0 * ff
    write = kernel_kib(args.write, "WRITE_SIZE", args.kernel, args.dispatches) * 1024.0 * fw
    table = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            table = json.load(f)
    table.setdefault(args.source_hash, {})[args.workload] = {
        "bytes_per_launch": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
        "fetch_factor": ff, "write_factor": fw, "copy_fetch_kib": fk, "copy_write_kib": wk}
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps(table[args.source_hash][args.workload]))
    return 0


if __name__ == "__main__":
    sys.exit(main())
