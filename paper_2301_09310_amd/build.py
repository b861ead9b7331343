"""Build libsalo.so (the gfx950 HIP library) in-tree with hipcc.

Usage: python -m paper_2301_09310_amd.build [--jobs N]
"""
from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsalo.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC]
# device code: never let the compiler form packed fp32 ops; keep binary16
# denormals (IEEE mode): the 16-bit integer cells are compared as binary16
# numbers, and cell values 1..1023 are binary16 subnormals
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-fdenormal-fp-math=ieee"]
SOURCES = ["salo_kernels.hip", "salo_plan.hip", "salo_pack.hip", "salo_noalloc.hip",
           "salo_host.cpp"]
# the ceiling microbenchmarks: a library of their own, loaded only by bench.py
UBENCH_SOURCE = "salo_ubench.hip"
UBENCH_LIB = os.path.join(PKG, "libsalo_ubench.so")


TUNE_TABLE = os.path.join(PKG, "tune_gfx950.json")


def write_tune_table(json_path: str, out_dir: str) -> str:
    """The autotuner's record as the library's built-in bin table: writes
    salo_tune_table.inc (kDefaultBins) into out_dir."""
    import json
    with open(json_path) as f:
        rec = json.load(f)
    rows = []
    for b in rec["bins"]:
        cols = int(b.get("cols", 16))
        if cols not in (8, 16, 32) or int(b["lanes"]) not in (1, 2, 4, 8, 16, 32, 64):
            raise ValueError("bad bin in %s: %s" % (json_path, b))
        rows.append("    {%d, %d, %d, %d}," % (int(b["m_hi"]), int(b["packed"]),
                                               int(b["lanes"]), cols))
    path = os.path.join(out_dir, "salo_tune_table.inc")
    with open(path, "w") as f:
        f.write("// Written by build.py from %s (%s, %s): m_hi, packed, lanes, cols.\n"
                % (os.path.basename(json_path), rec.get("device", "?"), rec.get("date", "?")))
        f.write("const salo_bin_t kDefaultBins[] = {\n%s\n};\n" % "\n".join(rows))
    return path


def _compile(src: str, obj: str, inc: str = "") -> None:
    path = src if os.path.isabs(src) else os.path.join(CSRC, src)
    cmd = [HIPCC] + COMMON + (["-I" + inc] if inc else [])
    if src.endswith(".hip"):
        cmd += DEVICE + ["-x", "hip"]
    cmd += ["-c", path, "-o", obj]
    subprocess.run(cmd, check=True)


def build(jobs: int = 4, verbose: bool = True, out: str | None = None,
          csrc: str | None = None) -> str:
    """Compile the sources in `csrc` (default: the package's csrc/) into
    `out` (default: the package's libsalo.so)."""
    global CSRC
    if csrc:
        CSRC = csrc
    target = out or LIB
    missing = [s for s in SOURCES if not os.path.exists(os.path.join(CSRC, s))]
    if missing:
        raise FileNotFoundError("libsalo sources missing from %s: %s" % (CSRC, ", ".join(missing)))
    srcs = list(SOURCES)
    tmp = tempfile.mkdtemp(prefix="salo_build_")
    try:
        objs = [os.path.join(tmp, s + ".o") for s in srcs]
        write_tune_table(TUNE_TABLE, tmp)
        with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
            list(ex.map(lambda so: _compile(so[0], so[1], tmp), zip(srcs, objs)))
        out_tmp = target + ".tmp%d" % os.getpid()
        subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH,
                        "-o", out_tmp] + objs, check=True)
        os.replace(out_tmp, target)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    if verbose:
        print("built", target)
    if out is None:
        build_ubench(verbose)
    return target


def build_ubench(verbose: bool = True) -> str:
    """Compile the ceiling microbenchmarks into libsalo_ubench.so."""
    tmp = UBENCH_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + COMMON + DEVICE + ["-x", "hip", "-shared",
                                       os.path.join(PKG, "csrc", UBENCH_SOURCE), "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, UBENCH_LIB)
    if verbose:
        print("built", UBENCH_LIB)
    return UBENCH_LIB


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    args = ap.parse_args(argv)
    build(args.jobs)
    return 0


if __name__ == "__main__":
    sys.exit(main())
