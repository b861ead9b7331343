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
# device code: never let the compiler form packed fp32 ops
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops"]
SOURCES = ["salo_kernels.hip", "salo_plan.hip", "salo_pack.hip", "salo_host.cpp"]


def _compile(src: str, obj: str) -> None:
    path = src if os.path.isabs(src) else os.path.join(CSRC, src)
    cmd = [HIPCC] + COMMON
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
        with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
            list(ex.map(lambda so: _compile(*so), zip(srcs, objs)))
        out_tmp = target + ".tmp%d" % os.getpid()
        subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH,
                        "-o", out_tmp] + objs, check=True)
        os.replace(out_tmp, target)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    if verbose:
        print("built", target)
    return target


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    args = ap.parse_args(argv)
    build(args.jobs)
    return 0


if __name__ == "__main__":
    sys.exit(main())
