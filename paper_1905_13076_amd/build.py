"""Build the HIP library ``libppcmh.so`` in-tree for gfx950.

    python -m paper_1905_13076_amd.build [--debug]

Compiles every ``csrc/*.hip`` translation unit with hipcc into one shared library next
to this file.  Packed-FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libppcmh.so")
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def build(debug: bool = False, verbose: bool = False) -> str:
    cc = hipcc()
    flags = [f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
    flags += ["-O0", "-g"] if debug else ["-O3"]
    fd, tmp = tempfile.mkstemp(prefix="libppcmh.", suffix=".so.tmp", dir=HERE)
    os.close(fd)
    objdir = tempfile.mkdtemp(prefix="ppcmh_obj.")
    srcs = sources()
    objs = [os.path.join(objdir, os.path.basename(f) + ".o") for f in srcs]
    compile_flags = [f for f in flags if f != "-shared"]
    cmds = [[cc, *compile_flags, "-c", f, "-o", o] for f, o in zip(srcs, objs)]
    link = [cc, *flags, *objs, "-o", tmp]
    try:
        # translation units compile in parallel (the fine-sweep kernels dominate), then link
        procs = []
        for c in cmds:
            if verbose:
                print(" ".join(c), flush=True)
            procs.append(subprocess.Popen(c))
        failed = [c for c, p in zip(cmds, procs) if p.wait() != 0]
        if failed:
            raise subprocess.CalledProcessError(1, failed[0])
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
        os.replace(tmp, LIB)
    finally:
        if os.path.exists(tmp):
            os.remove(tmp)
        shutil.rmtree(objdir, ignore_errors=True)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--debug", action="store_true")
    a = ap.parse_args()
    print(build(debug=a.debug, verbose=True))


if __name__ == "__main__":
    sys.exit(main())
