"""Build libmttkrp.so in-tree with hipcc for gfx950.

Usage: python -m paper_2411_04785_amd.build  (or __graft_entry__.build()).
Objects go to _build/ at the repository root; the shared library is written
next to this file.  Every call recompiles every source.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libmttkrp.so")
ARCH = os.environ.get("MTK_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

# Packed FP32 instructions are switched off for all device code.
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
          f"-I{os.path.join(ROOT, 'include')}"]

SOURCES = ["mttkrp_kernels.hip", "dimtree.hip", "als_kernels.hip", "quant_kernels.hip", "nway.hip", "sparse.hip", "api.hip",
           "server.hip"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # hipcc's host pass does not know the device-only feature flag; drop that noise.
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    return p.returncode, out


def build(verbose: bool = False, jobs: int = 0) -> str:
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objs = [os.path.join(bdir, os.path.splitext(s)[0] + ".o") for s in srcs]

    def comp(pair):
        s, o = pair
        return s, _run([HIPCC, *COMMON, "-c", os.path.join(CSRC, s), "-o", o])

    jobs = jobs or min(len(srcs), os.cpu_count() or 1, 8)
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(comp, zip(srcs, objs)))
    for s, (rc, out) in results:
        if out.strip() and (verbose or rc != 0):
            print(f"--- {s}\n{out}", file=sys.stderr)
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {s}")
    tmp = OUT + ".tmp"
    rc, out = _run([HIPCC, *COMMON, "-shared", *objs, "-o", tmp, "-lpthread", "-Wl,--no-undefined"])
    if rc != 0:
        print(out, file=sys.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
