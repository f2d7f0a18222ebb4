"""Build ``libsparsefusion.so`` (HIP for gfx950) and the microbenchmark.

Every translation unit under ``csrc/`` is compiled with hipcc for gfx950;
kernels get ``-packed-fp32-ops`` disabled (packed FP32 instructions are not
generated) and the atomic optimizer off (see COMMON).  The result is placed next to this file so it travels with the
source tree.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libsparsefusion.so")
MICRO = os.path.join(BUILD, "sf_microbench")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# -amdgpu-atomic-optimizer-strategy=None: the executors' work-claiming
# atomics are issued by one lane; the optimizer's wave-wide rewrite of them
# would wait for each result at once instead of where it is first used.
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
          "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function",
          "-Wno-unused-command-line-argument"]

UNITS = ["inspect.cpp", "static_plan.cpp", "api.cpp", "k_ts.hip", "k_ic0.hip", "k_ilu.hip", "k_bwd.hip", "k_refine.hip",
         "k_layout.hip", "k_probe.hip", "scratch.hip", "k_rfused.hip", "k_region.hip"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + COMMON + lang + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [os.path.join(CSRC, u) for u in UNITS]
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    micro_tmp = MICRO + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC] + COMMON + ["-o", micro_tmp, os.path.join(CSRC, "microbench.hip")],
                          stderr=subprocess.DEVNULL)
    os.replace(micro_tmp, MICRO)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
