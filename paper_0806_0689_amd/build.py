"""Builds the HIP library ``libme.so`` for gfx950 with hipcc (no GPU needed)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libme.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["me_api.hip", "me_batch.hip", "me_proposer.hip"]
# Stand-alone calibration program (VALU issue rates of the SAD instructions),
# run by bench.py as a child process.
RATES_SRC = "valu_rates.hip"
RATES = os.path.join(HERE, "valu_rates")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # Packed FP32 instructions stay off in every device build.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-fvisibility=hidden",
]


def build(verbose: bool = False) -> str:
    """Compiles every source to an object in parallel, then links libme.so."""
    from concurrent.futures import ThreadPoolExecutor
    tag = "%d" % os.getpid()
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(CSRC, "%s.%s.o" % (src, tag))
        objs.append(obj)
        cmds.append([HIPCC, *[f for f in FLAGS if f != "-shared"], "-c", "-I", os.path.join(ROOT, "include"),
                     "-I", CSRC, "-o", obj, os.path.join(CSRC, src)])
    tmp = LIB + ".tmp" + tag
    rates_tmp = RATES + ".tmp" + tag
    cmds.append([HIPCC, *[f for f in FLAGS if f not in ("-shared", "-fPIC", "-fvisibility=hidden")], "-o", rates_tmp,
                 os.path.join(CSRC, RATES_SRC)])
    try:
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            for cmd in cmds:
                if verbose:
                    print(" ".join(cmd), flush=True)
            for f in [ex.submit(subprocess.check_call, cmd) for cmd in cmds]:
                f.result()
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
        os.replace(tmp, LIB)
        os.replace(rates_tmp, RATES)
    finally:
        for o in objs + [tmp, rates_tmp]:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
