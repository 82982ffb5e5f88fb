"""Build the gfx950 shared library libsph_mi355x.so in-tree with hipcc.

The launch sequences are instantiated once per (dimension, kernel, pair
precision) in csrc/sph_part.hip; the build compiles those twelve objects and
the C ABI (csrc/sph.hip) in parallel, then links them."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SRC = os.path.join(CSRC, "sph.hip")
PART = os.path.join(CSRC, "sph_part.hip")
DEPS = [SRC, PART] + [os.path.join(CSRC, f) for f in
                      ("sph_engine.hpp", "sph_kernels.hpp", "sph_adjoint.hpp", "sph_tiles.hpp")] + \
       [os.path.join(ROOT, "include", "sph.h")]
LIB = os.path.join(HERE, "libsph_mi355x.so")
OBJDIR = os.path.join(HERE, "_build")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds fused only within one source expression, so an inlined
    # helper rounds the same wherever it is used (the pair arithmetic is
    # bitwise the same whether a neighbour comes from a list or a cell walk)
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function",
]

COMBOS = [(d, k, t) for d in (2, 3) for t in ("float", "double") for k in (0, 1, 2)]


def _compile(args):
    cmd, verbose = args
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False, jobs: int = 0) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    cmds, objs = [], []
    # the heaviest (3D) objects first
    for d, k, t in sorted(COMBOS, key=lambda c: -c[0]):
        obj = os.path.join(OBJDIR, f"part_{d}d_k{k}_{t}.o")
        cmds.append([hipcc, *HIPCC_FLAGS, *inc, f"-DSPH_PART_DIM={d}", f"-DSPH_PART_KERNEL={k}",
                     f"-DSPH_PART_T={t}", "-c", "-o", obj, PART])
        objs.append(obj)
    abi_obj = os.path.join(OBJDIR, "sph_abi.o")
    cmds.append([hipcc, *HIPCC_FLAGS, *inc, "-c", "-o", abi_obj, SRC])
    objs.append(abi_obj)
    jobs = jobs or min(len(cmds), max(1, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, [(c, verbose) for c in cmds]))
    for c, r in zip(cmds, results):
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed ({' '.join(c[-1:])}):\n{r.stderr[-4000:]}")
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
