"""Build libmpm.so (the gfx950 HIP library behind include/mpm.h) in-tree.

    python -m paper_2111_00699_amd.build

Each HIP source is compiled with hipcc for gfx950 only; packed-FP32 VALU
instructions are disabled and float atomics are emitted as the native
hardware instructions.  Variants are linked for the ablations:
libmpm.so (the default, fast-math flags), libmpm_precise.so (IEEE division,
square root and denormals), libmpm_aosoa.so (grouped particle layout) and
libmpm_lds_weights.so (P2G weights kept in LDS); the binding loads a variant
when MPM_LIBRARY names it.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmpm.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["mpm_bin.hip", "mpm_p2g.hip", "mpm_step.hip", "mpm_surrogate.hip", "mpm_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
BASE_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
# The paper's "Adopt fast-math intrinsics": FP32 denormals flushed (no
# scaling code around sqrt, rcp, log, exp), divisions by reciprocal, and the
# hardware's square root and reciprocal (1 ulp) instead of the correctly
# rounded expansions.  NaN and Inf keep their meaning (no finite-math), so
# the state checks still see them.
FAST_MATH_FLAGS = ["-fgpu-flush-denormals-to-zero", "-fno-signed-zeros", "-freciprocal-math",
                   "-fno-hip-fp32-correctly-rounded-divide-sqrt"]
# Library variants: the default build and, for the ablations, one with IEEE
# division, square root and denormals, one with the grouped particle layout
# (array of structures of arrays, 64 particles a group) instead of one array
# per field, and one whose P2G keeps the stencil weights in LDS instead of
# registers.
VARIANTS = {"fast": ("libmpm.so", FAST_MATH_FLAGS),
            "precise": ("libmpm_precise.so", []),
            "aosoa": ("libmpm_aosoa.so", FAST_MATH_FLAGS + ["-DMPM_AOSOA=1"]),
            "lds_weights": ("libmpm_lds_weights.so", FAST_MATH_FLAGS + ["-DMPM_WEIGHTS_IN_LDS=1"])}


def _compile(src: str, variant: str) -> str:
    out_dir = os.path.join(OBJ, variant)
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *BASE_FLAGS, *VARIANTS[variant][1], "-c", os.path.join(SRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if err.strip() and variant == "fast":
        print(err, file=sys.stderr)
    return obj


def build(verbose: bool = False, variants=tuple(VARIANTS)) -> str:
    jobs = [(src, v) for v in variants for src in SOURCES]
    for v in variants:
        os.makedirs(os.path.join(OBJ, v), exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(jobs), 8)) as ex:
        objs = list(ex.map(lambda j: _compile(*j), jobs))
    for v in variants:
        out = os.path.join(HERE, VARIANTS[v][0])
        mine = [o for o, (_, jv) in zip(objs, jobs) if jv == v]
        tmp = out + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *mine]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stderr)
        os.replace(tmp, out)
        if verbose:
            print(out)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
