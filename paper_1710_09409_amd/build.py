"""Build libsu3.so in-tree for gfx950 with hipcc.

The kernel unit su3_kprec.hip is compiled once per storage precision
(-DSU3_PREC=0..3) in parallel, then linked with the batch/yardstick unit,
the Wilson hopping unit, the expression-program unit, the host expression
compiler and the host C-ABI unit.  Always recompiles.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsu3.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # loadable by the HIP runtime that ships with PyTorch
    "-mcode-object-version=5",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _units():
    units = []
    for p in range(4):
        units.append(([f"-DSU3_PREC={p}", "-x", "hip",
                       os.path.join(CSRC, "su3_kprec.hip")],
                      os.path.join(OBJ, f"su3_kprec_p{p}.o")))
    units.append((["-x", "hip", os.path.join(CSRC, "su3_kmisc.hip")],
                  os.path.join(OBJ, "su3_kmisc.o")))
    units.append((["-x", "hip", os.path.join(CSRC, "su3_kdslash.hip")],
                  os.path.join(OBJ, "su3_kdslash.o")))
    units.append((["-x", "hip", os.path.join(CSRC, "su3_kprog.hip")],
                  os.path.join(OBJ, "su3_kprog.o")))
    units.append((["-x", "hip", os.path.join(CSRC, "su3_program.cpp")],
                  os.path.join(OBJ, "su3_program.o")))
    units.append((["-x", "hip", os.path.join(CSRC, "su3_api.cpp")],
                  os.path.join(OBJ, "su3_api.o")))
    return units


def _compile(unit):
    args, out = unit
    cmd = [HIPCC] + COMMON + args + ["-c", "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature; that warning
    # is expected
    noise = [ln for ln in (r.stdout + r.stderr).splitlines()
             if ln.strip() and "packed-fp32-ops" not in ln]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" +
                           "\n".join(noise))
    return "\n".join(noise)


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    units = _units()
    jobs = min(len(units), max(1, min(os.cpu_count() or 1, 8)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        logs = list(ex.map(_compile, units))
    if verbose:
        for lg in logs:
            if lg:
                print(lg, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-mcode-object-version=5", "-shared",
           "-fPIC", "-o", tmp] + \
        [u[1] for u in units]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
