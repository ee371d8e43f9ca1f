"""The library's kernels and C ABI compiled for the host against an
emulation of HIP's launch API (tests/cpu_emu) and run under
AddressSanitizer/UBSan, compared with the oracle: out-of-bounds indexing or
a wrong result fails here, on the CPU, before any GPU run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "cpu_emu")
CSRC = os.path.join(ROOT, "paper_1710_09409_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"
CLANG_C = "/opt/rocm/llvm/bin/clang"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="needs ROCm's clang")
def test_kernels_under_asan(tmp_path):
    fl = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-I", EMU, "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    units = [([f"-DSU3_PREC={p}", "-x", "c++", os.path.join(CSRC, "su3_kprec.hip")], f"kp{p}.o")
             for p in range(4)]
    units += [(["-x", "c++", os.path.join(CSRC, "su3_kmisc.hip")], "km.o"),
              (["-x", "c++", os.path.join(CSRC, "su3_kdslash.hip")], "kd.o"),
              (["-x", "c++", os.path.join(CSRC, "su3_kprog.hip")], "kg.o"),
              ([os.path.join(CSRC, "su3_program.cpp")], "pg.o"),
              ([os.path.join(CSRC, "su3_api.cpp")], "api.o"),
              ([os.path.join(EMU, "emu_globals.cpp")], "g.o"),
              ([os.path.join(EMU, "harness.cpp")], "h.o")]
    procs = [subprocess.Popen([CLANG, "-std=c++20"] + fl + args + ["-c", "-o", str(tmp_path / out)],
                              stderr=subprocess.PIPE, text=True) for args, out in units]
    procs.append(subprocess.Popen([CLANG_C, "-O2", "-g", "-fsanitize=address", "-c",
                                   os.path.join(ROOT, "testgen", "gen.c"), "-o",
                                   str(tmp_path / "gen.o")], stderr=subprocess.PIPE, text=True))
    procs.append(subprocess.Popen([CLANG_C, "-O2", "-g", "-ffp-contract=off", "-fsanitize=address",
                                   "-c", os.path.join(ROOT, "oracle", "oracle.c"), "-o",
                                   str(tmp_path / "or.o")], stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err
    objs = [str(tmp_path / o) for o in ("kp0.o", "kp1.o", "kp2.o", "kp3.o", "km.o", "kd.o", "kg.o", "pg.o", "api.o",
                                        "g.o", "h.o", "gen.o", "or.o")]
    subprocess.check_call([CLANG, "-fsanitize=address,undefined"] + objs +
                          ["-o", str(tmp_path / "harness"), "-lm"])
    r = subprocess.run([str(tmp_path / "harness")], capture_output=True, text=True,
                       timeout=900)
    tail = "\n".join((r.stdout + r.stderr).splitlines()[-30:])
    assert r.returncode == 0, tail
    assert "fails 0" in r.stdout, tail
    assert "shift cases done" in r.stdout, tail
    assert "dslash cases done" in r.stdout, tail
    assert "vnode cases done" in r.stdout, tail
    assert "program cases done" in r.stdout, tail
