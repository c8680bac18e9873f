"""Build libstiffchem.so (host compiler + HIP kernels for gfx950) in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libstiffchem.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["mech.cpp", "sparse.cpp", "thermo_fit.cpp", "capi.cpp", "kernels.hip", "adjoint.hip", "transport.hip", "sparse.hip", "mapping.hip"]
HEADERS = ["mech.hpp", "devmech.hpp", "core.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("STIFFCHEM_ARCH", "gfx950")
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions are kept out of every HIP build
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # multiply-adds are fused per source expression only, so every
         # inlined copy of the step routine (the integrator's, the adjoint's
         # recording pass and its replays) rounds identically
         "-ffp-contract=on",
         f"-I{INC}", f"-I{CSRC}"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build failed: " + " ".join(cmd))


def build(force=True, jobs=3):
    """Compile every source (in parallel) and link the shared library."""
    os.makedirs(OBJDIR, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, src + ".o")
        objs.append(obj)
        path = os.path.join(CSRC, src)
        deps = [path] + [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(INC, "stiffchem.h")]
        if not force and os.path.exists(obj) and all(os.path.getmtime(obj) >= os.path.getmtime(d) for d in deps):
            continue
        procs.append((subprocess.Popen([HIPCC, *FLAGS, "-c", path, "-o", obj], stdout=subprocess.PIPE,
                                       stderr=subprocess.PIPE, text=True), src))
    failed = []
    for p, src in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out + err)
            failed.append(src)
    if failed:
        raise RuntimeError("build failed: " + ", ".join(failed))
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


C_CHECK_SRC = os.path.join(ROOT, "tests", "c", "c_abi_check.c")
C_CHECK = os.path.join(OBJDIR, "c_abi_check")


def build_c_check():
    """The plain-C program that drives the C ABI without Python (used by the
    GPU tests): gcc, HIP runtime headers, linked against the library."""
    os.makedirs(OBJDIR, exist_ok=True)
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    _run(["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include", f"-I{INC}",
          C_CHECK_SRC, "-o", C_CHECK, f"-L{rocm}/lib", "-lamdhip64", f"-L{HERE}", "-lstiffchem",
          f"-Wl,-rpath,{rocm}/lib", "-Wl,-rpath,$ORIGIN/.."])
    return C_CHECK


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
    print(build_c_check())
