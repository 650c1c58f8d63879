"""Build the HIP library libqg.so for gfx950 in-tree (hipcc, no JIT cache).

The library links the roctx marker library of ROCm (ranges around qg_step,
qg_adjoint_step and qg_step_noalloc for rocprofv3 --marker-trace).

Sources are compiled in parallel (the kernel file once per slice of its
launchers, QG_PART = 0..4), then linked into paper_2508_06678_amd/libqg.so.
All device code is built with packed-FP32 instruction generation disabled.
A debug variant, libqg_ldspoison.so, is linked from the same sources with
QG_LDS_POISON defined: every kernel sets its LDS to NaN before use and every
transform pass poisons its buffer before writing, so that a read of LDS
nothing wrote carries NaN into the result (tests/test_gpu_lds_poison.py).
A second one, libqg_stamps.so (QG_STAMPS, kernels and API), writes per-wave
phase stamps for qg_stamp_steps (paper_2508_06678_amd/stamps.py).
Then the C example program qg_example (plain C99 against include/qg.h,
linked to libqg.so and the HIP runtime) is built beside it.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
# (source, extra defines, object name)
UNITS = [("qg_kernels.hip", [f"-DQG_PART={i}"], f"qg_kernels_{i}.o") for i in range(5)] + \
        [("qg_api.hip", [], "qg_api.o")]
POISON_UNITS = [("qg_kernels.hip", [f"-DQG_PART={i}", "-DQG_LDS_POISON"], f"qg_kernels_poison_{i}.o")
                for i in range(5)]
STAMP_UNITS = [("qg_kernels.hip", [f"-DQG_PART={i}", "-DQG_STAMPS"], f"qg_kernels_stamps_{i}.o")
               for i in range(5)] + [("qg_api.hip", ["-DQG_STAMPS"], "qg_api_stamps.o")]
LIB = os.path.join(PKG, "libqg.so")
LIB_POISON = os.path.join(PKG, "libqg_ldspoison.so")
LIB_STAMPS = os.path.join(PKG, "libqg_stamps.so")
ARCH = os.environ.get("QG_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def _hipcc():
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose=False):
    out_dir = os.path.join(ROOT, "_build")
    os.makedirs(out_dir, exist_ok=True)
    hipcc = _hipcc()

    def compile_one(unit):
        src, defs, name = unit
        obj = os.path.join(out_dir, name)
        cmd = [hipcc, *FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    units = UNITS + POISON_UNITS + STAMP_UNITS
    workers = max(1, min(len(units), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(compile_one, units))
    n0, n1 = len(UNITS), len(UNITS) + len(POISON_UNITS)
    api = objs[n0 - 1]
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    for lib, lib_objs in ((LIB, objs[:n0]), (LIB_POISON, objs[n0:n1] + [api]), (LIB_STAMPS, objs[n1:])):
        tmp = lib + ".tmp"
        cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *lib_objs, "-o", tmp,
               "-L", rocm_lib, "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + rocm_lib]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    build_example(verbose)
    return LIB


EXAMPLE = os.path.join(PKG, "qg_example")


def build_example(verbose=False):
    """The C program, compiled by the host C compiler: nothing in it is
    device code."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cc = os.environ.get("CC", "gcc")
    tmp = EXAMPLE + ".tmp"
    cmd = [cc, "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(rocm, "include"), os.path.join(CSRC, "qg_example.c"), "-o", tmp,
           "-L", PKG, "-lqg", "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(rocm, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, EXAMPLE)
    return EXAMPLE


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
