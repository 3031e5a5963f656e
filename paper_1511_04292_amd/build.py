"""Build libsrj.so for gfx950 in-tree with hipcc.

Every HIP translation unit is compiled with -ffp-contract=off (the sweep association is
part of the results' definition) and with packed-FP32 instruction generation disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libsrj.so")
SOURCES = ["kernels.hip", "sweep2d_tb.hip", "sweep3d_tb.hip", "batch.hip", "residual_static.hip", "small_solve.hip", "sweep2d_lds.hip",
           "api.cpp",
           "batch_api.cpp", "planner.cpp"]
ARCH = "gfx950"


def hipcc():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(verbose=False, jobs=4):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall",
              f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
    hip_flags = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".", "_") + ".o")
        objs.append(obj)
        path = os.path.join(CSRC, src)
        if src.endswith(".hip") or src in ("api.cpp", "batch_api.cpp"):
            cmd = [hipcc(), "-x", "hip"] + hip_flags + common + ["-c", path, "-o", obj]
        else:
            cmd = ["g++"] + common + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
    for cmd, pr in procs:
        if pr.wait() != 0:
            raise RuntimeError("compile failed: " + " ".join(cmd))
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", SO + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(SO + ".tmp", SO)
    return SO


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(SO)
