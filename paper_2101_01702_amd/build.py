"""Build the HIP library liblbm.so (gfx950) in-tree.

    python -m paper_2101_01702_amd.build
"""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblbm.so")
BUILD_DIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed FP32 instructions are disabled for all device code
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, extra_device_flags=None) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    t0 = time.time()
    dev_obj = os.path.join(BUILD_DIR, "lbm_device.o")
    adj_obj = os.path.join(BUILD_DIR, "lbm_adjoint.o")
    api_obj = os.path.join(BUILD_DIR, "lbm_api.o")
    procs = [
        subprocess.Popen([HIPCC, "-x", "hip", f"--offload-arch={ARCH}", *COMMON, *DEVICE_FLAGS,
                          *(extra_device_flags or []), "-c", os.path.join(CSRC, "lbm_device.hip"),
                          "-o", dev_obj]),
        subprocess.Popen([HIPCC, "-x", "hip", f"--offload-arch={ARCH}", *COMMON, *DEVICE_FLAGS,
                          "-c", os.path.join(CSRC, "lbm_adjoint.hip"), "-o", adj_obj]),
        subprocess.Popen([HIPCC, f"--offload-arch={ARCH}", *COMMON, "-c",
                          os.path.join(CSRC, "lbm_api.cpp"), "-o", api_obj]),
    ]
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", dev_obj, adj_obj, api_obj, "-o", LIB + ".tmp"],
         verbose)
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f} s", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
