"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_AD = os.path.join(HERE, "liboracle_ad.so")


def build(verbose: bool = False, src: str = None, out: str = None) -> str:
    """Compile ``src`` (default oracle/oracle.c) into ``out`` (default liboracle.so)."""
    src = src or os.path.join(HERE, "oracle.c")
    out = out or LIB
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-I", HERE, src, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build_ad(verbose: bool = False, src: str = None, out: str = None) -> str:
    """Compile the reverse sweep (oracle_ad.cpp: oracle.c on a recording type) into
    ``out`` (default liboracle_ad.so)."""
    src = src or os.path.join(HERE, "oracle_ad.cpp")
    out = out or LIB_AD
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-Wno-unknown-pragmas", "-I", HERE, src, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    build_ad(verbose=True)
    sys.exit(0)
