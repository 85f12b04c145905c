"""Build the CPU oracle shared library (test infrastructure only).

Compiles oracle/chsim_oracle.cpp with g++ into oracle/liboracle.so.  The
oracle is plain C++ and needs no GPU toolchain.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "chsim_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


# The same source with AddressSanitizer and UndefinedBehaviorSanitizer, for
# checking runs (load it through CHSIM_ORACLE_LIB with libasan preloaded).
SAN_LIB = os.path.join(os.path.dirname(HERE), "_build", "oracle_san", "liboracle_san.so")


def build_sanitized(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(SAN_LIB), exist_ok=True)
    cmd = ["g++", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-std=c++17", "-fPIC", "-shared", "-pthread", SRC, "-o", SAN_LIB]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return SAN_LIB


def asan_runtime() -> str:
    """The libasan that g++ links sanitized code against."""
    out = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not (out and os.path.isabs(out) and os.path.exists(out)):
        raise RuntimeError("libasan not found")
    return out


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose=True))
    else:
        build(verbose=True)
    sys.exit(0)
