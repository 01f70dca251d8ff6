"""Build the CPU oracle library (test infrastructure; see gs_oracle.c).

    python oracle/build.py [--sanitize]

Compiles gs_oracle.c with gcc into oracle/libgs_oracle.so: IEEE FP64, no
floating-point contraction, no fast-math, OpenMP for the outer loops.

--sanitize builds oracle/libgs_oracle_san.so instead, with AddressSanitizer
and UndefinedBehaviorSanitizer (every finding aborts).  Load it by setting
GS_ORACLE_LIB to its path and preloading gcc's ASan runtime (the Python
interpreter itself is not instrumented); tests/test_sanitize_cpu.py runs the
oracle's pins that way.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gs_oracle.c")
LIB = os.path.join(HERE, "libgs_oracle.so")
LIB_SAN = os.path.join(HERE, "libgs_oracle_san.so")

CFLAGS = ["-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp",
          "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"]
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = LIB_SAN if sanitize else LIB
    flags = CFLAGS + (SAN_FLAGS if sanitize else [])
    cmd = ["gcc", *flags, SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def asan_runtime() -> str:
    """Path of gcc's AddressSanitizer runtime, to preload into Python."""
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                       check=True)
    return r.stdout.strip()


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
