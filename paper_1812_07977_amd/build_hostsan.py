"""Host-sanitized build of the library, for CPU checks of its host code.

    python -m paper_1812_07977_amd.build_hostsan

Compiles the same sources with the same flags as build.py, and the host half
of every source also with AddressSanitizer and UndefinedBehaviorSanitizer
(every finding aborts); the device code is built exactly as for the product.
The result, libgs_fluid_hostsan.so, is loaded by setting GS_FLUID_LIB to its
path and preloading the compiler's ASan runtime (asan_runtime()).  It is for
the CPU: tests/test_sanitize_cpu.py runs the C-ABI argument-validation tests
against it.  It is never loaded on a GPU.
"""
import glob
import os
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

from . import build as B

LIB = os.path.join(B.HERE, "libgs_fluid_hostsan.so")
# host-only instrumentation: each sanitizer flag goes to the host pass only
HOST_SAN = ["-Xarch_host", "-fsanitize=address,undefined",
            "-Xarch_host", "-fno-sanitize-recover=all",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def build(verbose: bool = False, out: str = LIB) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(B.ROOT, "include"), "-I", os.path.join(B.HERE, "csrc")]
    with tempfile.TemporaryDirectory(prefix="gs_hostsan_") as tmp:
        jobs = []
        for src, own in B.SRCS.items():
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            jobs.append((obj, [hipcc, *B.FLAGS, *own, *HOST_SAN, *inc, "-c", src, "-o", obj]))
        with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
            for f in [ex.submit(B._run, cmd, verbose) for _, cmd in jobs]:
                f.result()
        B._run([hipcc, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *[o for o, _ in jobs],
                "-o", out + ".tmp"], verbose)
    os.replace(out + ".tmp", out)
    return out


def asan_runtime() -> str:
    """The compiler's shared ASan runtime (it also carries the UBSan
    handlers), to preload into an uninstrumented Python."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found under /opt/rocm/llvm")
    return hits[-1]


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
