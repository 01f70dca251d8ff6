"""Sanitizer runs on the CPU: the oracle's pins against an ASan/UBSan build
of the oracle, and the C ABI's argument-validation tests against a build of
the library whose host code carries ASan/UBSan (device code unchanged).
Each runs in a child Python with the sanitizer runtime preloaded; any
finding aborts the child, so the check is its exit status.  Leak detection
is off: the interpreter and the runtimes it loads keep allocations until
exit by design."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}

MAPS_CHECK = ("import sys; sys.path.insert(0, {root!r}); import {mod} as m; m.{load}(); "
              "maps = open('/proc/self/maps').read(); "
              "assert {lib!r} in maps and {rt!r} in maps, 'sanitized build not loaded'; "
              "print('loaded', {lib!r})")


def _run(args, env, timeout):
    r = subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=timeout)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    return r.stdout


def test_oracle_pins_pass_under_asan_and_ubsan():
    from oracle import build as ob
    lib = ob.build(sanitize=True)
    rt = ob.asan_runtime()
    env = dict(os.environ, GS_ORACLE_LIB=lib, LD_PRELOAD=rt, OMP_NUM_THREADS="4", **SAN_ENV)
    _run(["-c", MAPS_CHECK.format(root=ROOT, mod="oracle", load="lib",
                                  lib=os.path.basename(lib), rt=os.path.basename(rt))], env, 120)
    out = _run(["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                "tests/test_oracle_pointwise.py", "tests/test_oracle_physics.py",
                "tests/test_exact_riemann.py"], env, 600)
    assert " passed" in out and "failed" not in out


def test_c_abi_validation_passes_under_host_asan_and_ubsan(tmp_path):
    pytest.importorskip("paper_1812_07977_amd._lib")
    from paper_1812_07977_amd import build_hostsan as hb
    try:
        rt = hb.asan_runtime()
    except FileNotFoundError as e:
        pytest.skip(str(e))
    lib = hb.build(out=str(tmp_path / "libgs_fluid_hostsan.so"))
    env = dict(os.environ, GS_FLUID_LIB=lib, LD_PRELOAD=rt, **SAN_ENV)
    _run(["-c", MAPS_CHECK.format(root=ROOT, mod="paper_1812_07977_amd._lib", load="lib",
                                  lib=os.path.basename(lib), rt=os.path.basename(rt))], env, 120)
    out = _run(["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_api_cpu.py"],
               env, 600)
    assert " passed" in out and "failed" not in out
