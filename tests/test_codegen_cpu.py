"""Code generation checks on the CPU: the device code of each source, built
with the library's own flags, contains no instruction forms this project
keeps out of its kernels, and the stage kernels keep the register budgets
their measured performance depends on.

- No scalar-cache writes: no scalar memory stores or atomics, no write-back
  or discard of the scalar data cache.  Every store is a vector store.
- No packed FP32 arithmetic: the build disables the feature, so that the
  compiler never forms those instructions from ordinary float code.
- The FP64 stage kernels (16 x 16 tiles) and the FP64 batched kernels with
  16 x 16 tiles fit three waves per SIMD: at most 168 VGPRs, no spills.
"""
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1812_07977_amd import build as B  # noqa: E402

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SCALAR_WRITE = re.compile(r"^\s+s_(store|atomic|buffer_store|scratch_store|dcache_wb|dcache_discard)\w*\b",
                          re.M)
PACKED_F32 = re.compile(r"^\s+v_pk_(add|mul|fma)_f32\b", re.M)


def _asm(src, own):
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(B.HERE, "csrc")]
    cmd = [HIPCC, *B.FLAGS, *own, *inc, "--offload-device-only", "-S", src, "-o", "-"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return r.stdout


@pytest.fixture(scope="module")
def asm():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    with ThreadPoolExecutor(max_workers=len(B.SRCS)) as ex:
        futs = {os.path.basename(s): ex.submit(_asm, s, own) for s, own in B.SRCS.items()}
        return {k: f.result() for k, f in futs.items()}


def _kernel_meta(text):
    """(name, vgpr_count, vgpr_spill_count) of every kernel in the metadata."""
    md = text[text.index("amdhsa.kernels"):]
    out = []
    for blk in re.split(r"\n  - ", md)[1:]:
        m = re.search(r"\.name:\s+(\S+)", blk)
        if not m:
            continue
        v = re.search(r"\.vgpr_count:\s+(\d+)", blk)
        sp = re.search(r"\.vgpr_spill_count:\s+(\d+)", blk)
        out.append((m.group(1), int(v.group(1)) if v else None, int(sp.group(1)) if sp else 0))
    return out


def test_every_source_compiles_for_the_device(asm):
    assert set(asm) == {os.path.basename(s) for s in B.SRCS}
    for name, text in asm.items():
        assert "amdhsa.kernels" in text, name


def test_no_scalar_cache_writes(asm):
    for name, text in asm.items():
        hits = SCALAR_WRITE.findall(text)
        assert not hits, (name, hits[:5])


def test_no_packed_fp32_arithmetic(asm):
    for name, text in asm.items():
        hits = PACKED_F32.findall(text)
        assert not hits, (name, hits[:5])


def test_fp64_stage_kernels_fit_three_waves(asm):
    checked = 0
    for src, pat in (("gs_fluid.hip", r"stage_kernelIdLi16ELi16E"),
                     ("gs_batch.hip", r"batch_stage_kernelIdLi16ELi16E")):
        for name, vgpr, spill in _kernel_meta(asm[src]):
            if re.search(pat, name):
                checked += 1
                assert vgpr is not None and vgpr <= 168, (name, vgpr)
                assert spill == 0, (name, spill)
    assert checked >= 10
