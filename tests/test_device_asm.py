"""Device-code checks on the gfx950 assembly of the library's own sources.

Two checks: no matrix instruction under an unguarded exec mask (below), and
no write through the scalar data cache anywhere (vector stores only).

A matrix instruction (v_mfma_*) placed in a region where EXEC has been
narrowed by a vector branch, with no branch that skips the region when EXEC
is empty, still updates its accumulator in a wavefront that should have
skipped it.  This was observed on the network adjoint, where a
wavefront-role branch written as `if (q == 1)` on a per-lane value
corrupted the other role's accumulator.  Role branches must be scalar
(wavefront index through readfirstlane).  The check walks each kernel's
instruction stream linearly and flags such an MFMA.  It is a heuristic
over straight-line code, so a clean result means no flagged pattern, not a
proof.
"""

import os
import re
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2111_11215_amd import build as B

MFMA_SOURCES = ["render.hip", "proposal.hip"]
ALL_SOURCES = ["abi.hip", "sampler.hip", "render.hip", "optim.hip", "proposal.hip", "scene.hip"]

_NARROW = re.compile(r"s_(and|or|andn2|xor|nand|nor|orn2)_saveexec_b64|s_mov_b64 exec, (?!-1)|"
                     r"s_(and|andn2|xor)_b64 exec, ")
_RESTORE = re.compile(r"s_or_b64 exec, exec, |s_mov_b64 exec, -1")


def masked_mfmas(asm: str):
    """(function, line, instruction) of every MFMA in a narrowed region that
    no execz branch guards."""
    found = []
    func, masked, guarded = None, False, False
    for no, line in enumerate(asm.splitlines(), 1):
        m = re.match(r"^(_Z\w+):", line)
        if m:
            func, masked, guarded = m.group(1), False, False
            continue
        t = line.strip()
        if _RESTORE.match(t):
            masked = False
        elif _NARROW.match(t):
            masked, guarded = True, False
        elif t.startswith("s_cbranch_execz") or t.startswith("s_cbranch_execnz"):
            guarded = True
        elif t.startswith("v_mfma") and masked and not guarded:
            found.append((func, no, t))
    return found


def _device_asm(src, out_dir):
    out = os.path.join(out_dir, os.path.splitext(src)[0] + ".s")
    flags = [f for f in B.HIPCC_FLAGS if f != "-fPIC"]
    cmd = [B.hipcc(), *flags, "-I", B.INCLUDE, "-I", B.CSRC, "--cuda-device-only", "-S",
           os.path.join(B.CSRC, src), "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    with open(out) as f:
        return f.read()


def _have_hipcc():
    try:
        B.hipcc()
        return True
    except RuntimeError:
        return False


def test_detector_flags_an_unguarded_masked_mfma():
    bad = "\n".join([
        "_Zkernel:",
        "\ts_and_saveexec_b64 s[4:5], s[8:9]",
        "\tv_mfma_f32_32x32x16_bf16 v[0:15], v[16:19], v[20:23], v[0:15]",
        "\ts_or_b64 exec, exec, s[4:5]",
    ])
    good = bad.replace("s[8:9]\n", "s[8:9]\n\ts_cbranch_execz .LBB0_2\n")
    assert len(masked_mfmas(bad)) == 1
    assert masked_mfmas(good) == []
    assert masked_mfmas(bad.replace("s_and_saveexec_b64 s[4:5], s[8:9]", "s_cbranch_scc1 .LBB0_2")) == []


@pytest.mark.skipif(not _have_hipcc(), reason="hipcc not available")
def test_no_matrix_instruction_under_an_unguarded_exec_mask(tmp_path):
    with ThreadPoolExecutor(max_workers=len(MFMA_SOURCES)) as ex:
        asms = list(ex.map(lambda s: _device_asm(s, str(tmp_path)), MFMA_SOURCES))
    total = sum(a.count("v_mfma") for a in asms)
    assert total > 100, "expected the network kernels' matrix instructions in the assembly"
    bad = [x for a in asms for x in masked_mfmas(a)]
    assert bad == [], bad[:5]


_SCALAR_WRITE = re.compile(r"^\s*(s_store_|s_buffer_store|s_scratch_store|s_atomic_|s_buffer_atomic_|s_dcache_wb|s_dcache_discard)")


def test_scalar_write_pattern():
    assert _SCALAR_WRITE.match("\ts_store_dword s4, s[2:3], 0x10")
    assert _SCALAR_WRITE.match("\ts_atomic_add s4, s[2:3], 0x0")
    assert _SCALAR_WRITE.match("\ts_dcache_wb")
    assert not _SCALAR_WRITE.match("\ts_load_dwordx2 s[0:1], s[4:5], 0x0")
    assert not _SCALAR_WRITE.match("\tglobal_store_dword v0, v1, s[2:3]")


@pytest.mark.skipif(not _have_hipcc(), reason="hipcc not available")
def test_no_scalar_cache_writes(tmp_path):
    """Device code writes memory through vector stores only: no scalar-cache
    stores, atomics, write-backs or discards in any kernel."""
    with ThreadPoolExecutor(max_workers=len(ALL_SOURCES)) as ex:
        asms = list(ex.map(lambda s: _device_asm(s, str(tmp_path)), ALL_SOURCES))
    bad = [(src, no, line.strip()) for src, asm in zip(ALL_SOURCES, asms)
           for no, line in enumerate(asm.splitlines(), 1) if _SCALAR_WRITE.match(line)]
    assert bad == [], bad[:5]
