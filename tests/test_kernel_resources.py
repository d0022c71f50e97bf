"""CPU check of the compiled kernels' resources: every gfx950 kernel of the
library runs without private (scratch) memory and without vector-register
spills (which go to scratch).  A kernel that indexes a private array or
struct with a run-time index gets a scratch segment, and each access becomes
a memory round trip; the batched control kernel once lost a third of its
time that way.  Scalar-register spills are allowed: they go to lanes of
vector registers, not to memory.  The device code is compiled here with the
library's flags to assembly and the kernels' metadata read back.  No device
work is done."""
import os
import re
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_1209_5553_amd import build as B

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1209_5553_amd", "csrc")
INCLUDE = os.path.join(os.path.dirname(CSRC), "..", "include")


def _hipcc():
    try:
        return B.hipcc()
    except RuntimeError:
        return None


def _kernel_metadata(asm):
    """(kernel name, private segment bytes, VGPR spills) per kernel."""
    out = []
    for m in re.finditer(r"^\s+\.name:\s+(\S+)\s*$", asm, flags=re.M):
        start = asm.rfind("- .agpr_count", 0, m.start())
        end = asm.find("- .agpr_count", m.end())
        blk = asm[start:end if end > 0 else len(asm)]

        def field(key):
            f = re.search(r"\." + key + r":\s+(\d+)", blk)
            return int(f.group(1)) if f else 0

        out.append((m.group(1), field("private_segment_fixed_size"), field("vgpr_spill_count")))
    return out


@pytest.fixture(scope="module")
def kernels():
    hipcc = _hipcc()
    if hipcc is None or not shutil.which(hipcc) and not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    sources = [s for s in B.SOURCES if s.endswith(".hip")]
    flags = [f for f in B.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    tmp = tempfile.mkdtemp(prefix="erem_asm_")

    def compile_one(src):
        out = os.path.join(tmp, src + ".s")
        subprocess.run([hipcc, *flags, "--cuda-device-only", "-S", "-I", INCLUDE, "-I", CSRC,
                        os.path.join(CSRC, src), "-o", out], check=True, capture_output=True)
        return src, open(out).read()

    try:
        with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as pool:
            asm = dict(pool.map(compile_one, sources))
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return {src: _kernel_metadata(text) for src, text in asm.items()}


def test_kernels_are_found(kernels):
    # every source but the allocation-free entry point (launchers only) defines kernels
    names = [name for ks in kernels.values() for name, _, _ in ks]
    assert any("k_bt_ctrl" in n for n in names) and any("k_leja_terms" in n for n in names)
    assert all(ks for src, ks in kernels.items() if src != "noalloc.hip")


def test_no_kernel_uses_scratch_or_spills_vector_registers(kernels):
    bad = [(src, name, priv, vs) for src, ks in kernels.items() for name, priv, vs in ks if priv or vs]
    assert not bad, "kernels with private memory or VGPR spills: " + "; ".join(
        f"{src} {name}: private {priv} B, VGPR spills {vs}" for src, name, priv, vs in bad)
