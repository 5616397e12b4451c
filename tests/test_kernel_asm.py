"""Static checks of the gfx950 code of the triplet kernel (CPU only: hipcc
cross-compiles).  The kernel addresses LDS through 32-bit LDS addresses; a
generic pointer made from such an address is not an LDS reference (the
compiler may fold the conversion to a plain global address), so the kernel
must contain no flat stores, must declare no static LDS (its LDS map starts
at address 0) and must not spill."""
from __future__ import annotations

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1708_08619_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not HIPCC:
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("asm") / "kernels.s"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-x", "hip",
                           "--cuda-device-only", "-S", os.path.join(CSRC, "g3_kernels.hip"),
                           "-o", str(out)], stderr=subprocess.DEVNULL)
    return out.read_text()


def _bodies(text, name):
    out = {}
    for m in re.finditer(r"^(_Z\w*%s\w*):\s*;" % name, text, re.M):
        end = text.index("s_endpgm", m.end())
        out[m.group(1)] = text[m.end():end]
    return out


def test_triplet_kernel_has_no_flat_stores(asm):
    bodies = _bodies(asm, "k_triplet")
    assert len(bodies) == 9
    for sym, body in bodies.items():
        assert "flat_store" not in body, sym


def test_triplet_kernel_has_no_static_lds_and_no_spills(asm):
    for sym in _bodies(asm, "k_triplet"):
        i = asm.index(".name:           " + sym)
        # the kernel's metadata map runs from its list item marker to the next
        meta = asm[asm.rindex("\n  - ", 0, i):asm.find("\n  - ", i)]
        assert re.search(r"\.group_segment_fixed_size:\s+0\b", meta), sym
        assert re.search(r"\.private_segment_fixed_size:\s+0\b", meta), sym
        assert re.search(r"\.vgpr_spill_count:\s+0\b", meta), sym


def test_hot_kernels_use_no_flat_memory_instructions(asm):
    """Flat loads, stores and atomics also count against the LDS wait counter,
    so an LDS wait would also wait for outstanding global accesses: the
    neighbour build and the triplet kernel address global memory through
    global-address-space pointers only."""
    for name, count in (("k_triplet", 9), ("k_nbr_build", 4), ("k_nbr_wave", 3)):
        bodies = _bodies(asm, name)
        assert len(bodies) == count, name
        for sym, body in bodies.items():
            assert not re.search(r"^\s+flat_", body, re.M), sym


def test_wave_build_fits_its_occupancy(asm):
    """The per-wave neighbour build runs up to seven 4-wave workgroups per CU
    (seven waves per SIMD): at most 72 VGPRs, no spills, no static LDS."""
    bodies = _bodies(asm, "k_nbr_wave")
    assert len(bodies) == 3
    for sym in bodies:
        i = asm.index(".name:           " + sym)
        meta = asm[asm.rindex("\n  - ", 0, i):asm.find("\n  - ", i)]
        assert int(re.search(r"\.vgpr_count:\s+(\d+)", meta).group(1)) <= 72, sym
        assert re.search(r"\.private_segment_fixed_size:\s+0\b", meta), sym
        assert re.search(r"\.vgpr_spill_count:\s+0\b", meta), sym
        assert re.search(r"\.group_segment_fixed_size:\s+0\b", meta), sym
