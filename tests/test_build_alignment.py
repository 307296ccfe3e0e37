"""The build's code-alignment pass (paper_2111_11924_amd/build.py): kernel ids
read from mangled names, and the multiply-adds of the CRT-halves and blinded
kernels of 2048-4096-bit keys at addresses 0 modulo 8 in the built objects
(host-side reading of the compiled gfx950 code; no GPU)."""
import os

import pytest

from paper_2111_11924_amd import build


def test_code_ids_from_mangled_names():
    assert build._code_id("_ZN3pmk13halves_kernelILi4096EEEvNS_8ClassRunEmjj") == 2_040_960
    assert build._code_id("_ZN3pmk19halves_lanes_kernelILi4096ELi2EEEvNS_8ClassRunEmjj") == 4_040_962
    assert build._code_id("_ZN3pmk17batch_wide_kernelENS_9BatchArgsE") == 8_000_000
    assert build._code_id("_ZN3pmk14mp_part_kernelILi1EEEvPKjS2_PKNS_9ChunkDescEjS2_PjS6_miS6_") == 9_000_010
    assert build._code_id("_ZN3pmk11pack_kernelILi64ELi64EEEvPKhPKNS_9ChunkDescEPKjS7_iiPji") is None
    assert build._code_id("_Z5probePyj") is None


@pytest.mark.parametrize("src,kind,bits", [
    ("k2048.hip", 2, 2048), ("k3072.hip", 2, 3072), ("k4096.hip", 2, 4096),
    ("kjoint.hip", 3, 2048), ("kjoint.hip", 3, 3072), ("kjoint.hip", 3, 4096)])
def test_hot_kernels_keep_multiply_adds_aligned(src, kind, bits):
    obj = os.path.join(build.OBJ, src + ".o")
    if not os.path.exists(obj) or not build._align_tools():
        pytest.skip("objects or llvm tools not present (build first)")
    n, odd = build.mad_alignment(obj)[kind * 1_000_000 + bits * 10]
    assert n > 1000
    assert odd <= 0.02 * n, f"{odd} of {n} multiply-adds at 4 modulo 8"
