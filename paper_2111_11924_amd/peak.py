"""Measured VALU issue rates of the instructions the Montgomery kernels use.

    python -m paper_2111_11924_amd.peak

Runs the probe built from csrc/mad_rate.hip (built by the library build, or
here if missing) on GPU 0 and prints lane-operations per clock per compute
unit for v_mad_u64_u32 (4, 8 and 16 independent chains per thread) and the
helper instructions of a Montgomery column (v_mul_lo_u32, v_add_co_u32,
v_lshrrev_b64, v_and_b32).
"""
from __future__ import annotations

import os
import subprocess
import sys

from . import build as _build


def main() -> int:
    if not os.path.exists(_build.PROBE):
        os.makedirs(os.path.dirname(_build.PROBE), exist_ok=True)
        _build.build_probe()
    return subprocess.call([_build.PROBE])


if __name__ == "__main__":
    sys.exit(main())
