"""Measured VALU issue rates of the instructions the Montgomery kernels use.

    python -m paper_2111_11924_amd.peak

Runs the probe built from csrc/mad_rate.hip (built by the library build, or
here if missing) on GPU 0 and prints, per instruction, waves per SIMD and
independent chains per wave: lane-operations per second (event-timed), the
shader clock the waves measured, and lane-operations per cycle per compute
unit at that clock -- for v_mad_u64_u32 (carry-outs to VCC, and to a pair per
chain, the latter also with the multiply-adds placed at addresses 0 and at 4
modulo 8) and the helper instructions of a Montgomery column (v_mul_lo_u32,
v_add_co_u32, v_lshrrev_b64, v_and_b32).
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
