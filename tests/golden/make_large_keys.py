"""Writes tests/golden/large_keys.json: one seeded key pair per modulus size
2048, 3072, 4096, 6144 and 8192 bits, the inputs of the oracle's large-size
pins.

These are inputs, not expected values: every key comes from the seeded key
generator (``inputs.make_key``, stream 4242, index 0), stored only because the
8192-bit prime search takes minutes in pure Python.  The pins recheck each key
(primality with an independent routine, N = p q, e d = 1 mod lambda) before
using it.

    python tests/golden/make_large_keys.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2111_11924_amd import inputs  # noqa: E402

SIZES = (2048, 3072, 4096, 6144, 8192)
SEED = 4242


def main() -> None:
    keys = inputs.make_keys(list(SIZES), SEED)
    out = {"seed": SEED, "generator": "paper_2111_11924_amd.inputs.make_keys", "keys": [k.to_json() for k in keys]}
    with open(os.path.join(HERE, "large_keys.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
