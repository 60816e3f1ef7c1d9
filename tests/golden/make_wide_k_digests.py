"""Writes wide_k_digests.txt: per-limb SHA-256 digests of the oracle's k-input
multiply (tensor product, relinearisation with the relocated ModDown, k - 1
combined rescales) for seeded uniform inputs at the ring degrees and widths
where the oracle takes minutes (its tensor product sums over all 2^k
selections of eq. (d_u formula for n-ct mult)).

Calls only the oracle and the seeded input generator.  The GPU tests draw the
same inputs, run the library and compare the digests of every output limb.

    python tests/golden/make_wide_k_digests.py   # from the repository root
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from oracle import keys as okeys, mult, params as oparams  # noqa: E402
from seeded_inputs import limb_digests, uniform_cts  # noqa: E402

OUT = os.path.join(HERE, "wide_k_digests.txt")

# name: (log_n, L, K, dnum, key_seed, k_max, k, level, input_seed)
CASES = {
    "n16_k12_l32": (16, 32, 8, 4, 81, 12, 12, 32, 1612),
    "n16_k11_l16": (16, 32, 8, 4, 81, 12, 11, 16, 1611),
    "n16_k10_l13": (16, 32, 8, 4, 81, 12, 10, 13, 1610),
    "n16_k9_l12": (16, 32, 8, 4, 81, 12, 9, 12, 1609),
    "n15_k12_l16": (15, 16, 4, 4, 82, 12, 12, 16, 1512),
    "n15_k11_l13": (15, 16, 4, 4, 82, 12, 11, 13, 1511),
    "n14_k12_l12": (14, 12, 2, 4, 83, 12, 12, 12, 1412),
    "n14_k11_l12": (14, 12, 2, 4, 83, 12, 11, 12, 1411),
}


def main() -> None:
    keys = {}
    lines = ["# Per-limb digests of the oracle's k-input multiply on seeded uniform inputs",
             "# (tests/seeded_inputs.py: uniform_cts(input_seed, q_0..q_{level-1}, N, k)).",
             "# Written by tests/golden/make_wide_k_digests.py from the oracle alone.",
             "# name log_n L K dnum key_seed k_max k level input_seed digest(poly 0 limbs..., poly 1 limbs...)"]
    for name, (log_n, L, K, dnum, ks, kmax, k, level, iseed) in CASES.items():
        t0 = time.time()
        pk = (log_n, L, K, dnum, ks, kmax)
        if pk not in keys:
            op = oparams.make_params(log_n, L, K, dnum)
            keys[pk] = (op, okeys.keygen(op, ks, kmax))
        op, ok = keys[pk]
        cts = uniform_cts(iseed, op.q[:level], op.N, k)
        out = mult.mul_relin_rescale(op, ok, cts, level)
        d = limb_digests(out)
        lines.append(" ".join([name] + [str(v) for v in (log_n, L, K, dnum, ks, kmax, k, level, iseed)] + d))
        print("%s: %.1f s" % (name, time.time() - t0), flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
