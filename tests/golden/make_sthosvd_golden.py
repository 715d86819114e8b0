"""Writes sthosvd_1024x1024x512.txt: the oracle's deterministic STHOSVD (Alg. 2.2, numpy SVD
per mode, float64) of the 1024 x 1024 x 512 smooth-field workload at ranks (32, 32, 32), for
the full-size GPU test.  Calls only the oracle and the seeded input generator.

    python tests/golden/make_sthosvd_golden.py      # a few minutes, about 20 GB of memory
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import tucker as T  # noqa: E402


def main():
    dims, r = (1024, 1024, 512), [32, 32, 32]
    X = synth.bumps_field(dims, nbumps=200, noise_rel=1e-4, seed=synth.DATA_SEED).astype(np.float64)
    G, Vs = T.sthosvd(X, r)
    e = T.rel_error(X, G, Vs)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sthosvd_1024x1024x512.txt")
    with open(out, "w") as f:
        f.write("# Oracle STHOSVD (Alg. 2.2) of the 1024x1024x512 smooth field (data seed 1, binary32 values),\n")
        f.write("# ranks (32, 32, 32); written by tests/golden/make_sthosvd_golden.py\n")
        f.write(f"rel_error {e:.15e}\n")
        f.write("core_norm " + f"{float(np.linalg.norm(G)):.15e}\n")
    print(f"rel_error {e:.15e}")


if __name__ == "__main__":
    main()
