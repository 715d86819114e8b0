"""Subsampled randomized Hadamard factors for the Kronecker sketch (Sec. 5.1).

TEST INFRASTRUCTURE ONLY (see ``oracle.tucker``).

A factor is Phi = R H D: D a diagonal of random signs, H the N x N Walsh-Hadamard
matrix scaled by 1/sqrt(N) (orthogonal), R the selection of s distinct rows (the paper
samples s columns of H for Omega = Phi^T).  N is a power of two; a mode of size n < N is
read as zero-padded to N, so only the first n columns of R H D act on the data.  The
random draws (the sampled rows and the n signs) are inputs.  The Hadamard matrix is
built by Sylvester's doubling H_1 = [1], H_2m = [[H_m, H_m], [H_m, -H_m]].
"""
from __future__ import annotations

import numpy as np


def padded_size(n: int) -> int:
    """Smallest power of two >= n (the zero-padded length of a mode of size n)."""
    N = 1
    while N < n:
        N *= 2
    return N


def walsh_hadamard(N: int) -> np.ndarray:
    """Unnormalised N x N Walsh-Hadamard matrix (entries +-1) by Sylvester's doubling."""
    if N < 1 or N & (N - 1):
        raise ValueError("N must be a power of two")
    H = np.ones((1, 1))
    while H.shape[0] < N:
        H = np.block([[H, H], [H, -H]])
    return H


def srht_factor(n: int, rows, signs) -> np.ndarray:
    """Phi = (R H D)[:, :n] (s x n, float64) for sampled rows ``rows`` (s distinct integers
    in [0, N)) and signs ``signs`` (n values +-1), N = padded_size(n)."""
    N = padded_size(n)
    rows = np.asarray(rows, dtype=np.int64)
    signs = np.asarray(signs, dtype=np.float64)
    if signs.shape != (n,) or np.any(np.abs(signs) != 1.0):
        raise ValueError("need n signs of +-1")
    if rows.ndim != 1 or np.any(rows < 0) or np.any(rows >= N) or len(set(rows.tolist())) != len(rows):
        raise ValueError("rows must be distinct integers in [0, N)")
    H = walsh_hadamard(N) / np.sqrt(N)
    return H[rows, :n] * signs[None, :]
