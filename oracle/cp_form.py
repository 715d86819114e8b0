"""The randomized algorithms applied to a tensor held in Kruskal (CP) form.

TEST INFRASTRUCTURE ONLY (see ``oracle.tucker``).

X = sum_i lam_i a_{1,i} o a_{2,i} o ... o a_{d,i} is never assembled: a TTM X x_k M maps
the factor A_k to M A_k (Sec. 2.1), so every sketch, every contraction with U_hat^T and
the core G_hat (a few dozen entries per mode) are formed from the factors.  The steps are
those of Alg. 4.3 / Alg. 4.4 / App. A in the same order as ``oracle.tucker``; only the
representation of X differs.  Because U_j = U_hat_j V_j is orthonormal and G = X x_j U_j^T,
the error follows from ||X - X_hat||^2 = ||X||^2 - ||G||^2 (Sec. 5.2); with relative
errors near 1e-4 that difference keeps about 8 significant digits in float64.  Used for
the accuracy experiment at the paper's size (500^3), which a dense float64 oracle would
need 1 GB per trial for.
"""
from __future__ import annotations

import numpy as np

from . import tucker as T


def full(lam, A) -> np.ndarray:
    """Assemble the (small) tensor sum_i lam_i a_{1,i} o ... o a_{d,i}."""
    d = len(A)
    letters = "abcdefgh"[:d]
    spec = "z," + ",".join(f"{c}z" for c in letters) + "->" + letters
    return np.einsum(spec, np.asarray(lam, dtype=np.float64), *A, optimize=True)


def norm2(lam, A) -> float:
    """||X||^2 = sum_{i,j} lam_i lam_j prod_k (A_k^T A_k)_{ij}."""
    M = np.outer(lam, lam)
    for Ak in A:
        M = M * (Ak.T @ Ak)
    return float(M.sum())


def sketch(lam, A, mats, n) -> np.ndarray:
    """Y_(n) for Y = X x_{k != n} M_k (mats[k] for k != n)."""
    B = [A[k] if k == n else mats[k] @ A[k] for k in range(len(A))]
    return T.unfold(full(lam, B), n)


def _finish(lam, A, Uhat, Ghat, r):
    G, Vs = T.sthosvd(Ghat, r)
    Us = [Uh @ V for Uh, V in zip(Uhat, Vs)]
    x2 = norm2(lam, A)
    e2 = max(x2 - float(np.sum(G * G)), 0.0) / x2
    return G, Us, float(np.sqrt(e2))


def rhkron(lam, A, r, phis):
    """Alg. 4.4 (factor reuse) on a CP tensor; returns (G, [U_j], relative error)."""
    d = len(A)
    Uhat = [T.qr_pos(sketch(lam, A, phis, n))[0] for n in range(d)]
    Ghat = full(lam, [Uhat[k].T @ A[k] for k in range(d)])
    return _finish(lam, A, Uhat, Ghat, r)


def rhkron_noreuse(lam, A, r, phis):
    """App. A (an independent factor set per mode) on a CP tensor."""
    d = len(A)
    Uhat = [T.qr_pos(sketch(lam, A, phis[j], j))[0] for j in range(d)]
    Ghat = full(lam, [Uhat[k].T @ A[k] for k in range(d)])
    return _finish(lam, A, Uhat, Ghat, r)


def rsthkron(lam, A, r, phis):
    """Alg. 4.3 (sequentially truncated) on a CP tensor."""
    d = len(A)
    B = list(A)
    Uhat = []
    for j in range(d):
        Q = T.qr_pos(sketch(lam, B, phis[j], j))[0]
        Uhat.append(Q)
        B[j] = Q.T @ B[j]
    return _finish(lam, A, Uhat, full(lam, B), r)
