"""FP64 oracle for the multi-TTM and its adjoint (gradients by the chain rule).

TEST INFRASTRUCTURE ONLY (see ``oracle.tucker``).

For Y = X x_1 A_1 ... x_d A_d (A_k of shape m_k x I_k, Sec. 2.1) and an
incoming gradient dY:
    dX   = dY x_1 A_1^T ... x_d A_d^T
    dA_n = dY_(n) Z_(n)^T   with  Z = X x_{k != n} A_k
(both unfoldings in the same C column order).  The Tucker reconstruction loss
L = ||X - (X x_k U_k^T) x_k U_k||^2 is differentiated through two multi-TTMs.
"""
from __future__ import annotations

import numpy as np

from . import tucker as T


def multi_ttm_all(X, As):
    return T.multi_ttm(np.asarray(X, dtype=np.float64), {k: A for k, A in enumerate(As)})


def multi_ttm_grads(X, As, dY):
    """Gradients (dX, [dA_k]) of <dY, X x_k A_k> with respect to X and each A_k."""
    X = np.asarray(X, dtype=np.float64)
    d = X.ndim
    dX = T.multi_ttm(dY, {k: A.T for k, A in enumerate(As)})
    dAs = []
    for n in range(d):
        Z = T.multi_ttm(X, {k: As[k] for k in range(d) if k != n})
        dAs.append(T.unfold(dY, n) @ T.unfold(Z, n).T)
    return dX, dAs


def recon_loss(X, Us):
    """L = ||X - X_hat||^2 with G = X x_k U_k^T and X_hat = G x_k U_k."""
    G = multi_ttm_all(X, [U.T for U in Us])
    Xh = multi_ttm_all(G, Us)
    R = np.asarray(X, dtype=np.float64) - Xh
    return float(np.sum(R * R)), G, Xh


def recon_loss_grads(X, Us):
    """(L, dL/dX, [dL/dU_k]) for the reconstruction loss, by the chain rule."""
    X = np.asarray(X, dtype=np.float64)
    L, G, Xh = recon_loss(X, Us)
    R = X - Xh
    dXh = -2.0 * R
    # X_hat = G x_k U_k
    dG, dU_rec = multi_ttm_grads(G, Us, dXh)
    # G = X x_k U_k^T  (A_k = U_k^T, so dU_k = dA_k^T)
    dX_fwd, dA_fwd = multi_ttm_grads(X, [U.T for U in Us], dG)
    dX = 2.0 * R + dX_fwd
    dUs = [a + b.T for a, b in zip(dU_rec, dA_fwd)]
    return L, dX, dUs
