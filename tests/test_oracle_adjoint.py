"""Pins of the oracle's multi-TTM adjoint and reconstruction-loss gradients
(Sec. 2.1 multi-TTM; chain rule through G = X x_k U_k^T, X_hat = G x_k U_k).

Each check is independent of the formulas it tests: explicit Kronecker
matrices, finite differences (exact for the linear and quadratic cases),
the projector closed form, and the zero gradient at an exact fit."""
import numpy as np

import synth
from oracle import adjoint as AD
from oracle import tucker as T


def _kron_all(As):
    K = np.ones((1, 1))
    for A in As:  # C order: the first mode is the slowest index
        K = np.kron(K, A)
    return K


def test_multi_ttm_is_kronecker_matrix():
    rng = np.random.default_rng(11)
    X = rng.standard_normal((4, 3, 5))
    As = [rng.standard_normal((2, 4)), rng.standard_normal((3, 3)), rng.standard_normal((4, 5))]
    Y = AD.multi_ttm_all(X, As)
    assert np.allclose(Y.reshape(-1), _kron_all(As) @ X.reshape(-1), rtol=0, atol=1e-13)


def test_multi_ttm_adjoint_dx_is_kronecker_transpose():
    rng = np.random.default_rng(12)
    X = rng.standard_normal((4, 3, 5))
    As = [rng.standard_normal((2, 4)), rng.standard_normal((3, 3)), rng.standard_normal((4, 5))]
    dY = rng.standard_normal((2, 3, 4))
    dX, _ = AD.multi_ttm_grads(X, As, dY)
    assert np.allclose(dX.reshape(-1), _kron_all(As).T @ dY.reshape(-1), rtol=0, atol=1e-13)


def test_multi_ttm_grads_match_unit_differences():
    """f(X, A) = <dY, X x_k A_k> is linear in X and in each A_k separately, so a
    unit step gives each partial derivative exactly (up to rounding)."""
    rng = np.random.default_rng(13)
    X = rng.standard_normal((3, 4, 2))
    As = [rng.standard_normal((2, 3)), rng.standard_normal((5, 4)), rng.standard_normal((3, 2))]
    dY = rng.standard_normal((2, 5, 3))

    def f(X_, As_):
        return float(np.sum(dY * AD.multi_ttm_all(X_, As_)))

    dX, dAs = AD.multi_ttm_grads(X, As, dY)
    f0 = f(X, As)
    for idx in np.ndindex(X.shape):
        Xp = X.copy()
        Xp[idx] += 1.0
        assert abs((f(Xp, As) - f0) - dX[idx]) < 1e-12
    for k in range(3):
        for idx in np.ndindex(As[k].shape):
            Ap = [A.copy() for A in As]
            Ap[k][idx] += 1.0
            assert abs((f(X, Ap) - f0) - dAs[k][idx]) < 1e-12


def test_recon_loss_grads_match_central_differences():
    """L is quadratic in X (central differences exact) and quartic in each U_k."""
    rng = np.random.default_rng(14)
    X = rng.standard_normal((5, 4, 3))
    Us = [rng.standard_normal((5, 2)), rng.standard_normal((4, 3)), rng.standard_normal((3, 2))]
    L, dX, dUs = AD.recon_loss_grads(X, Us)
    assert abs(L - AD.recon_loss(X, Us)[0]) == 0.0
    for idx in np.ndindex(X.shape):
        Xp, Xm = X.copy(), X.copy()
        Xp[idx] += 0.5
        Xm[idx] -= 0.5
        fd = AD.recon_loss(Xp, Us)[0] - AD.recon_loss(Xm, Us)[0]
        assert abs(fd - dX[idx]) <= 1e-10 * max(1.0, abs(dX[idx]))
    h = 1e-5
    for k in range(3):
        for idx in np.ndindex(Us[k].shape):
            Up = [U.copy() for U in Us]
            Um = [U.copy() for U in Us]
            Up[k][idx] += h
            Um[k][idx] -= h
            fd = (AD.recon_loss(X, Up)[0] - AD.recon_loss(X, Um)[0]) / (2 * h)
            assert abs(fd - dUs[k][idx]) <= 1e-6 * max(1.0, abs(dUs[k][idx]))


def test_recon_loss_projector_closed_form():
    """Orthonormal U_k make P = (x) U_k U_k^T an orthogonal projector, so
    L = ||(I - P) X||^2 and dL/dX = 2 (X - P X)."""
    X, _, _ = synth.random_tucker((12, 10, 8), (4, 4, 3), 0.3, seed=5)
    Us = synth.fixed_factors((12, 10, 8), (3, 3, 2), seed=6)
    L, dX, _ = AD.recon_loss_grads(X, Us)
    Pk = [U @ U.T for U in Us]
    PX = (_kron_all(Pk) @ X.reshape(-1)).reshape(X.shape)
    assert np.allclose(dX, 2.0 * (X - PX), rtol=0, atol=1e-12)
    assert abs(L - float(np.sum((X - PX) ** 2))) <= 1e-12 * L


def test_recon_loss_zero_at_exact_fit():
    """X = C x_k U_k with orthonormal U_k is reproduced exactly: L = 0 and every gradient is 0."""
    rng = np.random.default_rng(7)
    Us = synth.fixed_factors((12, 10, 8), (3, 3, 2), seed=8)
    C = rng.standard_normal((3, 3, 2))
    X = T.multi_ttm(C, {k: U for k, U in enumerate(Us)})
    L, dX, dUs = AD.recon_loss_grads(X, Us)
    assert L < 1e-26
    assert np.max(np.abs(dX)) < 1e-13
    for g in dUs:
        assert np.max(np.abs(g)) < 1e-13
