"""Plain FP64 CPU oracle for randomized Tucker decomposition with Kronecker sketches.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports or calls this module; only the tests, the package's
``smoke()`` check and the benchmark's CPU-baseline leg do.  It shares no code
with the GPU path.

Everything is written in the paper's order and notation, in float64, with
numpy as the only library (tensordot for each TTM, LAPACK QR and SVD).  Tensors
are C-ordered numpy arrays; mode indices are 0-based here (paper mode j is
index j-1).  The mode-n unfolding is taken in C order, which permutes the
columns of the paper's (column-major) unfolding: ranges and singular values
are unchanged, and the Kronecker factors of a multi-TTM appear in ascending
mode order (Sec. 2.1, multi-TTM unfolding identity).

Readings of the paper taken here (each also listed with the design notes):
  * "rHKron" is the factor-reuse algorithm (Alg. 4.4, Sec. 4.3): one Phi_k per mode.
  * The number of columns of U_hat_n is every column of the sketch,
    ltilde_n = prod_{k != n} s_k (clipped to I_n); it is never cut back to r_n + p
    (Sec. 4.2, "choosing subranks": a larger product is extra oversampling).
  * The subrank formula of Sec. 4.3 is read with the product over k != j and the
    (d-1)-th root.
  * QR factors are normalised so that diag(R) >= 0.
  * STHOSVD takes modes in order 1..d; singular vector signs are fixed so that
    the largest-magnitude entry of each vector is positive.
"""
from __future__ import annotations

from math import prod

import numpy as np


# --------------------------------------------------------------------------
# Tensor operations (Sec. 2.1)
# --------------------------------------------------------------------------

def ttm(X: np.ndarray, A: np.ndarray, k: int) -> np.ndarray:
    """Mode-k tensor-times-matrix X x_k A with A of shape m x I_k (Sec. 2.1).

    Its mode-k unfolding is A times the mode-k unfolding of X.
    """
    A = np.asarray(A, dtype=np.float64)
    if A.shape[1] != X.shape[k]:
        raise ValueError(f"ttm: A has {A.shape[1]} columns, mode {k} has size {X.shape[k]}")
    Y = np.tensordot(A, X, axes=([1], [k]))  # shape m x (other modes, in order)
    return np.moveaxis(Y, 0, k)


def multi_ttm(X: np.ndarray, mats: dict) -> np.ndarray:
    """Multi-TTM X x_k A_k over the modes k that are keys of ``mats`` (Sec. 2.1).

    Distinct modes commute, so the order of application does not change the
    exact result; ascending mode order is used.
    """
    Y = X
    for k in sorted(mats):
        Y = ttm(Y, mats[k], k)
    return Y


def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding, C order: rows indexed by i_n, columns by the other modes (last fastest)."""
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1)


def fold(M: np.ndarray, n: int, shape) -> np.ndarray:
    """Inverse of ``unfold`` for a tensor of the given shape."""
    rest = [s for i, s in enumerate(shape) if i != n]
    return np.moveaxis(M.reshape([shape[n]] + rest), 0, n)


# --------------------------------------------------------------------------
# Sketch sizes (Sec. 4.2 and Sec. 4.3, "choosing subranks")
# --------------------------------------------------------------------------

def subranks_reuse(ell) -> list[int]:
    """Subrank vector of the factor-reuse algorithm (Sec. 4.3).

    s_i = ceil( (prod_j ell_j)^(1/(d-1)) / ell_i ), evaluated exactly in
    integers: s_i is the least s with (s * ell_i)^(d-1) >= prod_j ell_j.
    """
    ell = [int(v) for v in ell]
    d = len(ell)
    if d < 2:
        raise ValueError("need d >= 2")
    P = prod(ell)
    out = []
    for li in ell:
        s = 1
        while (s * li) ** (d - 1) < P:
            s += 1
        out.append(s)
    return out


def sketch_widths(s) -> list[int]:
    """ltilde_n = prod_{k != n} s_k: number of columns of the mode-n sketch (Sec. 4.2)."""
    return [prod(int(v) for i, v in enumerate(s) if i != n) for n in range(len(s))]


def _factor_splits(n: int, parts: int, lo: int = 2):
    """All non-increasing tuples of ``parts`` integers >= lo whose product is n."""
    if parts == 1:
        if n >= lo:
            yield (n,)
        return
    f = lo
    while f ** parts <= n:
        if n % f == 0:
            for rest in _factor_splits(n // f, parts - 1, f):
                yield rest + (f,)
        f += 1


def subrank_row_sth(ell_j: int, parts: int) -> tuple[int, ...]:
    """One row of the subrank matrix for the sequentially truncated algorithm (Sec. 4.2).

    The row is made of ``parts`` = d-1 integer factors of ell_j; when ell_j has no
    such split the oversampling is raised: ell_j is increased to the least value
    that splits into ``parts`` factors, each at least 2.  Among the splits of
    that value the most balanced one is taken (smallest largest factor, then
    smallest next factor, ...).  Returned in non-increasing order.
    """
    v = int(ell_j)
    while True:
        splits = list(_factor_splits(v, parts))
        if splits:
            return min(splits)  # tuples are non-increasing; min = most balanced
        v += 1


def subrank_matrix_sth(ell) -> list[list[int]]:
    """Subrank matrix S (diagonal 1) for the sequentially truncated algorithm.

    Row j holds the factors of ``subrank_row_sth(ell_j, d-1)`` assigned to the
    modes k != j in ascending mode order, largest factor first.  The paper does
    not fix this assignment.
    """
    d = len(ell)
    S = []
    for j in range(d):
        fac = list(subrank_row_sth(ell[j], d - 1))
        row = []
        for k in range(d):
            row.append(1 if k == j else fac.pop(0))
        S.append(row)
    return S


# --------------------------------------------------------------------------
# Randomized range finder pieces (Alg. 2.3, with a Kronecker Omega)
# --------------------------------------------------------------------------

def qr_pos(Y: np.ndarray):
    """Thin QR Y = Q R with diag(R) >= 0 (the range-finder's QR step).

    Returns Q (m x min(m,n)) and R (min(m,n) x n).
    """
    Q, R = np.linalg.qr(np.asarray(Y, dtype=np.float64), mode="reduced")
    sgn = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    return Q * sgn[None, :], R * sgn[:, None]


def kron_sketch(X: np.ndarray, phis, n: int) -> np.ndarray:
    """Mode-n sketch Y = X x_{k != n} Phi_k, returned as its mode-n unfolding (I_n x prod s_k).

    This is the multi-TTM of the factor-reuse algorithm's sketch step: the mode-n
    unfolding of X times the transposed Kronecker product of the Phi_k, k != n.
    """
    Y = multi_ttm(X, {k: phis[k] for k in range(X.ndim) if k != n})
    return unfold(Y, n)


# --------------------------------------------------------------------------
# STHOSVD (Alg. 2.2) used as the core truncation
# --------------------------------------------------------------------------

def _sign_fix(V: np.ndarray) -> np.ndarray:
    idx = np.argmax(np.abs(V), axis=0)
    sgn = np.where(V[idx, np.arange(V.shape[1])] < 0.0, -1.0, 1.0)
    return V * sgn[None, :]


def sthosvd(G: np.ndarray, r):
    """Deterministic STHOSVD in mode order 1..d (Alg. 2.2).

    For each mode j: V_j = first r_j left singular vectors of the current core's
    mode-j unfolding, then G <- G x_j V_j^T.  Returns (G, [V_j]).
    """
    G = np.asarray(G, dtype=np.float64)
    Vs = []
    for j in range(G.ndim):
        Uj, _, _ = np.linalg.svd(unfold(G, j), full_matrices=False)
        V = _sign_fix(Uj[:, : int(r[j])])
        Vs.append(V)
        G = ttm(G, V.T, j)
    return G, Vs


def hosvd(X: np.ndarray, r):
    """Deterministic HOSVD (Alg. 2.1): every U_j from X itself, then G = X x_j U_j^T."""
    Us = []
    for j in range(X.ndim):
        Uj, _, _ = np.linalg.svd(unfold(X, j), full_matrices=False)
        Us.append(_sign_fix(Uj[:, : int(r[j])]))
    G = multi_ttm(X, {j: U.T for j, U in enumerate(Us)})
    return G, Us


# --------------------------------------------------------------------------
# The two randomized algorithms with Kronecker sketches
# --------------------------------------------------------------------------

def core_order(dims) -> list[int]:
    """Modes sorted by size, largest first (ties by mode index); any order is exact."""
    return sorted(range(len(dims)), key=lambda k: (-dims[k], k))


def rhkron(X: np.ndarray, r, phis, *, return_parts: bool = False):
    """Randomized HOSVD with Kronecker factor reuse (Alg. 4.4, Sec. 4.3).

    ``phis[k]`` is Phi_k (s_k x I_k).  For every mode n: sketch
    Y = X x_{k != n} Phi_k, thin QR of Y_(n) gives U_hat_n.  Then
    G_hat = X x_1 U_hat_1^T ... x_d U_hat_d^T, STHOSVD(G_hat, r) -> (G, V_j),
    and U_j = U_hat_j V_j.
    """
    X = np.asarray(X, dtype=np.float64)
    d = X.ndim
    Uhat = []
    for n in range(d):
        Q, _ = qr_pos(kron_sketch(X, phis, n))
        Uhat.append(Q)
    Ghat = X
    for k in core_order(X.shape):
        Ghat = ttm(Ghat, Uhat[k].T, k)
    G, Vs = sthosvd(Ghat, r)
    Us = [Uh @ V for Uh, V in zip(Uhat, Vs)]
    if return_parts:
        return G, Us, {"Uhat": Uhat, "Ghat": Ghat, "V": Vs}
    return G, Us


def rhkron_noreuse(X: np.ndarray, r, phis, *, return_parts: bool = False):
    """Randomized HOSVD with an independent set of Kronecker factors per mode (App. A).

    ``phis[j][k]`` is Phi_{j,k} (s_{j,k} x I_k) for k != j; row j of the subrank matrix
    S follows the rule of Sec. 4.2 (``subrank_matrix_sth``).  For every mode j: sketch
    Y = X x_{k != j} Phi_{j,k}, thin QR of Y_(j) gives U_hat_j.  Then, as in the reuse
    algorithm, G_hat = X x_1 U_hat_1^T ... x_d U_hat_d^T, STHOSVD(G_hat, r) and
    U_j = U_hat_j V_j.
    """
    X = np.asarray(X, dtype=np.float64)
    d = X.ndim
    Uhat = []
    for j in range(d):
        Y = multi_ttm(X, {k: phis[j][k] for k in range(d) if k != j})
        Q, _ = qr_pos(unfold(Y, j))
        Uhat.append(Q)
    Ghat = X
    for k in core_order(X.shape):
        Ghat = ttm(Ghat, Uhat[k].T, k)
    G, Vs = sthosvd(Ghat, r)
    Us = [Uh @ V for Uh, V in zip(Uhat, Vs)]
    if return_parts:
        return G, Us, {"Uhat": Uhat, "Ghat": Ghat, "V": Vs}
    return G, Us


def noreuse_phi_shapes(dims, S):
    """Shapes of Phi_{j,k} for the no-reuse algorithm (App. A): s_{j,k} x I_k (X is never
    truncated before it is sketched).  Diagonal entries are None."""
    d = len(dims)
    return [[None if k == j else (int(S[j][k]), int(dims[k])) for k in range(d)] for j in range(d)]


def sth_phi_shapes(dims, S):
    """Shapes of Phi_{j,k} for the sequentially truncated algorithm (Sec. 4.2).

    Phi_{j,k} is s_{j,k} x (current size of mode k at step j): the truncated size
    c_k = min(I_k, prod_{i != k} s_{k,i}) for k < j, the original I_k for k > j.
    Diagonal entries are None.
    """
    d = len(dims)
    c = [min(int(dims[k]), prod(int(S[k][i]) for i in range(d) if i != k)) for k in range(d)]
    shapes = []
    for j in range(d):
        row = []
        for k in range(d):
            if k == j:
                row.append(None)
            else:
                row.append((int(S[j][k]), c[k] if k < j else int(dims[k])))
        shapes.append(row)
    return shapes


def rsthkron(X: np.ndarray, r, phis, *, return_parts: bool = False):
    """Randomized STHOSVD with Kronecker products (Alg. 4.3, Sec. 4.2).

    ``phis[j][k]`` is Phi_{j,k}.  For j = 1..d: Y = G_hat x_{k != j} Phi_{j,k},
    thin QR of Y_(j) gives U_hat_j, and G_hat <- G_hat x_j U_hat_j^T.  Then
    STHOSVD(G_hat, r) and U_j = U_hat_j V_j.
    """
    X = np.asarray(X, dtype=np.float64)
    d = X.ndim
    Ghat = X
    Uhat = []
    for j in range(d):
        Y = multi_ttm(Ghat, {k: phis[j][k] for k in range(d) if k != j})
        Q, _ = qr_pos(unfold(Y, j))
        Uhat.append(Q)
        Ghat = ttm(Ghat, Q.T, j)
    G, Vs = sthosvd(Ghat, r)
    Us = [Uh @ V for Uh, V in zip(Uhat, Vs)]
    if return_parts:
        return G, Us, {"Uhat": Uhat, "Ghat": Ghat, "V": Vs}
    return G, Us


# --------------------------------------------------------------------------
# Error (Sec. 5)
# --------------------------------------------------------------------------

def reconstruct(G: np.ndarray, Us) -> np.ndarray:
    """X_hat = G x_1 U_1 ... x_d U_d."""
    return multi_ttm(np.asarray(G, dtype=np.float64), {j: U for j, U in enumerate(Us)})


def rel_error(X: np.ndarray, G: np.ndarray, Us) -> float:
    """Relative reconstruction error ||X - G x_j U_j|| / ||X||, by explicit residual."""
    X = np.asarray(X, dtype=np.float64)
    return float(np.linalg.norm(X - reconstruct(G, Us)) / np.linalg.norm(X))
