"""Pins for the FP64 oracle: each check is fixed by the paper or by mathematics,
not by re-typing the oracle's own formulas.

Each oracle function is hit by at least one check that a plausible mistake
(dropped term, wrong sign, transposed operand, wrong index) would fail.
"""
import itertools
import os
from math import prod

import numpy as np
import pytest

import synth
from oracle import tucker as T
from oracle import lowp as L

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            out[key] = [float(v) for v in vals]
    return out


# ----------------------------------------------------------------- TTM / multi-TTM

def test_ttm_brute_force_3way():
    rng = np.random.default_rng(10)
    X = rng.standard_normal((4, 5, 6))
    for k in range(3):
        A = rng.standard_normal((3, X.shape[k]))
        Y = T.ttm(X, A, k)
        ref = np.zeros(Y.shape)
        for idx in itertools.product(*[range(n) for n in Y.shape]):
            acc = 0.0
            for t in range(X.shape[k]):
                src = list(idx)
                src[k] = t
                acc += A[idx[k], t] * X[tuple(src)]
            ref[idx] = acc
        np.testing.assert_allclose(Y, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dims", [(5, 6, 7), (3, 4, 5, 6)])
def test_kronecker_unfolding_identity(dims):
    """Sketch multi-TTM equals X_(n) times the transposed Kronecker product of the Phi_k,
    k != n, in ascending mode order for C-order unfoldings (Sec. 2.1 identity; Sec. 4.2
    definition of Omega_j as a Kronecker product)."""
    rng = np.random.default_rng(11)
    X = rng.standard_normal(dims)
    d = len(dims)
    s = [2, 3, 2, 3][:d]
    phis = [rng.standard_normal((s[k], dims[k])) for k in range(d)]
    for n in range(d):
        Y = T.kron_sketch(X, phis, n)
        K = np.ones((1, 1))
        for k in range(d):
            if k != n:
                K = np.kron(K, phis[k])
        ref = T.unfold(X, n) @ K.T
        assert Y.shape == (dims[n], prod(s[k] for k in range(d) if k != n))
        np.testing.assert_allclose(Y, ref, rtol=1e-13, atol=1e-12)


def test_sketch_brute_force_loops():
    rng = np.random.default_rng(12)
    X = rng.standard_normal((3, 4, 5))
    phis = [rng.standard_normal((2, n)) for n in X.shape]
    Y1 = T.kron_sketch(X, phis, 0)  # 3 x (2*2), columns (c2, c3) with c3 fastest
    for i, c2, c3 in itertools.product(range(3), range(2), range(2)):
        acc = 0.0
        for j, k in itertools.product(range(4), range(5)):
            acc += X[i, j, k] * phis[1][c2, j] * phis[2][c3, k]
        assert abs(Y1[i, c2 * 2 + c3] - acc) < 1e-12


def test_unfold_fold_roundtrip():
    rng = np.random.default_rng(13)
    X = rng.standard_normal((3, 4, 5, 2))
    for n in range(4):
        M = T.unfold(X, n)
        assert M.shape == (X.shape[n], X.size // X.shape[n])
        np.testing.assert_array_equal(T.fold(M, n, X.shape), X)
        # row i of the unfolding is the slice with i_n = i, flattened in C order
        np.testing.assert_array_equal(M[1], np.take(X, 1, axis=n).ravel())


def test_multi_ttm_mode_order_invariance():
    rng = np.random.default_rng(14)
    X = rng.standard_normal((6, 7, 8))
    As = {k: rng.standard_normal((3 + k, X.shape[k])) for k in range(3)}
    ref = T.multi_ttm(X, As)
    for perm in itertools.permutations(range(3)):
        Y = X
        for k in perm:
            Y = T.ttm(Y, As[k], k)
        np.testing.assert_allclose(Y, ref, rtol=1e-12, atol=1e-12)


def test_core_multi_ttm_kron_form():
    """G_hat_(1) = U1^T X_(1) (U2 kron U3) for C-order unfoldings."""
    rng = np.random.default_rng(15)
    X = rng.standard_normal((5, 6, 7))
    Us = [np.linalg.qr(rng.standard_normal((n, 3)))[0] for n in X.shape]
    G = T.multi_ttm(X, {k: U.T for k, U in enumerate(Us)})
    ref = Us[0].T @ T.unfold(X, 0) @ np.kron(Us[1], Us[2])
    np.testing.assert_allclose(T.unfold(G, 0), ref, rtol=1e-12, atol=1e-13)


# ----------------------------------------------------------------- sketch sizes

def test_subranks_reuse_workloads():
    """s = 4, 7, 3 for the three standard workloads (ell = 13^3, 40^3, 22^4)."""
    assert T.subranks_reuse([13, 13, 13]) == [4, 4, 4]
    assert T.subranks_reuse([40, 40, 40]) == [7, 7, 7]
    assert T.subranks_reuse([22, 22, 22, 22]) == [3, 3, 3, 3]
    # real-valued formula on non-borderline inputs
    for ell in ([8, 20, 20], [15, 15, 15], [7, 30, 11, 9], [36, 43, 40, 11, 16]):
        d = len(ell)
        Pr = float(prod(ell)) ** (1.0 / (d - 1))
        want = [int(np.ceil(Pr / li - 1e-12)) for li in ell]
        assert T.subranks_reuse(ell) == want


def test_subranks_reuse_feasible_and_minimal():
    rng = np.random.default_rng(16)
    for _ in range(200):
        d = int(rng.integers(2, 6))
        ell = [int(v) for v in rng.integers(2, 60, size=d)]
        s = T.subranks_reuse(ell)
        w = T.sketch_widths(s)
        assert all(w[n] >= ell[n] for n in range(d)), (ell, s, w)


def test_printed_reuse_vectors_feasible():
    g = read_golden("subranks.txt")
    for rkey, skey in (("miranda_r", "miranda_reuse_s"), ("sp_r", "sp_reuse_s")):
        ell = [int(v) + 5 for v in g[rkey]]
        s = [int(v) for v in g[skey]]
        w = T.sketch_widths(s)
        formula = T.subranks_reuse(ell)
        # printed vectors are component-wise no larger than the formula's
        assert all(a <= b for a, b in zip(s, formula))
        if rkey == "miranda_r":
            assert all(w[n] >= ell[n] for n in range(len(ell)))


def test_subrank_rows_match_paper_multisets():
    """With p = 5 the row rule reproduces every printed row of S as a multiset (Sec. 7.5, 7.6)."""
    g = read_golden("subranks.txt")
    for name, rkey in (("miranda", "miranda_r"), ("sp", "sp_r")):
        r = [int(v) for v in g[rkey]]
        d = len(r)
        for j in range(d):
            printed = [int(v) for k, v in enumerate(g[f"{name}_S_row{j + 1}"]) if k != j]
            row = T.subrank_row_sth(r[j] + 5, d - 1)
            assert sorted(row) == sorted(printed), (name, j, row, printed)
            assert prod(row) >= r[j] + 5


# ----------------------------------------------------------------- QR

@pytest.mark.parametrize("m,n", [(40, 7), (64, 16), (30, 30), (12, 20)])
def test_qr_pos_properties(m, n):
    rng = np.random.default_rng(17)
    Y = rng.standard_normal((m, n))
    Q, R = T.qr_pos(Y)
    c = min(m, n)
    assert Q.shape == (m, c) and R.shape == (c, n)
    np.testing.assert_allclose(Q.T @ Q, np.eye(c), atol=1e-13)
    np.testing.assert_allclose(Q @ R, Y, atol=1e-12 * np.linalg.norm(Y))
    assert np.all(np.diag(R) >= 0)
    assert np.allclose(np.tril(R, -1)[:, :c], 0.0)


def test_qr_pos_matches_gram_schmidt():
    """Unique thin QR with diag(R) > 0: equals modified Gram-Schmidt on a well-conditioned matrix."""
    rng = np.random.default_rng(18)
    Y = rng.standard_normal((50, 9))
    Q = np.zeros_like(Y)
    V = Y.copy()
    for j in range(9):
        for i in range(j):
            V[:, j] -= (Q[:, i] @ V[:, j]) * Q[:, i]
        Q[:, j] = V[:, j] / np.linalg.norm(V[:, j])
    Qo, _ = T.qr_pos(Y)
    np.testing.assert_allclose(Qo, Q, atol=1e-12)


# ----------------------------------------------------------------- STHOSVD / closed forms

def test_sthosvd_closed_form_e1():
    """Orthogonally decomposable tensor with lambda_i = 0.4^(i-1): STHOSVD at rank 10 has
    relative error 0.4^10 = 1.048576e-4, printed as 0.000104858 (Sec. 7.1)."""
    g = read_golden("e1_accuracy.txt")
    X, lam, _ = synth.superdiagonal(48, terms=48, seed=5)
    G, Us = T.sthosvd(X, [10, 10, 10])
    Us_full = [Us[j] for j in range(3)]
    # sthosvd returns V_j acting on X directly here
    e = T.rel_error(X, G, Us_full)
    closed = np.sqrt(np.sum(lam[10:] ** 2) / np.sum(lam ** 2))
    assert abs(closed - 0.4 ** 10) < 1e-18
    assert abs(e - closed) < 1e-12 * closed
    assert abs(e - g["sthosvd_rel_error"][0]) < 0.5e-9  # printed to 6 significant digits


def test_sthosvd_error_bound_and_subspace():
    """STHOSVD error^2 <= sum_j sum_{i > r_j} sigma_i^2(X_(j)) (Sec. 5, core bound), and the
    mode-1 factor spans the leading left singular subspace."""
    rng = np.random.default_rng(19)
    X = rng.standard_normal((9, 8, 7)) * np.exp(-np.arange(7))[None, None, :]
    r = [4, 3, 2]
    G, Us = T.sthosvd(X, r)
    err2 = np.linalg.norm(X - T.reconstruct(G, Us)) ** 2
    bound = sum(np.sum(np.linalg.svd(T.unfold(X, j), compute_uv=False)[r[j]:] ** 2) for j in range(3))
    assert err2 <= bound * (1 + 1e-12)
    U1, _, _ = np.linalg.svd(T.unfold(X, 0))
    P = U1[:, :4] @ U1[:, :4].T
    np.testing.assert_allclose(Us[0] @ Us[0].T, P, atol=1e-10)


def test_hosvd_equals_sthosvd_on_exact_rank():
    X, _, _ = synth.random_tucker((10, 9, 8), (3, 2, 4), 0.0, seed=20)
    for fn in (T.hosvd, T.sthosvd):
        G, Us = fn(X, [3, 2, 4])
        assert T.rel_error(X, G, Us) < 1e-13


# ----------------------------------------------------------------- randomized algorithms

def _phis_reuse(dims, s, seed):
    return synth.gaussians(seed, [(s[k], dims[k]) for k in range(len(dims))])


def _phis_sth(dims, S, seed):
    shapes = T.sth_phi_shapes(dims, S)
    flat = synth.gaussians(seed, [sh for row in shapes for sh in row])
    d = len(dims)
    return [flat[j * d:(j + 1) * d] for j in range(d)]


@pytest.mark.parametrize("algo", ["rhkron", "rsthkron"])
def test_exact_tucker_rank_recovery(algo):
    dims, core = (20, 18, 16), (4, 3, 5)
    X, _, factors = synth.random_tucker(dims, core, 0.0, seed=21)
    r = list(core)
    if algo == "rhkron":
        s = T.subranks_reuse([v + 2 for v in r])
        G, Us = T.rhkron(X, r, _phis_reuse(dims, s, 22))
    else:
        S = T.subrank_matrix_sth([v + 2 for v in r])
        G, Us = T.rsthkron(X, r, _phis_sth(dims, S, 22))
    assert T.rel_error(X, G, Us) < 1e-12
    for U, F in zip(Us, factors):
        np.testing.assert_allclose(U @ U.T, F @ F.T, atol=1e-10)
        np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-13)


def test_full_width_sketch_equals_sthosvd():
    """ltilde_n = I_n: U_hat_n is square orthogonal, so rHKron's error equals STHOSVD's."""
    rng = np.random.default_rng(23)
    X = rng.standard_normal((16, 16, 16)) + 3 * synth.random_tucker((16, 16, 16), (3, 3, 3), 0.0, seed=24)[0]
    s = [4, 4, 4]
    r = [5, 4, 6]
    G, Us, parts = T.rhkron(X, r, _phis_reuse(X.shape, s, 25), return_parts=True)
    for U in parts["Uhat"]:
        assert U.shape == (16, 16)
    Gs, Vs = T.sthosvd(X, r)
    assert abs(T.rel_error(X, G, Us) - T.rel_error(X, Gs, Vs)) < 1e-12
    for U, V in zip(Us, Vs):
        np.testing.assert_allclose(U @ U.T, V @ V.T, atol=1e-9)


def test_norm_identity_and_orthonormality():
    """||X - X_hat||^2 = ||X||^2 - ||G||^2 when U_j are orthonormal and G = X x_j U_j^T (Sec. 5)."""
    X, _, _ = synth.random_tucker((24, 20, 16), (5, 5, 5), 1e-2, seed=26)
    s = T.subranks_reuse([9, 9, 9])
    G, Us = T.rhkron(X, [5, 5, 5], _phis_reuse(X.shape, s, 27))
    for U in Us:
        np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-13)
    lhs = np.linalg.norm(X - T.reconstruct(G, Us)) ** 2
    rhs = np.linalg.norm(X) ** 2 - np.linalg.norm(G) ** 2
    assert abs(lhs - rhs) <= 1e-10 * np.linalg.norm(X) ** 2
    # G is the projection of X: G = X x_j U_j^T
    np.testing.assert_allclose(G, T.multi_ttm(X, {j: U.T for j, U in enumerate(Us)}), atol=1e-12)


def test_core_singular_values_bounded_by_input():
    """sigma_i(G_hat_(j)) <= sigma_i(X_(j)) for orthonormal U_hat (appendix lemma on core singular values)."""
    rng = np.random.default_rng(28)
    X = rng.standard_normal((16, 16, 16))
    s = [3, 3, 3]
    _, _, parts = T.rhkron(X, [4, 4, 4], _phis_reuse(X.shape, s, 29), return_parts=True)
    Gh = parts["Ghat"]
    for j in range(3):
        sg = np.linalg.svd(T.unfold(Gh, j), compute_uv=False)
        sx = np.linalg.svd(T.unfold(X, j), compute_uv=False)
        assert np.all(sg <= sx[: len(sg)] * (1 + 1e-12))


def test_error_split_and_projection_lemma():
    """eps_total <= eps_rand + eps_core (Sec. 5), eps_core equals the STHOSVD error of G_hat, and
    ||X - X x_j P_j||^2 = sum_j ||X x_{i<j} P_i x_j (I - P_j)||^2 (projection lemma, Sec. 5.2)."""
    X, _, _ = synth.random_tucker((18, 16, 14), (6, 6, 6), 5e-2, seed=30)
    r = [4, 4, 4]
    s = T.subranks_reuse([7, 7, 7])
    G, Us, parts = T.rhkron(X, r, _phis_reuse(X.shape, s, 31), return_parts=True)
    Uh, Gh, Vs = parts["Uhat"], parts["Ghat"], parts["V"]
    That = T.reconstruct(Gh, Uh)
    Tr = T.reconstruct(G, Us)
    eps_total = np.linalg.norm(X - Tr)
    eps_rand = np.linalg.norm(X - That)
    eps_core = np.linalg.norm(That - Tr)
    assert eps_total <= eps_rand + eps_core + 1e-12
    assert abs(eps_core - np.linalg.norm(Gh - T.reconstruct(G, Vs))) < 1e-10
    # STHOSVD bound on the core
    bound = sum(np.sum(np.linalg.svd(T.unfold(Gh, j), compute_uv=False)[r[j]:] ** 2) for j in range(3))
    assert eps_core ** 2 <= bound * (1 + 1e-10)
    # projection lemma
    P = [U @ U.T for U in Uh]
    lhs = np.linalg.norm(X - T.multi_ttm(X, {j: P[j] for j in range(3)})) ** 2
    rhs = 0.0
    for j in range(3):
        Z = T.multi_ttm(X, {i: P[i] for i in range(j)})
        Z = T.ttm(Z, np.eye(P[j].shape[0]) - P[j], j)
        rhs += np.linalg.norm(Z) ** 2
    assert abs(lhs - rhs) < 1e-10 * np.linalg.norm(X) ** 2


def test_rsthkron_phi_shapes_follow_truncation():
    S = [[1, 3, 5], [5, 1, 3], [3, 5, 1]]
    shapes = T.sth_phi_shapes((40, 30, 20), S)
    assert shapes[0] == [None, (3, 30), (5, 20)]
    assert shapes[1] == [(5, 15), None, (3, 20)]
    assert shapes[2] == [(3, 15), (5, 15), None]


def test_rsthkron_sketch_is_on_truncated_core():
    """Step j sketches the partially truncated core G_hat (Alg. 4.3): check mode-2 step by hand."""
    rng = np.random.default_rng(32)
    X = rng.standard_normal((10, 9, 8))
    S = [[1, 2, 3], [3, 1, 2], [2, 3, 1]]
    phis = _phis_sth(X.shape, S, 33)
    _, _, parts = T.rsthkron(X, [2, 2, 2], phis, return_parts=True)
    U1 = parts["Uhat"][0]
    G1 = T.ttm(X, U1.T, 0)
    Y = T.ttm(T.ttm(G1, phis[1][0], 0), phis[1][2], 2)
    Q, _ = np.linalg.qr(T.unfold(Y, 1))
    np.testing.assert_allclose(np.abs(Q.T @ parts["Uhat"][1]), np.eye(Q.shape[1]), atol=1e-10)


# ----------------------------------------------------------------- accuracy experiment (statistical)

@pytest.mark.slow
def test_e1_distribution_matches_paper():
    """Accuracy experiment (Sec. 7.1) at reduced size.  With Gaussian Phi and
    X = diag(0.4^(i-1)) x_k Q_k, the sketch only sees Phi_k Q_k, which is Gaussian for any
    n >= number of terms, so the error distribution does not depend on n; 64^3 stands in
    for 500^3 (terms beyond the 40th are below double precision)."""
    g = read_golden("e1_accuracy.txt")
    r = [10, 10, 10]
    s = T.subranks_reuse([15, 15, 15])
    assert s == [4, 4, 4]
    S = T.subrank_matrix_sth([15, 15, 15])
    e_re, e_st = [], []
    for trial in range(100):
        X, _, _ = synth.superdiagonal(64, seed=1000 + trial)
        G, Us = T.rhkron(X, r, _phis_reuse(X.shape, s, 5000 + trial))
        e_re.append(T.rel_error(X, G, Us))
        G, Us = T.rsthkron(X, r, _phis_sth(X.shape, S, 5000 + trial))
        e_st.append(T.rel_error(X, G, Us))
    e_re, e_st = np.array(e_re), np.array(e_st)
    opt = 0.4 ** 10
    # best multilinear rank-10 error of an orthogonally decomposable tensor is 0.4^10
    assert e_re.min() >= opt * (1 - 1e-9) and e_st.min() >= opt * (1 - 1e-9)
    for e, key in ((e_re, "rhkron_reuse"), (e_st, "rsthkron")):
        med = np.median(e)
        assert abs(med - g["sthosvd_rel_error"][0]) <= 0.01 * g["sthosvd_rel_error"][0]
        assert np.percentile(e, 75) <= g[f"{key}_upper_quartile"][0] * 1.02


# ----------------------------------------------------------------- emulated rounding

def test_round_bf16_against_bit_truncation_reference():
    """bf16 RNE from float32: compare the frexp/rint rounding with numpy float32 bit arithmetic."""
    rng = np.random.default_rng(34)
    x32 = np.concatenate([rng.standard_normal(20000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 20000),
                          np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -8 + 2 ** -20, 3.0e38, 1e-40,
                                    -1e-39, 0.0, -0.0], dtype=np.float32)]).astype(np.float32)
    got = L.round_bf16(x32.astype(np.float64))
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    ref = (((u + 0x7FFF + lsb) >> 16) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    np.testing.assert_array_equal(got, ref)
    # ties go to even
    assert L.round_bf16(1.0 + 2 ** -8) == 1.0
    assert L.round_bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def test_round_f32_matches_numpy_cast():
    rng = np.random.default_rng(35)
    x = rng.standard_normal(50000) * 10.0 ** rng.integers(-40, 38, 50000)
    np.testing.assert_array_equal(L.round_f32(x), x.astype(np.float32).astype(np.float64))


def test_round_f8_enumerated_grid():
    """Every E4M3 value is a fixed point; midpoints round to the even neighbour; saturation at 448."""
    vals = L.f8_decode(np.arange(256, dtype=np.uint8))
    fin = np.isfinite(vals)
    assert np.sum(~fin) == 2  # 0x7f and 0xff
    pos = np.unique(vals[fin & (vals >= 0)])
    assert pos.max() == 448.0 and len(pos) == 127
    assert pos[1] == 2.0 ** -9  # smallest subnormal
    np.testing.assert_array_equal(L.round_f8(pos), pos)
    np.testing.assert_array_equal(L.f8_bits(pos), np.arange(127, dtype=np.uint8))
    mids = 0.5 * (pos[1:] + pos[:-1])
    r = L.round_f8(mids)
    lo_bits = np.arange(126)
    want = np.where(lo_bits % 2 == 0, pos[:-1], pos[1:])
    np.testing.assert_array_equal(r, want)
    assert L.round_f8(1000.0) == 448.0 and L.round_f8(-460.0) == -448.0


def test_emulated_f64_equals_plain():
    X, _, _ = synth.random_tucker((12, 11, 10), (3, 3, 3), 1e-3, seed=36)
    s = T.subranks_reuse([5, 5, 5])
    ph = _phis_reuse(X.shape, s, 37)
    G1, U1 = T.rhkron(X, [3, 3, 3], ph)
    G2, U2 = L.rhkron_emulated(X, [3, 3, 3], ph, "f64", "f64")
    assert abs(T.rel_error(X, G1, U1) - T.rel_error(X, G2, U2)) < 1e-14
