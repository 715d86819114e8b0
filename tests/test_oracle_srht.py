"""CPU pins of the oracle's no-reuse algorithm (App. A), its subsampled randomized Hadamard
factors (Sec. 5.1) and its CP-form evaluation of the randomized algorithms, ending in the
SRHT panel of the accuracy experiment (Sec. 7.1) at the paper's size."""
import os

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import cp_form as CP
from oracle import srht as H
from oracle import tucker as T

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                key, *vals = line.split()
                out[key] = [float(v) for v in vals]
    return out


# ----------------------------------------------------------------- Hadamard factors

@pytest.mark.parametrize("N", [1, 2, 8, 64, 512])
def test_walsh_hadamard_definitions(N):
    Hm = H.walsh_hadamard(N)
    np.testing.assert_array_equal(Hm, scipy.linalg.hadamard(N))  # library's Sylvester matrix
    # closed form of the Sylvester ordering: H[i, j] = (-1)^popcount(i & j)
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    pop = np.vectorize(lambda v: bin(int(v)).count("1"))(i & j)
    np.testing.assert_array_equal(Hm, np.where(pop % 2 == 0, 1.0, -1.0))
    np.testing.assert_array_equal(Hm.T @ Hm, N * np.eye(N))


def test_srht_factor_rows_orthonormal_and_padding():
    rng = np.random.default_rng(3)
    (rows, signs), = synth.srht_draws(4, [(6, 64, 64)])
    Phi = H.srht_factor(64, rows, signs)
    np.testing.assert_allclose(Phi @ Phi.T, np.eye(6), atol=1e-15)
    assert np.all(np.abs(np.abs(Phi) - 1 / 8) == 0)
    # a mode of 50 is zero-padded to 64: the factor is the first 50 columns of the padded one
    (rows, signs), = synth.srht_draws(5, [(5, 64, 50)])
    Phi50 = H.srht_factor(50, rows, signs)
    full_signs = np.concatenate([signs, rng.choice([-1.0, 1.0], 14)])
    np.testing.assert_array_equal(Phi50, H.srht_factor(64, rows, full_signs)[:, :50])
    x = rng.standard_normal(50)
    xp = np.concatenate([x, np.zeros(14)])
    np.testing.assert_allclose(Phi50 @ x, H.srht_factor(64, rows, full_signs) @ xp, atol=1e-14)
    with pytest.raises(ValueError):
        H.srht_factor(50, [1, 1], signs)
    with pytest.raises(ValueError):
        H.srht_factor(50, [64], signs)


def test_srht_factor_is_sampled_transform_of_signed_data():
    """Phi x equals the FWHT of D x (zero-padded) sampled at the rows: checked with a
    plain recursive fast transform written here."""
    def fwht(v):
        v = v.copy()
        h = 1
        while h < len(v):
            for a in range(0, len(v), 2 * h):
                x, y = v[a:a + h].copy(), v[a + h:a + 2 * h].copy()
                v[a:a + h], v[a + h:a + 2 * h] = x + y, x - y
            h *= 2
        return v
    (rows, signs), = synth.srht_draws(6, [(7, 128, 100)])
    x = np.random.default_rng(7).standard_normal(100)
    want = fwht(np.concatenate([signs * x, np.zeros(28)]))[rows] / np.sqrt(128)
    np.testing.assert_allclose(H.srht_factor(100, rows, signs) @ x, want, atol=1e-13)


# ----------------------------------------------------------------- no-reuse algorithm (App. A)

def _noreuse_phis(dims, S, seed):
    shapes = T.noreuse_phi_shapes(dims, S)
    flat = synth.gaussians(seed, [sh for row in shapes for sh in row])
    d = len(dims)
    return [flat[j * d:(j + 1) * d] for j in range(d)]


def test_noreuse_with_shared_factors_is_the_reuse_algorithm():
    X, _, _ = synth.random_tucker((14, 12, 10), (3, 3, 3), 1e-2, seed=50)
    s = [3, 3, 3]
    phis = synth.gaussians(51, [(3, n) for n in X.shape])
    G1, U1 = T.rhkron(X, [3, 3, 3], phis)
    G2, U2 = T.rhkron_noreuse(X, [3, 3, 3], [[None if k == j else phis[k] for k in range(3)] for j in range(3)])
    np.testing.assert_allclose(G1, G2, atol=1e-13)
    for a, b in zip(U1, U2):
        np.testing.assert_allclose(a, b, atol=1e-13)
    assert s == [3, 3, 3]


def test_noreuse_sketch_is_explicit_kronecker():
    X = np.random.default_rng(52).standard_normal((5, 6, 7, 4))
    S = T.subrank_matrix_sth([4, 6, 6, 4])
    phis = _noreuse_phis(X.shape, S, 53)
    _, _, parts = T.rhkron_noreuse(X, [2, 2, 2, 2], phis, return_parts=True)
    for j in range(4):
        K = np.ones((1, 1))
        for k in range(4):
            if k != j:
                K = np.kron(K, phis[j][k].T)
        Q, _ = T.qr_pos(T.unfold(X, j) @ K)
        np.testing.assert_allclose(parts["Uhat"][j], Q, atol=1e-12)


@pytest.mark.parametrize("dims,r", [((20, 18, 16), (4, 3, 5)), ((9, 8, 7, 6), (2, 3, 2, 2))])
def test_noreuse_exact_rank_recovery(dims, r):
    X, _, F = synth.random_tucker(dims, r, 0.0, seed=54)
    S = T.subrank_matrix_sth([v + 2 for v in r])
    G, Us = T.rhkron_noreuse(X, list(r), _noreuse_phis(dims, S, 55))
    assert T.rel_error(X, G, Us) < 1e-12
    for U, A in zip(Us, F):
        assert np.linalg.norm(U @ U.T - A @ A.T, 2) < 1e-10


def test_noreuse_avoids_the_reuse_rank_cap():
    """With skewed ranks the reuse subranks cap a sketch's rank at prod_{k != n} min(r_k, s_k)
    (Sec. 4.3 recommends against reuse there); the no-reuse subrank matrix gives every mode
    a sketch of its own width, and an exact tensor is recovered."""
    dims, r, p = (40, 36, 30), (16, 4, 15), 4
    X, _, _ = synth.random_tucker(dims, r, 0.0, seed=56)
    s = T.subranks_reuse([v + p for v in r])
    cap = [int(np.prod([min(r[k], s[k]) for k in range(3) if k != n])) for n in range(3)]
    assert any(cap[n] < r[n] for n in range(3))
    Gr, Ur = T.rhkron(X, list(r), synth.gaussians(57, [(s[k], dims[k]) for k in range(3)]))
    assert T.rel_error(X, Gr, Ur) > 1e-3
    S = T.subrank_matrix_sth([v + p for v in r])
    G, Us = T.rhkron_noreuse(X, list(r), _noreuse_phis(dims, S, 58))
    assert T.rel_error(X, G, Us) < 1e-12


# ----------------------------------------------------------------- CP-form evaluation

@pytest.mark.parametrize("algo", ["rhkron", "rsthkron", "noreuse"])
def test_cp_form_equals_dense_oracle(algo):
    rng = np.random.default_rng(60)
    dims, K, r = (30, 26, 22), 12, [4, 4, 4]
    lam = 0.6 ** np.arange(K)
    A = [np.linalg.qr(rng.standard_normal((n, K)))[0] for n in dims]
    X = CP.full(lam, A)
    assert abs(CP.norm2(lam, A) - np.sum(X * X)) < 1e-13
    if algo == "rhkron":
        s = T.subranks_reuse([7, 7, 7])
        phis = synth.gaussians(61, [(s[k], dims[k]) for k in range(3)])
        Gd, Ud = T.rhkron(X, r, phis)
        Gc, Uc, e = CP.rhkron(lam, A, r, phis)
    elif algo == "rsthkron":
        S = T.subrank_matrix_sth([7, 7, 7])
        shapes = T.sth_phi_shapes(dims, S)
        flat = synth.gaussians(61, [sh for row in shapes for sh in row])
        phis = [flat[j * 3:(j + 1) * 3] for j in range(3)]
        Gd, Ud = T.rsthkron(X, r, phis)
        Gc, Uc, e = CP.rsthkron(lam, A, r, phis)
    else:
        S = T.subrank_matrix_sth([7, 7, 7])
        phis = _noreuse_phis(dims, S, 61)
        Gd, Ud = T.rhkron_noreuse(X, r, phis)
        Gc, Uc, e = CP.rhkron_noreuse(lam, A, r, phis)
    np.testing.assert_allclose(Gc, Gd, atol=1e-12)
    ed = T.rel_error(X, Gd, Ud)
    assert abs(e - ed) <= 1e-8 * ed


# ----------------------------------------------------------------- SRHT accuracy experiment

def _srht_phis(specs, seed):
    """SRHT factors for a list of (s, n) shapes (None kept)."""
    draws = synth.srht_draws(seed, [None if sp is None else (sp[0], H.padded_size(sp[1]), sp[1]) for sp in specs])
    return [None if sp is None else H.srht_factor(sp[1], *dr) for sp, dr in zip(specs, draws)]


@pytest.mark.slow
def test_e1_srht_panel_matches_paper():
    """Accuracy experiment (Sec. 7.1, SRHT panel) at the paper's size: 500^3 super-diagonal
    tensor with entries 0.4^(i-1) (40 terms; the rest are below double precision) rotated by
    random orthogonal matrices, rank (10, 10, 10), p = 5, 100 trials, Kronecker products of
    SRHT factors (modes of 500 zero-padded to 512, truncated modes of 15 to 16).  The paper
    prints the medians and quartiles of both algorithms; ours must have medians within 1 %
    and upper quartiles within 2 % of them."""
    g = read_golden("e1_accuracy.txt")
    n, K, r = 500, 40, [10, 10, 10]
    lam = 0.4 ** np.arange(K)
    s = T.subranks_reuse([15, 15, 15])
    S = T.subrank_matrix_sth([15, 15, 15])
    e_re, e_st = [], []
    for trial in range(100):
        rng = np.random.default_rng(1000 + trial)
        A = [synth.orthonormal(rng, n, K) for _ in range(3)]
        phis = _srht_phis([(s[k], n) for k in range(3)], 5000 + trial)
        e_re.append(CP.rhkron(lam, A, r, phis)[2])
        shapes = T.sth_phi_shapes((n, n, n), S)
        flat = _srht_phis([sh for row in shapes for sh in row], 7000 + trial)
        e_st.append(CP.rsthkron(lam, A, r, [flat[j * 3:(j + 1) * 3] for j in range(3)])[2])
    opt = 0.4 ** 10
    for e, key in ((np.array(e_re), "srht_rhkron_reuse"), (np.array(e_st), "srht_rsthkron")):
        assert e.min() >= opt * (1 - 1e-6)
        med = np.median(e)
        assert abs(med - g[f"{key}_median"][0]) <= 0.01 * g[f"{key}_median"][0], (key, med)
        assert np.percentile(e, 75) <= g[f"{key}_upper_quartile"][0] * 1.02, (key, np.percentile(e, 75))
