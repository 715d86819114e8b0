"""Pins of the emulated-precision oracle's low-precision branches (CPU only).

The emulated rHKron (Alg. 4.4) and rSTHKron (Alg. 4.3) round operands at the
points where the GPU stores them in a narrow format.  Here every intermediate
they return is rebuilt independently from the definitions: the sketch as the
mode-n unfolding times an explicit Kronecker product of the rounded factors
(np.kron, the Kronecker form of the multi-TTM in Sec. 2.1), the core as explicit
products of unfoldings, bfloat16 rounding by integer arithmetic on binary64 bit
patterns (checked against torch's conversion) and binary32 rounding by numpy's
cast (neither is the oracle's own rounding routine).  A wrong
rounding point (a factor left unrounded, U_hat rounded to the wrong format, a
missing binary32 store) changes these intermediates by far more than the 1e-12
tolerance; each test also checks that the roundings it pins do change them.
"""
import numpy as np
import pytest

import synth
from oracle import lowp as L
from oracle import tucker as T

torch = pytest.importorskip("torch")


def bf16(a):
    """bfloat16 rounding (nearest, ties to even) of float64 values by integer arithmetic
    on their bit patterns: keep the sign, the exponent and 7 fraction bits.  Valid in
    the normal range of binary32, which every value here is in."""
    a = np.asarray(a, dtype=np.float64)
    tiny = np.abs(a[a != 0])
    assert tiny.size == 0 or (tiny.min() > 2.0 ** -126 and tiny.max() < 2.0 ** 127)
    u = a.view(np.uint64)
    drop = np.uint64(45)
    lsb = (u >> drop) & np.uint64(1)
    out = ((u + (np.uint64(1) << np.uint64(44)) - np.uint64(1) + lsb) >> drop) << drop
    return out.view(np.float64)


def test_bf16_helper_agrees_with_torch_on_binary32_inputs():
    x = np.random.default_rng(39).standard_normal(4096).astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(bf16(x), ref)


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def unf(X, n):
    perm = [n] + [k for k in range(X.ndim) if k != n]
    return np.transpose(X, perm).reshape(X.shape[n], -1)


def fld(M, n, shape):
    rest = [shape[k] for k in range(len(shape)) if k != n]
    perm = list(range(1, n + 1)) + [0] + list(range(n + 1, len(shape)))
    return np.transpose(M.reshape([shape[n]] + rest), perm)


def kron_all(mats):
    out = np.ones((1, 1))
    for M in mats:
        out = np.kron(out, M)
    return out


def kron_sketch(X, factors, n):
    """Y_(n) = X_(n) (Phi_a^T kron Phi_b^T kron ...), modes a < b < ... other than n."""
    return unf(X, n) @ kron_all([factors[k].T for k in range(X.ndim) if k != n])


def contract(X, U, n):
    """X x_n U^T as an explicit product of the mode-n unfolding."""
    shape = list(X.shape)
    shape[n] = U.shape[1]
    return fld(U.T @ unf(X, n), n, shape)


def qr_plus(Y):
    Q, R = np.linalg.qr(Y)
    return Q * np.where(np.diag(R) < 0, -1.0, 1.0)[None, :]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _inputs(dims, s, seed):
    """binary32-exact tensor and factors (the GPU's inputs are binary32 tensors)."""
    X, _, _ = synth.random_tucker(dims, [min(4, n) for n in dims], 1e-2, seed=seed)
    X = f32(X)
    phis = [f32(p) for p in synth.gaussians(seed + 1, [(s[k], dims[k]) for k in range(len(dims))])]
    return X, phis


@pytest.mark.parametrize("sketch_fmt,ttm_fmt", [("bf16", "bf16"), ("f8e4m3", "f32"), ("f8e4m3", "bf16")])
def test_rhkron_emulated_rounding_points(sketch_fmt, ttm_fmt):
    dims, s = (12, 10, 8), [3, 3, 3]
    X, phis = _inputs(dims, s, 40)
    rs = bf16 if sketch_fmt == "bf16" else L.round_f8  # E4M3 has no independent library rounding here
    rt = bf16 if ttm_fmt == "bf16" else f32
    _, _, parts = L.rhkron_emulated(X, [3, 3, 3], phis, sketch_fmt, ttm_fmt, return_parts=True)
    for n in range(3):
        want = kron_sketch(rs(X), [rs(p) for p in phis], n)
        assert rel(parts["Y"][n], want) <= 1e-13
        # the sketch's rounding points matter: unrounded factors give another sketch
        assert rel(kron_sketch(rs(X), phis, n), want) > 1e-4
        np.testing.assert_allclose(parts["Uhat"][n], qr_plus(want), atol=1e-10)
    U = parts["Uhat"]
    # core: largest mode first (0, 1, 2 here), first contraction on the rounded X and U_hat,
    # binary32 stores between contractions, binary64 result
    G1 = f32(contract(rt(X), rt(U[0]), 0))
    G2 = f32(contract(G1, f32(U[1]), 1))
    want = contract(G2, f32(U[2]), 2)
    assert rel(parts["Ghat"], want) <= 1e-13
    exact = contract(contract(contract(X, U[0], 0), U[1], 1), U[2], 2)
    assert rel(exact, want) > (1e-4 if ttm_fmt == "bf16" else 1e-8)  # the core's roundings are visible


def test_rhkron_emulated_f8_sketch_matches_bitwise_decoder():
    """The FP8 sketch operand equals the E4M3 value whose bit pattern the encoder gives."""
    X, phis = _inputs((12, 10, 8), [3, 3, 3], 41)
    q = L.round_f8(X)
    np.testing.assert_array_equal(L.f8_decode(L.f8_bits(q)), q)


@pytest.mark.parametrize("dims,S", [((12, 10, 8), [[1, 3, 3], [3, 1, 3], [3, 3, 1]]),
                                    ((6, 7, 5, 6), [[1, 2, 2, 2], [2, 1, 2, 2], [2, 2, 1, 2], [2, 2, 2, 1]])])
@pytest.mark.parametrize("fmt", ["bf16", "f32"])
def test_rsthkron_emulated_rounding_points(dims, S, fmt):
    d = len(dims)
    X, _ = _inputs(dims, [2] * d, 42)
    shapes = T.sth_phi_shapes(dims, S)
    flat = synth.gaussians(43, [sh for row in shapes for sh in row])
    phis = [[None if f is None else f32(f) for f in flat[j * d:(j + 1) * d]] for j in range(d)]
    r = [2] * d
    _, _, parts = L.rsthkron_emulated(X, r, phis, fmt, return_parts=True)
    first = bf16 if fmt == "bf16" else f32
    G = first(X)
    for j in range(d):
        rj = first if j == 0 else f32  # after the first step the core is binary32
        fac = {k: rj(phis[j][k]) for k in range(d) if k != j}
        Y = unf(G, j) @ kron_all([fac[k].T for k in range(d) if k != j])
        assert rel(parts["Y"][j], Y) <= 1e-13, j
        if fmt == "bf16" and j == 0:
            unrounded = unf(G, j) @ kron_all([phis[j][k].T for k in range(d) if k != j])
            assert rel(unrounded, Y) > 1e-4
        Q = qr_plus(Y)
        np.testing.assert_allclose(parts["Uhat"][j], Q, atol=1e-10)
        G = contract(G, rj(parts["Uhat"][j]), j)
        if j < d - 1:
            G = f32(G)
    assert rel(parts["Ghat"], G) <= 1e-13


def test_rsthkron_emulated_f64_equals_plain():
    dims, S = (12, 10, 8), [[1, 3, 3], [3, 1, 3], [3, 3, 1]]
    X, _ = _inputs(dims, [3, 3, 3], 44)
    shapes = T.sth_phi_shapes(dims, S)
    flat = synth.gaussians(45, [sh for row in shapes for sh in row])
    phis = [flat[j * 3:(j + 1) * 3] for j in range(3)]
    G1, U1 = T.rsthkron(X, [3, 3, 3], phis)
    G2, U2 = L.rsthkron_emulated(X, [3, 3, 3], phis, "f64")
    assert abs(T.rel_error(X, G1, U1) - T.rel_error(X, G2, U2)) < 1e-14


def test_emulated_error_floor_scales_with_unit_roundoff():
    """On an exact low-rank tensor the emulated error is set by the rounding of X and the
    factors: about u = 2^-8 for bfloat16 and 2^-24 for binary32 (a dropped rounding gives
    a far smaller error, a misplaced one a far larger)."""
    X, _, _ = synth.random_tucker((24, 20, 16), (3, 3, 3), 0.0, seed=46)
    X = f32(X)
    s = T.subranks_reuse([5, 5, 5])
    phis = synth.gaussians(47, [(s[k], X.shape[k]) for k in range(3)])
    eb = T.rel_error(X, *L.rhkron_emulated(X, [3, 3, 3], phis, "bf16", "bf16"))
    e32 = T.rel_error(X, *L.rhkron_emulated(X, [3, 3, 3], phis, "f32", "f32"))
    assert 2 ** -8 / 8 < eb < 2 ** -8 * 2
    assert e32 < 2 ** -24 * 8
