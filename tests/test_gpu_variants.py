"""GPU parity of the sketch variants: the no-reuse algorithm (App. A) and subsampled
randomized Hadamard factors (Sec. 5.1), against the oracle on the same random draws."""
import numpy as np
import pytest

from gpu_common import T, dev, host, pytestmark_skip, rt, say, subspace_gap, synth, torch
from oracle import srht as H

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(pytestmark_skip, reason="needs a GPU")]


def noreuse_phis(dims, S, seed):
    shapes = T.noreuse_phi_shapes(dims, S)
    flat = synth.gaussians(seed, [sh for row in shapes for sh in row])
    d = len(dims)
    return [flat[j * d:(j + 1) * d] for j in range(d)]


def srht_pair(s, n, seed):
    """(oracle factor, device factor) from the same draws."""
    (rows, signs), = synth.srht_draws(seed, [(s, H.padded_size(n), n)])
    host_phi = H.srht_factor(n, rows, signs)
    dev_phi = rt.rtucker_srht_factor(n, torch.as_tensor(rows, device="cuda:0"), dev(signs))
    return host_phi, dev_phi


@pytest.mark.parametrize("s,n", [(1, 1), (4, 64), (7, 1024), (7, 512), (5, 500), (3, 15), (16, 16), (6, 1000)])
def test_srht_factor_bit_exact(s, n):
    say("srht factor", s, n)
    hp, dp = srht_pair(s, n, 10 + s + n)
    np.testing.assert_array_equal(host(dp), hp)


def test_srht_factor_rejects_bad_sizes():
    rows = torch.zeros(3, dtype=torch.int64, device="cuda:0")
    with pytest.raises(rt.RtuckerError):
        rt.rtucker_srht_factor(2, rows, dev(np.ones(2)))  # s = 3 > N = 2


def _noreuse_case(dims, r, p, seed, dtype):
    X = synth.bumps_field(dims, nbumps=25, noise_rel=1e-4, seed=seed).astype(np.float64)
    if dtype == torch.float32:
        X = X.astype(np.float32).astype(np.float64)
    S = rt.rtucker_sketch_sizes(dims, r, p, "rhkron_noreuse")
    assert S == T.subrank_matrix_sth([v + p for v in r])
    phis = noreuse_phis(dims, S, seed + 1)
    return X, S, phis


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
@pytest.mark.parametrize("dims,r,p", [((64, 72, 80), (6, 6, 6), 4), ((40, 36, 32, 28), (4, 5, 3, 4), 3),
                                      ((100, 90, 70), (16, 4, 15), 4)])
def test_decompose_noreuse_matches_oracle(dtype, tol, dims, r, p):
    say("noreuse", dims, r, dtype)
    X, S, phis = _noreuse_case(dims, list(r), p, 20, dtype)
    d = len(dims)
    pd = [[None if f is None else dev(f) for f in row] for row in phis]
    G, Us = rt.rtucker_decompose(dev(X, dtype), list(r), p, pd, algo="rhkron_noreuse", s=S)
    Gh, Uh = host(G), [host(u) for u in Us]
    Go, Uo = T.rhkron_noreuse(X, list(r), phis)
    e_g, e_o = T.rel_error(X, Gh, Uh), T.rel_error(X, Go, Uo)
    say(f"  e_gpu={e_g:.10e} e_oracle={e_o:.10e}")
    assert abs(e_g - e_o) <= tol
    for k in range(d):
        np.testing.assert_allclose(Uh[k].T @ Uh[k], np.eye(r[k]), atol=1e-12)


@pytest.mark.parametrize("algo", ["rhkron", "rsthkron", "rhkron_noreuse"])
def test_decompose_with_srht_factors(algo):
    """Every algorithm with SRHT factors made on the device, against the oracle's own
    factors from the same draws (FP64 64^3 random Tucker tensor, |de| <= 1e-10)."""
    say("srht decompose", algo)
    dims, r, p = (64, 64, 64), [8, 8, 8], 5
    X, _, _ = synth.random_tucker(dims, (8, 8, 8), 1e-6, seed=30)
    S = rt.rtucker_sketch_sizes(dims, r, p, algo)
    if algo == "rhkron":
        pairs = [srht_pair(S[k], dims[k], 40 + k) for k in range(3)]
        ph_h, ph_d = [a for a, _ in pairs], [b for _, b in pairs]
        Go, Uo = T.rhkron(X, r, ph_h)
    else:
        shapes = T.sth_phi_shapes(dims, S) if algo == "rsthkron" else T.noreuse_phi_shapes(dims, S)
        ph_h, ph_d = [], []
        for j in range(3):
            row = [None if sh is None else srht_pair(sh[0], sh[1], 50 + 3 * j + k) for k, sh in enumerate(shapes[j])]
            ph_h.append([None if q is None else q[0] for q in row])
            ph_d.append([None if q is None else q[1] for q in row])
        Go, Uo = (T.rsthkron if algo == "rsthkron" else T.rhkron_noreuse)(X, r, ph_h)
    G, Us = rt.rtucker_decompose(dev(X), r, p, ph_d, algo=algo, s=S)
    e_g = T.rel_error(X, host(G), [host(u) for u in Us])
    e_o = T.rel_error(X, Go, Uo)
    say(f"  e_gpu={e_g:.12e} e_oracle={e_o:.12e}")
    assert abs(e_g - e_o) <= 1e-10


def test_noreuse_recovers_where_reuse_is_capped():
    """Skewed ranks (16, 4, 15): the reuse sketch of mode 1 has rank at most 12, the
    no-reuse sketches are full; on an exact tensor only no-reuse recovers it (Sec. 4.3)."""
    dims, r, p = (100, 90, 70), [16, 4, 15], 4
    X, _, F = synth.random_tucker(dims, r, 0.0, seed=60)
    s = rt.rtucker_sketch_sizes(dims, r, p, "rhkron")
    ph = [dev(f) for f in synth.gaussians(61, [(s[k], dims[k]) for k in range(3)])]
    G, Us = rt.rtucker_decompose(dev(X), r, p, ph, s=s)
    e_reuse, _ = rt.rtucker_rel_error(dev(X), G, Us)
    S = rt.rtucker_sketch_sizes(dims, r, p, "rhkron_noreuse")
    pd = [[None if f is None else dev(f) for f in row] for row in noreuse_phis(dims, S, 62)]
    G, Us = rt.rtucker_decompose(dev(X), r, p, pd, algo="rhkron_noreuse", s=S)
    e_nr, _ = rt.rtucker_rel_error(dev(X), G, Us)
    say(f"  reuse e={e_reuse:.3e} no-reuse e={e_nr:.3e}")
    assert e_reuse > 1e-3 and e_nr < 1e-12
    for U, A in zip(Us, F):
        assert subspace_gap(host(U), A) < 1e-10


@pytest.mark.parametrize("shape,s", [((37, 150, 530), 7), ((5, 64), 4), ((3, 10), 5), ((2, 4096), 64), ((7, 3, 1), 1),
                                     ((64, 33, 512), 7), ((9, 2000), 20)])
def test_srht_fast_transform_sketch(shape, s):
    """The fast-transform SRHT sketch of the last mode against the oracle's dense factor,
    entry by entry (binary32 adds over log2 N stages)."""
    say("srht fast transform", shape, s)
    Q = shape[-1]
    (rows, signs), = synth.srht_draws(70 + Q + s, [(s, H.padded_size(Q), Q)])
    X = np.random.default_rng(71).standard_normal(shape).astype(np.float32).astype(np.float64)
    Z = rt.rtucker_srht_sketch_last(dev(X, torch.float32), torch.as_tensor(rows, device="cuda:0"), dev(signs))
    Phi = H.srht_factor(Q, rows, signs)
    want = T.ttm(X, Phi, len(shape) - 1)
    bound = T.ttm(np.abs(X), np.abs(Phi), len(shape) - 1)
    from gpu_common import assert_entrywise
    assert_entrywise(host(Z), want, bound, 2e-6 * max(1, int(np.log2(H.padded_size(Q)))), "SRHT sketch")


def test_srht_fast_transform_rejects_long_modes():
    X = torch.zeros((2, 5000), dtype=torch.float32, device="cuda:0")
    with pytest.raises(rt.RtuckerError):
        rt.rtucker_srht_sketch_last(X, torch.zeros(3, dtype=torch.int64, device="cuda:0"), dev(np.ones(5000)))
