"""GPU parity: each entry point of the C ABI against the FP64 oracle on the same
seeded inputs (sizes span several tiles and ragged tails)."""
import numpy as np
import pytest

from gpu_common import (DEV, T, assert_entrywise, dev, host, pytestmark_skip, reuse_phis, rt, say, sth_phis,
                        subspace_gap, synth, torch)
from oracle import lowp as L

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(pytestmark_skip, reason="needs a GPU")]


# ------------------------------------------------------------------ conversion (bit-exact)
def _convert_inputs():
    rng = np.random.default_rng(100)
    x = rng.standard_normal(1 << 18) * np.exp2(rng.integers(-140, 128, 1 << 18))
    grid = L.f8_decode(np.arange(0, 127, dtype=np.uint8))
    mids = 0.5 * (grid[1:] + grid[:-1])
    special = np.array([0.0, -0.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 2 ** -126, 2 ** -130, -2 ** -133, 2 ** -134,
                        3.3e38, 448.0, 464.0, 500.0, -1e6, 2 ** -10, 2 ** -9 * 1.5])
    return np.concatenate([x, grid, -grid, mids, -mids, special])


@pytest.mark.parametrize("src", ["f32", "f64"])
def test_convert_bf16_bit_exact(src):
    say("convert bf16", src)
    x = _convert_inputs()
    if src == "f32":
        x = x.astype(np.float32).astype(np.float64)
    t = dev(x, torch.float32 if src == "f32" else torch.float64)
    got = rt.rtucker_convert(t, torch.bfloat16)
    got_bits = got.view(torch.int16).cpu().numpy().view(np.uint16)
    want = L.round_bf16(x)
    fin = np.isfinite(want)
    want_bits = L.bf16_bits(want[fin])
    np.testing.assert_array_equal(got_bits[fin], want_bits)
    assert np.all((got_bits[~fin] & 0x7fff) == 0x7f80)


@pytest.mark.parametrize("src", ["f32", "f64"])
def test_convert_f8_bit_exact(src):
    say("convert f8", src)
    x = _convert_inputs()
    x = x[np.abs(x) < 1e30]
    if src == "f32":
        x = x.astype(np.float32).astype(np.float64)
    t = dev(x, torch.float32 if src == "f32" else torch.float64)
    got = rt.rtucker_convert(t, torch.float8_e4m3fn)
    got_bits = got.view(torch.uint8).cpu().numpy()
    want_bits = L.f8_bits(L.round_f8(x))
    np.testing.assert_array_equal(got_bits, want_bits)
    # torch's own decoding of the bytes agrees with the format definition
    np.testing.assert_array_equal(got.float().cpu().numpy().astype(np.float64), L.f8_decode(got_bits))


@pytest.mark.parametrize("dst", ["bf16", "f8"])
@pytest.mark.parametrize("n,offset", [(1, 0), (3, 1), (4097, 0), (4097, 3), (1 << 20, 2), ((1 << 20) + 5, 0)])
def test_convert_f32_vector_and_scalar_paths(dst, n, offset):
    """The vectorised binary32 cast (16-byte aligned source) and the element-wise one
    (misaligned source) give the same bits as the format definition, tails included."""
    say("convert paths", dst, n, offset)
    rng = np.random.default_rng(101 + n + offset)
    x = (rng.standard_normal(n + offset) * np.exp2(rng.integers(-20, 10, n + offset))).astype(np.float32)
    t = dev(x, torch.float32)[offset:]
    tdt = torch.bfloat16 if dst == "bf16" else torch.float8_e4m3fn
    got = rt.rtucker_convert(t, tdt)
    xv = x[offset:].astype(np.float64)
    if dst == "bf16":
        bits = got.view(torch.int16).cpu().numpy().view(np.uint16)
        np.testing.assert_array_equal(bits, L.bf16_bits(L.round_bf16(xv)))
    else:
        bits = got.view(torch.uint8).cpu().numpy()
        np.testing.assert_array_equal(bits, L.f8_bits(L.round_f8(xv)))
    out = torch.empty_like(got)
    assert rt.rtucker_convert(t, tdt, out=out) is out and torch.equal(out.view(torch.uint8), got.view(torch.uint8))


def test_convert_scale_exponent():
    x = np.array([1.0, 3.0, -0.75, 100.0])
    got = rt.rtucker_convert(dev(x, torch.float32), torch.float32, scale_exp=-3)
    np.testing.assert_array_equal(host(got), x / 8)


# ------------------------------------------------------------------ sketch
SKETCH_CASES = [
    ((37, 150, 530), (3, 5, 7)),     # two column blocks (530 > 512), row split, ragged tails
    ((64, 64, 64), (4, 4, 4)),
    ((9, 33, 1000), (2, 8, 6)),
    ((11, 13, 17, 70), (2, 3, 4, 5)),  # 4-way: tree beyond the first level
    ((300, 517), (6, 5)),            # 2-way
    ((20, 24, 30), (4, 10, 3)),      # subrank > 8: generic first level
    ((4, 512, 264), (3, 7, 5)),      # bf16 matrix-core pass: 4 row blocks, ragged column tail
    ((16, 96, 1040), (2, 8, 8)),     # bf16 matrix-core pass: 3 column blocks
    ((6, 72, 136), (3, 5, 7)),       # bf16 matrix-core pass: the last 32-row step ends past the rows
                                     # (three of its 8-row groups are clamped and zeroed), and two
                                     # of the four waves have no columns
    ((20, 18, 16, 12), (4, 4, 4, 4)),  # 4-way: one tree level's matrix-core contractions share one
                                       # launch, the next level's differ in K % 4 (one launch each)
    ((6, 7, 5, 9, 40), (2, 2, 3, 2, 3)),  # 5-way: memoised tree, two shared prefixes below W
    ((4, 5, 3, 6, 4, 36), (2, 3, 2, 2, 3, 2)),  # 6-way
    ((12, 16, 20, 24, 64), (3, 3, 3, 3, 3)),  # 5-way with matrix-core tree contractions
]


@pytest.mark.parametrize("dims,s", SKETCH_CASES)
@pytest.mark.parametrize("dt", ["f64", "f32", "bf16", "f8"])
def test_sketch_parity(dims, s, dt):
    say("sketch", dims, s, dt)
    rng = np.random.default_rng(200)
    X = rng.standard_normal(dims)
    phis = reuse_phis(dims, s, seed=201)
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f8": torch.float8_e4m3fn}[dt]
    rnd = {"f64": lambda v: v, "f32": L.round_f32, "bf16": L.round_bf16, "f8": L.round_f8}[dt]
    Xr = rnd(X)
    Xd = dev(Xr, torch.float64).to(tdt) if dt != "f64" else dev(Xr)
    Ys = rt.rtucker_sketch(Xd, [dev(p) for p in phis], s)
    tol = 1e-13 if dt == "f64" else 2e-5
    for n in range(len(dims)):
        want = T.kron_sketch(Xr, [rnd(p) for p in phis], n)
        bound = T.kron_sketch(np.abs(Xr), [np.abs(rnd(p)) for p in phis], n)
        assert_entrywise(host(Ys[n]), want, bound, tol, f"sketch mode {n}")


def test_sketch_single_mode_masks():
    dims, s = (21, 40, 66), (3, 4, 5)
    X = np.random.default_rng(202).standard_normal(dims)
    phis = reuse_phis(dims, s, seed=203)
    for n in range(3):
        Ys = rt.rtucker_sketch(dev(X), [dev(p) for p in phis], s, modes=[n])
        assert all(Ys[k] is None for k in range(3) if k != n)
        want = T.kron_sketch(X, phis, n)
        bound = T.kron_sketch(np.abs(X), [np.abs(p) for p in phis], n)
        assert_entrywise(host(Ys[n]), want, bound, 1e-13, f"sketch mode {n}")


# ------------------------------------------------------------------ QR
QR_CASES = [(1024, 49), (300, 64), (130, 27), (64, 16), (600, 20), (257, 33), (5000, 8), (40, 60), (3, 5)]


@pytest.mark.parametrize("m,n", QR_CASES)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_qr_parity(m, n, dt):
    say("qr", m, n, dt)
    rng = np.random.default_rng(300 + m + n)
    Y = rng.standard_normal((m, n))
    if dt == "f32":
        Y = L.round_f32(Y)
    Yd = dev(Y, torch.float64 if dt == "f64" else torch.float32)
    Q, R = rt.rtucker_qr(Yd, want_r=True)
    Q, R = host(Q), host(R)
    Qo, Ro = T.qr_pos(Y)
    c = min(m, n)
    assert Q.shape == (m, c) and R.shape == (c, n)
    np.testing.assert_allclose(Q.T @ Q, np.eye(c), atol=1e-13)
    np.testing.assert_allclose(Q, Qo, atol=1e-11)
    np.testing.assert_allclose(R, Ro, atol=1e-11 * np.abs(Ro).max())
    assert np.all(np.diag(R) >= 0)


@pytest.mark.parametrize("m", [90, 700])
def test_qr_rank_deficient(m):
    rng = np.random.default_rng(310)
    Y = rng.standard_normal((m, 3)) @ rng.standard_normal((3, 12))
    Q = host(rt.rtucker_qr(dev(Y)))
    np.testing.assert_allclose(Q.T @ Q, np.eye(12), atol=1e-12)
    assert np.linalg.norm(Y - Q @ (Q.T @ Y)) <= 1e-12 * np.linalg.norm(Y)
    Qo, _ = T.qr_pos(Y)
    assert subspace_gap(Q[:, :3], Qo[:, :3]) < 1e-10


def test_qr_zero_matrix():
    Q = host(rt.rtucker_qr(dev(np.zeros((50, 6)))))
    np.testing.assert_allclose(Q.T @ Q, np.eye(6), atol=1e-14)


# ------------------------------------------------------------------ core multi-TTM
CORE_CASES = [
    ((264, 136, 40), (30, 49, 17)),   # first contraction on MFMA (B = 5440), then generic
    ((70, 90, 130), (20, 33, 64)),    # generic first (B = 1), MFMA second with a ragged K = 90
    ((256, 64, 96), (49, 16, 5)),     # m = 49 padded to 64 rows
    ((1024, 16, 24), (49, 8, 8)),     # split-K partial sums
    ((12, 11, 10, 200), (3, 4, 5, 27)),
]


@pytest.mark.parametrize("dims,l", CORE_CASES)
@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_core_parity(dims, l, dt):
    say("core", dims, l, dt)
    rng = np.random.default_rng(400)
    X = rng.standard_normal(dims)
    Us = [np.linalg.qr(rng.standard_normal((n, k)))[0] for n, k in zip(dims, l)]
    if dt == "bf16":
        X = L.round_bf16(X)
        Xd = dev(X).to(torch.bfloat16)
    elif dt == "f32":
        X = L.round_f32(X)
        Xd = dev(X, torch.float32)
    else:
        Xd = dev(X)
    G = host(rt.rtucker_core(Xd, [dev(U) for U in Us]))
    # emulate the rounding points: first (largest) mode's U in X's dtype, later ones binary32
    order = T.core_order(dims)
    rnd1 = {"f64": lambda v: v, "f32": L.round_f32, "bf16": L.round_bf16}[dt]
    rnd2 = (lambda v: v) if dt == "f64" else L.round_f32
    want = T.ttm(X, rnd1(Us[order[0]]).T, order[0])
    bound = T.ttm(np.abs(X), np.abs(rnd1(Us[order[0]])).T, order[0])
    for k in order[1:]:
        want = T.ttm(rnd2(want), rnd2(Us[k]).T, k)
        bound = T.ttm(bound, np.abs(rnd2(Us[k])).T, k)
    # the binary32 store between contractions rounds each entry by 2^-24 relative:
    # part of the accumulation scale for the later products
    tol = 1e-13 if dt == "f64" else 2e-5
    assert_entrywise(G, want, bound, tol, "core")


def test_core_single_modes():
    dims = (33, 64, 80)
    rng = np.random.default_rng(401)
    X = L.round_f32(rng.standard_normal(dims))
    Us = [np.linalg.qr(rng.standard_normal((n, 9)))[0] for n in dims]
    for k in range(3):
        G = host(rt.rtucker_core(dev(X, torch.float32), [dev(U) for U in Us], modes=[k]))
        want = T.ttm(X, L.round_f32(Us[k]).T, k)
        bound = T.ttm(np.abs(X), np.abs(L.round_f32(Us[k])).T, k)
        assert_entrywise(G, want, bound, 2e-5, f"core mode {k}")


@pytest.mark.parametrize("m", [17, 18, 33, 34, 49, 50, 48, 19])
@pytest.mark.parametrize("K", [1024, 92, 90])
def test_core_first_contraction_tail_rows(m, K):
    """Factor widths one or two rows past a whole 16-row tile take the vector-ALU tail in
    the binary32 matrix-core contraction (K % 4 == 0), the others the padded tiles."""
    say("core tail rows", m, K)
    rng = np.random.default_rng(402 + m + K)
    dims = (K, 24, 40)
    X = L.round_f32(rng.standard_normal(dims))
    U = np.linalg.qr(rng.standard_normal((K, m)))[0]
    G = host(rt.rtucker_core(dev(X, torch.float32), [dev(U), None, None], modes=[0]))
    Ur = L.round_f32(U)
    want = T.ttm(X, Ur.T, 0)
    bound = T.ttm(np.abs(X), np.abs(Ur).T, 0)
    assert_entrywise(G, want, bound, 2e-5, f"core m={m} K={K}")


@pytest.mark.parametrize("m", [17, 49, 50])
@pytest.mark.parametrize("K", [92, 212])
def test_core_first_contraction_unsplit(m, K):
    """Enough columns that k is not split (2049 128-column units: the last workgroup has
    three idle waves, the last unit 124 columns), so the binary32 tail-row contraction stages
    U_hat in LDS: one partial window of k (K = 92) or a full one and a partial one (K = 212)."""
    say("core unsplit", m, K)
    rng = np.random.default_rng(403 + m + K)
    B = 128 * 2049 - 4
    dims = (K, 4, B // 4)
    X = L.round_f32(rng.standard_normal((K, B), dtype=np.float32).astype(np.float64)).reshape(dims)
    U = np.linalg.qr(rng.standard_normal((K, m)))[0]
    G = host(rt.rtucker_core(dev(X, torch.float32), [dev(U), None, None], modes=[0])).reshape(m, B)
    Ur = L.round_f32(U)
    cols = np.r_[0:512, B - 700:B]  # the first units and the ragged last ones
    Xc = X.reshape(K, B)[:, cols]
    want = Ur.T @ Xc
    bound = np.abs(Ur).T @ np.abs(Xc)
    assert_entrywise(G[:, cols], want, bound, 2e-5, f"core unsplit m={m} K={K}")


@pytest.mark.parametrize("m", [17, 49])
@pytest.mark.parametrize("K", [96, 200])
def test_core_first_contraction_unsplit_bf16(m, K):
    """The bfloat16 matrix-core contraction without a split over k: 2049 units (three idle
    waves in the last workgroup, a ragged last unit), K = 96 and 200."""
    say("core unsplit bf16", m, K)
    rng = np.random.default_rng(404 + m + K)
    B = 128 * 2049 - 8
    dims = (K, 8, B // 8)
    X = L.round_bf16(rng.standard_normal((K, B), dtype=np.float32).astype(np.float64)).reshape(dims)
    U = np.linalg.qr(rng.standard_normal((K, m)))[0]
    Xd = rt.rtucker_convert(dev(X, torch.float32), torch.bfloat16)
    G = host(rt.rtucker_core(Xd, [dev(U), None, None], modes=[0])).reshape(m, B)
    Ur = L.round_bf16(U)
    cols = np.r_[0:512, B - 700:B]
    Xc = X.reshape(K, B)[:, cols]
    want = Ur.T @ Xc
    bound = np.abs(Ur).T @ np.abs(Xc)
    assert_entrywise(G[:, cols], want, bound, 2e-5, f"core unsplit bf16 m={m} K={K}")


# ------------------------------------------------------------------ decomposition
def _decompose_and_compare(X, Xd, r, p, algo, phis, s, tol_e, Xsk=None, emulate=None):
    phis_d = [dev(f) for f in phis] if algo == "rhkron" else [[dev(f) if f is not None else None for f in row]
                                                                for row in phis]
    G, Us = rt.rtucker_decompose(Xd, r, p, phis_d, algo=algo, s=s, X_sketch=Xsk)
    G, Us = host(G), [host(U) for U in Us]
    if emulate is not None:
        Go, Uo = emulate
    elif algo == "rhkron":
        Go, Uo = T.rhkron(X, r, phis)
    else:
        Go, Uo = T.rsthkron(X, r, phis)
    e_o = T.rel_error(X, Go, Uo)
    e_g = T.rel_error(X, G, Us)
    e_dev, norms = rt.rtucker_rel_error(Xd, dev(G), [dev(U) for U in Us])
    e_seen = T.rel_error(host(Xd), G, Us)  # error against the tensor the device holds (maybe rounded)
    say(f"  e_gpu={e_g:.12e} e_oracle={e_o:.12e} e_device={e_dev:.12e}")
    assert abs(e_g - e_o) <= tol_e
    assert abs(e_dev - e_seen) <= 1e-12 + 1e-9 * e_seen
    for U in Us:
        np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
    return G, Us, Go, Uo


def test_decompose_config1_fp64():
    """64^3 FP64 random Tucker (core 8^3, noise 1e-6), r = 8, p = 5, s = 4: |de| <= 1e-10."""
    say("decompose config1")
    X, _, _ = synth.random_tucker((64, 64, 64), (8, 8, 8), 1e-6)
    s = [4, 4, 4]
    phis = reuse_phis(X.shape, s)
    G, Us, Go, Uo = _decompose_and_compare(X, dev(X), [8, 8, 8], 5, "rhkron", phis, s, 1e-10)
    for U, V in zip(Us, Uo):
        assert subspace_gap(U, V) < 1e-8
    np.testing.assert_allclose(G, Go, atol=1e-9 * np.abs(Go).max())


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_decompose_rsthkron_4way(dt):
    say("decompose rsthkron 4way", dt)
    dims = (20, 18, 16, 14)
    core = synth.tucker_core_decay((6, 6, 6, 6), tau=3.0, seed=5)
    X, _, _ = synth.random_tucker(dims, None, 1e-3, seed=6, core=core)
    r = [4, 4, 4, 4]
    S = T.subrank_matrix_sth([6, 6, 6, 6])
    phis = sth_phis(dims, S, seed=7)
    if dt == "f32":
        X = L.round_f32(X)
    Xd = dev(X) if dt == "f64" else dev(X, torch.float32)
    _decompose_and_compare(X, Xd, r, 2, "rsthkron", phis, S, 1e-10 if dt == "f64" else 1e-5)


@pytest.mark.parametrize("algo", ["rhkron", "rsthkron"])
def test_decompose_bumps_fp32(algo):
    say("decompose bumps fp32", algo)
    dims = (96, 80, 72)
    X = synth.bumps_field(dims, nbumps=30, noise_rel=1e-4, seed=8).astype(np.float64)
    r, p = [8, 8, 8], 4
    if algo == "rhkron":
        s = T.subranks_reuse([12, 12, 12])
        phis = reuse_phis(dims, s, seed=9)
    else:
        s = T.subrank_matrix_sth([12, 12, 12])
        phis = sth_phis(dims, s, seed=9)
    _decompose_and_compare(X, dev(X, torch.float32), r, p, algo, phis, s, 1e-5)


def test_decompose_bf16_against_emulation():
    say("decompose bf16")
    dims = (96, 80, 72)
    X = synth.bumps_field(dims, nbumps=30, noise_rel=1e-4, seed=8).astype(np.float64)
    r, p = [8, 8, 8], 4
    s = T.subranks_reuse([12, 12, 12])
    phis = reuse_phis(dims, s, seed=9)
    Xb = L.round_bf16(X)
    emu = L.rhkron_emulated(X, r, phis, "bf16", "bf16")
    _decompose_and_compare(X, dev(Xb).to(torch.bfloat16), r, p, "rhkron", phis, s, 1e-5, emulate=emu)


def test_decompose_fp8_sketch_against_emulation():
    say("decompose fp8 sketch")
    dims = (96, 80, 72)
    X = synth.bumps_field(dims, nbumps=30, noise_rel=1e-4, seed=8).astype(np.float64)  # binary32 values
    r, p = [8, 8, 8], 4
    s = T.subranks_reuse([12, 12, 12])
    phis = reuse_phis(dims, s, seed=9)
    Xf = dev(X, torch.float32)
    X8 = rt.rtucker_convert(Xf, torch.float8_e4m3fn)
    emu = L.rhkron_emulated(X, r, phis, "f8e4m3", "f32")
    _decompose_and_compare(X, Xf, r, p, "rhkron", phis, s, 1e-5, Xsk=X8, emulate=emu)


def test_decompose_exact_rank_and_full_width():
    """Exact Tucker rank: error at rounding level.  Full-width sketch (ltilde = I): equals STHOSVD."""
    say("decompose exact rank")
    X, _, F = synth.random_tucker((30, 26, 22), (4, 3, 5), 0.0, seed=10)
    s = T.subranks_reuse([6, 5, 7])
    phis = reuse_phis(X.shape, s, seed=11)
    G, Us = rt.rtucker_decompose(dev(X), [4, 3, 5], 2, [dev(f) for f in phis], s=s)
    assert T.rel_error(X, host(G), [host(U) for U in Us]) < 1e-12
    rng = np.random.default_rng(12)
    Y = rng.standard_normal((16, 16, 16))
    phis = reuse_phis(Y.shape, [4, 4, 4], seed=13)
    G, Us = rt.rtucker_decompose(dev(Y), [5, 4, 6], 3, [dev(f) for f in phis], s=[4, 4, 4])
    Gs, Vs = T.sthosvd(Y, [5, 4, 6])
    assert abs(T.rel_error(Y, host(G), [host(U) for U in Us]) - T.rel_error(Y, Gs, Vs)) < 1e-12


def test_decompose_rank_above_32_fp64():
    """r > 32 leading eigenpairs per truncation: the eigensolver's Jacobi path.  |de| <= 1e-10."""
    say("decompose rank > 32")
    dims = (72, 70, 68)
    core = synth.tucker_core_decay((40, 40, 40), tau=12.0, seed=21)
    X, _, _ = synth.random_tucker(dims, None, 1e-6, seed=22, core=core)
    r, p = [34, 33, 35], 4
    s = rt.rtucker_sketch_sizes(dims, r, p)
    assert all(34 <= int(np.prod([s[k] for k in range(3) if k != n])) <= 64 for n in range(3))
    phis = reuse_phis(dims, s, seed=23)
    _decompose_and_compare(X, dev(X), r, p, "rhkron", phis, s, 1e-10)


def test_decompose_repeated_singular_values_fp64():
    """A core whose unfoldings have six equal singular values: the tridiagonal path's checks
    reject the cluster (inverse iteration gives non-orthogonal vectors there) and the Jacobi
    path takes over.  The error depends only on the retained subspace: |de| <= 1e-10."""
    say("decompose repeated singular values")
    core = np.zeros((6, 6, 6))
    for i in range(6):
        core[i, i, i] = 1.0
    X, _, _ = synth.random_tucker((40, 36, 32), None, 1e-7, seed=24, core=core)
    s = [4, 4, 4]
    phis = reuse_phis(X.shape, s, seed=25)
    _decompose_and_compare(X, dev(X), [6, 6, 6], 3, "rhkron", phis, s, 1e-10)


def test_decompose_bitwise_repeatable():
    X = synth.bumps_field((64, 72, 80), nbumps=20, noise_rel=1e-4, seed=14)
    Xd = dev(X, torch.float32)
    s = [4, 4, 4]
    phis = [dev(f) for f in reuse_phis(X.shape, s, seed=15)]
    G1, U1 = rt.rtucker_decompose(Xd, [6, 6, 6], 4, phis, s=s)
    G2, U2 = rt.rtucker_decompose(Xd, [6, 6, 6], 4, phis, s=s)
    torch.cuda.synchronize()
    assert torch.equal(G1, G2) and all(torch.equal(a, b) for a, b in zip(U1, U2))


def test_decompose_two_streams_in_flight():
    """Decompositions enqueued alternately on two streams (own workspaces and outputs, one
    shared input) return the one-at-a-time results bit for bit."""
    X = synth.bumps_field((96, 80, 72), nbumps=20, noise_rel=1e-4, seed=16)
    Xd = dev(X, torch.float32)
    s = [4, 4, 4]
    phis = [dev(f) for f in reuse_phis(X.shape, s, seed=17)]
    G0, U0 = rt.rtucker_decompose(Xd, [6, 6, 6], 4, phis, s=s)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    nb = rt.rtucker_decompose_workspace(Xd, [6, 6, 6], 4, "rhkron", s)
    wss = [torch.empty(max(nb, 256), dtype=torch.uint8, device=DEV) for _ in range(2)]
    outs = []
    for i in range(6):
        k = i % 2
        with torch.cuda.stream(streams[k]):
            G = torch.empty((6, 6, 6), dtype=torch.float64, device=DEV)
            Us = [torch.empty((n, 6), dtype=torch.float64, device=DEV) for n in X.shape]
            rt.rtucker_decompose(Xd, [6, 6, 6], 4, phis, s=s, G=G, Us=Us, ws=wss[k])
            outs.append((G, Us))
    torch.cuda.synchronize()
    for G, Us in outs:
        assert torch.equal(G, G0) and all(torch.equal(a, b) for a, b in zip(Us, U0))


@pytest.mark.parametrize("algo", ["rhkron", "rsthkron"])
def test_decompose_phases_bitwise_and_positive(algo):
    """The phase-timed call returns the plain call's results bit for bit, and a positive time
    for each of sketch, QR, core and truncation."""
    X = synth.bumps_field((64, 72, 80), nbumps=20, noise_rel=1e-4, seed=14)
    Xd = dev(X, torch.float32)
    if algo == "rhkron":
        s = [4, 4, 4]
        phis = [dev(f) for f in reuse_phis(X.shape, s, seed=15)]
    else:
        s = T.subrank_matrix_sth([10, 10, 10])
        phis = [[None if f is None else dev(f) for f in row] for row in sth_phis(X.shape, s, seed=15)]
    G1, U1 = rt.rtucker_decompose(Xd, [6, 6, 6], 4, phis, algo=algo, s=s)
    G2, U2, ph = rt.rtucker_decompose_phases(Xd, [6, 6, 6], 4, phis, algo=algo, s=s)
    torch.cuda.synchronize()
    assert torch.equal(G1, G2) and all(torch.equal(a, b) for a, b in zip(U1, U2))
    assert set(ph) == {"sketch", "qr", "core", "truncate"}
    assert all(v > 0.0 for v in ph.values()), ph


def test_rel_error_matches_oracle():
    rng = np.random.default_rng(16)
    X = rng.standard_normal((50, 40, 30))
    G = rng.standard_normal((5, 4, 3))
    Us = [np.linalg.qr(rng.standard_normal((n, k)))[0] for n, k in zip(X.shape, G.shape)]
    e, norms = rt.rtucker_rel_error(dev(X), dev(G), [dev(U) for U in Us])
    assert abs(e - T.rel_error(X, G, Us)) <= 1e-13
    assert abs(norms["g2"] - np.sum(G * G)) <= 1e-12 * np.sum(G * G)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_rel_error_counts_nonfinite(dt):
    """NaN and +-Inf entries of X are counted and left out of both norms; the binding
    raises on them unless asked for the count."""
    rng = np.random.default_rng(17)
    X = rng.standard_normal((40, 33, 21))
    bad = [(0, 0, 0), (7, 12, 3), (39, 32, 20), (20, 1, 9), (5, 5, 5)]
    vals = [np.nan, np.inf, -np.inf, np.nan, np.inf]
    for idx, v in zip(bad, vals):
        X[idx] = v
    G = rng.standard_normal((4, 3, 2))
    Us = [np.linalg.qr(rng.standard_normal((n, k)))[0] for n, k in zip(X.shape, G.shape)]
    rnd = {"f64": lambda v: v, "f32": L.round_f32, "bf16": L.round_bf16}[dt]
    Xr = rnd(X)
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dt]
    Xd = dev(Xr).to(tdt)
    with pytest.raises(rt.RtuckerError):
        rt.rtucker_rel_error(Xd, dev(G), [dev(U) for U in Us])
    e, norms = rt.rtucker_rel_error(Xd, dev(G), [dev(U) for U in Us], allow_nonfinite=True)
    assert norms["nonfinite"] == len(bad)
    fin = np.isfinite(Xr)
    R = Xr - T.reconstruct(G, Us)
    res2, x2 = float(np.sum(R[fin] ** 2)), float(np.sum(Xr[fin] ** 2))
    assert abs(norms["res2"] - res2) <= 1e-12 * res2
    assert abs(norms["x2"] - x2) <= 1e-12 * x2


# ------------------------------------------------------------------ the streaming sketch pass alone
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f8"])
@pytest.mark.parametrize("shape,sp,sl", [((37, 150, 530), 7, 7), ((64, 64, 64), 4, 4), ((11, 13, 17, 70), 3, 5),
                                         ((20, 24, 30), 9, 10), ((1024, 1024 // 8, 512 // 4), 7, 7),
                                         ((8, 40, 132), 9, 12)])  # s of the last mode past 8 (PhiQ not in LDS)
def test_sketch_pass(dtype, shape, sp, sl):
    say("sketch pass", shape, sp, sl, dtype)
    rng = np.random.default_rng(51)
    X = rng.standard_normal(shape)
    Pp, Pl = rng.standard_normal((sp, shape[-2])), rng.standard_normal((sl, shape[-1]))
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f8": torch.float8_e4m3fn}[dtype]
    if dtype in ("f64", "f32"):
        Xd = dev(X, torch.float64).to(tdt)
    else:
        Xd = rt.rtucker_convert(dev(X, torch.float32), tdt)
    Z, W = rt.rtucker_sketch_pass(Xd, dev(Pp), dev(Pl))
    Xs = host(Xd) if dtype != "f8" else L.f8_decode(Xd.view(torch.uint8).cpu().numpy())
    if dtype == "bf16":
        Pp_, Pl_ = L.round_bf16(Pp), L.round_bf16(Pl)
    elif dtype == "f8":
        Pp_, Pl_ = L.round_f8(Pp), L.round_f8(Pl)
    elif dtype == "f32":
        Pp_, Pl_ = Pp.astype(np.float32).astype(np.float64), Pl.astype(np.float32).astype(np.float64)
    else:
        Pp_, Pl_ = Pp, Pl
    d = len(shape)
    Zr = T.ttm(Xs, Pl_, d - 1)
    Wr = T.ttm(Xs, Pp_, d - 2)
    tol = 1e-13 if dtype == "f64" else 2e-5
    assert_entrywise(host(Z), Zr, T.ttm(np.abs(Xs), np.abs(Pl_), d - 1), tol, "Z")
    assert_entrywise(host(W), Wr, T.ttm(np.abs(Xs), np.abs(Pp_), d - 2), tol, "W")
    # one output only
    Z2, W2 = rt.rtucker_sketch_pass(Xd, dev(Pp), dev(Pl), want=(True, False))
    assert W2 is None and np.array_equal(host(Z2), host(Z))
    Z3, W3 = rt.rtucker_sketch_pass(Xd, dev(Pp), dev(Pl), want=(False, True))
    assert Z3 is None
    assert_entrywise(host(W3), Wr, T.ttm(np.abs(Xs), np.abs(Pp_), d - 2), tol, "W alone")
