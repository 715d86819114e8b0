"""Full-size parity on the benchmark workload (1024 x 1024 x 512 smooth field,
r = 32, p = 8, s = 7), in the launch configuration the benchmark times.

The FP64 oracle runs the whole decomposition on the host (seconds), so the
relative reconstruction errors are compared directly: FP32 GPU vs FP64 oracle,
BF16 / FP8-sketch GPU (rHKron and rSTHKron) vs the emulated-precision oracle
(|de| <= 1e-5), plus
sampled sketch rows and the QR of the GPU sketch against the oracle."""
import numpy as np
import pytest

from gpu_common import DEV, T, dev, host, pytestmark_skip, rt, say, subspace_gap, synth, torch
from oracle import lowp as L

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(pytestmark_skip, reason="needs a GPU")]

DIMS = (1024, 1024, 512)
R = [32, 32, 32]
P = 8


@pytest.fixture(scope="module")
def work():
    say("full size: generating the field")
    Xh = synth.bumps_field(DIMS, nbumps=200, noise_rel=1e-4, seed=synth.DATA_SEED)
    s = rt.rtucker_sketch_sizes(DIMS, R, P)
    assert s == [7, 7, 7]
    phis = synth.gaussians(synth.PHI_SEED, [(s[k], DIMS[k]) for k in range(3)])
    X32 = torch.from_numpy(Xh).to(DEV)
    return {"Xh": Xh, "X32": X32, "s": s, "phis": phis, "phis_d": [dev(f) for f in phis]}


def test_fullsize_sketch_rows_and_qr(work):
    Xh, s, phis = work["Xh"], work["s"], work["phis"]
    say("full size: sketch rows")
    Ys = rt.rtucker_sketch(work["X32"], work["phis_d"], s)
    Ys = [host(Y) for Y in Ys]
    rng = np.random.default_rng(7)
    p32 = [L.round_f32(f) for f in phis]
    for _ in range(6):
        i, j, k = (int(rng.integers(0, n)) for n in DIMS)
        y1 = (p32[1] @ Xh[i].astype(np.float64) @ p32[2].T).ravel()
        y2 = (p32[0] @ Xh[:, j, :].astype(np.float64) @ p32[2].T).ravel()
        y3 = (p32[0] @ Xh[:, :, k].astype(np.float64) @ p32[1].T).ravel()
        for got, want in ((Ys[0][i], y1), (Ys[1][j], y2), (Ys[2][k], y3)):
            assert np.linalg.norm(got - want) <= 2e-6 * np.linalg.norm(want)
    say("full size: QR of the device sketch")
    for n in range(3):
        Q = host(rt.rtucker_qr(torch.from_numpy(Ys[n]).to(DEV)))
        Qo, _ = T.qr_pos(Ys[n])
        np.testing.assert_allclose(Q.T @ Q, np.eye(49), atol=1e-13)
        np.testing.assert_allclose(Q, Qo, atol=1e-9)


def test_fullsize_core_first_contraction_samples(work):
    Xh = work["Xh"]
    rng = np.random.default_rng(8)
    U = np.linalg.qr(rng.standard_normal((1024, 49)))[0]
    C = host(rt.rtucker_core(work["X32"], [dev(U), None, None], modes=[0]))
    U32 = L.round_f32(U)
    for _ in range(200):
        a, j, k = int(rng.integers(0, 49)), int(rng.integers(0, 1024)), int(rng.integers(0, 512))
        col = Xh[:, j, k].astype(np.float64)
        want = U32[:, a] @ col
        assert abs(C[a, j, k] - want) <= 2e-6 * (np.abs(U32[:, a]) @ np.abs(col))


@pytest.mark.parametrize("path", ["f32", "bf16", "f8sketch", "rsthkron_f32", "rsthkron_bf16", "noreuse_f32",
                                  "srht_f32"])
def test_fullsize_decompose_error(work, path):
    Xh, s, phis = work["Xh"], work["s"], work["phis"]
    X = Xh.astype(np.float64)
    say(f"full size decompose {path}")
    if path.startswith("rsthkron"):
        S = rt.rtucker_sketch_sizes(DIMS, R, P, "rsthkron")
        cdim = [min(DIMS[k], int(np.prod([S[k][i] for i in range(3) if i != k]))) for k in range(3)]
        shapes = [None if k == j else (S[j][k], cdim[k] if k < j else DIMS[k]) for j in range(3) for k in range(3)]
        flat = synth.gaussians(synth.PHI_SEED, shapes)
        sph = [flat[j * 3:(j + 1) * 3] for j in range(3)]
        Xin = work["X32"] if path == "rsthkron_f32" else rt.rtucker_convert(work["X32"], torch.bfloat16)
        G, Us = rt.rtucker_decompose(Xin, R, P, [[None if f is None else dev(f) for f in row] for row in sph],
                                     algo="rsthkron", s=S)
        if path == "rsthkron_f32":
            Go, Uo = T.rsthkron(X, R, sph)
        else:
            Go, Uo = L.rsthkron_emulated(X, R, sph, "bf16")
    elif path == "f32":
        G, Us = rt.rtucker_decompose(work["X32"], R, P, work["phis_d"], s=s)
        Go, Uo = T.rhkron(X, R, phis)
    elif path == "noreuse_f32":
        S = rt.rtucker_sketch_sizes(DIMS, R, P, "rhkron_noreuse")
        shapes = T.noreuse_phi_shapes(DIMS, S)
        flat = synth.gaussians(synth.PHI_SEED, [sh for row in shapes for sh in row])
        nph = [flat[j * 3:(j + 1) * 3] for j in range(3)]
        G, Us = rt.rtucker_decompose(work["X32"], R, P, [[None if f is None else dev(f) for f in row] for row in nph],
                                     algo="rhkron_noreuse", s=S)
        Go, Uo = T.rhkron_noreuse(X, R, nph)
    elif path == "srht_f32":
        from oracle import srht as H
        draws = synth.srht_draws(synth.PHI_SEED, [(s[k], H.padded_size(DIMS[k]), DIMS[k]) for k in range(3)])
        sph = [H.srht_factor(DIMS[k], *draws[k]) for k in range(3)]
        sph_d = [rt.rtucker_srht_factor(DIMS[k], torch.as_tensor(draws[k][0], device=DEV), dev(draws[k][1]))
                 for k in range(3)]
        G, Us = rt.rtucker_decompose(work["X32"], R, P, sph_d, s=s)
        Go, Uo = T.rhkron(X, R, sph)
    elif path == "bf16":
        X16 = rt.rtucker_convert(work["X32"], torch.bfloat16)
        G, Us = rt.rtucker_decompose(X16, R, P, work["phis_d"], s=s)
        Go, Uo = L.rhkron_emulated(X, R, phis, "bf16", "bf16")
    else:
        X16 = rt.rtucker_convert(work["X32"], torch.bfloat16)
        X8 = rt.rtucker_convert(work["X32"], torch.float8_e4m3fn)
        G, Us = rt.rtucker_decompose(X16, R, P, work["phis_d"], s=s, X_sketch=X8)
        Go, Uo = L.rhkron_emulated(X, R, phis, "f8e4m3", "bf16")
    e_dev, norms = rt.rtucker_rel_error(work["X32"], G, Us)
    say(f"  oracle error ...")
    e_o = T.rel_error(X, Go, Uo)
    say(f"  {path}: e_device={e_dev:.9e} e_oracle={e_o:.9e}")
    assert abs(e_dev - e_o) <= 1e-5
    for U in Us:
        Uh = host(U)
        np.testing.assert_allclose(Uh.T @ Uh, np.eye(32), atol=1e-12)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_fullsize_rsthkron_128_4way(dtype):
    """128^4 FP32 tensor with a decaying 16^4 core, rSTHKron with every subrank 3, r = 16,
    p = 6, in the launch configuration the benchmark times: the binary32 run against the
    FP64 oracle, the bfloat16 run (X converted on the device) against the emulated-precision
    oracle, both to |de| <= 1e-5."""
    dims4, r4 = (128, 128, 128, 128), [16, 16, 16, 16]
    say(f"full size: generating the 128^4 tensor ({dtype})")
    core = synth.tucker_core_decay((16, 16, 16, 16), 6.0, seed=synth.DATA_SEED)
    Xh, _, _ = synth.random_tucker(dims4, (16, 16, 16, 16), 1e-3, seed=synth.DATA_SEED, core=core)
    Xh = Xh.astype(np.float32)
    S = [[1 if k == j else 3 for k in range(4)] for j in range(4)]
    shapes = T.sth_phi_shapes(dims4, S)
    flat = synth.gaussians(synth.PHI_SEED, [sh for row in shapes for sh in row])
    ph = [flat[j * 4:(j + 1) * 4] for j in range(4)]
    X32 = torch.from_numpy(Xh).to(DEV)
    phd = [[None if f is None else dev(f) for f in row] for row in ph]
    Xin = X32 if dtype == "f32" else rt.rtucker_convert(X32, torch.bfloat16)
    G, Us = rt.rtucker_decompose(Xin, r4, 6, phd, algo="rsthkron", s=S)
    e_dev, _ = rt.rtucker_rel_error(X32, G, Us)
    say(f"full size: 128^4 oracle ({dtype})")
    X64 = Xh.astype(np.float64)
    if dtype == "f32":
        Go, Uo = T.rsthkron(X64, r4, ph)
    else:
        Go, Uo = L.rsthkron_emulated(X64, r4, ph, "bf16")
    e_or = T.rel_error(X64, Go, Uo)
    say(f"  128^4 {dtype}: e_device={e_dev:.9e} e_oracle={e_or:.9e}")
    assert abs(e_dev - e_or) <= 1e-5, (e_dev, e_or)


def test_fullsize_sthosvd_matches_oracle_golden(work):
    """The deterministic STHOSVD of the workload against the oracle's value, stored by
    tests/golden/make_sthosvd_golden.py (numpy SVD per mode, float64)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sthosvd_1024x1024x512.txt")
    want = {ln.split()[0]: float(ln.split()[1]) for ln in open(path) if ln.strip() and not ln.startswith("#")}
    say("full size: deterministic STHOSVD")
    G, Us, it = rt.rtucker_sthosvd(work["X32"], R)
    e_dev, _ = rt.rtucker_rel_error(work["X32"], G, Us)
    say(f"  sthosvd: e_device={e_dev:.9e} e_oracle={want['rel_error']:.9e} iterations={it}")
    assert abs(e_dev - want["rel_error"]) <= 1e-5
    assert abs(float(torch.linalg.norm(G)) - want["core_norm"]) <= 1e-5 * want["core_norm"]
    for U in Us:
        Uh = host(U)
        np.testing.assert_allclose(Uh.T @ Uh, np.eye(32), atol=1e-12)
