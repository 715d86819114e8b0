"""Workloads at the paper's own scale, generated on the device as exact Tucker tensors
(the oracle's closed forms need only the core and the factors):

* the dimension-tree experiment (Sec. 7.3), (d, n, s) = (4, 500, 5) and (5, 145, 3) in
  binary32 (about 256 GB each): sampled rows of every mode's sketch from one call (tree
  on) against the closed form, and the one-mode-per-call sketches (tree off) against them;
* the strong-scaling tensor (Sec. 7.4): 410^4 binary32 (113 GB), exact rank 20, r = 20,
  p = 3: rHKron and rSTHKron recover the tensor (error at binary32 rounding level) and the
  factor subspaces, and sampled sketch rows match the closed form.
Each test skips when the device has too little free memory."""
import numpy as np
import pytest

from gpu_common import T, assert_entrywise, dev, host, pytestmark_skip, reuse_phis, rt, say, synth, torch

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(pytestmark_skip, reason="needs a GPU")]


def _room(nbytes):
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes + (24 << 30):
        pytest.skip(f"needs {nbytes / 2**30:.0f} GiB + 24 GiB of device memory, {free / 2**30:.0f} GiB free")


def closed_form_sketch_rows(core, F, phis, n, rows):
    """Rows of Y_(n) for X = core x_k F_k: core x_n F_n[rows] x_{k != n} (Phi_k F_k), and the
    same over absolute values (a bound on |X| x_{k != n} |Phi_k| for the entry-wise check)."""
    d = core.ndim
    mats = {k: phis[k] @ F[k] for k in range(d) if k != n}
    mats[n] = F[n][rows]
    amats = {k: np.abs(phis[k]) @ np.abs(F[k]) for k in range(d) if k != n}
    amats[n] = np.abs(F[n][rows])
    return T.unfold(T.multi_ttm(core, mats), n), T.unfold(T.multi_ttm(np.abs(core), amats), n)


E4_CASES = [(4, 500, 5), (5, 145, 3)]


@pytest.mark.parametrize("d,n,s", E4_CASES)
def test_e4_full_size_sampled(d, n, s):
    dims, sv = (n,) * d, [s] * d
    need = 4 * n ** d
    _room(need)
    say(f"E4 ({d}, {n}, {s}): generating {need / 2**30:.0f} GiB on the device")
    core, F = synth.tucker_factors(dims, [6] * d, seed=80 + d)
    X = synth.tucker_on_device(core, F, "cuda:0", torch.float32)
    phis = reuse_phis(dims, sv, seed=90 + d)
    pd = [dev(p) for p in phis]
    pr = [p.astype(np.float32).astype(np.float64) for p in phis]
    say("  tree on")
    Ys = [host(Y) for Y in rt.rtucker_sketch(X, pd, sv)]
    rng = np.random.default_rng(100 + d)
    for m in range(d):
        rows = np.sort(rng.choice(n, 8, replace=False))
        want, bound = closed_form_sketch_rows(core, F, pr, m, rows)
        # X is stored in binary32: its rounding (2^-24 of |X| per entry) and the binary32
        # accumulation are within 2e-5 of the absolute-value bound
        assert_entrywise(Ys[m][rows], want, bound, 2e-5, f"mode {m} sampled rows")
    say("  tree off")
    for m in (0, d - 2, d - 1):
        off = host(rt.rtucker_sketch(X, pd, sv, modes=[m])[m])
        scale = np.abs(Ys[m]).max()
        assert np.max(np.abs(off - Ys[m])) <= 1e-5 * scale, m
    del X
    torch.cuda.empty_cache()


@pytest.mark.parametrize("algo", ["rhkron", "rsthkron"])
def test_410_exact_rank(algo):
    dims, r, p = (410,) * 4, [20] * 4, 3
    _room(int(4 * 410 ** 4 * 1.25))
    say(f"410^4 {algo}: generating 113 GB on the device")
    core, F = synth.tucker_factors(dims, r, seed=synth.DATA_SEED)
    X = synth.tucker_on_device(core, F, "cuda:0", torch.float32)
    S = rt.rtucker_sketch_sizes(dims, r, p, algo)
    if algo == "rhkron":
        assert S == [3, 3, 3, 3]
        phis = reuse_phis(dims, S)
        ph = [dev(f) for f in phis]
        # sampled rows of the sketches against the closed form
        Ys = rt.rtucker_sketch(X, ph, S, modes=[0, 3])
        pr = [f.astype(np.float32).astype(np.float64) for f in phis]
        rows = np.array([0, 17, 205, 409])
        for m in (0, 3):
            want, bound = closed_form_sketch_rows(core, F, pr, m, rows)
            assert_entrywise(host(Ys[m])[rows], want, bound, 2e-5, f"410^4 sketch mode {m}")
        del Ys
    else:
        cdim = [min(dims[k], int(np.prod([S[k][i] for i in range(4) if i != k]))) for k in range(4)]
        assert cdim == [24] * 4
        shapes = [None if k == j else (S[j][k], cdim[k] if k < j else dims[k]) for j in range(4) for k in range(4)]
        flat = synth.gaussians(synth.PHI_SEED, shapes)
        ph = [[None if f is None else dev(f) for f in flat[j * 4:(j + 1) * 4]] for j in range(4)]
    say("  decompose")
    G, Us = rt.rtucker_decompose(X, r, p, ph, algo=algo, s=S)
    e, _ = rt.rtucker_rel_error(X, G, Us)
    say(f"  410^4 {algo}: e = {e:.3e}")
    # exact rank 20 stored in binary32: the error is the binary32 rounding of X and of the
    # contractions (a few units of 2^-24), far below 1e-5
    assert e < 1e-5
    for U, A in zip(Us, F):
        u = host(U)
        np.testing.assert_allclose(u.T @ u, np.eye(20), atol=1e-10)
        assert np.linalg.norm(u @ u.T - A @ A.T, 2) < 1e-4
    del X, G, Us
    torch.cuda.empty_cache()
