"""The allocation-free decomposition (static device scratch) against the plain entry point:
two calls in a row on one GPU, the second on a smaller tensor, each equal to
rtucker_decompose on the same inputs; an input whose workspace exceeds the scratch is
rejected before anything is launched."""
import numpy as np
import pytest

from gpu_common import T, dev, host, pytestmark_skip, reuse_phis, rt, say, sth_phis, synth, torch

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(pytestmark_skip, reason="needs a GPU")]


def _case(dims, r, p, seed, dtype, algo="rhkron"):
    X = synth.bumps_field(dims, nbumps=20, noise_rel=1e-4, seed=seed).astype(np.float64)
    if algo == "rhkron":
        s = T.subranks_reuse([v + p for v in r])
        phis = [dev(f) for f in reuse_phis(dims, s, seed=seed + 1)]
    else:
        s = T.subrank_matrix_sth([v + p for v in r])
        phis = [[None if f is None else dev(f) for f in row] for row in sth_phis(dims, s, seed=seed + 1)]
    Xd = dev(X, dtype)
    return Xd, s, phis


def _compare(Xd, r, p, phis, s, algo):
    G1, U1 = rt.rtucker_decompose(Xd, r, p, phis, algo=algo, s=s)
    G2 = torch.full_like(G1, float("nan"))
    U2 = [torch.full_like(u, float("nan")) for u in U1]
    rt.rtucker_decompose_noalloc(Xd, r, p, phis, G2, U2, algo=algo, s=s)
    torch.cuda.synchronize()
    e1, _ = rt.rtucker_rel_error(Xd, G1, U1)
    e2, _ = rt.rtucker_rel_error(Xd, G2, U2)
    tol = 1e-10 if Xd.dtype == torch.float64 else 1e-5
    assert abs(e1 - e2) <= tol, (e1, e2)
    assert torch.equal(G1, G2) and all(torch.equal(a, b) for a, b in zip(U1, U2))


@pytest.mark.parametrize("algo", ["rhkron", "rsthkron"])
def test_noalloc_two_calls_second_smaller(algo):
    say("noalloc", algo, "first call 160x144x128 f32")
    Xd, s, phis = _case((160, 144, 128), [10, 9, 8], 4, 60, torch.float32, algo)
    _compare(Xd, [10, 9, 8], 4, phis, s, algo)
    say("noalloc", algo, "second call 40x36x30 f64")
    Xd, s, phis = _case((40, 36, 30), [5, 4, 3], 3, 62, torch.float64, algo)
    _compare(Xd, [5, 4, 3], 3, phis, s, algo)


def test_noalloc_rejects_workspace_above_scratch():
    X = torch.empty((1024, 1024, 512), dtype=torch.float32, device="cuda:0")
    s = [7, 7, 7]
    assert rt.rtucker_decompose_workspace(X, [32, 32, 32], 8, "rhkron", s) > rt.NOALLOC_SCRATCH_BYTES
    phis = [torch.zeros((7, n), dtype=torch.float64, device="cuda:0") for n in X.shape]
    G = torch.empty((32, 32, 32), dtype=torch.float64, device="cuda:0")
    Us = [torch.empty((n, 32), dtype=torch.float64, device="cuda:0") for n in X.shape]
    with pytest.raises(rt.RtuckerError, match="workspace"):
        rt.rtucker_decompose_noalloc(X, [32, 32, 32], 8, phis, G, Us, s=s)
