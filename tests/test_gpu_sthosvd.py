"""GPU parity of the deterministic STHOSVD (Alg. 2.2), the baseline of the paper's timing
comparisons: against the oracle's STHOSVD (numpy SVD per mode) on the same tensor, the
closed form of the super-diagonal tensor of the accuracy experiment, and exact recovery."""
import os

import numpy as np
import pytest

from gpu_common import T, dev, host, pytestmark_skip, rt, say, subspace_gap, synth, torch

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(pytestmark_skip, reason="needs a GPU")]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _compare(X, Xd, r, tol_e, tol_u=None):
    G, Us, it = rt.rtucker_sthosvd(Xd, r)
    Gh, Uh = host(G), [host(u) for u in Us]
    Go, Vo = T.sthosvd(X, r)
    e_g, e_o = T.rel_error(X, Gh, Uh), T.rel_error(X, Go, Vo)
    say(f"  e_gpu={e_g:.12e} e_oracle={e_o:.12e} subspace iterations={it}")
    assert abs(e_g - e_o) <= tol_e
    for U, V in zip(Uh, Vo):
        np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
        if tol_u is not None:
            np.testing.assert_allclose(U, V, atol=tol_u)
    return Gh, Uh, Go, Vo, it


def test_sthosvd_small_modes_fp64():
    """Every mode <= 64: the one-workgroup eigensolver; columns and core equal the oracle's."""
    say("sthosvd small fp64")
    X, _, _ = synth.random_tucker((40, 36, 32), (6, 5, 4), 1e-3, seed=90)
    Gh, Uh, Go, Vo, it = _compare(X, dev(X), [5, 4, 3], 1e-10, tol_u=1e-8)
    assert it == 0
    np.testing.assert_allclose(Gh, Go, atol=1e-9 * np.abs(Go).max())


@pytest.mark.parametrize("dims,r", [((100, 90, 70), (6, 5, 4)), ((300, 80, 66), (10, 8, 12)),
                                    ((130, 20, 70, 9), (5, 4, 6, 3))])
def test_sthosvd_subspace_modes_fp64(dims, r):
    """Modes above 64: subspace iteration to its residual tolerance matches the oracle's SVD."""
    say("sthosvd fp64", dims, r)
    core = synth.tucker_core_decay([v + 4 for v in r], tau=4.0, seed=91)
    X, _, _ = synth.random_tucker(dims, None, 1e-4, seed=92, core=core)
    _compare(X, dev(X), list(r), 1e-10, tol_u=1e-7)


def test_sthosvd_fp32_bumps():
    say("sthosvd fp32 bumps")
    X = synth.bumps_field((160, 150, 140), nbumps=40, noise_rel=1e-4, seed=93).astype(np.float64)
    _compare(X, dev(X, torch.float32), [8, 8, 8], 1e-5)


def test_sthosvd_superdiagonal_closed_form():
    """The accuracy experiment's tensor (Sec. 7.1) at 100^3: super-diagonal 0.4^(i-1) rotated
    by orthogonal factors; STHOSVD at rank 10 has error exactly 0.4^10 = 1.048576e-4."""
    X, _, _ = synth.superdiagonal(100, seed=94, terms=60)
    G, Us, _ = rt.rtucker_sthosvd(dev(X), [10, 10, 10])
    e = T.rel_error(X, host(G), [host(u) for u in Us])
    assert abs(e - 0.4 ** 10) <= 1e-10


def test_sthosvd_exact_rank_recovery_fp32():
    dims, r = (200, 180, 90), (7, 5, 6)
    X, _, F = synth.random_tucker(dims, r, 0.0, seed=95)
    G, Us, _ = rt.rtucker_sthosvd(dev(X, torch.float32), list(r))
    e, _ = rt.rtucker_rel_error(dev(X, torch.float32), G, Us)
    assert e < 1e-5
    for U, A in zip(Us, F):
        assert subspace_gap(host(U), A) < 1e-5


def test_sthosvd_rejects_bad_arguments():
    X = torch.zeros((100, 10, 10), dtype=torch.float32, device="cuda:0")
    with pytest.raises(rt.RtuckerError):
        rt.rtucker_sthosvd(X, [40, 5, 5])  # r > 32 on a mode above 64
    with pytest.raises(rt.RtuckerError):
        rt.rtucker_sthosvd(X.to(torch.bfloat16), [4, 4, 4])
