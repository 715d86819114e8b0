"""GPU parity of the differentiable multi-TTM (forward and hand-written
adjoint) against the FP64 oracle, finite differences (gradcheck) and the
projector closed form, at the gradcheck size 12 x 10 x 8 with ranks (3, 3, 2)
and at the 256^3 loss with fixed rank-24 factors."""
import numpy as np
import pytest

from gpu_common import assert_entrywise, dev, host, pytestmark_skip, rt, say, synth, torch
from oracle import adjoint as AD

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(pytestmark_skip, reason="needs a GPU")]

if not pytestmark_skip:
    from paper_2211_13028_amd import autograd as RA


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dt,tol", [(torch.float64, 1e-13), (torch.float32, 2e-6)])
@pytest.mark.parametrize("shape,ms", [((12, 10, 8), (3, 3, 2)), ((37, 5, 130), (9, 4, 17)),
                                      ((64, 48, 70, 3), (256, 7, 1, 2)), ((300, 2), (5, 256))])
@pytest.mark.parametrize("transpose", [False, True])
def test_multi_ttm_forward(dt, tol, shape, ms, transpose):
    say("multi_ttm", shape, ms, dt, transpose)
    rng = np.random.default_rng(21)
    X = rng.standard_normal(shape)
    As = [rng.standard_normal((n, m) if transpose else (m, n)) for n, m in zip(shape, ms)]
    Y = rt.rtucker_multi_ttm(dev(X, dt), [dev(A, dt) for A in As], None, transpose)
    opA = [A.T for A in As] if transpose else As
    ref = AD.multi_ttm_all(X, opA)
    bound = AD.multi_ttm_all(np.abs(X), [np.abs(A) for A in opA])
    assert_entrywise(host(Y), ref, bound, 10 * tol, "multi-TTM")


@pytest.mark.parametrize("dt,tol", [(torch.float64, 1e-13), (torch.float32, 2e-6)])
@pytest.mark.parametrize("transpose", [False, True])
def test_multi_ttm_backward_matches_oracle(dt, tol, transpose):
    shape, ms = (33, 20, 70), (7, 12, 5)
    say("multi_ttm backward", dt, transpose)
    rng = np.random.default_rng(22)
    X = rng.standard_normal(shape)
    As = [rng.standard_normal((n, m) if transpose else (m, n)) for n, m in zip(shape, ms)]
    dY = rng.standard_normal(ms)
    Xd = dev(X, dt).requires_grad_(True)
    Ad = [dev(A, dt).requires_grad_(True) for A in As]
    Y = RA.multi_ttm(Xd, Ad, transpose)
    Y.backward(dev(dY, dt))
    opA = [A.T for A in As] if transpose else As
    dX, dAs = AD.multi_ttm_grads(X, opA, dY)
    bX, bAs = AD.multi_ttm_grads(np.abs(X), [np.abs(A) for A in opA], np.abs(dY))
    assert_entrywise(host(Xd.grad), dX, bX, 10 * tol, "dX")
    for k in range(3):
        want = dAs[k].T if transpose else dAs[k]
        bound = bAs[k].T if transpose else bAs[k]
        assert_entrywise(host(Ad[k].grad), want, bound, 10 * tol, f"dA_{k}")


def test_multi_ttm_partial_modes_backward():
    rng = np.random.default_rng(23)
    X = rng.standard_normal((9, 11, 13, 6))
    A1 = rng.standard_normal((4, 11))
    A3 = rng.standard_normal((2, 6))
    dY = rng.standard_normal((9, 4, 13, 2))
    Xd = dev(X).requires_grad_(True)
    a1 = dev(A1).requires_grad_(True)
    a3 = dev(A3).requires_grad_(True)
    Y = RA.multi_ttm(Xd, [None, a1, None, a3])
    Y.backward(dev(dY))
    from oracle import tucker as T
    dX = T.multi_ttm(dY, {1: A1.T, 3: A3.T})
    assert _rel(host(Xd.grad), dX) <= 1e-13
    Z1 = T.multi_ttm(X, {3: A3})
    assert _rel(host(a1.grad), T.unfold(dY, 1) @ T.unfold(Z1, 1).T) <= 1e-13
    Z3 = T.multi_ttm(X, {1: A1})
    assert _rel(host(a3.grad), T.unfold(dY, 3) @ T.unfold(Z3, 3).T) <= 1e-13


def _cfg4_small():
    X, _, _ = synth.random_tucker((12, 10, 8), (4, 4, 3), 1e-6, seed=synth.DATA_SEED)
    Us = synth.fixed_factors((12, 10, 8), (3, 3, 2))
    return X, Us


def test_gradcheck_projection_loss_fp64():
    say("gradcheck ProjectionLoss 12x10x8 ranks (3,3,2)")
    X, Us = _cfg4_small()
    # perturb the factors off orthonormality so every gradient term is exercised
    rng = np.random.default_rng(31)
    Us = [U + 0.1 * rng.standard_normal(U.shape) for U in Us]
    inputs = [dev(X).requires_grad_(True)] + [dev(U).requires_grad_(True) for U in Us]
    assert torch.autograd.gradcheck(lambda x, *u: RA.projection_loss(x, list(u)), inputs, eps=1e-6, atol=1e-7,
                                    rtol=1e-6)


def test_gradcheck_composed_multi_ttm_fp64():
    say("gradcheck MultiTTM + SqResidual 12x10x8")
    X, Us = _cfg4_small()
    inputs = [dev(X).requires_grad_(True)] + [dev(U).requires_grad_(True) for U in Us]

    def loss(x, *u):
        G = RA.multi_ttm(x, list(u), True)
        return RA.sq_residual(x, RA.multi_ttm(G, list(u), False))

    assert torch.autograd.gradcheck(loss, inputs, eps=1e-6, atol=1e-7, rtol=1e-6)


def test_gradcheck_multi_ttm_fp64():
    rng = np.random.default_rng(32)
    X = rng.standard_normal((5, 4, 6))
    As = [rng.standard_normal((3, 5)), rng.standard_normal((2, 4)), rng.standard_normal((4, 6))]
    inputs = [dev(X).requires_grad_(True)] + [dev(A).requires_grad_(True) for A in As]
    assert torch.autograd.gradcheck(lambda x, *a: RA.multi_ttm(x, list(a)), inputs, eps=1e-6, atol=1e-8,
                                    rtol=1e-6)


@pytest.mark.parametrize("perturb", [0.0, 0.05])
def test_projection_loss_grads_match_oracle_fp64(perturb):
    X, _, _ = synth.random_tucker((40, 36, 70), (6, 5, 7), 1e-2, seed=synth.DATA_SEED)
    Us = synth.fixed_factors((40, 36, 70), (5, 4, 9))
    rng = np.random.default_rng(33)
    Us = [U + perturb * rng.standard_normal(U.shape) for U in Us]
    L, dX, dUs = AD.recon_loss_grads(X, Us)
    Xd = dev(X).requires_grad_(True)
    Ud = [dev(U).requires_grad_(True) for U in Us]
    Ld = RA.projection_loss(Xd, Ud)
    Ld.backward()
    assert abs(float(Ld.detach()) - L) <= 1e-12 * L
    assert _rel(host(Xd.grad), dX) <= 1e-12
    for k in range(3):
        assert _rel(host(Ud[k].grad), dUs[k]) <= 1e-11


def test_projection_loss_closed_form_and_exact_fit():
    Us = synth.fixed_factors((24, 20, 16), (3, 3, 2))
    rng = np.random.default_rng(34)
    C = rng.standard_normal((3, 3, 2))
    from oracle import tucker as T
    X0 = T.multi_ttm(C, {k: U for k, U in enumerate(Us)})
    # exact fit: zero loss and zero gradients
    Xd = dev(X0).requires_grad_(True)
    Ud = [dev(U).requires_grad_(True) for U in Us]
    RA.projection_loss(Xd, Ud).backward()
    assert float(host(Xd.grad).__abs__().max()) < 1e-13
    for u in Ud:
        assert float(host(u.grad).__abs__().max()) < 1e-12
    # off the fit: dL/dX = 2 (X - P X) with P the orthogonal projector
    X = X0 + rng.standard_normal(X0.shape)
    Xd = dev(X).requires_grad_(True)
    RA.projection_loss(Xd, [dev(U) for U in Us]).backward()
    PX = T.multi_ttm(T.multi_ttm(X, {k: U.T for k, U in enumerate(Us)}), {k: U for k, U in enumerate(Us)})
    assert np.max(np.abs(host(Xd.grad) - 2.0 * (X - PX))) < 1e-12


def test_projection_loss_256_fp32():
    """The 256^3 loss with fixed rank-24 factors, FP32 kernels vs the FP64 oracle."""
    n, r = 256, 24
    say("projection loss 256^3 fp32")
    X, _, _ = synth.random_tucker((n, n, n), (r, r, r), 1e-6, seed=synth.DATA_SEED)
    Us = synth.fixed_factors((n, n, n), (r, r, r))
    X32 = X.astype(np.float32).astype(np.float64)
    U32 = [U.astype(np.float32).astype(np.float64) for U in Us]
    L, dX, dUs = AD.recon_loss_grads(X32, U32)
    Xd = dev(X32, torch.float32).requires_grad_(True)
    Ud = [dev(U, torch.float32).requires_grad_(True) for U in U32]
    Ld = RA.projection_loss(Xd, Ud)
    Ld.backward()
    assert abs(float(Ld.detach()) - L) <= 1e-5 * L
    assert _rel(host(Xd.grad), dX) <= 1e-5
    for k in range(3):
        assert _rel(host(Ud[k].grad), dUs[k]) <= 1e-5


def test_projection_loss_graph_replays_match_eager():
    """The captured forward + backward (64^3 FP32, rank 8) against the eager step on every
    replay, with eager work and synchronisations between the replays; the gradients of
    every replay equal the eager ones bit for bit (same kernels, same order)."""
    n, r = 64, 8
    say("projection loss graph capture")
    X, _, _ = synth.random_tucker((n, n, n), (r, r, r), 1e-3, seed=synth.DATA_SEED)
    Us = synth.fixed_factors((n, n, n), (r, r, r))
    Xe = dev(X, torch.float32).requires_grad_(True)
    Ue = [dev(U, torch.float32).requires_grad_(True) for U in Us]
    Le = RA.projection_loss(Xe, Ue)
    Le.backward()
    want = [host(Xe.grad)] + [host(u.grad) for u in Ue]
    Xg = dev(X, torch.float32).requires_grad_(True)
    Ug = [dev(U, torch.float32).requires_grad_(True) for U in Us]
    graph, Lg = RA.capture_projection_step(Xg, Ug)
    for rep in range(4):
        Xg.grad.zero_()
        for u in Ug:
            u.grad.fill_(7.0)
        graph.replay()
        torch.cuda.synchronize()
        got = [host(Xg.grad)] + [host(u.grad) for u in Ug]
        assert float(Lg.detach()) == float(Le.detach()), rep
        for a, b in zip(got, want):
            np.testing.assert_array_equal(a, b)
        # eager work of the program between replays
        RA.projection_loss(Xe.detach().requires_grad_(True), [u.detach() for u in Ue]).backward()
        torch.cuda.synchronize()


def test_scaled_diff_and_sq_residual():
    rng = np.random.default_rng(35)
    a, b = rng.standard_normal(1000003), rng.standard_normal(1000003)
    for dt, tol in [(torch.float64, 1e-15), (torch.float32, 1e-6)]:
        A, B = dev(a, dt), dev(b, dt)
        ah, bh = host(A), host(B)
        g = torch.tensor([0.75], dtype=torch.float64, device=A.device)
        out = rt.rtucker_scaled_diff(A, B, g, -2.0)
        assert _rel(host(out), -1.5 * (ah - bh)) <= tol
        assert _rel(host(rt.rtucker_scaled_diff(A)), ah) == 0.0
        s, R = rt.rtucker_sq_residual(A, B)
        # the difference is formed in the tensor's dtype, its square summed in binary64
        dd = (ah.astype(np.float32) - bh.astype(np.float32)).astype(np.float64) if dt == torch.float32 else ah - bh
        assert np.array_equal(host(R), dd)
        want = float(np.sum(dd * dd))
        assert abs(float(host(s)[0]) - want) <= 1e-12 * want
    empty = torch.empty(0, dtype=torch.float32, device="cuda:0")
    rt.rtucker_scaled_diff(empty)


@pytest.mark.parametrize("dt,tol", [(torch.float64, 1e-13), (torch.float32, 3e-6)])
@pytest.mark.parametrize("shapeP,shapeQ,n", [
    ((256, 64, 48), (24, 64, 48), 0),     # long contiguous rows
    ((40, 130, 3), (40, 70, 3), 1),       # rows of 3: loads along the mode index
    ((33, 17, 200), (33, 17, 5), 2),      # last mode: rows of 1
    ((7, 2, 9, 65), (7, 2, 9, 1), 3),
    ((2, 1000), (3, 1000), 0),
    ((1000, 2), (1000, 3), 1),
    ((5, 300, 37), (5, 9, 37), 1),        # 37-long rows, ragged 32-wide stages
])
def test_mode_contract_layouts(dt, tol, shapeP, shapeQ, n):
    say("mode_contract", shapeP, shapeQ, n, dt)
    rng = np.random.default_rng(41)
    Pm, Qm = rng.standard_normal(shapeP), rng.standard_normal(shapeQ)
    from oracle import tucker as T
    want = T.unfold(Pm, n) @ T.unfold(Qm, n).T
    bound = np.abs(T.unfold(Pm, n)) @ np.abs(T.unfold(Qm, n)).T
    got = rt.rtucker_mode_contract(dev(Pm, dt), dev(Qm, dt), n)
    assert_entrywise(host(got), want, bound, 10 * tol, "mode contraction")
    # accumulate into an existing result
    base = rng.standard_normal(want.shape)
    acc = dev(base, dt)
    rt.rtucker_mode_contract(dev(Pm, dt), dev(Qm, dt), n, out=acc)
    assert_entrywise(host(acc), base + want, bound + np.abs(base), 10 * tol, "accumulated mode contraction")
