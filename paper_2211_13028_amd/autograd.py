"""Differentiable multi-TTM (Sec. 2.1) on the rtucker kernels.

The adjoint of Y = X x_1 op(A_1) ... x_d op(A_d) is
    dX   = dY x_k op(A_k)^T                        (one multi-TTM)
    dA_n = dY_(n) Z_(n)^T,  Z = X x_{k != n} op(A_k)  (a mode contraction)
and Z is recomputed in the backward pass instead of being kept from the
forward pass.  Every product runs in the library's HIP kernels through the
C ABI; these classes only order the calls.

* ``MultiTTM``     -- Y = X x_k op(A_k) over the modes whose factor is given.
* ``SqResidual``   -- L = sum (A - B)^2 (binary64 accumulation).
* ``ProjectionLoss`` -- L = ||X - (X x_k U_k^T) x_k U_k||^2, the Tucker
  reconstruction loss with fixed factors, with its whole backward pass fused
  into library calls (no gradient is summed outside the kernels).
* ``capture_projection_step`` -- one forward + backward of that loss recorded in a
  CUDA (HIP) graph: the library's calls neither synchronise nor copy to the host,
  so a replay re-runs every kernel of the step without the Python and launch
  overhead of about 60 calls.
"""
from __future__ import annotations

import torch

from . import (rtucker_mode_contract, rtucker_multi_ttm, rtucker_scaled_diff, rtucker_sq_residual)


def _modes(As):
    return [k for k, A in enumerate(As) if A is not None]


def _contig(t):
    return t if t.is_contiguous() else t.contiguous()


class MultiTTM(torch.autograd.Function):
    """Y = X x_k op(A_k) for every k with A_k given (None skips the mode).

    op(A) = A with A_k of shape m_k x I_k, or A^T (A_k: I_k x m_k) when
    ``transpose`` is true.  X and the A_k: float32 or float64, one dtype.
    """

    @staticmethod
    def forward(ctx, X, transpose, *As):
        modes = _modes(As)
        ctx.transpose = bool(transpose)
        ctx.modes = modes
        ctx.d = X.dim()
        X = _contig(X)
        As = [None if A is None else _contig(A) for A in As]
        ctx.save_for_backward(X, *[As[k] for k in modes])
        return rtucker_multi_ttm(X, As, modes, ctx.transpose)

    @staticmethod
    def backward(ctx, dY):
        X, *sel = ctx.saved_tensors
        d, modes, tr = ctx.d, ctx.modes, ctx.transpose
        As = [None] * d
        for k, A in zip(modes, sel):
            As[k] = A
        dY = _contig(dY)
        dX = None
        if ctx.needs_input_grad[0]:
            dX = rtucker_multi_ttm(dY, As, modes, not tr)
        dAs = [None] * d
        for k in modes:
            if not ctx.needs_input_grad[2 + k]:
                continue
            others = [j for j in modes if j != k]
            Z = rtucker_multi_ttm(X, As, others, tr) if others else X
            # op(A_k) = A_k: dA_k = dY_(k) Z_(k)^T;  op(A_k) = A_k^T: its transpose
            dAs[k] = rtucker_mode_contract(Z, dY, k) if tr else rtucker_mode_contract(dY, Z, k)
        return (dX, None, *dAs)


class SqResidual(torch.autograd.Function):
    """L = sum (A - B)^2 as a float64 scalar; dA = 2 g (A - B), dB = -2 g (A - B)."""

    @staticmethod
    def forward(ctx, A, B):
        out, R = rtucker_sq_residual(_contig(A), _contig(B), want_r=True)
        ctx.save_for_backward(R)
        return out.view(())

    @staticmethod
    def backward(ctx, g):
        (R,) = ctx.saved_tensors
        g = _contig(g.reshape(1))
        dA = rtucker_scaled_diff(R, None, g, 2.0) if ctx.needs_input_grad[0] else None
        dB = rtucker_scaled_diff(R, None, g, -2.0) if ctx.needs_input_grad[1] else None
        return dA, dB


class ProjectionLoss(torch.autograd.Function):
    """L = ||X - X_hat||^2 with G = X x_k U_k^T and X_hat = G x_k U_k (U_k: I_k x r_k).

    Backward, with R = X - X_hat, g the incoming gradient, S_k = R x_{j != k} U_j^T,
    Z'_k = X x_{j != k} U_j^T and RG = R x_j U_j^T:
        dX   = 2 g (R - RG x_j U_j)
        dU_k = -2 g [ (S_k)_(k) G_(k)^T + (Z'_k)_(k) RG_(k)^T ]
    (the first term is R_(k) (G x_{j != k} U_j)_(k)^T with the expansion moved
    onto R).  S_k and Z'_k are recomputed from two full-size passes each (over the
    first and the last mode), shared by all k.
    """

    @staticmethod
    def forward(ctx, X, *Us):
        X = _contig(X)
        Us = [_contig(U) for U in Us]
        G = rtucker_multi_ttm(X, Us, None, True)
        Xh = rtucker_multi_ttm(G, Us, None, False)
        out, R = rtucker_sq_residual(X, Xh, want_r=True)
        del Xh
        ctx.save_for_backward(X, G, R, *Us)
        return out.view(())

    @staticmethod
    def _all_but_one(T, Us):
        """[T x_{j != k} U_j^T for every k]: two passes over T (first and last mode)."""
        d = T.dim()
        L = d - 1

        def shrink(src, modes):
            if not modes:
                return src
            return rtucker_multi_ttm(src, [Us[j] if j in modes else None for j in range(d)], modes, True)

        TL = shrink(T, [L])
        T0 = shrink(T, [0])
        outs = [shrink(TL, [j for j in range(L) if j != k]) for k in range(L)]
        outs.append(shrink(T0, list(range(1, L))))
        return outs

    @staticmethod
    def backward(ctx, gL):
        X, G, R, *Us = ctx.saved_tensors
        d = X.dim()
        g = _contig(gL.reshape(1))
        need_u = any(ctx.needs_input_grad[1:])
        S = ProjectionLoss._all_but_one(R, Us)
        RG = rtucker_multi_ttm(S[0], [Us[0]] + [None] * (d - 1), [0], True)  # R x_j U_j^T (= dG / (-2 g))
        dX = None
        if ctx.needs_input_grad[0]:
            PR = rtucker_multi_ttm(RG, Us, None, False)
            dX = rtucker_scaled_diff(R, PR, g, 2.0)
            del PR
        dUs = [None] * d
        if need_u:
            Zp = ProjectionLoss._all_but_one(X, Us)
            for k in range(d):
                if not ctx.needs_input_grad[1 + k]:
                    continue
                acc = rtucker_mode_contract(S[k], G, k)
                rtucker_mode_contract(Zp[k], RG, k, out=acc)
                dUs[k] = rtucker_scaled_diff(acc, None, g, -2.0, out=acc)
        return (dX, *dUs)


def multi_ttm(X, As, transpose: bool = False):
    """Differentiable Y = X x_k op(A_k) (None entries skip a mode)."""
    return MultiTTM.apply(X, transpose, *As)


def sq_residual(A, B):
    """Differentiable sum (A - B)^2 (float64 scalar)."""
    return SqResidual.apply(A, B)


def projection_loss(X, Us):
    """Differentiable ||X - (X x_k U_k^T) x_k U_k||^2 (float64 scalar)."""
    return ProjectionLoss.apply(X, *Us)


def capture_projection_step(X, Us, warmup: int = 2):
    """Record one forward + backward of ``projection_loss(X, Us)`` in a CUDA graph.

    X and the U_k are static tensors (requires_grad set as wanted).  Returns
    ``(graph, loss)``: each ``graph.replay()`` recomputes ``loss`` and rewrites
    X.grad and U_k.grad in place (the gradients are allocated inside the graph, so
    they are overwritten, not accumulated).  The warm-up runs on a side stream of
    default priority, as graph capture requires."""
    ts = [X, *Us]
    side = torch.cuda.Stream(device=X.device)
    side.wait_stream(torch.cuda.current_stream(X.device))
    with torch.cuda.stream(side):
        for _ in range(warmup):
            for t in ts:
                t.grad = None
            projection_loss(X, Us).backward()
    torch.cuda.current_stream(X.device).wait_stream(side)
    for t in ts:
        t.grad = None
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        loss = projection_loss(X, Us)
        loss.backward()
    return graph, loss
