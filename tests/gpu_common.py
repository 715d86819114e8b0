"""Helpers shared by the GPU parity tests (inputs from ``synth``, expected values from ``oracle``)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

if not torch.cuda.is_available():  # CPU container: GPU tests are collected but skipped
    pytestmark_skip = True
else:
    pytestmark_skip = False

import paper_2211_13028_amd as rt  # noqa: E402
import synth  # noqa: E402
from oracle import tucker as T  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy() if t.dtype != torch.float64 else t.cpu().numpy()


def reuse_phis(dims, s, seed=synth.PHI_SEED):
    return synth.gaussians(seed, [(s[k], dims[k]) for k in range(len(dims))])


def sth_phis(dims, S, seed=synth.PHI_SEED):
    shapes = T.sth_phi_shapes(dims, S)
    flat = synth.gaussians(seed, [sh for row in shapes for sh in row])
    d = len(dims)
    return [flat[j * d:(j + 1) * d] for j in range(d)]


def subspace_gap(U, V):
    return float(np.linalg.norm(U @ U.T - V @ V.T, 2))


def assert_entrywise(got, want, bound, tol, what=""):
    """Element-by-element check |got - want| <= tol * bound, where ``bound`` is the same
    contraction taken over the absolute values of its (rounded) operands: the scale of the
    accumulation error of each entry, so cancellation in one entry cannot hide an error."""
    got, want, bound = (np.asarray(a, dtype=np.float64) for a in (got, want, bound))
    assert got.shape == want.shape == bound.shape, (got.shape, want.shape, bound.shape)
    err = np.abs(got - want)
    lim = tol * bound
    bad = ~(err <= lim)
    if bad.any():
        ratio = np.max(err[bad] / np.maximum(lim[bad], 1e-300))
        raise AssertionError(f"{what}: {int(bad.sum())} of {got.size} entries off, worst err/limit {ratio:.3g}")
