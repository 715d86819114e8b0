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
