"""Seeded synthetic inputs shared by the CPU oracle tests, the GPU parity tests and the benchmark.

This module only draws random numbers and assembles input tensors.  It holds
none of the decomposition's arithmetic: sketch sizes, sketches, QR, core
contractions and truncation live in the oracle (CPU) and in the HIP library
(GPU), which share no code.  The random Kronecker factors that the method
draws are produced here and handed to both sides as inputs.

All generators use numpy's PCG64 (`numpy.random.default_rng`) and build in
float64; callers cast to the working dtype.
"""
from __future__ import annotations

import numpy as np

DATA_SEED = 1
PHI_SEED = 2
FIXED_U_SEED = 3


def gaussians(seed: int, shapes):
    """Draw one standard-normal float64 matrix per entry of ``shapes`` in order.

    Used for the Kronecker factors Phi (one per mode for the factor-reuse
    algorithm, one per (step, mode) pair for the sequentially truncated one);
    the caller supplies the shapes, so this function knows nothing about how
    sketch sizes are chosen.  ``None`` entries yield ``None``.
    """
    rng = np.random.default_rng(seed)
    out = []
    for sh in shapes:
        out.append(None if sh is None else rng.standard_normal(tuple(int(v) for v in sh)))
    return out


def orthonormal(rng, n: int, k: int) -> np.ndarray:
    """Orthonormal n x k matrix: Q factor of an n x k standard-normal draw."""
    q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    return q


def _expand(core: np.ndarray, factors) -> np.ndarray:
    """Assemble core x_1 F_1 ... x_d F_d for input construction (einsum, float64)."""
    d = core.ndim
    letters = "abcdefgh"[:d]
    outs = "ijklmnop"[:d]
    spec = letters + "," + ",".join(o + l for o, l in zip(outs, letters)) + "->" + outs
    return np.einsum(spec, core, *factors, optimize=True)


def _add_noise(rng, x: np.ndarray, rel: float) -> np.ndarray:
    if rel == 0.0:
        return x
    e = rng.standard_normal(x.shape)
    e *= rel * np.linalg.norm(x) / np.linalg.norm(e)
    return x + e


def random_tucker(dims, core_dims, noise_rel: float, seed: int = DATA_SEED, core=None):
    """Random Tucker tensor C x_k Q_k (+ Gaussian noise at ``noise_rel`` relative Frobenius norm).

    C ~ N(0,1) unless ``core`` is given; Q_k orthonormal (QR of N(0,1) draws).
    Returns (X, core, factors) in float64.
    """
    rng = np.random.default_rng(seed)
    if core is None:
        core = rng.standard_normal(tuple(core_dims))
    factors = [orthonormal(rng, n, c) for n, c in zip(dims, core.shape)]
    x = _expand(core, factors)
    return _add_noise(rng, x, noise_rel), core, factors


def fixed_factors(dims, ranks, seed: int = FIXED_U_SEED):
    """Orthonormal I_k x r_k factors drawn independently of any tensor (QR of N(0,1))."""
    rng = np.random.default_rng(seed)
    return [orthonormal(rng, int(n), int(r)) for n, r in zip(dims, ranks)]


def superdiagonal(n: int, d: int = 3, rate: float = 0.4, terms: int | None = None, seed: int = DATA_SEED):
    """Super-diagonal core with entries rate**(i-1), rotated by random orthogonal matrices.

    This is the accuracy workload of the paper's accuracy experiment (Sec. 7.1):
    geometric decay 0.4, largest entry 1.  ``terms`` (default n) entries are kept.
    Returns (X, lambdas, factors).
    """
    rng = np.random.default_rng(seed)
    k = n if terms is None else terms
    lam = rate ** np.arange(k, dtype=np.float64)
    factors = [orthonormal(rng, n, k) for _ in range(d)]
    letters = "ijklmnop"[:d]
    spec = "a," + ",".join(l + "a" for l in letters) + "->" + letters
    x = np.einsum(spec, lam, *factors, optimize=True)
    return x, lam, factors


def bumps_field(dims, nbumps: int = 200, noise_rel: float = 1e-4, seed: int = DATA_SEED,
                out_dtype=np.float32, chunk: int = 64):
    """Smooth simulation-like field: sum of separable anisotropic Gaussian bumps plus white noise.

    f(x) = sum_b a_b prod_k exp(-(x_k - c_bk)^2 / (2 w_bk^2)), x_k = (i_k + 1/2)/I_k,
    c ~ U[0,1]^d, w ~ U[0.02, 0.2] per axis (width as a fraction of the domain),
    a ~ U[0.5, 1.5]; then N(0,1) noise scaled to ``noise_rel`` of ||f||_F.
    Built slab by slab along mode 1 (float64 products, ``out_dtype`` storage) so
    that a 1024 x 1024 x 512 field needs only the output array in memory.
    """
    rng = np.random.default_rng(seed)
    d = len(dims)
    cen = rng.uniform(0.0, 1.0, size=(nbumps, d))
    wid = rng.uniform(0.02, 0.2, size=(nbumps, d))
    amp = rng.uniform(0.5, 1.5, size=nbumps)
    prof = []
    for k, n in enumerate(dims):
        xk = (np.arange(n, dtype=np.float64) + 0.5) / n
        prof.append(np.exp(-((xk[:, None] - cen[None, :, k]) ** 2) / (2.0 * wid[None, :, k] ** 2)))
    # Khatri-Rao of modes 2..d (rows in C order), weighted by amplitudes
    kr = prof[1]
    for k in range(2, d):
        kr = (kr[:, None, :] * prof[k][None, :, :]).reshape(-1, nbumps)
    kr = kr * amp[None, :]
    out = np.empty(tuple(dims), dtype=out_dtype)
    flat = out.reshape(dims[0], -1)
    fnorm2 = 0.0
    for i0 in range(0, dims[0], chunk):
        blk = prof[0][i0:i0 + chunk] @ kr.T
        fnorm2 += float(np.dot(blk.ravel(), blk.ravel()))
        flat[i0:i0 + chunk] = blk
    if noise_rel > 0.0:
        nrng = np.random.default_rng(seed + 7919)
        total = out.size
        # noise scale fixed from the expected norm of N(0,1) draws
        scale = noise_rel * np.sqrt(fnorm2) / np.sqrt(total)
        step = 1 << 24
        v = out.reshape(-1)
        for j in range(0, total, step):
            m = min(step, total - j)
            v[j:j + m] += (scale * nrng.standard_normal(m, dtype=np.float32)).astype(out_dtype)
    return out


def tucker_core_decay(shape, tau: float = 6.0, seed: int = DATA_SEED):
    """Core z_{i..} * exp(-(i+j+k+...)/tau) with z ~ N(0,1), 0-based indices."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(tuple(shape))
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    return z * np.exp(-sum(grids) / tau)


def batch_specs(count: int = 512, lo: int = 32, hi: int = 192, rlo: int = 4, rhi: int = 16,
                seed: int = DATA_SEED):
    """Dims U{lo..hi}^3 and ranks U{rlo..rhi}^3 for a batch of independent 3-way tensors."""
    rng = np.random.default_rng(seed)
    dims = rng.integers(lo, hi + 1, size=(count, 3))
    ranks = rng.integers(rlo, rhi + 1, size=(count, 3))
    return [tuple(int(v) for v in a) for a in dims], [tuple(int(v) for v in b) for b in ranks]


def batch_tensor(i: int, dims, ranks, noise_rel: float = 1e-4, seed: int = DATA_SEED):
    """Item i of a batch: a random Tucker tensor of Tucker rank ``ranks`` plus noise (float64)."""
    x, _, _ = random_tucker(dims, ranks, noise_rel, seed=seed * 1_000_003 + i)
    return x


def batch_phis(dims_list, s_list, seed: int = PHI_SEED):
    """Phi_k (s_k x I_k) for every item of a batch, drawn item by item in mode order."""
    shapes = [(s[k], d[k]) for d, s in zip(dims_list, s_list) for k in range(3)]
    flat = gaussians(seed, shapes)
    return [flat[3 * i:3 * i + 3] for i in range(len(dims_list))]


def tucker_factors(dims, ranks, seed: int = DATA_SEED, core=None):
    """Core ~ N(0,1) (unless given) and orthonormal factors of a random Tucker tensor, without
    assembling it: the inputs of ``tucker_on_device`` for tensors too large for host memory."""
    rng = np.random.default_rng(seed)
    if core is None:
        core = rng.standard_normal(tuple(int(r) for r in ranks))
    factors = [orthonormal(rng, int(n), int(c)) for n, c in zip(dims, core.shape)]
    return core, factors


def tucker_on_device(core, factors, device, dtype, chunk_elems: int = 1 << 28):
    """Assemble core x_1 F_1 ... x_d F_d directly in device memory (torch matmuls in float64,
    stored in ``dtype``), slab by slab along mode 1, so that host memory holds only the small
    core and factors.  Input construction only: the decomposition's arithmetic runs elsewhere."""
    import torch

    d = core.ndim
    dims = [int(f.shape[0]) for f in factors]
    out = torch.empty(dims, dtype=dtype, device=device)
    C = torch.as_tensor(core, dtype=torch.float64, device=device)
    F = [torch.as_tensor(f, dtype=torch.float64, device=device) for f in factors]
    # T = core x_2 F_2 ... x_d F_d  would be too large; contract modes 2..d per slab instead
    rest = int(np.prod(dims[1:]))
    rows = max(1, min(dims[0], chunk_elems // max(rest, 1)))
    for i0 in range(0, dims[0], rows):
        i1 = min(dims[0], i0 + rows)
        T = torch.tensordot(F[0][i0:i1], C, dims=([1], [0]))  # (rows, r2, ..., rd)
        for k in range(1, d):
            T = torch.tensordot(T, F[k], dims=([1], [1]))  # contract the leading core mode, append I_k
        out[i0:i1] = T.to(dtype)
        del T
    return out


def srht_draws(seed: int, specs):
    """Random draws of subsampled randomized Hadamard factors: for each (s, N, n) in
    ``specs`` (None entries give None), s distinct row indices in [0, N) and n signs +-1
    (int64 and float64 arrays), drawn in order with PCG64.  How a factor is formed from
    them is the method's business, not this module's."""
    rng = np.random.default_rng(seed)
    out = []
    for sp in specs:
        if sp is None:
            out.append(None)
            continue
        s, N, n = (int(v) for v in sp)
        rows = rng.choice(N, size=s, replace=False).astype(np.int64)
        signs = rng.choice(np.array([-1.0, 1.0]), size=n)
        out.append((rows, signs))
    return out
