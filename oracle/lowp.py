"""Emulated low-precision rounding and the emulated-precision decomposition.

TEST INFRASTRUCTURE ONLY (see ``oracle.tucker``).  Rounding is written from
the format definitions, with frexp/rint in float64, independently of any GPU
conversion code:

  * binary32: 24 significant bits, normal exponents -126..127, subnormal
    spacing 2^-149, round-to-nearest-even, overflow to infinity.
  * bfloat16: 8 significant bits, same exponent range as binary32, subnormal
    spacing 2^-133, round-to-nearest-even, overflow to infinity.
  * FP8 E4M3 (OCP "e4m3fn"): 4 significant bits, exponent bias 7, normal
    exponents -6..8, subnormal spacing 2^-9, largest finite value 448, no
    infinities.  Round-to-nearest-even; finite values beyond 448 saturate to
    +-448 (the saturating conversion; this choice is ours).

The emulated decomposition rounds at exactly the points where the GPU path
stores a low-precision operand and otherwise computes in float64.
"""
from __future__ import annotations

import numpy as np

from . import tucker as T

_FORMATS = {
    # name: (significant bits, min normal exponent, max finite, saturate)
    "f32": (24, -126, float.fromhex("0x1.fffffep127"), False),
    "bf16": (8, -126, float.fromhex("0x1.fep127"), False),
    "f8e4m3": (4, -6, 448.0, True),
}


def round_to(x, fmt: str) -> np.ndarray:
    """Round float64 values to the nearest value of ``fmt`` (ties to even); returns float64."""
    p, emin, vmax, sat = _FORMATS[fmt]
    x = np.asarray(x, dtype=np.float64)
    out = np.array(x, copy=True)
    fin = np.isfinite(x) & (x != 0.0)
    a = np.abs(x[fin])
    _, e = np.frexp(a)  # a = m * 2^e, 0.5 <= m < 1  ->  unit in last place 2^(e-p)
    e = np.maximum(e, emin + 1)  # below the normal range the spacing is fixed
    q = np.ldexp(np.rint(np.ldexp(a, -(e - p))), e - p)  # rint = round half to even
    if sat:
        q = np.minimum(q, vmax)
    else:
        q = np.where(q > vmax, np.inf, q)
    out[fin] = np.copysign(q, x[fin])
    return out


def round_bf16(x):
    return round_to(x, "bf16")


def round_f32(x):
    return round_to(x, "f32")


def round_f8(x):
    return round_to(x, "f8e4m3")


def bf16_bits(x) -> np.ndarray:
    """uint16 bit patterns of the bf16 values nearest to ``x`` (x must already be bf16-exact)."""
    v = np.asarray(x, dtype=np.float32).view(np.uint32)
    return (v >> 16).astype(np.uint16)


def f8_bits(x) -> np.ndarray:
    """uint8 E4M3 bit patterns of values that are already E4M3-exact (finite)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape, dtype=np.uint8)
    sign = (np.signbit(x)).astype(np.uint8) << 7
    a = np.abs(x)
    nz = a > 0
    _, e = np.frexp(a[nz])
    e = e - 1  # a = 1.f * 2^e
    sub = e < -6
    exp_field = np.where(sub, 0, e + 7)
    scale = np.where(sub, -9, e - 3)
    mant = np.rint(np.ldexp(a[nz], -scale)).astype(np.int64)
    mant = np.where(sub, mant, mant - 8)
    out[nz] = (exp_field.astype(np.int64) << 3 | mant).astype(np.uint8)
    return out | sign


def f8_decode(bits) -> np.ndarray:
    """float64 values of E4M3 bit patterns (0x7f / 0xff are NaN)."""
    b = np.asarray(bits, dtype=np.uint8).astype(np.int64)
    s = np.where(b & 0x80, -1.0, 1.0)
    ef = (b >> 3) & 0xF
    m = b & 0x7
    val = np.where(ef == 0, np.ldexp(m.astype(np.float64), -9),
                   np.ldexp((8 + m).astype(np.float64), ef - 10))
    val = np.where((ef == 15) & (m == 7), np.nan, val)
    return s * val


_ROUND = {"f64": lambda v: np.asarray(v, dtype=np.float64), "f32": round_f32,
          "bf16": round_bf16, "f8e4m3": round_f8}


def rhkron_emulated(X, r, phis, sketch_fmt: str, ttm_fmt: str, *, return_parts: bool = False):
    """Factor-reuse rHKron (Alg. 4.4, Sec. 4.3) with low-precision rounding at the GPU's rounding points.

    Sketch: X and every Phi_k rounded to ``sketch_fmt``; products exact (float64).
    QR, truncation: float64.  Core: the first contraction (largest mode) takes X
    and U_hat rounded to ``ttm_fmt``; its result is stored in binary32, and the
    later contractions take binary32 operands (the last one's result is kept in
    float64, as the GPU writes the core in binary64).
    """
    rs, rt = _ROUND[sketch_fmt], _ROUND[ttm_fmt]
    X = np.asarray(X, dtype=np.float64)
    d = X.ndim
    Xs = rs(X)
    ph = [rs(p) for p in phis]
    Uhat, Ys = [], []
    for n in range(d):
        Y = T.kron_sketch(Xs, ph, n)
        Q, _ = T.qr_pos(Y)
        Ys.append(Y)
        Uhat.append(Q)
    order = T.core_order(X.shape)
    Ghat = T.ttm(rt(X), rt(Uhat[order[0]]).T, order[0])
    lowp = ttm_fmt != "f64"
    for k in order[1:]:
        if lowp:
            Ghat = round_f32(Ghat)
        Ghat = T.ttm(Ghat, (round_f32(Uhat[k]) if lowp else Uhat[k]).T, k)
    G, Vs = T.sthosvd(Ghat, r)
    Us = [Uh @ V for Uh, V in zip(Uhat, Vs)]
    if return_parts:
        return G, Us, {"Uhat": Uhat, "Ghat": Ghat, "V": Vs, "Y": Ys}
    return G, Us


def rsthkron_emulated(X, r, phis, fmt: str, *, return_parts: bool = False):
    """Sequentially truncated rSTHKron (Alg. 4.3, Sec. 4.2) with low-precision rounding
    at the GPU's rounding points.

    The working core starts as X rounded to ``fmt``.  Step j (modes in order
    1..d) computes in the dtype of the current core: at the first step that is
    ``fmt``, afterwards binary32.  The step's factors Phi_{j,k} and its U_hat_j
    are rounded to that dtype; the sketch products and the contraction are exact
    (float64), the sketch's QR is float64, and the contracted core is stored in
    binary32 (except after the last step, whose result the GPU writes in
    binary64).  The final STHOSVD truncation is float64.
    """
    X = np.asarray(X, dtype=np.float64)
    d = X.ndim
    lowp = fmt != "f64"
    Ghat = _ROUND[fmt](X)
    Uhat, Ys = [], []
    for j in range(d):
        rj = _ROUND[fmt] if (j == 0 or not lowp) else round_f32
        Y = T.unfold(T.multi_ttm(Ghat, {k: rj(phis[j][k]) for k in range(d) if k != j}), j)
        Q, _ = T.qr_pos(Y)
        Ys.append(Y)
        Uhat.append(Q)
        Ghat = T.ttm(Ghat, rj(Q).T, j)
        if lowp and j < d - 1:
            Ghat = round_f32(Ghat)
    G, Vs = T.sthosvd(Ghat, r)
    Us = [Uh @ V for Uh, V in zip(Uhat, Vs)]
    if return_parts:
        return G, Us, {"Uhat": Uhat, "Ghat": Ghat, "V": Vs, "Y": Ys}
    return G, Us
