"""Python binding of librtucker (randomized Tucker with Kronecker sketches on MI355X).

Thin ctypes marshalling over the C ABI in include/rtucker.h: every function
here has the name of the C entry point it calls, turns torch tensors into
device pointers, allocates outputs and workspace with torch (device memory
only) and passes torch's current HIP stream.  All arithmetic happens in the
library's HIP kernels; there is no fallback: if the library is not built, or a
call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtucker.so")
MAX_D = 8

RT_F64, RT_F32, RT_BF16, RT_F8E4M3 = 0, 1, 2, 3
RT_RHKRON, RT_RSTHKRON = 0, 1
RT_RHKRON_NOREUSE = 2
ALGOS = {"rhkron": RT_RHKRON, "rsthkron": RT_RSTHKRON, "rhkron_noreuse": RT_RHKRON_NOREUSE}


class RtuckerError(RuntimeError):
    pass


class rt_tensor(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("dims", ctypes.c_int64 * MAX_D), ("dtype", ctypes.c_int),
                ("data", ctypes.c_void_p)]


class rt_batch_item(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("dims", ctypes.c_int64 * 3), ("r", ctypes.c_int32 * 3),
                ("s", ctypes.c_int64 * 3), ("phi", ctypes.c_void_p * 3), ("G", ctypes.c_void_p),
                ("U", ctypes.c_void_p * 3)]


_lib = None

_SIGS = {
    "rtucker_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rtucker_version": (ctypes.c_char_p, []),
    "rtucker_sketch_sizes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_int, ctypes.c_void_p]),
    "rtucker_sketch_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]),
    "rtucker_sketch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "rtucker_sketch_pass_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]),
    "rtucker_sketch_pass": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_size_t, ctypes.c_void_p]),
    "rtucker_qr_workspace": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]),
    "rtucker_qr": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "rtucker_core_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]),
    "rtucker_core": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "rtucker_decompose_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                                   ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "rtucker_decompose": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "rtucker_decompose_phases": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                                ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                                ctypes.c_void_p]),
    "rtucker_decompose_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                                 ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p]),
    "rtucker_sthosvd_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rtucker_sthosvd": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "rtucker_rel_error_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rtucker_rel_error": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "rtucker_convert": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.c_void_p]),
    "rtucker_srht_factor": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "rtucker_srht_sketch_last": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p]),
    "rtucker_multi_ttm_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                                   ctypes.c_void_p]),
    "rtucker_multi_ttm": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_void_p]),
    "rtucker_mode_contract_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                                       ctypes.c_void_p]),
    "rtucker_mode_contract": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "rtucker_sq_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "rtucker_scaled_diff": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "rtucker_decompose_batched_workspace": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                                           ctypes.c_int, ctypes.c_void_p]),
    "rtucker_decompose_batched": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int,
                                                 ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "rtucker_decompose_batched_upload": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int,
                                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "rtucker_decompose_batched_launch": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int,
                                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "rtucker_decompose_batched_autotune": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                                          ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                                          ctypes.c_void_p, ctypes.c_void_p]),
    "rtucker_decompose_batched_tuning": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                                        ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load librtucker.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RtuckerError(f"{LIB_PATH} is missing: build it with `python -m paper_2211_13028_amd.build`")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def _check(status: int, what: str):
    if status != 0:
        msg = lib().rtucker_status_string(status).decode()
        raise RtuckerError(f"{what} failed: {msg} ({status})")


# ------------------------------------------------------------------ marshalling helpers
def _torch():
    import torch
    return torch


def dtype_code(t) -> int:
    torch = _torch()
    m = {torch.float64: RT_F64, torch.float32: RT_F32, torch.bfloat16: RT_BF16}
    f8 = getattr(torch, "float8_e4m3fn", None)
    if f8 is not None:
        m[f8] = RT_F8E4M3
    if t.dtype not in m:
        raise RtuckerError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _tensor(t) -> rt_tensor:
    if not t.is_contiguous():
        raise RtuckerError("tensors must be contiguous (C order)")
    x = rt_tensor()
    x.d = t.dim()
    for i, v in enumerate(t.shape):
        x.dims[i] = int(v)
    x.dtype = dtype_code(t)
    x.data = _ptr(t)
    return x


def _i64(vals) -> ctypes.Array:
    return (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])


def _i32(vals) -> ctypes.Array:
    return (ctypes.c_int32 * len(vals))(*[int(v) for v in vals])


def _ptrs(ts) -> ctypes.Array:
    return (ctypes.c_void_p * len(ts))(*[_ptr(t) for t in ts])


def _stream(device=None) -> int:
    torch = _torch()
    return int(torch.cuda.current_stream(device).cuda_stream)


def _workspace(nbytes: int, device):
    torch = _torch()
    if nbytes == 0:
        return None, 0
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
    return ws, int(nbytes)


def _mask(modes, d) -> int:
    if modes is None:
        return (1 << d) - 1
    m = 0
    for k in modes:
        m |= 1 << int(k)
    return m


def _prod(vals):
    p = 1
    for v in vals:
        p *= int(v)
    return p


# ------------------------------------------------------------------ entry points
def rtucker_version() -> str:
    return lib().rtucker_version().decode()


def rtucker_sketch_sizes(dims: Sequence[int], r: Sequence[int], p: int, algo: str = "rhkron"):
    """Subranks: list of d (rhkron) or d x d nested list (rsthkron)."""
    d = len(dims)
    a = ALGOS[algo]
    out = (ctypes.c_int64 * (d if a == RT_RHKRON else d * d))()
    _check(lib().rtucker_sketch_sizes(d, _i64(dims), _i32(r), int(p), a, out), "rtucker_sketch_sizes")
    vals = list(out)
    return vals if a == RT_RHKRON else [vals[j * d:(j + 1) * d] for j in range(d)]


def rtucker_sketch(X, phis, s: Sequence[int], modes=None):
    """Sketch unfoldings Y_n = X x_{k != n} Phi_k (I_n x prod_{k != n} s_k); list with None for skipped modes."""
    torch = _torch()
    d = X.dim()
    mask = _mask(modes, d)
    xt = _tensor(X)
    nb = ctypes.c_size_t()
    _check(lib().rtucker_sketch_workspace(ctypes.byref(xt), _i64(s), mask, ctypes.byref(nb)), "rtucker_sketch_workspace")
    ydt = torch.float64 if X.dtype == torch.float64 else torch.float32
    Ys = []
    for n in range(d):
        if mask >> n & 1:
            Ys.append(torch.empty((X.shape[n], _prod(s[k] for k in range(d) if k != n)), dtype=ydt, device=X.device))
        else:
            Ys.append(None)
    ws, wb = _workspace(nb.value, X.device)
    _check(lib().rtucker_sketch(ctypes.byref(xt), _ptrs(phis), _i64(s), mask, _ptrs(Ys), _ptr(ws), wb,
                                _stream(X.device)), "rtucker_sketch")
    return Ys


def rtucker_sketch_pass(X, phi_prev, phi_last, Z=None, W=None, ws=None, want=(True, True)):
    """(Z, W) = (X x_d Phi_d, X x_{d-1} Phi_{d-1}) in one pass over X (either skipped via ``want``)."""
    torch = _torch()
    d = X.dim()
    xt = _tensor(X)
    s_prev, s_last = int(phi_prev.shape[0]), int(phi_last.shape[0])
    ct = torch.float64 if X.dtype == torch.float64 else torch.float32
    if want[0] and Z is None:
        Z = torch.empty(tuple(X.shape[:-1]) + (s_last,), dtype=ct, device=X.device)
    if want[1] and W is None:
        W = torch.empty(tuple(X.shape[:d - 2]) + (s_prev, X.shape[-1]), dtype=ct, device=X.device)
    if ws is None:
        nb = ctypes.c_size_t()
        _check(lib().rtucker_sketch_pass_workspace(ctypes.byref(xt), s_prev, s_last, ctypes.byref(nb)),
               "rtucker_sketch_pass_workspace")
        ws, wb = _workspace(nb.value, X.device)
    else:
        wb = int(ws.numel())
    _check(lib().rtucker_sketch_pass(ctypes.byref(xt), _ptr(phi_prev), s_prev, _ptr(phi_last), s_last,
                                     _ptr(Z if want[0] else None), _ptr(W if want[1] else None), _ptr(ws), wb,
                                     _stream(X.device)), "rtucker_sketch_pass")
    return (Z if want[0] else None), (W if want[1] else None)


def rtucker_qr(Y, want_r: bool = False):
    """Thin QR (binary64, diag(R) >= 0) of a device matrix (float32 or float64)."""
    torch = _torch()
    m, n = Y.shape
    c = min(m, n)
    nb = ctypes.c_size_t()
    _check(lib().rtucker_qr_workspace(m, n, ctypes.byref(nb)), "rtucker_qr_workspace")
    Q = torch.empty((m, c), dtype=torch.float64, device=Y.device)
    R = torch.empty((c, n), dtype=torch.float64, device=Y.device) if want_r else None
    ws, wb = _workspace(nb.value, Y.device)
    _check(lib().rtucker_qr(m, n, _ptr(Y.contiguous()), dtype_code(Y), _ptr(Q), _ptr(R), _ptr(ws), wb,
                            _stream(Y.device)), "rtucker_qr")
    return (Q, R) if want_r else Q


def rtucker_core(X, Us, modes=None):
    """G = X x_k U_k^T over ``modes`` (default all); U_k float64 I_k x l_k."""
    torch = _torch()
    d = X.dim()
    mask = _mask(modes, d)
    l = [int(Us[k].shape[1]) if (mask >> k & 1) else 0 for k in range(d)]
    xt = _tensor(X)
    nb = ctypes.c_size_t()
    _check(lib().rtucker_core_workspace(ctypes.byref(xt), _i64(l), mask, ctypes.byref(nb)), "rtucker_core_workspace")
    gdims = [l[k] if (mask >> k & 1) else X.shape[k] for k in range(d)]
    G = torch.empty(gdims, dtype=torch.float64 if X.dtype == torch.float64 else torch.float32, device=X.device)
    ws, wb = _workspace(nb.value, X.device)
    Up = [Us[k] if (mask >> k & 1) else None for k in range(d)]
    _check(lib().rtucker_core(ctypes.byref(xt), _ptrs(Up), _i64(l), mask, _ptr(G), _ptr(ws), wb, _stream(X.device)),
           "rtucker_core")
    return G


def _s_array(s, algo, d):
    if s is None:
        return None
    if ALGOS[algo] != RT_RHKRON:
        flat = [int(v) for row in s for v in row]
    else:
        flat = [int(v) for v in s]
    return _i64(flat)


def rtucker_decompose_workspace(X, r, p, algo="rhkron", s=None, X_sketch=None) -> int:
    xt = _tensor(X)
    xs = _tensor(X_sketch) if X_sketch is not None else None
    nb = ctypes.c_size_t()
    _check(lib().rtucker_decompose_workspace(ctypes.byref(xt), ctypes.byref(xs) if xs is not None else None, _i32(r),
                                             int(p), _s_array(s, algo, X.dim()), ALGOS[algo], ctypes.byref(nb)),
           "rtucker_decompose_workspace")
    return nb.value


def _decompose_args(X, r, p, phis, algo, s, X_sketch, G, Us, ws):
    torch = _torch()
    d = X.dim()
    xt = _tensor(X)
    xs = _tensor(X_sketch) if X_sketch is not None else None
    nb = rtucker_decompose_workspace(X, r, p, algo, s, X_sketch)
    if G is None:
        G = torch.empty([int(v) for v in r], dtype=torch.float64, device=X.device)
    if Us is None:
        Us = [torch.empty((X.shape[j], int(r[j])), dtype=torch.float64, device=X.device) for j in range(d)]
    if ws is None:
        ws, wb = _workspace(nb, X.device)
    else:
        wb = int(ws.numel())
    if ALGOS[algo] != RT_RHKRON:
        flat = [phis[j][k] if k != j else None for j in range(d) for k in range(d)]
    else:
        flat = list(phis)
    args = (ctypes.byref(xt), ctypes.byref(xs) if xs is not None else None, _i32(r), int(p), _s_array(s, algo, d),
            ALGOS[algo], _ptrs(flat), _ptr(G), _ptrs(Us), _ptr(ws), wb, _stream(X.device))
    return args, G, Us, (xt, xs, ws, flat)


def rtucker_decompose(X, r, p, phis, algo="rhkron", s=None, X_sketch=None, G=None, Us=None, ws=None):
    """Randomized Tucker decomposition; returns (G, [U_j]) in float64 on X's device.

    ``phis``: rhkron -> d float64 device matrices (s_k x I_k); rsthkron -> d x d nested
    list (None on the diagonal).  Preallocated ``G``, ``Us`` and workspace ``ws``
    (uint8 tensor) may be passed to avoid allocations (e.g. under graph capture).
    """
    args, G, Us, _keep = _decompose_args(X, r, p, phis, algo, s, X_sketch, G, Us, ws)
    _check(lib().rtucker_decompose(*args), "rtucker_decompose")
    return G, Us


NOALLOC_SCRATCH_BYTES = 64 << 20


def rtucker_decompose_noalloc(X, r, p, phis, G, Us, algo="rhkron", s=None, X_sketch=None):
    """rtucker_decompose into the caller's G and U_j, with the library's static device scratch
    as workspace (the C call allocates nothing; at most 64 MiB of workspace)."""
    d = X.dim()
    xt = _tensor(X)
    xs = _tensor(X_sketch) if X_sketch is not None else None
    if ALGOS[algo] != RT_RHKRON:
        flat = [phis[j][k] if k != j else None for j in range(d) for k in range(d)]
    else:
        flat = list(phis)
    _check(lib().rtucker_decompose_noalloc(ctypes.byref(xt), ctypes.byref(xs) if xs is not None else None, _i32(r),
                                           int(p), _s_array(s, algo, d), ALGOS[algo], _ptrs(flat), _ptr(G), _ptrs(Us),
                                           _stream(X.device)), "rtucker_decompose_noalloc")
    return G, Us


def rtucker_sthosvd_workspace(X, r) -> int:
    nb = ctypes.c_size_t()
    xt = _tensor(X)
    _check(lib().rtucker_sthosvd_workspace(ctypes.byref(xt), _i32(r), ctypes.byref(nb)), "rtucker_sthosvd_workspace")
    return int(nb.value)


def rtucker_sthosvd(X, r, G=None, Us=None, ws=None):
    """Deterministic STHOSVD (Alg. 2.2) on the device; returns (G, [U_j], subspace iterations).
    Synchronises."""
    torch = _torch()
    d = X.dim()
    xt = _tensor(X)
    nb = ctypes.c_size_t()
    _check(lib().rtucker_sthosvd_workspace(ctypes.byref(xt), _i32(r), ctypes.byref(nb)), "rtucker_sthosvd_workspace")
    if G is None:
        G = torch.empty([int(v) for v in r], dtype=torch.float64, device=X.device)
    if Us is None:
        Us = [torch.empty((X.shape[j], int(r[j])), dtype=torch.float64, device=X.device) for j in range(d)]
    if ws is None:
        ws, wb = _workspace(nb.value, X.device)
    else:
        wb = int(ws.numel())
    it = ctypes.c_int32(0)
    _check(lib().rtucker_sthosvd(ctypes.byref(xt), _i32(r), _ptr(G), _ptrs(Us), ctypes.byref(it), _ptr(ws), wb,
                                 _stream(X.device)), "rtucker_sthosvd")
    return G, Us, int(it.value)


PHASES = ("sketch", "qr", "core", "truncate")


def rtucker_decompose_phases(X, r, p, phis, algo="rhkron", s=None, X_sketch=None, G=None, Us=None, ws=None):
    """rtucker_decompose with the device time split by phase (synchronises):
    returns (G, [U_j], {"sketch": ms, "qr": ms, "core": ms, "truncate": ms})."""
    args, G, Us, _keep = _decompose_args(X, r, p, phis, algo, s, X_sketch, G, Us, ws)
    ms = (ctypes.c_float * 4)()
    _check(lib().rtucker_decompose_phases(*args, ms), "rtucker_decompose_phases")
    return G, Us, {name: float(ms[i]) for i, name in enumerate(PHASES)}


def rtucker_rel_error(X, G, Us, allow_nonfinite: bool = False):
    """(relative error, dict of squared norms) by explicit residual on the device (synchronises).

    Raises RtuckerError when X holds NaN or Inf entries, unless ``allow_nonfinite``:
    then the norms cover the finite entries and ``nonfinite`` counts the others."""
    torch = _torch()
    xt = _tensor(X)
    r = [int(v) for v in G.shape]
    nb = ctypes.c_size_t()
    _check(lib().rtucker_rel_error_workspace(ctypes.byref(xt), _i32(r), ctypes.byref(nb)), "rtucker_rel_error_workspace")
    out = torch.empty(4, dtype=torch.float64, device=X.device)
    ws, wb = _workspace(nb.value, X.device)
    _check(lib().rtucker_rel_error(ctypes.byref(xt), _ptr(G), _i32(r), _ptrs(Us), _ptr(out), _ptr(ws), wb,
                                   _stream(X.device)), "rtucker_rel_error")
    v = out.cpu().tolist()
    if v[3] > 0 and not allow_nonfinite:
        raise RtuckerError(f"input has {int(v[3])} non-finite entries")
    return (v[0] / v[1]) ** 0.5 if v[1] > 0 else float("nan"), {"res2": v[0], "x2": v[1], "g2": v[2], "nonfinite": v[3]}


def rtucker_convert(src, dst_dtype, scale_exp: int = 0, out=None):
    """Round src (float32/float64, device) * 2^scale_exp to float32 / bfloat16 / float8_e4m3fn
    (into ``out`` when given: contiguous, same shape, dtype dst_dtype)."""
    torch = _torch()
    if not src.is_contiguous():
        raise RtuckerError("rtucker_convert: src must be contiguous (C order)")
    if out is None:
        out = torch.empty(src.shape, dtype=dst_dtype, device=src.device)
    elif out.shape != src.shape or out.dtype != dst_dtype or out.device != src.device or not out.is_contiguous():
        raise RtuckerError("rtucker_convert: out must be contiguous, of src's shape and device, of dst_dtype")
    _check(lib().rtucker_convert(_ptr(src), dtype_code(src), _ptr(out), dtype_code(out), src.numel(), int(scale_exp),
                                 _stream(src.device)), "rtucker_convert")
    return out


def rtucker_srht_factor(n: int, rows, signs):
    """SRHT factor (R H D)[:, :n] (s x n float64 on the device of ``rows``) from sampled rows
    (int64 device tensor, s distinct values below the padded size) and n signs (float64)."""
    torch = _torch()
    if rows.dtype != torch.int64 or signs.dtype != torch.float64 or signs.numel() != int(n):
        raise RtuckerError("rtucker_srht_factor: rows int64, signs float64 of length n")
    rows, signs = rows.contiguous(), signs.contiguous()
    phi = torch.empty((rows.numel(), int(n)), dtype=torch.float64, device=rows.device)
    _check(lib().rtucker_srht_factor(int(n), rows.numel(), _ptr(rows), _ptr(signs), _ptr(phi), _stream(rows.device)),
           "rtucker_srht_factor")
    return phi


def rtucker_srht_sketch_last(X, rows, signs, Z=None):
    """Z = X x_last (R H D)[:, :Q] by a fast Walsh-Hadamard transform (float32 X)."""
    torch = _torch()
    xt = _tensor(X)
    if rows.dtype != torch.int64 or signs.dtype != torch.float64 or signs.numel() != X.shape[-1]:
        raise RtuckerError("rtucker_srht_sketch_last: rows int64, signs float64 of the last mode's length")
    rows, signs = rows.contiguous(), signs.contiguous()
    shape = tuple(X.shape[:-1]) + (rows.numel(),)
    if Z is None:
        Z = torch.empty(shape, dtype=torch.float32, device=X.device)
    elif tuple(Z.shape) != shape or Z.dtype != torch.float32 or not Z.is_contiguous():
        raise RtuckerError("rtucker_srht_sketch_last: Z has the wrong shape, dtype or layout")
    _check(lib().rtucker_srht_sketch_last(ctypes.byref(xt), rows.numel(), _ptr(rows), _ptr(signs), _ptr(Z),
                                          _stream(X.device)), "rtucker_srht_sketch_last")
    return Z


def rtucker_multi_ttm(X, As, modes=None, transpose: bool = False):
    """Y = X x_k op(A_k) for k in modes; op = A (m_k x I_k) or A^T when transpose (A_k: I_k x m_k)."""
    torch = _torch()
    d = X.dim()
    mask = _mask(modes, d)
    m = [0] * d
    for k in range(d):
        if mask >> k & 1:
            m[k] = int(As[k].shape[1] if transpose else As[k].shape[0])
    xt = _tensor(X)
    nb = ctypes.c_size_t()
    _check(lib().rtucker_multi_ttm_workspace(ctypes.byref(xt), _i64(m), mask, ctypes.byref(nb)),
           "rtucker_multi_ttm_workspace")
    ydims = [m[k] if (mask >> k & 1) else X.shape[k] for k in range(d)]
    Y = torch.empty(ydims, dtype=X.dtype, device=X.device)
    ws, wb = _workspace(nb.value, X.device)
    Ap = [As[k].contiguous() if (mask >> k & 1) else None for k in range(d)]
    _check(lib().rtucker_multi_ttm(ctypes.byref(xt), _ptrs(Ap), _i64(m), mask, 1 if transpose else 0, _ptr(Y),
                                   _ptr(ws), wb, _stream(X.device)), "rtucker_multi_ttm")
    return Y


def rtucker_mode_contract(P, Q, n: int, out=None):
    """P_(n) Q_(n)^T (sum over every index but mode n); added to `out` when it is given."""
    torch = _torch()
    pt, qt = _tensor(P), _tensor(Q)
    nb = ctypes.c_size_t()
    _check(lib().rtucker_mode_contract_workspace(ctypes.byref(pt), ctypes.byref(qt), int(n), ctypes.byref(nb)),
           "rtucker_mode_contract_workspace")
    acc = out is not None
    if out is None:
        out = torch.empty((P.shape[n], Q.shape[n]), dtype=P.dtype, device=P.device)
    elif tuple(out.shape) != (P.shape[n], Q.shape[n]) or out.dtype != P.dtype or not out.is_contiguous():
        raise RtuckerError("rtucker_mode_contract: out has the wrong shape, dtype or layout")
    ws, wb = _workspace(nb.value, P.device)
    _check(lib().rtucker_mode_contract(ctypes.byref(pt), ctypes.byref(qt), int(n), 1 if acc else 0, _ptr(out),
                                       _ptr(ws), wb, _stream(P.device)), "rtucker_mode_contract")
    return out


SQ_RESIDUAL_WS = 8192


def rtucker_sq_residual(A, B, want_r: bool = True):
    """(sum (A-B)^2 as a 1-element float64 device tensor, R = A - B or None)."""
    torch = _torch()
    at = _tensor(A)
    if B.shape != A.shape or B.dtype != A.dtype or B.device != A.device or not B.is_contiguous():
        raise RtuckerError("rtucker_sq_residual: B must match A in shape, dtype and device, and be contiguous")
    R = torch.empty_like(A) if want_r else None
    out = torch.empty(1, dtype=torch.float64, device=A.device)
    ws, wb = _workspace(SQ_RESIDUAL_WS, A.device)
    _check(lib().rtucker_sq_residual(ctypes.byref(at), _ptr(B), _ptr(R), _ptr(out), _ptr(ws), wb,
                                     _stream(A.device)), "rtucker_sq_residual")
    return out, R


def rtucker_scaled_diff(A, B=None, g=None, alpha: float = 1.0, out=None):
    """out = alpha * g * (A - B) elementwise (g: device float64 scalar tensor or None = 1; B None = 0)."""
    torch = _torch()
    at = _tensor(A)
    if B is not None and (B.shape != A.shape or B.dtype != A.dtype or B.device != A.device or not B.is_contiguous()):
        raise RtuckerError("rtucker_scaled_diff: B must match A")
    if g is not None and (g.dtype != torch.float64 or g.numel() != 1 or g.device != A.device):
        raise RtuckerError("rtucker_scaled_diff: g must be one float64 value on A's device")
    if out is None:
        out = torch.empty_like(A)
    _check(lib().rtucker_scaled_diff(ctypes.byref(at), _ptr(B), _ptr(g), float(alpha), _ptr(out),
                                     _stream(A.device)), "rtucker_scaled_diff")
    return out


def make_batch_items(Xs, ranks, phis, Gs, Us, s=None):
    items = (rt_batch_item * len(Xs))()
    for i, X in enumerate(Xs):
        it = items[i]
        it.X = _ptr(X)
        for k in range(3):
            it.dims[k] = int(X.shape[k])
            it.r[k] = int(ranks[i][k])
            it.s[k] = int(s[i][k]) if s is not None else 0
            it.phi[k] = _ptr(phis[i][k])
            it.U[k] = _ptr(Us[i][k])
        it.G = _ptr(Gs[i])
    return items


def batched_tuning(items, count: int, p: int, dtype: int):
    """Host query: (row tile, slabs per wave, signature key) that the batched calls would use
    for these items now (the tuning cache, else the defaults)."""
    tun = (ctypes.c_int32 * 2)()
    key = ctypes.c_uint64()
    _check(lib().rtucker_decompose_batched_tuning(int(count), items, int(p), int(dtype), tun, ctypes.byref(key)),
           "rtucker_decompose_batched_tuning")
    return int(tun[0]), int(tun[1]), int(key.value)


def rtucker_decompose_batched(Xs, ranks, p, phis, s=None, Gs=None, Us=None, ws=None):
    """Factor-reuse decomposition of many 3-way tensors (one dtype: float32 or bfloat16)."""
    torch = _torch()
    dev = Xs[0].device
    dt = dtype_code(Xs[0])
    if Gs is None:
        Gs = [torch.empty(tuple(int(v) for v in ranks[i]), dtype=torch.float64, device=dev) for i in range(len(Xs))]
    if Us is None:
        Us = [[torch.empty((int(Xs[i].shape[k]), int(ranks[i][k])), dtype=torch.float64, device=dev)
               for k in range(3)] for i in range(len(Xs))]
    items = make_batch_items(Xs, ranks, phis, Gs, Us, s)
    nb = ctypes.c_size_t()
    _check(lib().rtucker_decompose_batched_workspace(len(Xs), items, int(p), dt, ctypes.byref(nb)),
           "rtucker_decompose_batched_workspace")
    if ws is None:
        ws, wb = _workspace(nb.value, dev)
    else:
        wb = int(ws.numel())
    _check(lib().rtucker_decompose_batched(len(Xs), items, int(p), dt, _ptr(ws), wb, _stream(dev)),
           "rtucker_decompose_batched")
    return Gs, Us


class Batch:
    """A batch of 3-way tensors decomposed together by the grouped launches.

    Holds the item table, the outputs (G_i, U_i: float64) and the workspace, so
    that ``launch`` enqueues the whole batch with no host-device copy (it can be
    captured in a graph) once ``upload`` has written the job tables.
    """

    def __init__(self, Xs, ranks, p, phis, s=None):
        torch = _torch()
        self.Xs, self.ranks, self.p, self.phis = list(Xs), [tuple(int(v) for v in r) for r in ranks], int(p), phis
        self.device = self.Xs[0].device
        self.dt = dtype_code(self.Xs[0])
        for X in self.Xs:
            if dtype_code(X) != self.dt or X.dim() != 3 or not X.is_contiguous():
                raise RtuckerError("Batch: every tensor must be a contiguous 3-way tensor of one dtype")
        self.Gs = [torch.empty(r, dtype=torch.float64, device=self.device) for r in self.ranks]
        self.Us = [[torch.empty((int(X.shape[k]), r[k]), dtype=torch.float64, device=self.device) for k in range(3)]
                   for X, r in zip(self.Xs, self.ranks)]
        self.items = make_batch_items(self.Xs, self.ranks, phis, self.Gs, self.Us, s)
        nb = ctypes.c_size_t()
        _check(lib().rtucker_decompose_batched_workspace(len(self.Xs), self.items, self.p, self.dt, ctypes.byref(nb)),
               "rtucker_decompose_batched_workspace")
        self.ws, self.wb = _workspace(nb.value, self.device)

    def _args(self):
        return (len(self.Xs), self.items, self.p, self.dt, _ptr(self.ws), self.wb, _stream(self.device))

    def run(self):
        _check(lib().rtucker_decompose_batched(*self._args()), "rtucker_decompose_batched")
        return self.Gs, self.Us

    def upload(self):
        _check(lib().rtucker_decompose_batched_upload(*self._args()), "rtucker_decompose_batched_upload")

    def launch(self):
        _check(lib().rtucker_decompose_batched_launch(*self._args()), "rtucker_decompose_batched_launch")
        return self.Gs, self.Us

    def autotune(self):
        """Time every setting, keep the fastest; returns (row tile, slabs per wave)."""
        chosen = (ctypes.c_int32 * 2)()
        _check(lib().rtucker_decompose_batched_autotune(*self._args(), chosen), "rtucker_decompose_batched_autotune")
        return int(chosen[0]), int(chosen[1])

    def tuning(self):
        """The setting the batched calls use now: (row tile, slabs per wave, signature key)."""
        return batched_tuning(self.items, len(self.Xs), self.p, self.dt)

    def capture(self):
        """A torch CUDA graph whose replay runs ``launch`` (the tables must be uploaded)."""
        torch = _torch()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.launch()
        return g
