"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, and validates arguments and sizes workspace without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2211_13028_amd as rt
from oracle import tucker as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "rtucker.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rtucker_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = rt.lib()
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(rt.EXPORTED)
    assert "gfx950" in rt.rtucker_version()


def test_status_strings():
    L = rt.lib()
    for code in range(0, -8, -1):
        assert L.rtucker_status_string(code)
    assert L.rtucker_status_string(1) == b"unknown status"


@pytest.mark.parametrize("ell_r,p", [((8, 8, 8), 5), ((32, 32, 32), 8), ((16, 16, 16, 16), 6), ((4, 16, 16), 4),
                                     ((10, 10, 10), 5), ((3, 7, 2, 5), 3), ((31, 38, 35, 6, 11), 5)])
def test_sketch_sizes_match_oracle(ell_r, p):
    r = list(ell_r)
    dims = [max(200, v + p) for v in r]
    s = rt.rtucker_sketch_sizes(dims, r, p, "rhkron")
    assert s == T.subranks_reuse([v + p for v in r])
    S = rt.rtucker_sketch_sizes(dims, r, p, "rsthkron")
    want = T.subrank_matrix_sth([v + p for v in r])
    if len(r) == 2:
        want = [[1, r[0] + p], [r[1] + p, 1]]
    assert S == want


def test_sketch_sizes_workloads():
    assert rt.rtucker_sketch_sizes([64] * 3, [8] * 3, 5) == [4, 4, 4]
    assert rt.rtucker_sketch_sizes([1024, 1024, 512], [32] * 3, 8) == [7, 7, 7]
    assert rt.rtucker_sketch_sizes([128] * 4, [16] * 4, 6) == [3, 3, 3, 3]


def test_sketch_sizes_errors():
    L = rt.lib()
    out = (ctypes.c_int64 * 9)()
    dims = (ctypes.c_int64 * 3)(10, 10, 10)
    assert L.rtucker_sketch_sizes(3, dims, (ctypes.c_int32 * 3)(11, 2, 2), 2, 0, out) == -2
    assert L.rtucker_sketch_sizes(1, dims, (ctypes.c_int32 * 3)(2, 2, 2), 2, 0, out) == -1
    assert L.rtucker_sketch_sizes(3, dims, (ctypes.c_int32 * 3)(2, 2, 2), -1, 0, out) == -1
    assert L.rtucker_sketch_sizes(3, dims, (ctypes.c_int32 * 3)(2, 2, 2), 2, 7, out) == -1
    # s exceeding the mode size
    small = (ctypes.c_int64 * 3)(2, 40, 40)
    assert L.rtucker_sketch_sizes(3, small, (ctypes.c_int32 * 3)(1, 30, 30), 5, 0, out) == -2


def _tensor(dims, dtype=rt.RT_F32, data=None):
    x = rt.rt_tensor()
    x.d = len(dims)
    for i, v in enumerate(dims):
        x.dims[i] = v
    x.dtype = dtype
    x.data = data
    return x


def test_workspace_queries_without_gpu():
    L = rt.lib()
    nb = ctypes.c_size_t()
    X = _tensor([1024, 1024, 512])
    s = (ctypes.c_int64 * 3)(7, 7, 7)
    assert L.rtucker_sketch_workspace(ctypes.byref(X), s, 7, ctypes.byref(nb)) == 0
    assert nb.value > 1024 * 1024 * 7 * 4  # holds Z
    r = (ctypes.c_int32 * 3)(32, 32, 32)
    assert L.rtucker_decompose_workspace(ctypes.byref(X), None, r, 8, None, 0, ctypes.byref(nb)) == 0
    big = nb.value
    assert big % 256 == 0 and big > 49 * 1024 * 512 * 4
    assert L.rtucker_decompose_workspace(ctypes.byref(X), None, r, 8, None, 1, ctypes.byref(nb)) == 0
    assert L.rtucker_qr_workspace(1024, 49, ctypes.byref(nb)) == 0 and nb.value > 0
    assert L.rtucker_qr_workspace(200, 49, ctypes.byref(nb)) == 0 and nb.value > 0
    assert L.rtucker_qr_workspace(40, 60, ctypes.byref(nb)) == 0 and nb.value == 0  # wide: no workspace
    assert L.rtucker_qr_workspace(100, 65, ctypes.byref(nb)) == -2
    l = (ctypes.c_int64 * 3)(49, 49, 49)
    assert L.rtucker_core_workspace(ctypes.byref(X), l, 7, ctypes.byref(nb)) == 0 and nb.value > 49 * 1024 * 512 * 4
    assert L.rtucker_rel_error_workspace(ctypes.byref(X), r, ctypes.byref(nb)) == 0


def test_validation_errors_without_gpu():
    L = rt.lib()
    nb = ctypes.c_size_t()
    r = (ctypes.c_int32 * 3)(8, 8, 8)
    bad_d = _tensor([64])
    assert L.rtucker_decompose_workspace(ctypes.byref(bad_d), None, r, 5, None, 0, ctypes.byref(nb)) == -2
    X = _tensor([64, 64, 64], dtype=rt.RT_F8E4M3)
    assert L.rtucker_decompose_workspace(ctypes.byref(X), None, r, 5, None, 0, ctypes.byref(nb)) == -3
    X = _tensor([64, 64, 64], dtype=9)
    assert L.rtucker_decompose_workspace(ctypes.byref(X), None, r, 5, None, 0, ctypes.byref(nb)) == -3
    X = _tensor([64, 64, 64])
    # sketch too narrow for r + p
    s = (ctypes.c_int64 * 3)(3, 3, 3)
    assert L.rtucker_decompose_workspace(ctypes.byref(X), None, r, 5, s, 0, ctypes.byref(nb)) == -2
    # rank above the mode size
    assert L.rtucker_decompose_workspace(ctypes.byref(X), None, (ctypes.c_int32 * 3)(65, 8, 8), 5, None, 0,
                                         ctypes.byref(nb)) == -2
    # sketch width beyond the 64-column QR limit
    s = (ctypes.c_int64 * 3)(9, 9, 9)
    X100 = _tensor([100, 100, 100])
    assert L.rtucker_decompose_workspace(ctypes.byref(X100), None, r, 5, s, 0, ctypes.byref(nb)) == -2
    # ... but a width clipped to the mode size is fine
    assert L.rtucker_decompose_workspace(ctypes.byref(X), None, r, 5, s, 0, ctypes.byref(nb)) == 0
    # compute calls reject null data / workspace before touching the GPU
    phi = (ctypes.c_void_p * 3)(0, 0, 0)
    G = ctypes.c_void_p(0)
    U = (ctypes.c_void_p * 3)(0, 0, 0)
    assert L.rtucker_decompose(ctypes.byref(X), None, r, 5, None, 0, phi, G, U, None, 0, None) == -1
    Xd = _tensor([64, 64, 64], data=ctypes.c_void_p(4096))
    assert L.rtucker_decompose(ctypes.byref(Xd), None, r, 5, None, 0, phi, G, U, None, 0, None) == -1
    # workspace too small / misaligned (valid-looking pointers never dereferenced on the host)
    fake = [ctypes.c_void_p(4096 * (i + 2)) for i in range(4)]
    phi = (ctypes.c_void_p * 3)(*fake[:3])
    U = (ctypes.c_void_p * 3)(*fake[:3])
    assert L.rtucker_decompose(ctypes.byref(Xd), None, r, 5, None, 0, phi, fake[3], U, None, 0, None) == -4
    assert L.rtucker_decompose(ctypes.byref(Xd), None, r, 5, None, 0, phi, fake[3], U, ctypes.c_void_p(4096 + 8),
                               1 << 30, None) == -4
    assert L.rtucker_convert(None, rt.RT_F32, None, rt.RT_F64, 10, 0, None) == -3
    assert L.rtucker_convert(None, rt.RT_BF16, None, rt.RT_F32, 10, 0, None) == -3
    assert L.rtucker_convert(None, rt.RT_F32, None, rt.RT_BF16, -1, 0, None) == -1
    assert L.rtucker_convert(None, rt.RT_F32, None, rt.RT_BF16, 0, 0, None) == 0


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(rt, "_lib", None)
    monkeypatch.setattr(rt, "LIB_PATH", "/nonexistent/librtucker.so")
    with pytest.raises(rt.RtuckerError):
        rt.lib()


def test_binding_rejects_mismatched_operands():
    """Operand checks that happen in the binding before any library call (no GPU needed)."""
    import torch
    A = torch.zeros((4, 5), dtype=torch.float64)
    for B in (torch.zeros((4, 5), dtype=torch.float32), torch.zeros((5, 4), dtype=torch.float64),
              torch.zeros((10, 5), dtype=torch.float64)[::2]):
        with pytest.raises(rt.RtuckerError):
            rt.rtucker_sq_residual(A, B)
        with pytest.raises(rt.RtuckerError):
            rt.rtucker_scaled_diff(A, B)
    with pytest.raises(rt.RtuckerError):
        rt.rtucker_convert(torch.zeros((6, 4), dtype=torch.float32).t(), torch.bfloat16)


def test_status_code_minus_five_unused():
    assert rt.lib().rtucker_status_string(-5) == b"unknown status"


def _fake_batch(dims_list, ranks_list):
    items = (rt.rt_batch_item * len(dims_list))()
    for i, (d, r) in enumerate(zip(dims_list, ranks_list)):
        it = items[i]
        it.X = 0x1000
        it.G = 0x1000
        for k in range(3):
            it.dims[k], it.r[k], it.s[k] = d[k], r[k], 0
            it.phi[k] = 0x1000
            it.U[k] = 0x1000
    return items


def test_batch_tuning_cache_file(tmp_path, monkeypatch):
    """The autotuner's cache: defaults without a file; a file line for the batch's signature
    key sets the tuning; unparsable lines and values the plan rejects are skipped."""
    items = _fake_batch([(37, 41, 43), (50, 33, 61)], [(5, 6, 7), (4, 4, 9)])
    monkeypatch.delenv("RTUCKER_TUNE_CACHE", raising=False)
    mt, spb, key = rt.batched_tuning(items, 2, 4, rt.RT_F32)
    assert (mt, spb) == (16, 4)
    other = rt.batched_tuning(items, 2, 5, rt.RT_F32)[2]
    assert other != key  # p is part of the signature
    path = tmp_path / "tune.txt"
    path.write_text(f"not a line\n{key:016x} 8 2\n{key:016x} 7 3\n{other:016x} 32 1\n")
    monkeypatch.setenv("RTUCKER_TUNE_CACHE", str(path))
    assert rt.batched_tuning(items, 2, 4, rt.RT_F32)[:2] == (8, 2)
    assert rt.batched_tuning(items, 2, 5, rt.RT_F32)[:2] == (32, 1)
    with pytest.raises(rt.RtuckerError):
        rt.batched_tuning(items, 2, 4, rt.RT_F64)


def test_batch_workspace_independent_of_tuning(tmp_path, monkeypatch):
    """The batched workspace holds the job tables for every setting the autotuner may pick:
    the query gives the same size whatever the cache says."""
    dims = [(150, 40, 70), (192, 100, 33), (64, 64, 64)]
    ranks = [(6, 5, 4), (8, 8, 8), (4, 9, 5)]
    items = _fake_batch(dims, ranks)
    L = rt.lib()
    nb = ctypes.c_size_t()
    monkeypatch.delenv("RTUCKER_TUNE_CACHE", raising=False)
    assert L.rtucker_decompose_batched_workspace(3, items, 4, rt.RT_F32, ctypes.byref(nb)) == 0
    base = nb.value
    key = rt.batched_tuning(items, 3, 4, rt.RT_F32)[2]
    for mt, spb in ((8, 1), (32, 2), (16, 4)):
        path = tmp_path / f"t{mt}_{spb}.txt"
        path.write_text(f"{key:016x} {mt} {spb}\n")
        monkeypatch.setenv("RTUCKER_TUNE_CACHE", str(path))
        assert rt.batched_tuning(items, 3, 4, rt.RT_F32)[:2] == (mt, spb)
        assert L.rtucker_decompose_batched_workspace(3, items, 4, rt.RT_F32, ctypes.byref(nb)) == 0
        assert nb.value == base, (mt, spb)
