#!/usr/bin/env python3
"""Benchmark: randomized Tucker (rHKron, factor reuse) on one MI355X.

Workload: 1024 x 1024 x 512 smooth simulation-like field (200 separable
anisotropic Gaussian bumps, widths U[0.02, 0.2] of the domain, amplitude
U[0.5, 1.5], white noise at 1e-4 of ||f||), ranks (32, 32, 32), p = 8,
subranks s = 7 (sketch width 49), Gaussian Kronecker factors.  Synthetic data.

One step = one full decomposition on the device (all-at-once sketch, FP64
QR of the three sketches, core multi-TTM, FP64 STHOSVD truncation of the
49^3 core, U = U_hat V), inputs resident in HBM.  The headline line times
the FP32 path (binary32 tensor, binary32 matrix-core contractions).  The
precision form is timed beside it: BF16 (sketch also FP8 e4m3) with X resident
in the narrow format, and with X arriving in binary32 and the cast counted in
the step; rSTHKron likewise.  Each path also reports its device time per phase
(sketch, QR, core, truncation).

value = algorithmic multi-TTM flops of one step (sketch + core contractions,
unpadded) / step time, in TFLOP/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DIMS = (1024, 1024, 512)
RANKS = (32, 32, 32)
P_OVER = 8
HBM_PEAK = 8.0e12          # B/s
MFMA_PEAK = {"f32": 157.3e12, "bf16": 2.5e15, "f8": 5.0e15}
# (d, n, s) of the dimension-tree experiment timed here (the paper's third point, (3, 4000, 20),
# needs subrank 20, beyond the one-pass sketch's limit of 8)
E4_CASES = ((4, 500, 5), (5, 145, 3))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` from its committed byte-counter summary
    (profiles/hbm_counters_<kernel>_1024x1024x512.md), or None when there is none or the
    kernel's source has changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"hbm_counters_{kernel}_1024x1024x512.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    m_k = re.search(r"^traffic_kernel: (\S+)", text, re.M)
    m_b = re.search(r"^traffic_bytes_per_launch: (\d+)", text, re.M)
    m_h = re.search(r"^source_sha256\((\S+)\): ([0-9a-f]+)", text, re.M)
    if not (m_k and m_b and m_h) or m_k.group(1) != kernel:
        return None
    try:
        src = open(os.path.join(ROOT, m_h.group(1)), "rb").read()
    except OSError:
        return None
    if hashlib.sha256(src).hexdigest() != m_h.group(2):
        return None
    return int(m_b.group(1))


def multi_ttm_flops(dims, s, ell):
    """Unpadded flops of the sketch (dimension tree, d = 3) and core contractions."""
    I1, I2, I3 = dims
    s1, s2, s3 = s
    N = I1 * I2 * I3
    sketch = 2 * N * (s3 + s2)                    # Z = X x3 Phi3, W = X x2 Phi2 (one pass)
    sketch += 2 * s2 * I1 * I2 * s3               # Y1 = Z x2 Phi2
    sketch += 2 * s1 * I1 * I2 * s3               # Y2 = Z x1 Phi1
    sketch += 2 * s1 * I1 * s2 * I3               # Y3 = W x1 Phi1
    l1, l2, l3 = ell
    core = 2 * l1 * N + 2 * l2 * (l1 * I2 * I3) + 2 * l3 * (l1 * l2 * I3)
    return sketch, core


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="time only the headline FP32 path")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device buffers three times (reference for the HBM byte counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 128^4 rSTHKron, 256^3 adjoint and 512-tensor batch measurements")
    ap.add_argument("--no-paper-scale", action="store_true",
                    help="skip the tensors of the paper's own scale (the dimension-tree experiment at ~256 GB "
                         "and the 410^4 exact-rank tensor)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "rtucker runs on one GPU only; sharding across GPUs is described in the "
                                   "design notes, not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = 1 << 28  # float32 elements: 1 GiB read and 1 GiB written per copy
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 3}))
        return

    import paper_2211_13028_amd as rt
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    log("generating the 1024x1024x512 field ...")
    Xh = synth.bumps_field(DIMS, nbumps=200, noise_rel=1e-4, seed=synth.DATA_SEED)
    log(f"  generated in {time.time() - t0:.1f} s")
    X32 = torch.from_numpy(Xh).to(dev)
    X16 = rt.rtucker_convert(X32, torch.bfloat16)
    X8 = rt.rtucker_convert(X32, torch.float8_e4m3fn)
    s = rt.rtucker_sketch_sizes(DIMS, RANKS, P_OVER, "rhkron")
    ell = [int(np.prod([s[k] for k in range(3) if k != n])) for n in range(3)]
    phis_h = synth.gaussians(synth.PHI_SEED, [(s[k], DIMS[k]) for k in range(3)])
    phis = [torch.from_numpy(f).to(dev) for f in phis_h]
    S = rt.rtucker_sketch_sizes(DIMS, RANKS, P_OVER, "rsthkron")
    stream = torch.cuda.current_stream()

    def make_run(X, algo="rhkron", Xs=None, sizes=None, ph=None):
        nb = rt.rtucker_decompose_workspace(X, RANKS, P_OVER, algo, sizes, Xs)
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
        G = torch.empty(RANKS, dtype=torch.float64, device=dev)
        Us = [torch.empty((DIMS[j], RANKS[j]), dtype=torch.float64, device=dev) for j in range(3)]
        pp = ph if ph is not None else phis

        def run():
            rt.rtucker_decompose(X, RANKS, P_OVER, pp, algo=algo, s=sizes, X_sketch=Xs, G=G, Us=Us, ws=ws)
        return run, G, Us

    def time_steps(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps  # ms

    sk_flops, core_flops = multi_ttm_flops(DIMS, s, ell)
    step_flops = sk_flops + core_flops
    results = {}

    def phases_of(X, algo="rhkron", Xs=None, sizes=None, ph=None, reps=5):
        """Median device time per phase over `reps` calls of the phase-timed entry point."""
        nb = rt.rtucker_decompose_workspace(X, RANKS, P_OVER, algo, sizes, Xs)
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
        rows = []
        for _ in range(reps):
            _, _, pm = rt.rtucker_decompose_phases(X, RANKS, P_OVER, ph if ph is not None else phis, algo=algo,
                                                   s=sizes, X_sketch=Xs, ws=ws)
            rows.append(pm)
        return {k: round(float(np.median([r[k] for r in rows])), 4) for k in rows[0]}

    # ---------------------------------------------------------------- headline: FP32
    run32, G32, U32 = make_run(X32, sizes=s)
    log("timing FP32 rHKron (headline) ...")
    ms32 = time_steps(run32, args.steps, args.warmup)
    e32, _ = rt.rtucker_rel_error(X32, G32, U32)
    results["rhkron_f32"] = {"ms": ms32, "rel_err": e32, "phases_ms": phases_of(X32, sizes=s)}

    if not args.no_variants:
        # BF16 with X resident in bfloat16, and with X arriving in binary32 (the cast timed in the step)
        run16, G16, U16 = make_run(X16, sizes=s)
        log("timing BF16 rHKron ...")
        ms16 = time_steps(run16, args.steps, args.warmup)
        e16, _ = rt.rtucker_rel_error(X32, G16, U16)
        results["rhkron_bf16"] = {"ms": ms16, "rel_err": e16, "phases_ms": phases_of(X16, sizes=s)}

        def run16_cast():
            rt.rtucker_convert(X32, torch.bfloat16, out=X16)
            run16()
        ms = time_steps(run16_cast, args.steps, args.warmup)
        e, _ = rt.rtucker_rel_error(X32, G16, U16)
        results["rhkron_bf16_cast_counted"] = {"ms": ms, "rel_err": e}
        run8, G8, U8 = make_run(X16, Xs=X8, sizes=s)
        log("timing BF16 rHKron with FP8 sketch ...")
        ms8 = time_steps(run8, args.steps, args.warmup)
        e8, _ = rt.rtucker_rel_error(X32, G8, U8)
        results["rhkron_bf16_f8sketch"] = {"ms": ms8, "rel_err": e8, "phases_ms": phases_of(X16, Xs=X8, sizes=s)}

        def run8_cast():
            rt.rtucker_convert(X32, torch.bfloat16, out=X16)
            rt.rtucker_convert(X32, torch.float8_e4m3fn, out=X8)
            run8()
        ms = time_steps(run8_cast, args.steps, args.warmup)
        e, _ = rt.rtucker_rel_error(X32, G8, U8)
        results["rhkron_bf16_f8sketch_cast_counted"] = {"ms": ms, "rel_err": e}
        shapes = []
        cdim = [min(DIMS[k], int(np.prod([S[k][i] for i in range(3) if i != k]))) for k in range(3)]
        for j in range(3):
            for k in range(3):
                shapes.append(None if k == j else (S[j][k], cdim[k] if k < j else DIMS[k]))
        flat = synth.gaussians(synth.PHI_SEED, shapes)
        sphis = [[None if f is None else torch.from_numpy(f).to(dev) for f in flat[j * 3:(j + 1) * 3]]
                 for j in range(3)]
        # the sketch variants (FP32): an independent factor set per mode (App. A), and the reuse
        # algorithm with subsampled randomized Hadamard factors made on the device (Sec. 5.1)
        SN = rt.rtucker_sketch_sizes(DIMS, RANKS, P_OVER, "rhkron_noreuse")
        nshapes = [None if k == j else (SN[j][k], DIMS[k]) for j in range(3) for k in range(3)]
        nflat = synth.gaussians(synth.PHI_SEED, nshapes)
        nphis = [[None if f is None else torch.from_numpy(f).to(dev) for f in nflat[j * 3:(j + 1) * 3]]
                 for j in range(3)]
        fn, G, U = make_run(X32, algo="rhkron_noreuse", sizes=SN, ph=nphis)
        log("timing rhkron_noreuse_f32 ...")
        ms = time_steps(fn, max(3, args.steps // 2), 2)
        e, _ = rt.rtucker_rel_error(X32, G, U)
        results["rhkron_noreuse_f32"] = {"ms": ms, "rel_err": e,
                                         "phases_ms": phases_of(X32, "rhkron_noreuse", sizes=SN, ph=nphis)}
        pads = [1 << (int(n) - 1).bit_length() for n in DIMS]
        draws = synth.srht_draws(synth.PHI_SEED, [(s[k], pads[k], DIMS[k]) for k in range(3)])
        sr_phis = [rt.rtucker_srht_factor(DIMS[k], torch.from_numpy(draws[k][0]).to(dev),
                                          torch.from_numpy(draws[k][1]).to(dev)) for k in range(3)]
        fn, G, U = make_run(X32, sizes=s, ph=sr_phis)
        log("timing rhkron_srht_f32 ...")
        ms = time_steps(fn, max(3, args.steps // 2), 2)
        e, _ = rt.rtucker_rel_error(X32, G, U)
        results["rhkron_srht_f32"] = {"ms": ms, "rel_err": e}
        for name, X in (("rsthkron_f32", X32), ("rsthkron_bf16", X16)):
            fn, G, U = make_run(X, algo="rsthkron", sizes=S, ph=sphis)
            log(f"timing {name} ...")
            ms = time_steps(fn, max(3, args.steps // 2), 2)
            e, _ = rt.rtucker_rel_error(X32, G, U)
            results[name] = {"ms": ms, "rel_err": e, "phases_ms": phases_of(X, "rsthkron", sizes=S, ph=sphis)}
            if name == "rsthkron_bf16":
                def fn_cast():
                    rt.rtucker_convert(X32, torch.bfloat16, out=X16)
                    fn()
                ms = time_steps(fn_cast, max(3, args.steps // 2), 2)
                e, _ = rt.rtucker_rel_error(X32, G, U)
                results["rsthkron_bf16_cast_counted"] = {"ms": ms, "rel_err": e}

    if not args.no_variants:
        # the deterministic STHOSVD (Alg. 2.2) on the device: the baseline of the paper's
        # "randomized vs STHOSVD" comparisons
        Gd = torch.empty(RANKS, dtype=torch.float64, device=dev)
        Ud = [torch.empty((DIMS[j], RANKS[j]), dtype=torch.float64, device=dev) for j in range(3)]
        nbs = rt.rtucker_sthosvd_workspace(X32, RANKS)
        wss = torch.empty(max(nbs, 256), dtype=torch.uint8, device=dev)
        its = []
        log("timing the deterministic STHOSVD ...")
        ms = time_steps(lambda: its.append(rt.rtucker_sthosvd(X32, RANKS, G=Gd, Us=Ud, ws=wss)[2]), 3, 1)
        e, _ = rt.rtucker_rel_error(X32, Gd, Ud)
        results["sthosvd_f32"] = {"ms": ms, "rel_err": e, "subspace_iterations": its[-1],
                                  "ratio_to_rhkron_f32": round(ms / ms32, 2)}
        del wss

    # ---------------------------------------------------------------- per-kernel rooflines
    N = int(np.prod(DIMS))
    kernels = {}
    Uh = [torch.linalg.qr(torch.randn((DIMS[k], ell[k]), dtype=torch.float64, device=dev))[0].contiguous()
          for k in range(3)]

    def kernel_time(fn, reps=10):
        return time_steps(fn, reps, 2)

    # the binary32 -> bfloat16 cast: 4 bytes read, 2 written per element
    ms = kernel_time(lambda: rt.rtucker_convert(X32, torch.bfloat16, out=X16))
    kernels["cast_f32_bf16"] = {"ms": ms, "GB/s": 6 * N / ms / 1e6, "alg_bytes": 6 * N}
    def in_step_time(fn, reps=10):
        """fn's duration (HIP events on the stream) when it runs as it does inside the headline
        step: each timed call follows one whole FP32 decomposition (untimed)."""
        tot = 0.0
        for i in range(reps + 1):
            run32()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            if i > 0:
                tot += a.elapsed_time(b)
        return tot / reps

    for tag, X, esz in (("f32", X32, 4), ("bf16", X16, 2)):
        # first core contraction: X x_1 U_hat_1^T (MFMA), plus a tiny operand-rounding kernel.
        # "ms" is its duration inside the step (after a decomposition, as in the timed steps);
        # "ms_back_to_back" the same call repeated without pause, where the matrix-core-heavy
        # FP32 kernel runs slower
        core = lambda: rt.rtucker_core(X, Uh, modes=[0])
        ms_b2b = kernel_time(core)
        ms = in_step_time(core)
        byts = N * esz + ell[0] * (N // DIMS[0]) * 4 + DIMS[0] * ell[0] * esz
        fl = 2 * ell[0] * N
        kernels[f"core_ttm1_{tag}"] = {"ms": ms, "GB/s": byts / ms / 1e6, "TFLOP/s": fl / ms / 1e9,
                                       "alg_bytes": byts, "alg_flops": fl, "ms_back_to_back": ms_b2b,
                                       "TFLOP/s_back_to_back": fl / ms_b2b / 1e9}
        # the streaming sketch pass: Z = X x3 Phi3 and W = X x2 Phi2 in one read of X
        # (launches: operand rounding, the pass, and the fixed-order sum of its row-range partials)
        Zb = torch.empty((DIMS[0], DIMS[1], s[2]), dtype=torch.float32, device=dev)
        Wb = torch.empty((DIMS[0], s[1], DIMS[2]), dtype=torch.float32, device=dev)
        Zb, Wb = rt.rtucker_sketch_pass(X, phis[1], phis[2], Z=Zb, W=Wb)
        ms = kernel_time(lambda: rt.rtucker_sketch_pass(X, phis[1], phis[2], Z=Zb, W=Wb))
        byts = N * esz + (Zb.numel() + Wb.numel()) * 4
        fl = 2 * N * (s[1] + s[2])
        kernels[f"sketch_pass_{tag}"] = {"ms": ms, "GB/s": byts / ms / 1e6, "TFLOP/s": fl / ms / 1e9,
                                         "alg_bytes": byts, "alg_flops": fl}
        # the whole sketch call (pass + the small contractions of the tree + unfolds)
        ms = kernel_time(lambda: rt.rtucker_sketch(X, phis, s))
        zbytes = (DIMS[0] * DIMS[1] * s[2] + DIMS[0] * s[1] * DIMS[2]) * 4
        byts = N * esz + zbytes
        fl = sk_flops
        kernels[f"sketch_{tag}"] = {"ms": ms, "GB/s": byts / ms / 1e6, "TFLOP/s": fl / ms / 1e9,
                                    "alg_bytes": byts, "alg_flops": fl}
        if tag == "f32":
            # the SRHT sketch of the last mode by a fast Walsh-Hadamard transform, beside the
            # dense-factor pass above (which also makes W): same read of X, s outputs per fiber
            pad = 1 << (DIMS[2] - 1).bit_length()
            (rows, signs), = synth.srht_draws(synth.PHI_SEED, [(s[2], pad, DIMS[2])])
            rows_d, signs_d = torch.from_numpy(rows).to(dev), torch.from_numpy(signs).to(dev)
            Zs = rt.rtucker_srht_sketch_last(X, rows_d, signs_d, Z=Zb)
            ms = kernel_time(lambda: rt.rtucker_srht_sketch_last(X, rows_d, signs_d, Z=Zs))
            byts = N * esz + Zb.numel() * 4
            kernels["srht_fwht_last_f32"] = {"ms": ms, "GB/s": byts / ms / 1e6, "alg_bytes": byts}
        del Zb, Wb

    # dominant kernel of the headline (FP32) step: the first core contraction, a dense contraction
    # on the binary32 matrix cores (arithmetic intensity 23 flop/B, above the ridge)
    dom = "core_ttm1_f32"
    kd = kernels[dom]
    roofline = {"kernel": dom, "bound": "mfma", "achieved": round(kd["TFLOP/s"], 2), "peak": MFMA_PEAK["f32"] / 1e12,
                "unit": "TFLOP/s", "frac": round(kd["TFLOP/s"] * 1e12 / MFMA_PEAK["f32"], 4),
                "traffic": counter_traffic(dom)}

    extras = {}
    if not args.no_extras:
        extras = run_extras(rt, synth, torch, dev, time_steps, log)
    if not args.no_paper_scale:
        extras.update(run_paper_scale(rt, synth, torch, dev, time_steps, log, keep=[X32, X16, X8]))

    # ---------------------------------------------------------------- CPU baseline (oracle, whole workload)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(Xh, phis_h, step_flops)

    value = step_flops / (ms32 / 1e3) / 1e12
    out = {
        "metric": "rHKron time + multi-TTM TFLOP/s, BF16-MFMA vs FP32 at stated rel. error",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rHKron 1024x1024x512 smooth field, r=32, p=8, s=7 (sketch width 49)",
                   "dims": list(DIMS), "ranks": list(RANKS), "p": P_OVER, "s": s,
                   "step_multi_ttm_gflop": round(step_flops / 1e9, 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paths": {k: {kk: (round(vv, 4) if kk == "ms" else vv) for kk, vv in v.items()} for k, v in results.items()},
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kernels.items()},
        "other_workloads": extras,
    }
    print(json.dumps(out))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(Xh, phis_h, step_flops):
    """The FP64 oracle on the whole workload: all host cores, then one core (threadpoolctl)."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import tucker as T

    Xd64 = Xh.astype(np.float64)

    def timed(reps):
        times = []
        for _ in range(reps):
            t1 = time.perf_counter()
            T.rhkron(Xd64, list(RANKS), phis_h)
            times.append(time.perf_counter() - t1)
        return float(np.median(times))

    log("timing the CPU oracle (numpy FP64) on the whole workload, all cores ...")
    info = [p for p in threadpool_info() if p.get("user_api") == "blas"]
    threads = max([int(p.get("num_threads", 1)) for p in info] or [1])
    blas = ", ".join(f"{p.get('internal_api')} {p.get('version')}" for p in info) or "unknown"
    dt_all = timed(3)
    log("timing the CPU oracle on one core ...")
    with threadpool_limits(limits=1):
        dt_one = timed(1)
    del Xd64
    return {"value": round(step_flops / dt_all / 1e12, 6), "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"whole workload (1024x1024x512, FP64 numpy rHKron incl. truncation), median of 3 runs on "
                      f"{threads} BLAS threads: {dt_all:.3f} s; one thread: {dt_one:.3f} s",
            "one_core": {"value": round(step_flops / dt_one / 1e12, 6), "seconds": round(dt_one, 3), "cores": 1},
            "cpu_model": cpu_model(), "blas": blas}


def run_paper_scale(rt, synth, torch, dev, time_steps, log, keep=()):
    """Workloads at the paper's own sizes, generated on the device (exact Tucker tensors):

    * the dimension-tree experiment (Sec. 7.3): the sketch of every mode of a d-way n^d
      binary32 tensor with s = subrank per mode, (d, n, s) = (4, 500, 5) and (5, 145, 3),
      about 256 GB each; "tree on" = all modes in one call (one read of X
      for the first level, memoised tree below it), "tree off" = one call per mode;
    * the strong-scaling tensor (Sec. 7.4): 410^4 binary32 (113 GB), exact rank 20,
      r = 20, p = 3, rHKron and rSTHKron on one GPU.
    Each is skipped when the device lacks the memory."""
    out = {}
    torch.cuda.empty_cache()
    held = sum(int(t.numel()) * t.element_size() for t in keep)

    def room(nbytes):
        free, _ = torch.cuda.mem_get_info()
        return free >= nbytes + (24 << 30)

    e4 = {}
    for d, n, sub in E4_CASES:
        key = f"d{d}_n{n}_s{sub}"
        nbytes = 4 * n ** d
        if not room(nbytes):
            e4[key] = {"skipped": f"needs {nbytes / 2**30:.0f} GiB + 24 GiB free ({held / 2**30:.1f} GiB held)"}
            continue
        log(f"dimension-tree experiment {key}: generating {nbytes / 1e9:.0f} GB on the device ...")
        core, F = synth.tucker_factors((n,) * d, [6] * d, seed=80 + d)
        X = synth.tucker_on_device(core, F, dev, torch.float32)
        sv = [sub] * d
        phis = [torch.from_numpy(f).to(dev) for f in synth.gaussians(90 + d, [(sub, n)] * d)]
        on = time_steps(lambda: rt.rtucker_sketch(X, phis, sv), 3, 1)

        def tree_off():
            for m in range(d):
                rt.rtucker_sketch(X, phis, sv, modes=[m])
        off = time_steps(tree_off, 2, 1)
        e4[key] = {"tree_on_ms": round(on, 3), "tree_off_ms": round(off, 3), "speedup": round(off / on, 3),
                   "tree_on_GB/s": round(nbytes / on / 1e6, 1),
                   "tree_on_hbm_frac": round(nbytes / on / 1e6 / (HBM_PEAK / 1e9), 4)}
        del X
        torch.cuda.empty_cache()
    out["e4_dimension_tree"] = e4

    dims, r, p = (410,) * 4, [20] * 4, 3
    nbytes = 4 * 410 ** 4
    if room(int(nbytes * 1.25)):
        log("generating the 410^4 exact-rank tensor (113 GB) on the device ...")
        core, F = synth.tucker_factors(dims, r, seed=synth.DATA_SEED)
        X = synth.tucker_on_device(core, F, dev, torch.float32)
        for algo in ("rhkron", "rsthkron"):
            S = rt.rtucker_sketch_sizes(dims, r, p, algo)
            if algo == "rhkron":
                shapes = [(S[k], dims[k]) for k in range(4)]
            else:
                cdim = [min(dims[k], int(np.prod([S[k][i] for i in range(4) if i != k]))) for k in range(4)]
                shapes = [None if k == j else (S[j][k], cdim[k] if k < j else dims[k]) for j in range(4)
                          for k in range(4)]
            flat = [None if f is None else torch.from_numpy(f).to(dev) for f in synth.gaussians(synth.PHI_SEED, shapes)]
            ph = flat if algo == "rhkron" else [flat[j * 4:(j + 1) * 4] for j in range(4)]
            nb = rt.rtucker_decompose_workspace(X, r, p, algo, S)
            ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
            G = torch.empty(r, dtype=torch.float64, device=dev)
            Us = [torch.empty((410, 20), dtype=torch.float64, device=dev) for _ in range(4)]
            log(f"timing 410^4 {algo} ...")
            ms = time_steps(lambda: rt.rtucker_decompose(X, r, p, ph, algo=algo, s=S, G=G, Us=Us, ws=ws), 5, 2)
            _, _, phases = rt.rtucker_decompose_phases(X, r, p, ph, algo=algo, s=S, G=G, Us=Us, ws=ws)
            del ws
            torch.cuda.empty_cache()
            e, _ = rt.rtucker_rel_error(X, G, Us)
            gap = max(float(np.linalg.norm(u @ u.T - f @ f.T, 2)) for u, f in zip([u.cpu().numpy() for u in Us], F))
            out[f"{algo}_410^4_f32"] = {"ms": round(ms, 3), "rel_err": e, "max_subspace_gap": gap,
                                        "phases_ms": {k: round(v, 3) for k, v in phases.items()},
                                        "read_GB/s": round(nbytes / ms / 1e6, 1)}
        G = torch.empty(r, dtype=torch.float64, device=dev)
        Us = [torch.empty((410, 20), dtype=torch.float64, device=dev) for _ in range(4)]
        nb = rt.rtucker_sthosvd_workspace(X, r)
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
        log("timing 410^4 deterministic STHOSVD ...")
        ms = time_steps(lambda: rt.rtucker_sthosvd(X, r, G=G, Us=Us, ws=ws), 2, 1)
        del ws
        torch.cuda.empty_cache()
        e, _ = rt.rtucker_rel_error(X, G, Us)
        out["sthosvd_410^4_f32"] = {"ms": round(ms, 3), "rel_err": e}
        for algo in ("rhkron", "rsthkron"):
            key = f"{algo}_410^4_f32"
            if key in out and "ms" in out[key]:
                out[key]["speedup_over_sthosvd"] = round(ms / out[key]["ms"], 2)
        del X
        torch.cuda.empty_cache()
    else:
        out["rhkron_410^4_f32"] = {"skipped": "not enough device memory"}
    return out


def run_extras(rt, synth, torch, dev, time_steps, log):
    """The other workloads, timed beside the headline (not part of its value)."""
    from paper_2211_13028_amd import autograd as RA
    out = {}
    # ---- 128^4 FP32, decaying 16^4 core, rSTHKron with subranks 3 (sketch width 27), r = 16, p = 6
    dims4, r4 = (128, 128, 128, 128), (16, 16, 16, 16)
    log("generating the 128^4 tensor ...")
    core = synth.tucker_core_decay((16, 16, 16, 16), 6.0, seed=synth.DATA_SEED)
    X4h, _, _ = synth.random_tucker(dims4, (16, 16, 16, 16), 1e-3, seed=synth.DATA_SEED, core=core)
    X4 = torch.from_numpy(X4h.astype(np.float32)).to(dev)
    del X4h
    S4 = [[1 if k == j else 3 for k in range(4)] for j in range(4)]
    cdim = [min(dims4[k], 27) for k in range(4)]
    shapes = [None if k == j else (3, cdim[k] if k < j else dims4[k]) for j in range(4) for k in range(4)]
    flat = synth.gaussians(synth.PHI_SEED, shapes)
    ph4 = [[None if f is None else torch.from_numpy(f).to(dev) for f in flat[j * 4:(j + 1) * 4]] for j in range(4)]
    for tag, X in (("f32", X4), ("bf16", rt.rtucker_convert(X4, torch.bfloat16))):
        nb = rt.rtucker_decompose_workspace(X, r4, 6, "rsthkron", S4)
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
        G = torch.empty(r4, dtype=torch.float64, device=dev)
        Us = [torch.empty((128, 16), dtype=torch.float64, device=dev) for _ in range(4)]

        def fn():
            rt.rtucker_decompose(X, r4, 6, ph4, algo="rsthkron", s=S4, G=G, Us=Us, ws=ws)
        log(f"timing 128^4 rSTHKron {tag} ...")
        ms = time_steps(fn, 10, 2)
        e, _ = rt.rtucker_rel_error(X4, G, Us)
        out[f"rsthkron_128^4_{tag}"] = {"ms": round(ms, 4), "rel_err": e}
        del ws
    del X4
    torch.cuda.empty_cache()
    # ---- 256^3 FP32 projection loss, fixed rank-24 factors: forward + hand-written backward
    n3, rr = 256, 24
    X3h, _, _ = synth.random_tucker((n3, n3, n3), (rr, rr, rr), 1e-6, seed=synth.DATA_SEED)
    X3 = torch.from_numpy(X3h.astype(np.float32)).to(dev).requires_grad_(True)
    U3 = [torch.from_numpy(u.astype(np.float32)).to(dev).requires_grad_(True)
          for u in synth.fixed_factors((n3, n3, n3), (rr, rr, rr))]

    def step():
        X3.grad = None
        for u in U3:
            u.grad = None
        RA.projection_loss(X3, U3).backward()
    log("timing the 256^3 projection loss forward + backward ...")
    ms = time_steps(step, 20, 3)
    # algorithmic traffic: X read by the forward (G, then the residual) and by the backward
    # recomputation (2 passes); R written and read 4 times; X_hat, P R and dX written once each
    nbytes = X3.numel() * 4
    alg = nbytes * (2 + 2) + nbytes * (1 + 4) + nbytes * 3
    # the same step recorded once in a graph and replayed (no Python or launch overhead)
    log("timing the 256^3 projection loss as a captured graph ...")
    graph, _ = RA.capture_projection_step(X3, U3)
    ms_g = time_steps(graph.replay, 20, 3)
    out["projection_loss_256^3_f32"] = {"ms": round(ms, 4), "alg_bytes": alg, "GB/s": round(alg / ms / 1e6, 1),
                                        "hbm_frac": round(alg / ms / 1e6 / (HBM_PEAK / 1e9), 4),
                                        "graph_ms": round(ms_g, 4),
                                        "graph_hbm_frac": round(alg / ms_g / 1e6 / (HBM_PEAK / 1e9), 4)}
    del graph
    del X3, U3
    torch.cuda.empty_cache()
    # ---- 512 tensors, dims U{32..192}^3, ranks U{4..16}^3, p = 4, grouped launches
    count = 512
    dims, ranks = synth.batch_specs(count)
    sb = [rt.rtucker_sketch_sizes(d, r, 4, "rhkron") for d, r in zip(dims, ranks)]
    phis = synth.batch_phis(dims, sb)
    log("generating the 512-tensor batch ...")
    X32 = [torch.from_numpy(synth.batch_tensor(i, d, r).astype(np.float32)).to(dev)
           for i, (d, r) in enumerate(zip(dims, ranks))]
    php = [[torch.from_numpy(f).to(dev) for f in ph] for ph in phis]
    nel = sum(int(x.numel()) for x in X32)
    for tag, Xs in (("f32", X32), ("bf16", [rt.rtucker_convert(x, torch.bfloat16) for x in X32])):
        B = rt.Batch(Xs, ranks, 4, php)
        B.run()
        mt, spb = B.autotune()
        B.upload()
        log(f"timing the 512-tensor batch {tag} ...")
        ms = time_steps(B.launch, 10, 2)
        graph = B.capture()  # the same launches replayed from a captured graph
        ms_g = time_steps(graph.replay, 10, 2)
        esz = 4 if tag == "f32" else 2
        alg = 2 * nel * esz  # two reads of every tensor: the sketch pass and the first core contraction
        errs = [rt.rtucker_rel_error(X32[i], B.Gs[i], B.Us[i])[0] for i in range(0, count, 64)]
        out[f"batch512_{tag}"] = {"ms": round(ms, 4), "tensors_per_s": round(count / (ms / 1e3), 1),
                                  "alg_bytes": alg, "GB/s": round(alg / ms / 1e6, 1),
                                  "hbm_frac": round(alg / ms / 1e6 / (HBM_PEAK / 1e9), 4),
                                  "graph_ms": round(ms_g, 4),
                                  "graph_tensors_per_s": round(count / (ms_g / 1e3), 1),
                                  "graph_hbm_frac": round(alg / ms_g / 1e6 / (HBM_PEAK / 1e9), 4),
                                  "core_row_tile": mt, "sketch_slabs_per_wave": spb,
                                  "max_rel_err_sampled": max(errs)}
        del graph
        del B
    return out


if __name__ == "__main__":
    main()
