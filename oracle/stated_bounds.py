"""Stated BF16 / FP8 error bounds for the benchmark workloads (run on the CPU).

TEST INFRASTRUCTURE ONLY.  For each workload it prints the FP64 oracle's
relative error and the emulated-precision oracle's (``oracle.lowp``), with the
stated bound = emulated error x 1.1.  Inputs and Phi are the seeded synthetic
ones the GPU tests and the benchmark use.

    python -m oracle.stated_bounds            # all workloads (several minutes, ~25 GB of host memory)
"""
from __future__ import annotations

import sys

import numpy as np

import synth
from oracle import lowp as L
from oracle import tucker as T


def field_1024():
    dims, r, p = (1024, 1024, 512), [32, 32, 32], 8
    X = synth.bumps_field(dims, nbumps=200, noise_rel=1e-4, seed=synth.DATA_SEED).astype(np.float64)
    s = T.subranks_reuse([ri + p for ri in r])
    phis = synth.gaussians(synth.PHI_SEED, [(s[k], dims[k]) for k in range(3)])
    G, U = T.rhkron(X, r, phis)
    e64 = T.rel_error(X, G, U)
    Gb, Ub = L.rhkron_emulated(X, r, phis, "bf16", "bf16")
    eb = T.rel_error(X, Gb, Ub)
    G8, U8 = L.rhkron_emulated(X, r, phis, "f8e4m3", "bf16")
    e8 = T.rel_error(X, G8, U8)
    S = T.subrank_matrix_sth([ri + p for ri in r])
    shapes = T.sth_phi_shapes(dims, S)
    flat = synth.gaussians(synth.PHI_SEED, [sh for row in shapes for sh in row])
    sph = [flat[j * 3:(j + 1) * 3] for j in range(3)]
    Gs, Us = T.rsthkron(X, r, sph)
    es = T.rel_error(X, Gs, Us)
    Gsb, Usb = L.rsthkron_emulated(X, r, sph, "bf16")
    esb = T.rel_error(X, Gsb, Usb)
    return {"1024x1024x512 rHKron": (e64, eb, e8), "1024x1024x512 rSTHKron": (es, esb, None)}


def tensor_128():
    dims, r = (128, 128, 128, 128), [16, 16, 16, 16]
    core = synth.tucker_core_decay((16, 16, 16, 16), 6.0, seed=synth.DATA_SEED)
    X, _, _ = synth.random_tucker(dims, (16, 16, 16, 16), 1e-3, seed=synth.DATA_SEED, core=core)
    X = X.astype(np.float32).astype(np.float64)
    S = [[1 if k == j else 3 for k in range(4)] for j in range(4)]
    shapes = T.sth_phi_shapes(dims, S)
    flat = synth.gaussians(synth.PHI_SEED, [sh for row in shapes for sh in row])
    sph = [flat[j * 4:(j + 1) * 4] for j in range(4)]
    G, U = T.rsthkron(X, r, sph)
    Gb, Ub = L.rsthkron_emulated(X, r, sph, "bf16")
    return {"128^4 rSTHKron": (T.rel_error(X, G, U), T.rel_error(X, Gb, Ub), None)}


def batch_512(count=512):
    dims, ranks = synth.batch_specs(count)
    s = [T.subranks_reuse([ri + 4 for ri in rk]) for rk in ranks]
    phis = synth.batch_phis(dims, s)
    e64, eb = [], []
    for i in range(count):
        X = synth.batch_tensor(i, dims[i], ranks[i]).astype(np.float32).astype(np.float64)
        G, U = T.rhkron(X, list(ranks[i]), phis[i])
        e64.append(T.rel_error(X, G, U))
        Gb, Ub = L.rhkron_emulated(X, list(ranks[i]), phis[i], "bf16", "bf16")
        eb.append(T.rel_error(X, Gb, Ub))
    return {"512 tensors rHKron (max over items)": (max(e64), max(eb), None)}


def main():
    parts = sys.argv[1:] or ["field", "t128", "batch"]
    out = {}
    if "field" in parts:
        out.update(field_1024())
    if "t128" in parts:
        out.update(tensor_128())
    if "batch" in parts:
        out.update(batch_512())
    print("| workload | e_fp64 | e_bf16 (emulated) | BF16 bound | e_fp8-sketch (emulated) | FP8 bound |")
    print("|---|---|---|---|---|---|")
    for k, (e64, eb, e8) in out.items():
        f = lambda v: "—" if v is None else f"{v:.4e}"
        b = lambda v: "—" if v is None else f"{1.1 * v:.4e}"
        print(f"| {k} | {f(e64)} | {f(eb)} | {b(eb)} | {f(e8)} | {b(e8)} |", flush=True)


if __name__ == "__main__":
    main()
