"""GPU parity of the batched decomposition (grouped launches): every item
against the FP64 oracle (bfloat16: the emulated-precision oracle) run on the same Phi, for uneven shapes of the
many-small-tensors workload (dims U{32..192}^3, ranks U{4..16}^3, p = 4),
plus graph capture, the autotuner and argument validation."""
import numpy as np
import pytest

from gpu_common import assert_entrywise, dev, host, pytestmark_skip, rt, say, synth, torch
from oracle import lowp as LP
from oracle import tucker as T

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(pytestmark_skip, reason="needs a GPU")]

P_OVER = 4


def _batch(count, lo=32, hi=192, seed=synth.DATA_SEED, extra=()):
    dims, ranks = synth.batch_specs(count, lo, hi, 4, 16, seed=seed)
    dims = list(dims) + [e[0] for e in extra]
    ranks = list(ranks) + [e[1] for e in extra]
    s = [rt.rtucker_sketch_sizes(d, r, P_OVER, "rhkron") for d, r in zip(dims, ranks)]
    phis = synth.batch_phis(dims, s)
    Xs = [synth.batch_tensor(i, d, r, 1e-4, seed=seed) for i, (d, r) in enumerate(zip(dims, ranks))]
    return dims, ranks, s, phis, Xs


def _device_phis(phis):
    return [[dev(f) for f in ph] for ph in phis]


def capped_modes(r, s, Ys):
    """Modes whose sketch cannot determine r_n directions (Sec. 4.3 reuse sketch).

    The mode-n sketch X_(n) (kron_{k != n} Phi_k^T) of a tensor of Tucker rank r has
    rank at most q_n = prod_{k != n} min(r_k, s_k); with unbalanced ranks q_n can fall
    below r_n although prod s_k >= r_n + p.  Near-deficiency counts too: q_n is also
    capped by the number of singular values of the oracle's sketch above 1e-3 of the
    largest (ten times the 1e-4 noise of the workload).  Returns {n: q_n} for the
    modes with q_n < r_n; the columns of U_hat_n beyond q_n then span directions set
    by the noise, any of which a correct QR may return."""
    out = {}
    for n in range(3):
        q = int(np.prod([min(r[k], s[k]) for k in range(3) if k != n]))
        sv = np.linalg.svd(Ys[n], compute_uv=False)
        q = min(q, int(np.sum(sv > 1e-3 * sv[0])))
        if q < r[n]:
            out[n] = q
    return out


def check_item(Xseen, G, Us, r, s, phis, dtype):
    """One batch item against the oracle on the same Phi (the emulated-precision oracle
    for bfloat16).  Uncapped items: |e_gpu - e_oracle| <= 1e-5 (bfloat16: 3e-5).  Capped items: what the
    sketch determines, i.e. the projection onto range(U_n) of the leading q_n left singular
    vectors of the oracle's sketch, equal entry by entry to 1e-4, and the core equal to
    X x_k U_k^T for the device's own factors.  Returns True when the item was capped."""
    r = list(r)
    if dtype == "f32":
        Go, Uo, parts = T.rhkron(Xseen, r, phis, return_parts=True)
        Ys = [T.kron_sketch(Xseen, phis, n) for n in range(3)]
    else:
        Go, Uo, parts = LP.rhkron_emulated(Xseen, r, phis, "bf16", "bf16", return_parts=True)
        Ys = parts["Y"]
    for k in range(3):
        assert np.max(np.abs(Us[k].T @ Us[k] - np.eye(r[k]))) < 1e-10
    e_dev = T.rel_error(Xseen, G, Us)
    e_or = T.rel_error(Xseen, Go, Uo)
    assert np.isfinite(e_dev)
    cap = capped_modes(r, s, Ys)
    if not cap:
        # bfloat16: the columns of U_hat past the ranks follow the sketch's noise (here the
        # rounding of X to bfloat16, about 2e-3 of each entry), and their bfloat16 roundings
        # in the first core contraction enter e.  A relative change of the sketch of a few
        # binary32 units (the device accumulates it in binary32, the oracle in binary64)
        # moves e by up to about 1.2e-5 on items of this workload (emulated oracle, sketch
        # perturbed by 32 units of 2^-24), so e is determined to that level only.
        tol = 1e-5 if dtype == "f32" else 3e-5
        assert abs(e_dev - e_or) <= tol, (e_dev, e_or)
        return False
    for n, q in cap.items():
        Sd = np.linalg.svd(Ys[n], full_matrices=False)[0][:, :q]
        pd = Us[n] @ (Us[n].T @ Sd)
        po = Uo[n] @ (Uo[n].T @ Sd)
        assert np.max(np.abs(pd - po)) <= 1e-4, (n, q, np.max(np.abs(pd - po)))
    # the core is the projection of X on the device's factors (U_hat rounded to bfloat16 in
    # the first contraction of the bfloat16 path: two bfloat16 units of the entry scale)
    want = T.multi_ttm(Xseen, {k: Us[k].T for k in range(3)})
    bound = T.multi_ttm(np.abs(Xseen), {k: np.abs(Us[k]).T for k in range(3)})
    assert_entrywise(G, want, bound, 2e-5 if dtype == "f32" else 2.0 ** -7, "core of a capped item")
    return True


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batched_matches_oracle(dtype):
    # uneven sizes, including dims that are not multiples of 8 and a clipped sketch (I_k < prod s)
    dims, ranks, s, phis, Xs = _batch(10, 32, 96, extra=[((17, 40, 33), (4, 5, 6)), ((12, 100, 9), (4, 4, 4))])
    say("batched", dtype, len(Xs), "items")
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    Xd = [rt.rtucker_convert(dev(X, torch.float32), tdt) if dtype == "bf16" else dev(X, torch.float32) for X in Xs]
    B = rt.Batch(Xd, ranks, P_OVER, _device_phis(phis))
    Gs, Us = B.run()
    capped = 0
    for i, X in enumerate(Xs):
        Xseen = host(Xd[i])  # the values the device decomposed
        capped += check_item(Xseen, host(Gs[i]), [host(u) for u in Us[i]], ranks[i], s[i], phis[i], dtype)
    say(f"  {capped} of {len(Xs)} items capped")


def test_batched_equals_single_tensor_path():
    dims, ranks, s, phis, Xs = _batch(6, 40, 120, seed=7)
    Xd = [dev(X, torch.float32) for X in Xs]
    B = rt.Batch(Xd, ranks, P_OVER, _device_phis(phis))
    Gs, Us = B.run()
    for i in range(len(Xs)):
        G1, U1 = rt.rtucker_decompose(Xd[i], list(ranks[i]), P_OVER, [dev(f) for f in phis[i]], s=s[i])
        e_b, _ = rt.rtucker_rel_error(Xd[i], Gs[i], Us[i])
        e_s, _ = rt.rtucker_rel_error(Xd[i], G1, U1)
        assert abs(e_b - e_s) <= 1e-6


def test_batched_graph_replay_and_autotune():
    dims, ranks, s, phis, Xs = _batch(8, 32, 80, seed=11)
    Xd = [dev(X, torch.float32) for X in Xs]
    B = rt.Batch(Xd, ranks, P_OVER, _device_phis(phis))
    Gs, Us = B.run()
    ref_G = [host(g).copy() for g in Gs]
    ref_U = [[host(u).copy() for u in us] for us in Us]
    chosen, spb = B.autotune()
    assert chosen in (8, 16, 32) and spb in (1, 2, 4)
    assert B.tuning()[:2] == (chosen, spb)
    B.upload()
    g = B.capture()
    for rep in range(3):
        for t in Gs:
            t.fill_(float("nan"))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(Xs)):
            if chosen == 16:  # same tiling as the reference: bitwise equal
                assert np.array_equal(host(Gs[i]), ref_G[i])
            else:
                assert np.allclose(host(Gs[i]), ref_G[i], rtol=1e-4, atol=1e-6 * np.abs(ref_G[i]).max())
            for k in range(3):
                a, b = host(Us[i][k]), ref_U[i][k]
                assert np.linalg.norm(a @ a.T - b @ b.T, 2) < 1e-4


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batched_full_size_all_items(dtype):
    """The 512-tensor workload (dims U{32..192}^3, ranks U{4..16}^3, p = 4), every item
    against the oracle on the host: strict on every item whose sketches determine the
    ranks, the determined part on the rest."""
    count = 512
    dims, ranks = synth.batch_specs(count)
    s = [rt.rtucker_sketch_sizes(d, r, P_OVER, "rhkron") for d, r in zip(dims, ranks)]
    phis = synth.batch_phis(dims, s)
    say(f"batched full size {dtype}: generating", count, "tensors")
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    Xd = []
    for i, (d, r) in enumerate(zip(dims, ranks)):
        x = dev(synth.batch_tensor(i, d, r), torch.float32)
        Xd.append(rt.rtucker_convert(x, tdt) if dtype == "bf16" else x)
    B = rt.Batch(Xd, ranks, P_OVER, _device_phis(phis))
    Gs, Us = B.run()
    torch.cuda.synchronize()
    capped = []
    for i in range(count):
        if i % 64 == 0:
            say(f"  item {i}")
        if check_item(host(Xd[i]), host(Gs[i]), [host(u) for u in Us[i]], ranks[i], s[i], phis[i], dtype):
            capped.append(i)
    say(f"  {len(capped)} of {count} items capped: {capped}")


def test_batched_validation():
    X = torch.zeros((20, 300, 20), dtype=torch.float32, device="cuda:0")
    phis = [[dev(np.ones((2, 20))), dev(np.ones((2, 300))), dev(np.ones((2, 20)))]]
    with pytest.raises(rt.RtuckerError):
        rt.Batch([X], [(2, 2, 2)], 1, phis, s=[(2, 2, 2)]).run()  # a mode longer than 256
    X = torch.zeros((20, 30, 20), dtype=torch.float32, device="cuda:0")
    phis = [[dev(np.ones((9, 20))), dev(np.ones((2, 30))), dev(np.ones((2, 20)))]]
    with pytest.raises(rt.RtuckerError):
        rt.Batch([X], [(2, 2, 2)], 1, phis, s=[(9, 2, 2)]).run()  # subrank above 8
