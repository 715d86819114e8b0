"""The all-at-once sketch through the memoised dimension tree (Sec. 4.4) against the oracle:
every mode's sketch from one call (tree on) and from one call per mode (tree off), for
4-, 5- and 6-way tensors."""
import numpy as np
import pytest

from gpu_common import T, assert_entrywise, dev, host, pytestmark_skip, reuse_phis, rt, say, synth, torch

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(pytestmark_skip, reason="needs a GPU")]


@pytest.mark.parametrize("dims,s", [((9, 10, 11, 12), (2, 3, 2, 3)), ((5, 6, 7, 8, 36), (2, 2, 3, 2, 2)),
                                    ((16, 20, 24, 28, 32), (3, 2, 3, 2, 3))])
def test_tree_on_equals_one_mode_per_call(dims, s):
    say("tree on/off", dims, s)
    X = np.random.default_rng(70).standard_normal(dims)
    phis = reuse_phis(dims, s, seed=71)
    Xd = dev(X, torch.float32)
    Xr = X.astype(np.float32).astype(np.float64)
    pr = [p.astype(np.float32).astype(np.float64) for p in phis]
    pd = [dev(p) for p in phis]
    on = rt.rtucker_sketch(Xd, pd, s)
    for n in range(len(dims)):
        off = rt.rtucker_sketch(Xd, pd, s, modes=[n])[n]
        want = T.kron_sketch(Xr, pr, n)
        bound = T.kron_sketch(np.abs(Xr), [np.abs(p) for p in pr], n)
        assert_entrywise(host(on[n]), want, bound, 2e-5, f"tree on, mode {n}")
        assert_entrywise(host(off), want, bound, 2e-5, f"tree off, mode {n}")


