"""The autotuner times the launch shapes of the path that runs and leaves the chains' decisions unchanged.

With delayed updates it tunes the window flush (grid, window length); the
candidate sweeps are real Metropolis sweeps, so after tuning every chain must
still match the oracle chain that ran the same number of sweeps.  A second
context with the same workload key takes the choice from the cache file.
"""
import os

import numpy as np
import pytest

from gpu_common import gpu_context, oracle_chain, say, spec_for

pytestmark = pytest.mark.gpu


def test_autotune_flush_path_keeps_decisions_and_caches(tmp_path):
    L, chains = 6, 3
    spec = spec_for(L, K=2)
    cache = os.path.join(str(tmp_path), "tune.txt")
    ctx = gpu_context([spec], [L] * chains, init=1)
    grid, window, third = ctx.autotune(1, cache)
    say(f"autotune: flush grid {grid}, window {window}")
    assert grid in (512, 1024, 2048) and window in (8, 16, 32) and third == 0
    ctx.sweep(2)
    tuned_sweeps = 9 + 2
    for c in range(chains):
        oc = oracle_chain(spec, L, c, init=1)[1]
        for _ in range(tuned_sweeps):
            oc.sweep()
        links, info = ctx.get_state(c)
        assert info["sweeps"] == tuned_sweeps
        assert np.array_equal(links, oc.k), c
        assert abs(info["logw"] - oc.logw) <= 1e-10 * abs(oc.logw)
    lines = open(cache).read().split()
    assert lines[0].startswith("flush_n288_p64_K2_c3") and [int(v) for v in lines[1:4]] == [grid, window, 0]
    ctx.close()
    ctx2 = gpu_context([spec], [L] * chains, init=1)
    assert ctx2.autotune(1, cache) == (grid, window, 0)
    assert ctx2.get_state(0)[1]["sweeps"] == 0           # the cached choice ran no sweeps
    ctx2.close()
