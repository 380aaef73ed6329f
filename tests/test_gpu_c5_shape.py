"""Sampled-chain parity at the shape of the 32x32 K=2 learned-proposal workload (256 chains, n = 8192).

The HIP path's hot start, one learned block sweep (64 Metropolis-Hastings
moves per chain on 4x4-site patches, rank-4m Woodbury updates) and the
observables, for chains 0 and 255 of the 256-chain launch, against results the
oracle stored from fresh factorisations (``tests/golden/make_c5.py``):

* float64: link fields after the start and after the sweep bit-exact, the
  proposed and accepted moves, log W within 1e-10 relative, every observable
  slot within 1e-9;
* float32 inverse with a float64 refactorisation every 4096 changed links (the
  benchmark's setting): the same link fields (a decision may differ only at a
  float32-level near tie, which fails the test), every observable slot within
  1e-6 of the oracle's float64 value (relative to max(1, |value|)).
"""
import importlib.util
import os

import numpy as np
import pytest

import synth
from gpu_common import gpu_context, say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden():
    spec = importlib.util.spec_from_file_location("make_c5", os.path.join(GOLDEN, "make_c5.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod, mod.load(os.path.join(GOLDEN, "c5_block_sweep.txt"))


@pytest.mark.parametrize("precision,refresh", [(64, 0), (32, 4096)])
def test_c5_shape_sampled_chains(precision, refresh):
    mod, ref = _golden()
    say(f"32x32 K=2, 256 chains, float{precision}: hot start, one block sweep, sampled chains {sorted(ref)}")
    spec = synth.make_tensor(mod.L, K=mod.K)
    ctx = gpu_context([spec], [mod.L] * 256, init=1, precision=precision, refresh_every=refresh)
    for c, r in ref.items():
        assert np.array_equal(ctx.get_state(c)[0], r["start"]), c
    ctx.nn_init(mod.P, 21)
    ctx.nn_params(mod.params())
    before = {c: ctx.block_stats(c) for c in ref}
    ctx.block_sweep(1)
    obs = ctx.measure()
    for c, r in ref.items():
        links, info = ctx.get_state(c)
        assert np.array_equal(links, r["after"]), f"chain {c}: link field differs after the block sweep"
        st = ctx.block_stats(c)
        assert st[0] - before[c][0] == r["proposed"] and st[1] - before[c][1] == r["accepted"], c
        err = np.abs(obs[c] - r["obs"]) / np.maximum(1.0, np.abs(r["obs"]))
        say(f"chain {c}: {r['accepted']}/{r['proposed']} moves accepted, log W {info['logw']:.12g} "
            f"(oracle {r['logw']:.12g}), worst observable error {err.max():.2e} (slot {int(err.argmax())})")
        if precision == 64:
            assert abs(info["logw"] - r["logw"]) <= 1e-10 * abs(r["logw"])
            assert err.max() < 1e-9
        else:
            assert abs(info["logw"] - r["logw"]) <= 1e-6 * abs(r["logw"])
            assert err.max() < 1e-6
    ctx.close()
