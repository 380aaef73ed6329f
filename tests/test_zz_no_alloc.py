"""ggf_measure_staged (the allocation-free host measurement) against ggf_measure with a host output.

Two calls in a row on one GPU, the second with fewer chains than the first (the
staging array keeps the first call's rows beyond the second's): every observable
slot bit-exact against the existing entry point, for the full mask and for the
electric-only kernel.  A context with more chains than the array holds is
refused with GGF_EINVAL.
"""
import ctypes

import numpy as np
import pytest

import synth
from gpu_common import say

pytestmark = pytest.mark.gpu


def _ctx(Ls, K, group, seed):
    from paper_2412_01737_amd.ggf import Context
    ctx = Context(0)
    tid = ctx.set_tensor_spec(synth.make_tensor(min(Ls), K=K, group=group))
    ctx.init_chains(np.asarray(Ls, np.int32), tid, seed, init=1, precision=64)
    return ctx


@pytest.mark.parametrize("mask", [15, 8])
def test_staged_measure_equals_measure(mask):
    say(f"staged measurement, mask {mask}: 96 chains, then 12 chains")
    big = _ctx([4, 6] * 48, 2, 3, 11)
    big.sweep(1)
    a = big.measure_staged(mask)
    b = big.measure(mask)
    assert a.shape == (96, 21) and np.array_equal(a, b)
    small = _ctx([4] * 12, 1, 2, 12)
    small.sweep(2)
    a2 = small.measure_staged(mask)
    b2 = small.measure(mask)
    assert a2.shape == (12, 21) and np.array_equal(a2, b2)
    assert np.array_equal(big.measure_staged(mask), b)       # the first context again, unchanged
    big.close()
    small.close()


def test_staged_measure_refuses_more_chains_than_the_array_holds():
    from paper_2412_01737_amd.ggf import GGF_EINVAL, GGF_STAGE_MAX_CHAINS, load
    ctx = _ctx([2] * (GGF_STAGE_MAX_CHAINS + 1), 1, 2, 13)
    out = np.zeros((GGF_STAGE_MAX_CHAINS + 1, 21))
    st = load().ggf_measure_staged(ctx.h, 15, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None)
    assert st == GGF_EINVAL
    assert b"at most" in load().ggf_last_error(ctx.h)
    ctx.close()
