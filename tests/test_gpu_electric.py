"""Electric-field observable on the GPU (Sec. 5.3) against the oracle.

Contexts whose chains all have K = 1 run the lean kernel (one 4x4 block of G per
link, rotated response table in LDS); any K > 1 chain selects the general one.
The general kernel evaluates, per link and pair (n, m) of the superposition, the mixed
occupation of the link's outgoing mode from the 4x4 block of M_nm^-1 (Woodbury
form for K > 1) and the bond's response matrix computed by the C ABI.  The
oracle reads the same quantity off a Pfaffian of the link's 8x8 patch matrix
at a finite phase angle (itself pinned against Fock-space sums), so the two
share only the input configuration.
"""
import numpy as np
import pytest

from gpu_common import ansatz_for, gpu_context, say, spec_for
from oracle.model import NOBS, OBS_ELECTRIC

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,K,group,precision", [
    (2, 1, 2, 64),     # 2x2: both links of a site end on the same neighbour pair
    (4, 1, 3, 64),
    (6, 1, 2, 64),
    (4, 2, 2, 64),
    (4, 3, 3, 64),
    (6, 4, 2, 64),
    (2, 3, 2, 64),     # patch links of every pair on a 2x2 lattice
    (6, 1, 2, 32),
])
def test_electric_slot(L, K, group, precision):
    say(f"electric L={L} K={K} Z{group} float{precision}")
    from paper_2412_01737_amd.ggf import OBS_ELECTRIC as BIT
    spec = spec_for(L, K, group)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * 2, init=1, precision=precision, refresh_every=16 if precision == 32 else 0)
    tol = 1e-10 if precision == 64 else 1e-6
    for _ in range(2):
        ctx.sweep(1)
        got = ctx.measure(BIT)
        for c in range(2):
            links, _ = ctx.get_state(c)
            ref = an.observables(links)[OBS_ELECTRIC]
            assert abs(got[c, OBS_ELECTRIC] - ref) < tol, (c, got[c, OBS_ELECTRIC], ref)
            others = np.delete(got[c], OBS_ELECTRIC)
            assert np.all(others == 0.0)
    ctx.close()


def test_electric_full_size_sampled():
    """4096 chains of 8x8 Z2 (n = 512, float64) measured in one launch; three chains checked
    against the oracle, every chain finite."""
    from paper_2412_01737_amd.ggf import OBS_ELECTRIC as BIT
    L, chains = 8, 4096
    say(f"electric full size L={L} chains={chains}")
    spec = spec_for(L, 1, 2)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * chains, init=1)
    ctx.sweep(1)
    got = ctx.measure(BIT)
    assert got.shape == (chains, NOBS)
    assert np.all(np.isfinite(got[:, OBS_ELECTRIC]))
    for c in (0, 1723, chains - 1):
        links, _ = ctx.get_state(c)
        ref = an.observables(links)[OBS_ELECTRIC]
        assert abs(got[c, OBS_ELECTRIC] - ref) < 1e-10, (c, got[c, OBS_ELECTRIC], ref)
    ctx.close()


def test_electric_mixed_batch():
    """One context with K = 1 and K = 3 chains of different L (general kernel for all of them)."""
    from paper_2412_01737_amd.ggf import OBS_ELECTRIC as BIT
    say("electric mixed batch")
    specs = [spec_for(2, 1, 2), spec_for(2, 3, 2)]
    Ls, tids = [4, 2, 6, 4], [0, 1, 0, 1]
    ctx = gpu_context(specs, Ls, tensor_ids=tids, init=1)
    ctx.sweep(1)
    got = ctx.measure(BIT)
    for c, (L, t) in enumerate(zip(Ls, tids)):
        links, _ = ctx.get_state(c)
        ref = ansatz_for(specs[t], L).observables(links)[OBS_ELECTRIC]
        assert abs(got[c, OBS_ELECTRIC] - ref) < 1e-10, (c, got[c, OBS_ELECTRIC], ref)
    ctx.close()
