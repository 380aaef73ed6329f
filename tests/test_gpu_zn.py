"""Z_N gauge groups beyond Z2/Z3 on the GPU (N up to 64) against the oracle.

The proposal step is 1 + (x2 mod (N - 1)), identical to the Z2 and Z3 rules
for N = 2, 3.  The link fields stay bit-exact against the oracle's Woodbury
chain, and the observables (the electric field included), the energy rows and
the K = 1 sensitivities match it.
"""
import numpy as np
import pytest

from gpu_common import ansatz_for, gpu_context, oracle_chain, say, spec_for
from oracle import energy as en

pytestmark = pytest.mark.gpu

CP = dict(t=0.7, mu=0.3, m=0.45, kb=-0.8, ke=1.3)


@pytest.mark.parametrize("L,K,group", [(4, 1, 4), (4, 2, 5), (6, 1, 8), (4, 1, 64)])
def test_zn_chains_bit_exact(L, K, group):
    say(f"Z{group} chains L={L} K={K}")
    spec = spec_for(L, K, group)
    ctx = gpu_context([spec], [L] * 2, init=1)
    orc = [oracle_chain(spec, L, c, init=1)[1] for c in range(2)]
    an = ansatz_for(spec, L)
    for s in range(3):
        ctx.sweep(1)
        for c, oc in enumerate(orc):
            oc.sweep()
            links, info = ctx.get_state(c)
            assert np.array_equal(links, oc.k), (s, c)
            assert abs(info["logw"] - oc.logw) <= 1e-10 * abs(oc.logw)
    obs = ctx.measure()
    rows = ctx.measure_energy(CP)
    for c in range(2):
        links, _ = ctx.get_state(c)
        ref = an.observables(links)
        assert np.abs(obs[c] - ref).max() < 1e-10, (c, obs[c], ref)
        rho, rh = en.pair_matrices(an, links, en.Couplings(**CP))
        S = np.conj(an.c) @ rho @ an.c
        e = (np.conj(an.c) @ rh @ an.c) / S
        assert abs(rows[c, 0] - e.real) <= 1e-10 * max(1.0, abs(e))
    if K == 1:
        sens = ctx.measure_sensitivity(CP)
        for c in range(2):
            _, Se, SN = en.sensitivities(an, ctx.get_state(c)[0], en.Couplings(**CP))
            assert np.abs(sens[c, :100].reshape(10, 10) - Se.real).max() <= 1e-10 * max(1.0, np.abs(Se).max())
            assert np.abs(sens[c, 100:].reshape(10, 10) - SN).max() <= 1e-10 * max(1.0, np.abs(SN).max())
    ctx.close()
