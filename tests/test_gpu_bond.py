"""GPU rows and gradient with respect to the patch bond states (Sec. 5 superposition, Sec. 6.3
outlook), through the C ABI, against the oracle on the same link fields.

* ggf_measure_bond_rows: the patch set, link values, G_SS and the antisymmetric part of R (the
  only part a gradient uses: the Woodbury factors Y are antisymmetric) against the oracle's
  contraction on a fresh inverse, float64 within 1e-9 (relative to the largest entry), float32
  within 2e-5;
* ggf_bond_gradient on the library's own energy and bond rows equals the oracle's definitional
  gradient over the same configurations (equal weights);
* the rows refuse s L^2 > 4096.
"""
import numpy as np
import pytest

import synth
from gpu_common import say
from oracle import bond as bd
from oracle import energy as en
from oracle.lattice import Lattice
from oracle.model import Ansatz

pytestmark = pytest.mark.gpu

CP = en.Couplings(t=0.7, mu=0.3, m=0.45, kb=-0.8, ke=1.3)
CPD = dict(t=CP.t, mu=CP.mu, m=CP.m, kb=CP.kb, ke=CP.ke)


def _context(spec, L, n_chains, precision, sweeps=2):
    from paper_2412_01737_amd.ggf import Context
    ctx = Context(0)
    tid = ctx.set_tensor_spec(spec)
    ctx.init_chains([L] * n_chains, tid, synth.SEED_CHAIN, init=1, precision=precision, refresh_every=256)
    ctx.sweep(sweeps)
    return ctx


@pytest.mark.parametrize("L,K,group,precision", [(4, 2, 2, 64), (8, 2, 2, 64), (4, 3, 3, 64), (4, 2, 2, 32)])
def test_bond_rows_against_oracle(L, K, group, precision):
    spec = synth.make_tensor(L, K=K, group=group)
    say(f"bond rows: L={L} K={K} Z{group} float{precision}")
    ctx = _context(spec, L, 3, precision)
    rows = ctx.measure_bond_rows(CPD)
    an = Ansatz(Lattice(L, L), spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k, spec.c)
    tol = 1e-9 if precision == 64 else 2e-5
    for c in range(3):
        links, _ = ctx.get_state(c)
        G = np.linalg.inv(an.assemble_M(links))
        S = an.S
        s = len(S)
        r = rows[c]
        assert int(r[0]) == s and int(r[1]) == L
        assert np.array_equal(r[2:2 + s].astype(int), S)
        for k in range(1, K):
            assert int(r[14 + k]) == links[int(an.patch_link[k])]
        gss = r[306:306 + 144].reshape(12, 12)[:s, :s]
        assert np.abs(gss - G[np.ix_(S, S)]).max() <= tol * max(1.0, np.abs(G).max())
        R = (r[18:18 + 288:2] + 1j * r[19:19 + 288:2]).reshape(12, 12)[:s, :s]
        Ro = bd.coefficient_contraction(an, links, CP, G)
        Ra, Roa = 0.5 * (R - R.T), 0.5 * (Ro - Ro.T)
        err = np.abs(Ra - Roa).max() / max(1.0, np.abs(Roa).max())
        assert err <= tol, (c, err)
    ctx.close()


@pytest.mark.parametrize("K,group", [(2, 2), (3, 3)])
def test_bond_gradient_end_to_end(K, group):
    from paper_2412_01737_amd.ggf import bond_gradient
    L, n = 4, 6
    spec = synth.make_tensor(L, K=K, group=group)
    ctx = _context(spec, L, n, 64, sweeps=3)
    erows = ctx.measure_energy(CPD)
    brows = ctx.measure_bond_rows(CPD)
    g = bond_gradient(spec, CPD, erows, brows)
    an = Ansatz(Lattice(L, L), spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k, spec.c)
    configs = [ctx.get_state(c)[0] for c in range(n)]
    worst = 0.0
    for k in range(1, K):
        for gi, pair in enumerate(bd.bond_pairs()):
            E = bd.bond_generator(*pair)
            es, des, dns = zip(*[bd.bond_sensitivities(an, links, CP, k, E) for links in configs])
            ref = bd.bond_gradient_from_samples(es, des, dns)
            err = abs(g[k - 1, gi] - ref) / max(1.0, abs(ref))
            worst = max(worst, err)
            assert err <= 1e-8, (k, pair, g[k - 1, gi], ref)
    say(f"bond gradient K={K} Z{group}: {n} chains, worst relative error {worst:.1e}")
    ctx.close()


def test_bond_rows_refuse_large_patch_sets():
    from paper_2412_01737_amd.ggf import GGFError
    spec = synth.make_tensor(20, K=4, group=2)        # s = 12, L^2 = 400
    from paper_2412_01737_amd.ggf import Context
    ctx = Context(0)
    tid = ctx.set_tensor_spec(spec)
    ctx.init_chains([20], tid, synth.SEED_CHAIN, init=0, precision=64)
    with pytest.raises(GGFError):
        ctx.measure_bond_rows(CPD)
    ctx.close()


def test_set_bond_recomputes_cross_terms():
    """ggf_set_bond: S(G) of every chain and its energy rows follow the rotated bond, log W and G
    stay (the patch bonds do not enter M_00)."""
    L, K, group = 4, 3, 3
    spec = synth.make_tensor(L, K=K, group=group)
    ctx = _context(spec, L, 3, 64)
    before = [ctx.get_state(c)[1] for c in range(3)]
    G0 = ctx.get_inverse(0)
    E = bd.bond_generator(0, 2)
    new_bond = bd.rotated_bond(np.asarray(spec.gamma_bond_k[2]), E, 0.3)
    ctx.set_bond(0, 2, new_bond)
    gk = [np.array(g) for g in spec.gamma_bond_k]
    gk[2] = new_bond
    an = Ansatz(Lattice(L, L), spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, gk, spec.c)
    erows = ctx.measure_energy(CPD)
    for c in range(3):
        links, info = ctx.get_state(c)
        S = an.s_factor_def(links)
        assert abs(complex(info["s_re"], info["s_im"]) - S) <= 1e-10 * abs(S)
        assert info["logw"] == before[c]["logw"]
        assert abs(erows[c, 0] - en.local_energy(an, links, CP).real) <= 1e-9 * max(1.0, abs(erows[c, 0]))
    assert np.array_equal(ctx.get_inverse(0), G0)
    ctx.close()
