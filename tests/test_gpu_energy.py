"""Local energy and the linear step for lambda on the GPU against the oracle (Sec. 2, 5.2, 5.3).

ggf_measure_energy returns per chain Re E_loc(G) and, per ordered pair (a, b) of
the superposition, rho_ab / S and rho_ab h_ab / S.  The oracle computes them from
the chain's link field alone: full Pfaffians for r_ab, a fresh float64 inverse
of each M_ab, Wick's theorem and the Pfaffian-lemma mixed occupation (itself
pinned against Fock-space sums).
"""
import numpy as np
import pytest

from gpu_common import ansatz_for, gpu_context, say, spec_for
from oracle import energy as en

pytestmark = pytest.mark.gpu

CP = dict(t=0.7, mu=0.3, m=0.45, kb=-0.8, ke=1.3)


def _oracle_row(an, links):
    cp = en.Couplings(**CP)
    rho, rh = en.pair_matrices(an, links, cp)
    S = np.conj(an.c) @ rho @ an.c
    e = (np.conj(an.c) @ rh @ an.c) / S
    return e, rho / S, rh / S


def _check(row, an, links, tol):
    K = an.K
    e, rs, rhs = _oracle_row(an, links)
    assert abs(row[0] - e.real) <= tol * max(1.0, abs(e)), (row[0], e)
    for p in range(K * K):
        i, j = divmod(p, K)
        g_rho = row[1 + 4 * p] + 1j * row[2 + 4 * p]
        g_rh = row[3 + 4 * p] + 1j * row[4 + 4 * p]
        assert abs(g_rho - rs[i, j]) <= tol * max(1.0, abs(rs[i, j])), (p, g_rho, rs[i, j])
        assert abs(g_rh - rhs[i, j]) <= tol * max(1.0, abs(rhs[i, j])), (p, g_rh, rhs[i, j])
    assert np.all(row[1 + 4 * K * K:] == 0.0)


@pytest.mark.parametrize("L,K,group,precision", [
    (2, 1, 2, 64), (4, 1, 3, 64), (6, 1, 2, 64), (4, 2, 2, 64), (4, 3, 3, 64), (2, 3, 2, 64), (6, 4, 2, 64),
    (6, 1, 2, 32),
])
def test_energy_rows(L, K, group, precision):
    say(f"energy L={L} K={K} Z{group} float{precision}")
    spec = spec_for(L, K, group)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * 2, init=1, precision=precision, refresh_every=16 if precision == 32 else 0)
    tol = 1e-10 if precision == 64 else 1e-5
    for _ in range(2):
        ctx.sweep(1)
        rows = ctx.measure_energy(CP)
        for c in range(2):
            _check(rows[c], an, ctx.get_state(c)[0], tol)
    ctx.close()


def test_energy_full_size_sampled():
    """4096 chains of 8x8 Z2 K=1 float64 in one launch; three chains checked, every row finite."""
    L, chains = 8, 4096
    say(f"energy full size L={L} chains={chains}")
    spec = spec_for(L, 1, 2)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * chains, init=1)
    ctx.sweep(1)
    rows = ctx.measure_energy(CP)
    assert np.all(np.isfinite(rows[:, 0]))
    for c in (0, 2961, chains - 1):
        _check(rows[c], an, ctx.get_state(c)[0], 1e-10)
    ctx.close()


def test_lambda_step_end_to_end():
    """Rows from GPU chains (K = 2, Z2, 4x4) over several sweeps: the library's step equals the
    oracle's linear method on matrices the oracle computes from the same link fields."""
    from paper_2412_01737_amd.ggf import lambda_step
    say("lambda step K=2")
    L, K, chains = 4, 2, 8
    spec = spec_for(L, K, 2)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * chains, init=1)
    rows, Hs, Ns = [], [], []
    for _ in range(3):
        ctx.sweep(1)
        r = ctx.measure_energy(CP)
        rows.append(r)
        for c in range(chains):
            _, rs, rhs = _oracle_row(an, ctx.get_state(c)[0])
            Hs.append(rhs)
            Ns.append(rs)
    e, lam = lambda_step(K, np.concatenate(rows))
    e0, lam0 = en.linear_method(np.mean(Hs, axis=0), np.mean(Ns, axis=0))
    assert abs(e - e0) <= 1e-9 * max(1.0, abs(e0))
    assert np.abs(lam - lam0).max() <= 1e-7 * np.abs(lam0).max()
    # the current lambda's estimate is never below the optimum over the same samples
    cur = np.concatenate(rows)[:, 0].mean()
    assert e <= cur + 1e-9
    ctx.close()


def test_set_lambda_recomputes_superposition():
    """After ggf_set_lambda, S(G) of every chain and its energy rows follow the new lambda."""
    import dataclasses
    say("set lambda K=3 Z3")
    L, K = 4, 3
    spec = spec_for(L, K, 3)
    ctx = gpu_context([spec], [L] * 3, init=1)
    ctx.sweep(1)
    c_new = np.array([0.8, -0.3 + 0.5j, 0.2 - 0.7j])
    ctx.set_lambda(0, c_new)
    an = ansatz_for(dataclasses.replace(spec, c=c_new), L)
    rows = ctx.measure_energy(CP)
    for c in range(3):
        links, info = ctx.get_state(c)
        S = an.s_factor_def(links)
        assert abs(info["s_re"] - S.real) <= 1e-10 * abs(S.real)
        _check(rows[c], an, links, 1e-10)
    ctx.close()


def test_optimise_lambda_rounds():
    """Three rounds of two sweeps on K = 3 Z3 chains: each round's optimum over its samples is not
    above the estimate with that round's lambda, and the chains end on the last lambda."""
    import dataclasses
    say("optimise lambda K=3 Z3")
    L, K, chains = 4, 3, 16
    spec = spec_for(L, K, 3)
    ctx = gpu_context([spec], [L] * chains, init=1)
    energies, e_opt, lam = ctx.optimise_lambda(0, CP, 3, 2, K)
    assert np.all(np.isfinite(energies)) and np.all(np.isfinite(e_opt))
    assert np.all(e_opt <= energies + 1e-9), (energies, e_opt)
    an = ansatz_for(dataclasses.replace(spec, c=lam), L)
    for c in range(0, chains, 5):
        links, info = ctx.get_state(c)
        S = an.s_factor_def(links)
        assert abs(info["s_re"] - S.real) <= 1e-10 * abs(S.real)
    ctx.close()


def test_energy_entry_points_reject_bad_input():
    """The variational entry points validate their arguments before any launch."""
    from paper_2412_01737_amd.ggf import Context, GGFError, GGF_EINVAL, GGF_ESTATE
    say("energy entry points: invalid input")
    ctx = Context(0)
    spec1, spec3 = spec_for(4, 1, 2), spec_for(2, 3, 2)
    t1 = ctx.set_tensor_spec(spec1)
    t3 = ctx.set_tensor_spec(spec3)
    with pytest.raises(GGFError) as e:
        ctx.measure_energy(CP)
    assert e.value.status == GGF_ESTATE
    ctx.init_chains([4, 2], [t1, t3], 1, init=1)
    with pytest.raises(GGFError) as e:
        ctx.measure_energy(dict(CP, t=float("nan")))
    assert e.value.status == GGF_EINVAL
    with pytest.raises(GGFError):
        ctx.set_lambda(t3 + 5, [1.0, 0.0, 0.0])
    with pytest.raises(GGFError):
        ctx.set_lambda(t3, [0.0, 0.0, 0.0])
    with pytest.raises(GGFError):
        ctx.set_lambda(t3, [1.0, float("inf"), 0.0])
    bad = spec1.gamma_loc.copy()
    bad[0, 1] += 0.1
    with pytest.raises(GGFError):
        ctx.set_gamma_loc(t1, bad)
    with pytest.raises(GGFError):
        ctx.optimise_lambda(t3, CP, 0, 1, 3)
    ctx.set_lambda(t1, [2.0])                    # K = 1: lambda only scales the state; no change
    rows = ctx.measure_energy(CP)
    assert np.all(np.isfinite(rows[:, 0]))
    ctx.close()
    big = Context(0)
    tb = big.set_tensor_spec(spec_for(18, 1, 2))
    big.init_chains([18], [tb], 1)
    assert np.all(np.isfinite(big.measure_sensitivity(CP)))   # K = 1: any L (up to 32)
    big.close()


def test_k3_full_size_sampled():
    """2048 chains of 16x16 Z2 K=3 in float32 with a float64 refresh every 64 flips (the shape
    of the K = 3 benchmark): electric slot and energy rows in one launch each, every chain
    finite, one chain checked against the oracle (float32 tolerance)."""
    from paper_2412_01737_amd.ggf import OBS_ELECTRIC as BIT
    from oracle.model import OBS_ELECTRIC
    L, K, chains = 16, 3, 2048
    say(f"electric + energy full size L={L} K={K} chains={chains}")
    spec = spec_for(L, K, 2)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * chains, init=1, precision=32, refresh_every=64)
    ctx.sweep(1)
    obs = ctx.measure(BIT)
    rows = ctx.measure_energy(CP)
    assert np.all(np.isfinite(obs[:, OBS_ELECTRIC])) and np.all(np.isfinite(rows[:, 0]))
    c = chains - 1
    links, _ = ctx.get_state(c)
    # reference with the oracle's patch-lemma cross ratios (pinned against full Pfaffians) and a
    # float64 inverse of every M_nm
    G = np.linalg.inv(an.assemble_M(links))
    rho = an.bond_overlaps() * an.cross_ratio_patch(G[np.ix_(an.S, an.S)], links)
    ginv = [[np.linalg.inv(an.assemble_M(links, n, m)) for m in range(K)] for n in range(K)]
    wts = np.conj(an.c)[:, None] * an.c[None, :] * rho
    ref = an.electric_mean(links, ginv, wts)
    assert abs(obs[c, OBS_ELECTRIC] - ref) < 1e-5, (obs[c, OBS_ELECTRIC], ref)
    cp = en.Couplings(**CP)
    rh = np.array([[rho[n, m] * en.pair_energy(an, links, ginv[n][m], n, m, cp) for m in range(K)]
                   for n in range(K)])
    S = np.conj(an.c) @ rho @ an.c
    e = (np.conj(an.c) @ rh @ an.c) / S
    assert abs(rows[c, 0] - e.real) <= 2e-5 * max(1.0, abs(e))
    for p in range(K * K):
        i, j = divmod(p, K)
        assert abs(rows[c, 1 + 4 * p] + 1j * rows[c, 2 + 4 * p] - rho[i, j] / S) <= 2e-5 * max(1.0, abs(rho[i, j] / S))
        assert abs(rows[c, 3 + 4 * p] + 1j * rows[c, 4 + 4 * p] - rh[i, j] / S) <= 2e-5 * max(1.0, abs(rh[i, j] / S))
    ctx.close()
