"""Gradient of <H> with respect to the on-site covariance on the GPU against the oracle.

ggf_measure_sensitivity returns per chain S_e (real part) and S_N with
d Re e(G) = tr(Delta S_e) and d log N(G) = tr(Delta S_N) for Delta = [E, Gamma_A].
The oracle builds them with dense NumPy products of a fresh float64 inverse and
reads the electric slopes off its own mixed occupation; its sensitivities are
pinned against finite differences and its gradient against the exactly
enumerated <H> (tests/test_oracle_energy.py).  For K > 1 the library forms each
pair's M_ab^-1 explicitly and combines the pair terms with the weights and
h_ab of the chain's energy row; the oracle inverts M_ab densely per pair.
"""
import dataclasses

import numpy as np
import pytest

import synth
from gpu_common import ansatz_for, gpu_context, say, spec_for
from oracle import energy as en

pytestmark = pytest.mark.gpu

CP = dict(t=0.7, mu=0.3, m=0.45, kb=-0.8, ke=1.3)


def _check_sens(row, an, links, tol):
    _, Se, SN = en.sensitivities(an, links, en.Couplings(**CP))
    got_e = row[:100].reshape(10, 10)
    got_n = row[100:].reshape(10, 10)
    scale = max(1.0, np.abs(Se.real).max())
    assert np.abs(got_e - Se.real).max() <= tol * scale, np.abs(got_e - Se.real).max()
    assert np.abs(got_n - SN.real).max() <= tol * max(1.0, np.abs(SN).max())
    assert np.abs(np.imag(SN)).max() <= 1e-9 * max(1.0, np.abs(SN).max())   # d log N is real


@pytest.mark.parametrize("L,group,precision", [(2, 2, 64), (4, 3, 64), (6, 2, 64), (4, 2, 32)])
def test_sensitivity_rows(L, group, precision):
    say(f"sensitivities L={L} Z{group} float{precision}")
    spec = spec_for(L, 1, group)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * 2, init=1, precision=precision, refresh_every=16 if precision == 32 else 0)
    ctx.sweep(1)
    rows = ctx.measure_sensitivity(CP)
    tol = 1e-10 if precision == 64 else 2e-5
    for c in range(2):
        _check_sens(rows[c], an, ctx.get_state(c)[0], tol)
    ctx.close()


@pytest.mark.parametrize("L,group", [(10, 2), (12, 3)])
def test_sensitivity_rows_large(L, group):
    """V = 100 (the largest lattice of the two-stage kernel, whose stripe and T_z fill its LDS) and
    V = 144 (the one-stage kernel with rows read from global memory)."""
    say(f"sensitivities L={L} Z{group} float64")
    spec = spec_for(L, 1, group)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * 2, init=1)
    ctx.sweep(1)
    rows = ctx.measure_sensitivity(CP)
    for c in range(2):
        _check_sens(rows[c], an, ctx.get_state(c)[0], 1e-10)
    ctx.close()


@pytest.mark.parametrize("L", [24, 32])
def test_sensitivity_rows_chunked(L):
    """Lattices above the one-chunk size: U_z formed on chunks of lattice rows (L = 24: rows 0-16 and
    17-23; L = 32: 0-12, 13-25, 26-31) with the next row as halo; one chain against the oracle."""
    say(f"sensitivities L={L} Z2 float64, row chunks")
    spec = spec_for(L, 1, 2)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L], init=1)
    ctx.sweep(1)
    rows = ctx.measure_sensitivity(CP)
    assert np.all(np.isfinite(rows))
    assert np.array_equal(ctx.measure_sensitivity(CP), rows)     # fixed summation order: reproducible
    _check_sens(rows[0], an, ctx.get_state(0)[0], 1e-10)
    ctx.close()


def test_sensitivity_full_size_sampled():
    """4096 chains of 8x8 Z2 (float64) in one launch; two chains checked, every row finite."""
    L, chains = 8, 4096
    say(f"sensitivities full size L={L} chains={chains}")
    spec = spec_for(L, 1, 2)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * chains, init=1)
    ctx.sweep(1)
    rows = ctx.measure_sensitivity(CP)
    assert np.all(np.isfinite(rows))
    for c in (0, chains - 1):
        _check_sens(rows[c], an, ctx.get_state(c)[0], 1e-10)
    ctx.close()


def test_gradient_end_to_end_and_update():
    """GPU rows -> library gradient = oracle gradient from oracle sensitivities of the same link
    fields; then a step exp(-eta g) on Gamma_A through ggf_set_gamma_loc refactorises the chains
    to the oracle's log W of the new tensor."""
    from paper_2412_01737_amd.ggf import gamma_gradient
    say("gradient end to end L=4 Z2")
    L, chains = 4, 6
    spec = spec_for(L, 1, 2)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * chains, init=1)
    ctx.sweep(2)
    er = ctx.measure_energy(CP)
    sr = ctx.measure_sensitivity(CP)
    g = gamma_gradient(spec.gamma_loc, er, sr)
    es, Ses, SNs = [], [], []
    for c in range(chains):
        e, Se, SN = en.sensitivities(an, ctx.get_state(c)[0], en.Couplings(**CP))
        es.append(e.real)
        Ses.append(Se.real)
        SNs.append(SN)
    ref = en.gradient_from_samples(spec.gamma_loc, es, Ses, SNs)
    assert np.abs(g - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
    new = en.rotated_gamma_loc(spec.gamma_loc, -0.05 * g / max(1e-12, np.abs(g).max()))
    ctx.set_gamma_loc(0, new)
    an2 = ansatz_for(dataclasses.replace(spec, gamma_loc=new), L)
    for c in range(chains):
        links, info = ctx.get_state(c)
        lw = an2.log_weight(links)
        assert abs(info["logw"] - lw) <= 1e-10 * abs(lw)
    rows = ctx.measure_energy(CP)
    for c in range(chains):
        e = en.local_energy(an2, ctx.get_state(c)[0], en.Couplings(**CP))
        assert abs(rows[c, 0] - e.real) <= 1e-10 * max(1.0, abs(e))
    ctx.close()


def test_optimise_gamma_round():
    """One round of ggf_optimise_gamma (one sweep): the returned Gamma_A is the oracle's
    exp(-eta g) Gamma_A exp(eta g) for the gradient the oracle computes on the same link fields,
    and the chains are refactorised to it.  Then a second call runs two more rounds."""
    say("optimise gamma L=4 Z2")
    L, chains, eta = 4, 8, 0.02
    spec = spec_for(L, 1, 2)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * chains, init=1)
    energies, gnorm, g_new = ctx.optimise_gamma(0, CP, 1, 1, eta)
    es, Ses, SNs = [], [], []
    for c in range(chains):
        e, Se, SN = en.sensitivities(an, ctx.get_state(c)[0], en.Couplings(**CP))
        es.append(e.real)
        Ses.append(Se.real)
        SNs.append(SN)
    g = en.gradient_from_samples(spec.gamma_loc, es, Ses, SNs)
    assert abs(energies[0] - np.mean(es)) <= 1e-10 * max(1.0, abs(np.mean(es)))
    assert abs(gnorm[0] - np.abs(g).max()) <= 1e-9 * max(1.0, np.abs(g).max())
    expect = en.rotated_gamma_loc(spec.gamma_loc, -eta * g)
    assert np.abs(g_new - expect).max() < 1e-10
    assert np.abs(g_new @ g_new + np.eye(10)).max() < 1e-10
    an2 = ansatz_for(dataclasses.replace(spec, gamma_loc=g_new), L)
    for c in range(chains):
        links, info = ctx.get_state(c)
        lw = an2.log_weight(links)
        assert abs(info["logw"] - lw) <= 1e-10 * abs(lw)
    energies2, gnorm2, _ = ctx.optimise_gamma(0, CP, 2, 1, eta)
    assert np.all(np.isfinite(energies2)) and np.all(np.isfinite(gnorm2))
    ctx.close()


@pytest.mark.parametrize("L,K,group,precision", [(4, 2, 2, 64), (4, 3, 3, 64), (2, 2, 2, 64), (6, 2, 2, 64),
                                                 (4, 2, 2, 32)])
def test_sensitivity_rows_pairs(L, K, group, precision):
    """K > 1: per pair (a, b) the K = 1 sensitivities with the complex M_ab^-1 and the pair's
    electric slopes, weighted by om_ab / S with (h_ab - E) on the log-norm part."""
    say(f"sensitivities K={K} L={L} Z{group} float{precision}")
    spec = spec_for(L, K, group)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * 3, init=1, precision=precision, refresh_every=16 if precision == 32 else 0)
    ctx.sweep(1)
    rows = ctx.measure_sensitivity(CP)
    tol = 1e-10 if precision == 64 else 2e-5
    for c in range(3):
        _check_sens(rows[c], an, ctx.get_state(c)[0], tol)
    ctx.close()


@pytest.mark.parametrize("L,K,group,precision", [(10, 2, 2, 64), (12, 2, 3, 64), (10, 3, 3, 64), (10, 2, 2, 32)])
def test_sensitivity_rows_pairs_large(L, K, group, precision):
    """K > 1 with n > 512: M_ab^-1 = G + (G_S Y_ab) G_S^T applied as a rank <= 8 correction of G,
    the electric part through its expansion, the d-block in chunks of lattice rows."""
    say(f"sensitivities K={K} L={L} Z{group} float{precision}, correction tables")
    spec = spec_for(L, K, group)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * 2, init=1, precision=precision, refresh_every=16 if precision == 32 else 0)
    ctx.sweep(1)
    rows = ctx.measure_sensitivity(CP)
    assert np.all(np.isfinite(rows))
    assert np.array_equal(ctx.measure_sensitivity(CP), rows)     # fixed summation order: reproducible
    _check_sens(rows[1], an, ctx.get_state(1)[0], 1e-10 if precision == 64 else 2e-5)
    ctx.close()


def test_sensitivity_rows_pairs_full_size_reduce_to_k1():
    """32x32 (n = 8192, six row chunks of the correction-table kernel): a K = 2 ansatz whose second
    amplitude is zero is the K = 1 ansatz of its reference bond.  Its rows, formed pair by pair through the
    correction tables in complex arithmetic, equal those of the real K = 1 kernel, a separate code path,
    on the same hot-start configuration, at a size the oracle does not reach."""
    L = 32
    say(f"sensitivities K=2 with lambda_1 = 0 against K=1, L={L} Z2 float64")
    s2 = dataclasses.replace(spec_for(L, 2, 2), c=np.array([1.0, 0.0], complex))
    s1 = dataclasses.replace(s2, K=1, patch_link=np.array([-1], np.int32), gamma_bond_k=np.zeros((1, 4, 4)),
                             c=np.ones(1, complex))
    ctx2 = gpu_context([s2], [L], init=1)
    ctx1 = gpu_context([s1], [L], init=1)
    assert np.array_equal(ctx2.get_state(0)[0], ctx1.get_state(0)[0])
    r2 = ctx2.measure_sensitivity(CP)
    r1 = ctx1.measure_sensitivity(CP)
    assert np.all(np.isfinite(r2))
    assert np.abs(r2 - r1).max() <= 1e-9 * max(1.0, np.abs(r1).max()), np.abs(r2 - r1).max()
    ctx2.close()
    ctx1.close()


def test_sensitivity_rows_pairs_large_mixed():
    """A K = 1 chain at L = 10 beside a K = 2 chain at L = 8 (n = 512 below the context's largest
    n = 800): both through the correction tables, each to its oracle."""
    say("sensitivities mixed K=1 L=10 / K=2 L=8 Z2, correction tables")
    specs = [spec_for(10, 1, 2), spec_for(8, 2, 2)]
    ctx = gpu_context(specs, [10, 8], init=1, tensor_ids=[0, 1])
    ctx.sweep(1)
    rows = ctx.measure_sensitivity(CP)
    for c, (t, L) in enumerate([(0, 10), (1, 8)]):
        _check_sens(rows[c], ansatz_for(specs[t], L), ctx.get_state(c)[0], 1e-10)
    ctx.close()


def test_sensitivity_rows_mixed_k():
    """K = 1 and K = 2 chains in one context: both go through the pair path, each to its oracle."""
    say("sensitivities mixed K=1 / K=2 L=4 Z2")
    specs = [spec_for(4, 1, 2), spec_for(4, 2, 2)]
    ctx = gpu_context(specs, [4, 4, 4], init=1, tensor_ids=[0, 1, 1])
    ctx.sweep(1)
    rows = ctx.measure_sensitivity(CP)
    for c, t in enumerate([0, 1, 1]):
        _check_sens(rows[c], ansatz_for(specs[t], 4), ctx.get_state(c)[0], 1e-10)
    ctx.close()


def test_gradient_pairs_end_to_end():
    """K = 2: GPU energy and sensitivity rows -> library gradient = oracle gradient from the oracle's
    K > 1 sensitivities of the same link fields."""
    from paper_2412_01737_amd.ggf import gamma_gradient
    say("gradient end to end K=2 L=4 Z2")
    L, chains = 4, 6
    spec = spec_for(L, 2, 2)
    an = ansatz_for(spec, L)
    ctx = gpu_context([spec], [L] * chains, init=1)
    ctx.sweep(2)
    er = ctx.measure_energy(CP)
    sr = ctx.measure_sensitivity(CP)
    g = gamma_gradient(spec.gamma_loc, er, sr)
    es, Ses, SNs = [], [], []
    for c in range(chains):
        e, Se, SN = en.sensitivities(an, ctx.get_state(c)[0], en.Couplings(**CP))
        assert abs(er[c, 0] - e.real) <= 1e-10 * max(1.0, abs(e))
        es.append(e.real)
        Ses.append(Se.real)
        SNs.append(SN.real)
    ref = en.gradient_from_samples(spec.gamma_loc, es, Ses, SNs)
    assert np.abs(g - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
    ctx.close()
