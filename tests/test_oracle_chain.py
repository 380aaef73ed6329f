"""Pins of the oracle's Metropolis chains (Sec. 5.1) and statistics.

* the Woodbury chain and the definitional chain make identical accept/reject
  decisions on shared Philox streams (Z2/Z3, K = 1, 2, cold/hot starts);
* Woodbury-maintained inverses equal fresh inverses after many updates;
* a long chain on 2x2 reproduces exhaustive enumeration of all 256 configs;
* tau_int of an AR(1) series matches its closed form.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import stats
from oracle.chain import DefinitionChain, WoodburyChain, hot_links
from oracle.lattice import Lattice
from oracle.model import Ansatz


def _ansatz(L, K=1, group=2):
    lat = Lattice(L, L)
    spec = synth.make_tensor(L, K=K, group=group)
    return Ansatz(lat, spec.gamma_loc, spec.gamma_bond, group, spec.patch_link,
                  spec.gamma_bond_k, spec.c)


@pytest.mark.parametrize("L,K,group,hot", [(2, 1, 2, False), (4, 1, 2, True), (4, 1, 3, False),
                                           (2, 2, 2, True), (2, 3, 3, False)])
def test_woodbury_and_definition_decide_alike(L, K, group, hot):
    an = _ansatz(L, K, group)
    l0 = hot_links(synth.SEED_CHAIN, 1, an.lat.n_links, group) if hot else None
    d = DefinitionChain(an, synth.SEED_CHAIN, 1, l0)
    w = WoodburyChain(an, synth.SEED_CHAIN, 1, l0, refresh_every=8)
    for _ in range(4):
        d.sweep()
        w.sweep()
        assert np.array_equal(d.k, w.k)
    assert abs(d.logn - w.logn) < 1e-10 * abs(d.logn)
    assert 0 < w.accepts <= 4 * an.lat.n_links


def test_woodbury_inverse_drift():
    an = _ansatz(4, 1, 3)
    w = WoodburyChain(an, 9, 0, refresh_every=0)
    for _ in range(8):
        w.sweep()
    assert w.accepts >= 64
    G = np.linalg.inv(an.assemble_M(w.k))
    assert np.abs(w.G - G).max() < 1e-10 * np.abs(G).max()
    assert np.abs(w.G + w.G.T).max() < 1e-12 * np.abs(G).max()
    assert abs(w.logw - an.log_weight(w.k)) < 1e-10 * abs(w.logw)


def _exact_2x2(an):
    ws, obs = [], []
    for k in itertools.product(range(2), repeat=an.lat.n_links):
        k = np.array(k, np.int8)
        ws.append(an.weight(k))
        obs.append(an.observables(k)[:3])
    ws = np.array(ws)
    return (ws[:, None] * np.array(obs)).sum(0) / ws.sum()


@pytest.mark.slow
def test_long_chain_matches_enumeration():
    """1 chain x 10^4 sweeps on the 2x2 lattice vs exact averages over all 256 configs."""
    an = _ansatz(2)
    exact = _exact_2x2(an)
    w = WoodburyChain(an, synth.SEED_CHAIN, 0, refresh_every=1024)
    n_sweeps, burn = 10000, 1000
    series = np.zeros((n_sweeps, 3))
    for s in range(n_sweeps):
        w.sweep()
        go = an.gamma_out(w.G)
        series[s, 0] = an.plaquette(w.k)
        series[s, 1] = an.wilson2x2(w.k)
        series[s, 2] = an.density_from(go).real
    series = series[burn:]
    for j in range(3):
        tau, _, _ = stats.tau_int(series[:, j])
        err = np.std(series[:, j]) * np.sqrt(2 * tau / len(series))
        assert abs(series[:, j].mean() - exact[j]) < 4 * err + 1e-12


def test_tau_int_ar1_closed_form():
    """AR(1) x_t = phi x_{t-1} + e_t has tau_int = (1 + phi) / (2 (1 - phi))."""
    rng = np.random.default_rng(0)
    phi, n = 0.8, 200000
    e = rng.standard_normal(n)
    x = np.zeros(n)
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    tau, err, _ = stats.tau_int(x[:20000])
    assert abs(tau - (1 + phi) / (2 * (1 - phi))) < 4 * err
    assert stats.tau_int(rng.standard_normal(5000))[0] == pytest.approx(0.5, abs=0.1)


def test_synthetic_inputs():
    g = synth.local_gamma()
    assert np.abs(g + g.T).max() < 1e-15
    assert np.abs(g @ g + np.eye(10)).max() < 1e-13
    from oracle.gaussian import pfaffian
    assert pfaffian(g) == pytest.approx(-1.0)       # even parity on 5 modes: (-1)^5 Pf = +1
    links, gk = synth.patch_bonds(128, 3)
    assert links[0] == -1 and len(set(links[1:].tolist())) == 2
    for k in range(3):
        assert np.abs(gk[k] @ gk[k] + np.eye(4)).max() < 1e-13
        assert pfaffian(gk[k]) == pytest.approx(pfaffian(synth.GAMMA_BOND0))
    L, K, grp = synth.mixed_batch(64)
    assert set(L) <= set(synth.MIX_L) and set(K) <= set(synth.MIX_K) and set(grp) <= {2, 3}


def test_proposal_rule_table():
    """Z_N moves k -> k + step (mod N) with step = 1 + (x2 mod (N - 1)) from the chain's Philox
    block: Z2 flips, Z3 steps by 1 + (x2 & 1), and the step is uniform over the N - 1 other
    elements (a symmetric proposal)."""
    from oracle.chain import propose
    from oracle import philox
    assert [propose(k, 1, 2) for k in (0, 1)] == [1, 0]
    assert [propose(k, s, 3) for k in (0, 1, 2) for s in (1, 2)] == [1, 2, 2, 0, 0, 1]
    x = philox.philox4x32_10((2, 5, 11, 0), (synth.SEED_CHAIN, 0))
    _, step = philox.draw(synth.SEED_CHAIN, 2, 5, 11)
    assert int(step) == 1 + (x[2] & 1)
    _, step2 = philox.draw(synth.SEED_CHAIN, 2, 5, 11, 2)
    assert int(step2) == 1
    _, s5 = philox.draw(synth.SEED_CHAIN, np.arange(8000), 3, 7, 5)
    counts = np.bincount(s5, minlength=6)
    assert counts[0] == 0 and counts[5] == 0
    assert np.all(np.abs(counts[1:5] - 2000) < 200)


def _golden(name):
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_t14", os.path.join(here, "make_t14.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.load(os.path.join(here, name))


def test_t14_c1_stored_sequence_reproduced_by_the_woodbury_chain():
    """The stored 10^4-sweep 2x2 decision sequence (fresh determinants) is reproduced sweep by sweep by
    the oracle's independent Woodbury route (rank-4 updates of the maintained inverse)."""
    ref = _golden("t14_c1.txt")[0]
    codes = "".join(ref["lines"])
    spec = synth.make_tensor(2)
    an = Ansatz(Lattice(2, 2), spec.gamma_loc, spec.gamma_bond, 2)
    ch = WoodburyChain(an, synth.SEED_CHAIN, 0, refresh_every=1024)
    for s in range(len(codes) // 2):
        ch.sweep()
        assert "%02x" % int(sum(int(v) << i for i, v in enumerate(ch.k))) == codes[2 * s:2 * s + 2], s
    assert ch.accepts == ref["accepts"] and ch.ties == ref["near_ties"] == 0
    assert abs(ch.logw - ref["logw"]) < 1e-11 * abs(ref["logw"])
