"""Pins of the covariance-form oracle against a dense Fock-space contraction.

The Fock evaluator builds |A>, applies U(G) and contracts the bonds mode by
mode (Sec. 3, 3.1, 4); nothing in it uses a covariance formula, so every
agreement below pins the oracle's weights, cross terms and observables
(Sec. 3.2, 5, 5.1, 5.2) independently.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import gaussian
from oracle.fock import FockPEPS
from oracle.lattice import Lattice
from oracle.model import Ansatz, OBS_DENSITY, OBS_MESON0


def _pair(Lx, Ly, K=1, group=2, **kw):
    lat = Lattice(Lx, Ly)
    spec = synth.make_tensor(max(Lx, 2), K=K, group=group, **kw)
    if K > 1:
        # patch links must exist on this lattice
        links, gk = synth.patch_bonds(lat.n_links, K)
        spec.patch_link, spec.gamma_bond_k = links, gk
    an = Ansatz(lat, spec.gamma_loc, spec.gamma_bond, group, spec.patch_link,
                spec.gamma_bond_k, spec.c)
    fk = FockPEPS(lat, spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k)
    return lat, spec, an, fk


def test_local_state_reproduces_covariance():
    g = synth.local_gamma()
    v = gaussian.state_of_covariance(g, 5)
    assert np.abs(gaussian.covariance_of_state(v, 5) - g).max() < 1e-13
    # even parity: amplitudes only on even occupation numbers
    odd = [s for s in range(32) if bin(s).count("1") % 2]
    assert np.abs(v[odd]).max() < 1e-12


@pytest.mark.parametrize("Lx,Ly,group", [(1, 1, 2), (1, 1, 3), (2, 1, 2), (2, 1, 3), (2, 2, 2)])
def test_weight_all_configs_small(Lx, Ly, group):
    """W(G) = 2^-4V sqrt det M(G) equals <psi(G)|psi(G)> for every configuration."""
    lat, _, an, fk = _pair(Lx, Ly, group=group)
    pf_signs = set()
    for k in itertools.product(range(group), repeat=lat.n_links):
        k = np.array(k)
        wf = fk.weight(k)
        M = an.assemble_M(k)
        wc = an.weight(k)
        assert 0 <= wf <= 1
        assert abs(wc - wf) <= 1e-12 * wf
        pf = gaussian.pfaffian(M)
        assert abs(pf * pf - np.linalg.det(M)) <= 1e-10 * abs(pf * pf)
        assert abs(pf * 2.0 ** (-4 * lat.V) - wf) <= 1e-12 * wf
        pf_signs.add(np.sign(pf))
    assert pf_signs == {1.0}           # Pf(M(G)) never changes sign


def test_weight_z3_2x2_sample():
    lat, _, an, fk = _pair(2, 2, group=3)
    rng = np.random.default_rng(2)
    for _ in range(30):
        k = rng.integers(0, 3, lat.n_links)
        wf = fk.weight(k)
        assert abs(an.weight(k) - wf) <= 1e-12 * wf


def test_gauge_invariance_z2_2x2():
    """Flipping the four links of a site leaves W unchanged (Gauss law); 256 configs fall into 32 orbits."""
    lat, _, an, _ = _pair(2, 2)
    vals = {}
    for k in itertools.product(range(2), repeat=lat.n_links):
        k = np.array(k)
        w = an.weight(k)
        for x in range(lat.V):
            k2 = k.copy()
            for ell in lat.site_links(x):
                k2[ell] ^= 1
            assert abs(an.weight(k2) - w) <= 1e-13 * w
        vals[tuple(k)] = w
    distinct = set(np.round(np.array(list(vals.values())) / max(vals.values()), 10))
    assert len(distinct) <= 32


def test_physical_covariance_and_purity():
    lat, _, an, fk = _pair(2, 2)
    rng = np.random.default_rng(4)
    for _ in range(6):
        k = rng.integers(0, 2, lat.n_links)
        G = np.linalg.inv(an.assemble_M(k))
        go = an.gamma_out(G)
        assert np.abs(go - fk.covariance_out(k)).max() < 1e-12
        assert np.abs(go @ go + np.eye(2 * lat.V)).max() < 1e-12
        n = np.array([(1 + go[2 * x, 2 * x + 1]) / 2 for x in range(lat.V)])
        assert np.all((n >= -1e-14) & (n <= 1 + 1e-14))


@pytest.mark.parametrize("K,group", [(2, 2), (3, 2), (2, 3), (3, 3)])
def test_cross_terms_against_fock(K, group):
    lat, spec, an, fk = _pair(2, 2, K=K, group=group)
    rng = np.random.default_rng(5 + K)
    for _ in range(3):
        k = rng.integers(0, group, lat.n_links)
        Nf = fk.cross_terms(k)
        Nc = an.cross_terms(k)
        assert np.abs(Nc - Nf).max() <= 1e-12 * np.abs(Nf).max()
        assert np.abs(Nc - Nc.conj().T).max() <= 1e-14 * np.abs(Nc).max()
        for n in range(K):
            for m in range(K):
                assert abs(Nc[n, m]) ** 2 <= Nc[n, n].real * Nc[m, m].real * (1 + 1e-12)
        N = an.norm(k)
        assert N >= 0
        psi_norm = np.real(np.conj(spec.c) @ Nf @ spec.c)
        assert abs(N - psi_norm) <= 1e-12 * psi_norm


@pytest.mark.parametrize("K", [2, 3, 4])
def test_patch_lemma_equals_full_pfaffians(K):
    lat, spec, an, _ = _pair(4, 4, K=K, group=3)
    rng = np.random.default_rng(K)
    for _ in range(2):
        k = rng.integers(0, 3, lat.n_links)
        G = np.linalg.inv(an.assemble_M(k))
        rp = an.cross_ratio_patch(G[np.ix_(an.S, an.S)], k)
        rd = an.cross_ratio_def(k)
        assert np.abs(rp - rd).max() < 1e-11 * np.abs(rd).max()


def test_superposition_closed_form_k2():
    """Footnote of Sec. 3.2: sqrt2 |b_0> - |vac pair> = psi_o^+ psi_i^+|0>, itself Gaussian.

    With b_1 = vacuum pair and c = (sqrt2, -1) the K = 2 norm N(G) equals the
    K = 1 weight of the lattice whose patch-link bond is the filled pair.
    """
    lat = Lattice(2, 2)
    g0 = synth.GAMMA_BOND0
    vac = gaussian.vacuum_covariance(2)
    ell = 5
    spec = synth.make_tensor(2)
    an2 = Ansatz(lat, spec.gamma_loc, g0, 2, np.array([-1, ell]), np.array([g0, vac]),
                 np.array([np.sqrt(2), -1.0]))
    assert abs(an2.bond_overlap(1, 0) - 1 / np.sqrt(2)) < 1e-14
    filled = -vac
    an1 = Ansatz(lat, spec.gamma_loc, g0, 2)
    rng = np.random.default_rng(9)
    for _ in range(6):
        k = rng.integers(0, 2, lat.n_links)
        # K = 1 weight with the filled pair on link ell: build M by hand from an1
        M = an1.assemble_M(k)
        u = lat.link_majoranas(ell)
        M[np.ix_(u, u)] += an1._rot_block(filled, k[ell]) - an1._rot_block(g0, k[ell])
        w_filled = 2.0 ** (-4 * lat.V) * np.sqrt(np.linalg.det(M))
        assert abs(an2.norm(k) - w_filled) <= 1e-12 * w_filled


def test_superposition_limits():
    lat, spec, an, _ = _pair(2, 2, K=3)
    k = np.array([0, 1, 1, 0, 1, 0, 0, 1])
    w = an.weight(k)
    an_k1 = Ansatz(lat, spec.gamma_loc, spec.gamma_bond, 2, spec.patch_link, spec.gamma_bond_k,
                   np.array([1.0, 0.0, 0.0]))
    assert abs(an_k1.norm(k) - w) <= 1e-13 * w
    # eps -> 0: every bond equals b_0, N -> |sum c|^2 W
    links, gk = synth.patch_bonds(lat.n_links, 3, eps=1e-9)
    an0 = Ansatz(lat, spec.gamma_loc, spec.gamma_bond, 2, links, gk, spec.c)
    assert abs(an0.norm(k) - abs(spec.c.sum()) ** 2 * w) <= 1e-7 * abs(spec.c.sum()) ** 2 * w


@pytest.mark.parametrize("K,group", [(1, 2), (2, 2), (3, 3)])
def test_fermionic_observables_against_fock(K, group):
    lat, spec, an, fk = _pair(2, 2, K=K, group=group)
    V = lat.V
    cs = gaussian.majorana_matrices(V)
    nops = gaussian.number_matrices(V)
    rng = np.random.default_rng(21)
    c = spec.c if K > 1 else None
    for _ in range(3):
        k = rng.integers(0, group, lat.n_links)
        obs = an.observables(k)
        dens = np.mean([fk.expect(k, nops[x], c).real for x in range(V)])
        assert abs(obs[OBS_DENSITY] - dens) < 1e-12
        tot = 0
        for x in range(V):
            y = lat.shift(x, 1, 0)
            line = np.exp(2j * np.pi * (k[lat.link(x, 0)] % group) / group)
            phx = (cs[2 * x] + 1j * cs[2 * x + 1]) / 2
            phy = (cs[2 * y] + 1j * cs[2 * y + 1]) / 2
            tot += 2 * line * fk.expect(k, phx.conj().T @ phy, c)
        assert abs(obs[OBS_MESON0] - (tot / V).real) < 1e-12
