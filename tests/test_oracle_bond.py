"""Pins of the oracle's gradient with respect to the patch bond states (Sec. 5 superposition,
Sec. 6.3 outlook: gradient descent on the variational parameters).

* the bond state's derivative against central differences of the state built from the rotated
  covariance (with the phase convention <b_0|b_k> > 0);
* per configuration, d e(G) and d log N(G) against central differences of the definitional
  E_loc(G) and log N(G) of the ansatz with the rotated bond (2x2 lattice; Z2 K = 2, Z3 K = 3;
  several generators; every coupling nonzero);
* a generator commuting with the bond covariance changes nothing;
* the route from G = M_00^-1 alone (G_SS and the coefficient contraction R) equals the
  definitional route;
* the p(G)-weighted gradient over every configuration of a 2x1 lattice against central
  differences of the exactly enumerated <H>(theta).
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import bond as bd
from oracle import energy as en
from oracle.lattice import Lattice
from oracle.model import Ansatz

CP = en.Couplings(t=0.7, mu=0.3, m=0.45, kb=-0.8, ke=1.3)


def _spec(lat, K, group):
    spec = synth.make_tensor(max(lat.Lx, 2), K=K, group=group)
    links, gk = synth.patch_bonds(lat.n_links, K)
    spec.patch_link, spec.gamma_bond_k = links, gk
    return spec


def _ansatz(lat, spec, gk=None):
    return Ansatz(lat, spec.gamma_loc, spec.gamma_bond, spec.group, spec.patch_link,
                  spec.gamma_bond_k if gk is None else gk, spec.c)


def _rotated(spec, k, E, theta):
    gk = [None if g is None else np.array(g) for g in spec.gamma_bond_k]
    gk[k] = bd.rotated_bond(np.asarray(spec.gamma_bond_k[k]), E, theta)
    return gk


def _log_n(an, links):
    return an.log_weight(links) + np.log(an.s_factor_def(links).real)


@pytest.mark.parametrize("k,pair", [(1, (0, 1)), (1, (1, 3)), (1, (0, 2))])
def test_bond_state_derivative(k, pair):
    lat = Lattice(2, 2)
    spec = _spec(lat, 2, 2)
    E = bd.bond_generator(*pair)
    an = _ansatz(lat, spec)
    dv = bd.bond_state_derivative(an, k, E)
    h = 1e-6
    vp = _ansatz(lat, spec, _rotated(spec, k, E, h)).bstate[k]
    vm = _ansatz(lat, spec, _rotated(spec, k, E, -h)).bstate[k]
    fd = (vp - vm) / (2 * h)
    assert np.abs(dv - fd).max() < 1e-7, (dv, fd)


@pytest.mark.parametrize("K,group", [(2, 2), (3, 3)])
def test_sensitivities_against_finite_differences(K, group):
    lat = Lattice(2, 2)
    spec = _spec(lat, K, group)
    an = _ansatz(lat, spec)
    rng = np.random.default_rng(17)
    h = 1e-5
    for trial in range(3):
        links = synth.random_links(rng, lat.n_links, group)
        for k in range(1, K):
            for pair in [(0, 1), (0, 2), (1, 3), (2, 3)][trial::2]:
                E = bd.bond_generator(*pair)
                e, de, dlogN = bd.bond_sensitivities(an, links, CP, k, E)
                assert abs(e - en.local_energy(an, links, CP)) < 1e-12 * max(1.0, abs(e))
                ap = _ansatz(lat, spec, _rotated(spec, k, E, h))
                am = _ansatz(lat, spec, _rotated(spec, k, E, -h))
                fe = (en.local_energy(ap, links, CP) - en.local_energy(am, links, CP)) / (2 * h)
                fn = (_log_n(ap, links) - _log_n(am, links)) / (2 * h)
                assert abs(de - fe) <= 1e-7 * max(1.0, abs(fe)), (k, pair, de, fe)
                assert abs(dlogN - fn) <= 1e-7 * max(1.0, abs(fn)), (k, pair, dlogN, fn)


def test_generator_in_the_stabiliser_changes_nothing():
    lat = Lattice(2, 2)
    spec = _spec(lat, 2, 2)
    an = _ansatz(lat, spec)
    g1 = np.asarray(spec.gamma_bond_k[1])
    E = 0.5 * (g1 - g1.T)                      # commutes with the bond's covariance
    links = synth.random_links(np.random.default_rng(3), lat.n_links, 2)
    e, de, dlogN = bd.bond_sensitivities(an, links, CP, 1, E)
    assert abs(de) < 1e-12 and abs(dlogN) < 1e-12


@pytest.mark.parametrize("K,group", [(2, 2), (3, 3)])
def test_patch_route_equals_definition(K, group):
    lat = Lattice(2, 2)
    spec = _spec(lat, K, group)
    an = _ansatz(lat, spec)
    rng = np.random.default_rng(23)
    for trial in range(2):
        links = synth.random_links(rng, lat.n_links, group)
        G = np.linalg.inv(an.assemble_M(links))
        rho, rh = en.pair_matrices(an, links, CP)
        R = bd.coefficient_contraction(an, links, CP, G)
        for k in range(1, K):
            for pair in bd.bond_pairs():
                E = bd.bond_generator(*pair)
                d = bd.bond_sensitivities(an, links, CP, k, E)
                p = bd.bond_sensitivities_patch(an, links, CP, k, E, G, rh / rho, rho, R)
                for x, y in zip(d, p):
                    assert abs(x - y) <= 1e-10 * max(1.0, abs(x)), (k, pair, d, p)


def test_gradient_against_exact_energy():
    lat = Lattice(2, 1)
    spec = _spec(lat, 2, 2)

    def exact(gk):
        a = _ansatz(lat, spec, gk)
        num = den = 0.0
        for G in itertools.product(range(2), repeat=lat.n_links):
            k = np.array(G)
            Nk = a.norm(k)
            num += Nk * en.local_energy(a, k, CP)
            den += Nk
        return (num / den).real

    an = _ansatz(lat, spec)
    h = 1e-5
    for pair in bd.bond_pairs():
        E = bd.bond_generator(*pair)
        es, des, dns, ws = [], [], [], []
        for G in itertools.product(range(2), repeat=lat.n_links):
            k = np.array(G)
            e, de, dn = bd.bond_sensitivities(an, k, CP, 1, E)
            es.append(e)
            des.append(de)
            dns.append(dn)
            ws.append(an.norm(k))
        g = bd.bond_gradient_from_samples(es, des, dns, weights=ws)
        fd = (exact(_rotated(spec, 1, E, h)) - exact(_rotated(spec, 1, E, -h))) / (2 * h)
        assert abs(g - fd) <= 1e-7 * max(1.0, abs(fd)), (pair, g, fd)
