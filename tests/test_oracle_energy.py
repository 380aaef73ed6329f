"""Pins of the oracle's local energy and linear variational step (Sec. 2, 5, 6.3).

* the pi-flux phases multiply to -1 around every plaquette (their defining property);
* E_loc(G) in covariance form (Wick's theorem on M_nm^-1, electric term through the
  mixed occupation) equals the dense Fock-space value
  [<psi(G)|H(G)|psi(G)> + ke sum_l sum_g' <g|J^2|g'> <psi(G)|psi(g'; G)>] / <psi|psi>,
  with the fermion operators built directly by Jordan-Wigner;
* sum_G N(G) E_loc(G) / N over every configuration equals <Psi|H|Psi> / <Psi|Psi>
  of the full gauge (x) fermion state (J^2 acting on each link's axis);
* the linear method on the reweighted matrices gives the lowest generalised
  eigenvalue of the dense K-dimensional subspace (<Psi_n|H|Psi_m>, <Psi_n|Psi_m>),
  whatever lambda the configurations were weighted with;
* E_loc is gauge invariant (Z2, flipping the links of a site).
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import energy as en
from oracle.fock import FockPEPS, annihilators, fock_local_energy, subspace_matrices
from oracle.gaussian import number_matrices
from oracle.lattice import Lattice
from oracle.model import Ansatz

CP = en.Couplings(t=0.7, mu=0.3, m=0.45, kb=-0.8, ke=1.3)


def _pair(Lx, Ly, K=1, group=2):
    lat = Lattice(Lx, Ly)
    spec = synth.make_tensor(max(Lx, 2), K=K, group=group)
    if K > 1:
        links, gk = synth.patch_bonds(lat.n_links, K)
        spec.patch_link, spec.gamma_bond_k = links, gk
    an = Ansatz(lat, spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k, spec.c)
    fk = FockPEPS(lat, spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k)
    return lat, an, fk


def _enumerate(an, c):
    """Exact p_c-averages of rho h / S and rho / S, and <H> = sum N E_loc / N."""
    K = an.K
    Hb = np.zeros((K, K), complex)
    Nb = np.zeros((K, K), complex)
    num = den = 0.0
    for G in itertools.product(range(an.group), repeat=an.lat.n_links):
        k = np.array(G)
        rho, rh = en.pair_matrices(an, k, CP)
        S = np.conj(c) @ rho @ c
        NG = an.weight(k) * S.real
        Hb += NG * rh / S
        Nb += NG * rho / S
        num += NG * (np.conj(c) @ rh @ c) / S
        den += NG
    return Hb / den, Nb / den, num / den


@pytest.mark.parametrize("L", [2, 4, 6])
def test_pi_flux(L):
    lat = Lattice(L, L)
    for x in range(lat.V):
        l1, l2, l3, l4 = lat.plaquette_links(x)
        sites = [x, lat.shift(x, 1, 0), lat.shift(x, 0, 1), x]
        dirs = [0, 1, 0, 1]
        prod = np.prod([en.eta(lat, s, d) for s, d in zip(sites, dirs)])
        assert prod == -1.0


def test_annihilators_are_canonical():
    V = 3
    a = annihilators(V)
    nm = number_matrices(V)
    for i in range(V):
        assert np.abs(a[i].conj().T @ a[i] - nm[i]).max() < 1e-15
        for j in range(V):
            anti = a[i] @ a[j].conj().T + a[j].conj().T @ a[i]
            assert np.abs(anti - (i == j) * np.eye(2 ** V)).max() < 1e-15
            assert np.abs(a[i] @ a[j] + a[j] @ a[i]).max() < 1e-15


@pytest.mark.parametrize("Lx,Ly,K,group", [(2, 1, 1, 2), (2, 1, 1, 3), (2, 1, 2, 3), (2, 2, 1, 2),
                                           (2, 2, 2, 2), (2, 2, 3, 3)])
def test_local_energy_against_fock(Lx, Ly, K, group):
    lat, an, fk = _pair(Lx, Ly, K, group)
    rng = np.random.default_rng(60 + K + group)
    for _ in range(2):
        k = rng.integers(0, group, lat.n_links)
        a = en.local_energy(an, k, CP)
        b = fock_local_energy(fk, k, CP, en.eta, an.c)
        assert abs(a - b) <= 1e-11 * max(1.0, abs(b)), (k, a, b)


@pytest.mark.parametrize("Lx,Ly,K,group", [(2, 1, 1, 2), (2, 1, 2, 3), (2, 2, 1, 2)])
def test_average_equals_full_space_expectation(Lx, Ly, K, group):
    lat, an, fk = _pair(Lx, Ly, K, group)
    Hm, Nm = subspace_matrices(fk, CP, en.eta)
    c = an.c
    exact = (np.conj(c) @ Hm @ c) / (np.conj(c) @ Nm @ c)
    assert abs(exact.imag) < 1e-12 * abs(exact)
    _, _, mc = _enumerate(an, c)
    assert abs(mc - exact) <= 1e-11 * abs(exact)


@pytest.mark.parametrize("Lx,Ly,K,group", [(2, 1, 2, 3), (2, 1, 3, 2)])
def test_linear_method_is_subspace_minimum(Lx, Ly, K, group):
    lat, an, fk = _pair(Lx, Ly, K, group)
    Hm, Nm = subspace_matrices(fk, CP, en.eta)
    w = scipy.linalg.eigh(0.5 * (Hm + Hm.conj().T), 0.5 * (Nm + Nm.conj().T), eigvals_only=True)
    rng = np.random.default_rng(8)
    for c in (an.c, rng.standard_normal(K) + 1j * rng.standard_normal(K)):
        Hb, Nb, e_now = _enumerate(an, c)
        e, lam = en.linear_method(Hb, Nb)
        assert abs(e - w[0]) <= 1e-10 * abs(w[0])
        assert e <= e_now.real + 1e-12
        # the returned lambda attains it in the dense subspace
        rq = (np.conj(lam) @ Hm @ lam) / (np.conj(lam) @ Nm @ lam)
        assert abs(rq - w[0]) <= 1e-10 * abs(w[0])


def test_gauge_invariance_z2():
    lat, an, _ = _pair(2, 2, 1, 2)
    rng = np.random.default_rng(13)
    for _ in range(3):
        k = rng.integers(0, 2, lat.n_links)
        k2 = k.copy()
        for ell in lat.site_links(int(rng.integers(lat.V))):
            k2[ell] ^= 1
        assert abs(en.local_energy(an, k, CP) - en.local_energy(an, k2, CP)) < 1e-12
