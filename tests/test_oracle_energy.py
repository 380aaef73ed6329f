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
* E_loc is gauge invariant (Z2, flipping the links of a site);
* gradient with respect to the on-site covariance Gamma_A (rotations
  exp(theta E) Gamma_A exp(-theta E), K = 1..3): the per-configuration
  sensitivities of e(G) and log N(G) against central differences, and the
  p(G)-weighted gradient over every configuration against central differences of
  the exactly enumerated <H>.
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


# ----- gradient with respect to Gamma_A (K = 1) -----
@pytest.mark.parametrize("K,group", [(1, 2), (1, 3), (2, 2), (3, 3)])
def test_sensitivities_against_finite_differences(K, group):
    """d e(G) and d log N(G) along generators of the on-site rotation, per configuration
    (K > 1: through every pair's M_nm^-1 and the cross-term weights)."""
    lat = Lattice(2, 2)
    spec = synth.make_tensor(2, K=K, group=group)
    if K > 1:
        links, gk = synth.patch_bonds(lat.n_links, K)
        spec.patch_link, spec.gamma_bond_k = links, gk

    def mk(g):
        return Ansatz(lat, g, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k, spec.c)

    an = mk(spec.gamma_loc)
    k = np.random.default_rng(1).integers(0, group, lat.n_links)
    e, Se, SN = en.sensitivities(an, k, CP)
    assert abs(e - en.local_energy(an, k, CP)) < 1e-12
    h = 1e-5
    for (a, b) in [(0, 1), (0, 5), (2, 7), (3, 9), (1, 4), (6, 8)]:
        E = en.generator(a, b)
        D = E @ spec.gamma_loc - spec.gamma_loc @ E
        ap, am = mk(en.rotated_gamma_loc(spec.gamma_loc, h * E)), mk(en.rotated_gamma_loc(spec.gamma_loc, -h * E))
        de = (en.local_energy(ap, k, CP) - en.local_energy(am, k, CP)) / (2 * h)
        dn = (np.log(ap.norm(k)) - np.log(am.norm(k))) / (2 * h)
        assert abs(np.sum(D * Se.T) - de) <= 1e-7 * max(1.0, abs(de))
        assert abs(np.sum(D * SN.T).real - dn) <= 1e-7 * max(1.0, abs(dn))


@pytest.mark.parametrize("K,group", [(1, 2), (1, 3), (2, 2)])
def test_gradient_against_exact_energy(K, group):
    """d<H>/d theta from per-configuration sensitivities weighted by p(G) over every configuration
    of a 2x1 lattice equals central differences of the exactly enumerated <H>(theta)."""
    lat = Lattice(2, 1)
    spec = synth.make_tensor(2, K=K, group=group)
    if K > 1:
        links, gk = synth.patch_bonds(lat.n_links, K)
        spec.patch_link, spec.gamma_bond_k = links, gk

    def mk(g):
        return Ansatz(lat, g, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k, spec.c)

    def exact(g):
        a = mk(g)
        num = den = 0.0
        for G in itertools.product(range(group), repeat=lat.n_links):
            k = np.array(G)
            Nk = a.norm(k)
            num += Nk * en.local_energy(a, k, CP)
            den += Nk
        return (num / den).real

    an = mk(spec.gamma_loc)
    es, Ses, SNs, ws = [], [], [], []
    for G in itertools.product(range(group), repeat=lat.n_links):
        k = np.array(G)
        e, Se, SN = en.sensitivities(an, k, CP)
        es.append(e)
        Ses.append(Se)
        SNs.append(SN)
        ws.append(an.norm(k))
    g = en.gradient_from_samples(spec.gamma_loc, es, Ses, SNs, weights=ws)
    assert np.abs(g + g.T).max() < 1e-14
    h = 1e-5
    for (a, b) in [(0, 1), (0, 6), (2, 9), (4, 5)]:
        E = en.generator(a, b)
        fd = (exact(en.rotated_gamma_loc(spec.gamma_loc, h * E))
              - exact(en.rotated_gamma_loc(spec.gamma_loc, -h * E))) / (2 * h)
        assert abs(g[a, b] - fd) <= 1e-7 * max(1.0, abs(fd)), (a, b, g[a, b], fd)


@pytest.mark.parametrize("group", [2, 3])
def test_bond_phase_is_an_on_site_rotation(group):
    """The one free parameter of an out-in coupled pure bond, the phase of its out mode, is
    absorbed by Gamma_A: rotating the bond's out pair by phi equals rotating the right and up
    virtual pairs of Gamma_A by -phi (same W(G) and E_loc(G) for every G).  So
    d<H>/d phi = -(g[r0, r1] + g[u0, u1]) in terms of the Gamma_A gradient."""
    from oracle.lattice import VSLOT_R, VSLOT_U
    from oracle.model import rotation
    lat = Lattice(2, 2)
    spec = synth.make_tensor(2, K=1, group=group)
    phi = 0.37
    o = np.eye(4)
    o[0:2, 0:2] = rotation(phi)
    a1 = Ansatz(lat, spec.gamma_loc, o @ spec.gamma_bond @ o.T, group)
    X = np.zeros((10, 10))
    for slot in (VSLOT_R, VSLOT_U):
        X -= phi * en.generator(2 + 2 * slot, 3 + 2 * slot)
    a2 = Ansatz(lat, en.rotated_gamma_loc(spec.gamma_loc, X), spec.gamma_bond, group)
    for G in itertools.islice(itertools.product(range(group), repeat=lat.n_links), 0, None, 7):
        k = np.array(G)
        assert abs(a1.log_weight(k) - a2.log_weight(k)) < 1e-12
        assert abs(en.local_energy(a1, k, CP) - en.local_energy(a2, k, CP)) < 1e-11
