"""Pins of the oracle's electric-field observable f_E(G) (Sec. 2.2 electric term, Sec. 5.3).

* the Casimir kernel <g|J^2|g'> has the irreps of Z_N as eigenvectors with the
  chosen spectrum as eigenvalues (its defining property);
* f_E from the Gaussian-trace definition equals the dense Fock-space sum over g'
  of <g|J^2|g'> <psi(G)|psi(g'; G)> / N(G), for K = 1..3 and complex spectra;
* the patch route (4x4 block of M_nm^-1) equals the definition;
* Gauss-law limits: a bond that never carries flux (|00>) gives e_0 exactly and
  one that always does (|11>) gives e_1;
* <J^2> = sum_G N(G) f_E(G) / sum_G N(G) over every configuration of a small
  lattice is real and lies within the spectrum (J^2 is Hermitian, its
  expectation a convex combination of its eigenvalues), although a single f_E(G)
  is complex;
* f_E is gauge invariant (flipping the four links of a site, Z2).
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import gaussian
from oracle.fock import FockPEPS
from oracle.lattice import Lattice
from oracle.model import Ansatz, OBS_ELECTRIC


def _pair(Lx, Ly, K=1, group=2, gamma_bond=None):
    lat = Lattice(Lx, Ly)
    spec = synth.make_tensor(max(Lx, 2), K=K, group=group)
    if K > 1:
        links, gk = synth.patch_bonds(lat.n_links, K)
        spec.patch_link, spec.gamma_bond_k = links, gk
    gb = spec.gamma_bond if gamma_bond is None else gamma_bond
    an = Ansatz(lat, spec.gamma_loc, gb, group, spec.patch_link, spec.gamma_bond_k, spec.c)
    fk = FockPEPS(lat, spec.gamma_loc, gb, group, spec.patch_link, spec.gamma_bond_k)
    return lat, an, fk


def _weights(an, k):
    K = an.K
    ginv = [[np.linalg.inv(an.assemble_M(k, n, m)) for m in range(K)] for n in range(K)]
    if K == 1:
        return ginv, np.ones((1, 1))
    wts = np.conj(an.c)[:, None] * an.c[None, :] * an.bond_overlaps() * an.cross_ratio_def(k)
    return ginv, wts


@pytest.mark.parametrize("group", [2, 3])
def test_casimir_kernel_diagonal_on_irreps(group):
    lat, an, _ = _pair(1, 1, group=group)
    rng = np.random.default_rng(11)
    e = rng.normal(size=group) + 1j * rng.normal(size=group)
    kap = an.casimir_kernel(e)
    J2 = np.array([[kap[(g - gp) % group] for gp in range(group)] for g in range(group)])
    w = np.exp(2j * np.pi / group)
    for j in range(group):
        v = np.array([w ** (j * g) for g in range(group)])
        assert np.abs(J2 @ v - e[j] * v).max() < 1e-14
    # a real spectrum gives a Hermitian J^2; a spectrum symmetric in j -> -j a real kernel
    er = rng.normal(size=group)
    k2 = an.casimir_kernel(er)
    J2r = np.array([[k2[(g - gp) % group] for gp in range(group)] for g in range(group)])
    assert np.abs(J2r - J2r.conj().T).max() < 1e-15
    es = np.array([0.0] + [1.0] * (group - 1))
    assert np.abs(an.casimir_kernel(es).imag).max() < 1e-15


@pytest.mark.parametrize("Lx,Ly,K,group", [(1, 1, 1, 2), (1, 1, 1, 3), (2, 1, 1, 2), (2, 1, 2, 3),
                                           (2, 2, 1, 2), (2, 2, 1, 3), (2, 2, 2, 2), (2, 2, 3, 3)])
def test_electric_definition_against_fock(Lx, Ly, K, group):
    lat, an, fk = _pair(Lx, Ly, K, group)
    rng = np.random.default_rng(20 + 7 * K + group)
    for _ in range(2):
        k = rng.integers(0, group, lat.n_links)
        e = rng.normal(size=group) + 1j * rng.normal(size=group)
        for ell in range(lat.n_links):
            ref = fk.electric(k, ell, e, an.c)
            got = an.electric_def(k, ell, e)
            assert abs(got - ref) <= 1e-11 * max(1.0, abs(ref)), (ell, got, ref)


@pytest.mark.parametrize("L,K,group", [(2, 1, 2), (4, 1, 2), (4, 2, 3), (2, 3, 2)])
def test_electric_patch_equals_definition(L, K, group):
    lat, an, _ = _pair(L, L, K, group)
    rng = np.random.default_rng(40 + L + K)
    k = rng.integers(0, group, lat.n_links)
    e = rng.normal(size=group)
    ginv, wts = _weights(an, k)
    links = range(lat.n_links) if L == 2 else rng.choice(lat.n_links, 6, replace=False)
    for ell in links:
        a = an.electric_def(k, int(ell), e)
        b = an.electric_patch(k, int(ell), e, ginv, wts)
        assert abs(a - b) <= 1e-11 * max(1.0, abs(a)), (ell, a, b)


@pytest.mark.parametrize("occ,group", [(0, 2), (1, 2), (0, 3), (1, 3)])
def test_gauss_law_limits(occ, group):
    """Bond |00> (out mode never occupied): f_E = e_0; bond |11>: f_E = e_1, for every G."""
    v = np.zeros(4, complex)
    v[3 * occ] = 1.0
    gb = gaussian.covariance_of_state(v, 2).real
    lat, an, fk = _pair(2, 1, 1, group, gamma_bond=gb)
    rng = np.random.default_rng(3)
    e = rng.normal(size=group)
    for k in itertools.product(range(group), repeat=lat.n_links):
        k = np.array(k)
        for ell in range(lat.n_links):
            f = an.electric_def(k, ell, e)
            assert abs(f - e[occ]) < 1e-12, (k, ell, f)
            assert abs(fk.electric(k, ell, e) - e[occ]) < 1e-12


@pytest.mark.parametrize("K,group", [(1, 2), (1, 3), (2, 2)])
def test_expectation_real_and_within_spectrum(K, group):
    lat, an, _ = _pair(2, 1, K, group)
    e = np.array([0.3, 1.7, 1.7][:group])           # real, symmetric in j -> -j for Z3
    imag_seen = 0.0
    for ell in range(lat.n_links):
        num = den = 0.0
        for k in itertools.product(range(group), repeat=lat.n_links):
            k = np.array(k)
            Nk = an.norm(k)
            f = an.electric_def(k, ell, e)
            imag_seen = max(imag_seen, abs(f.imag))
            num += Nk * f
            den += Nk
        ex = num / den
        assert abs(ex.imag) < 1e-12 * abs(ex.real)
        assert e.min() - 1e-12 <= ex.real <= e.max() + 1e-12
    assert imag_seen > 1e-6          # a single f_E(G) is complex in general


def test_gauge_invariance_z2():
    lat, an, _ = _pair(2, 2, 1, 2)
    rng = np.random.default_rng(9)
    e = np.array([0.0, 1.0])
    for _ in range(4):
        k = rng.integers(0, 2, lat.n_links)
        x = int(rng.integers(lat.V))
        k2 = k.copy()
        for ell in lat.site_links(x):
            k2[ell] ^= 1
        for ell in range(lat.n_links):
            assert abs(an.electric_def(k, ell, e) - an.electric_def(k2, ell, e)) < 1e-12


@pytest.mark.parametrize("K,group", [(1, 2), (2, 3)])
def test_observable_slot_is_link_mean(K, group):
    lat, an, _ = _pair(2, 2, K, group)
    rng = np.random.default_rng(12)
    k = rng.integers(0, group, lat.n_links)
    spec = np.array([0.0] + [1.0] * (group - 1))
    ref = np.mean([an.electric_def(k, ell, spec).real for ell in range(lat.n_links)])
    assert abs(an.observables(k)[OBS_ELECTRIC] - ref) < 1e-12
