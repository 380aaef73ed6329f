"""Z_N beyond Z2/Z3 (N <= 64, toward the continuous group U(1)): pins of the oracle.

One virtual fermion mode per leg carries flux 0 or 1, and the gauge field acts
as the phase exp(2 pi i k n_out / N).  The covariance-form weights, cross terms,
electric field and local energy are checked against the dense Fock-space
contraction for Z4 and Z5.  A Z4 chain on the 1x1 lattice, with its 16
configurations, reproduces the exact averages.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import energy as en
from oracle import stats
from oracle.chain import WoodburyChain
from oracle.fock import FockPEPS, fock_local_energy
from oracle.lattice import Lattice
from oracle.model import Ansatz


def _pair(Lx, Ly, K, group):
    lat = Lattice(Lx, Ly)
    spec = synth.make_tensor(max(Lx, 2), K=K, group=group)
    if K > 1:
        links, gk = synth.patch_bonds(lat.n_links, K)
        spec.patch_link, spec.gamma_bond_k = links, gk
    an = Ansatz(lat, spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k, spec.c)
    fk = FockPEPS(lat, spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k)
    return lat, an, fk


@pytest.mark.parametrize("Lx,Ly,group", [(1, 1, 4), (2, 1, 4), (1, 1, 5)])
def test_weight_all_configs(Lx, Ly, group):
    lat, an, fk = _pair(Lx, Ly, 1, group)
    for k in itertools.product(range(group), repeat=lat.n_links):
        k = np.array(k)
        wf = fk.weight(k)
        assert abs(an.weight(k) - wf) <= 1e-12 * wf


@pytest.mark.parametrize("K,group", [(2, 4), (3, 5)])
def test_cross_terms_and_electric_against_fock(K, group):
    lat, an, fk = _pair(2, 2, K, group)
    rng = np.random.default_rng(31 + group)
    e = rng.normal(size=group) + 1j * rng.normal(size=group)
    for _ in range(2):
        k = rng.integers(0, group, lat.n_links)
        Nf = fk.cross_terms(k)
        assert np.abs(an.cross_terms(k) - Nf).max() <= 1e-12 * np.abs(Nf).max()
        for ell in (0, 3, 6):
            ref = fk.electric(k, ell, e, an.c)
            assert abs(an.electric_def(k, ell, e) - ref) <= 1e-11 * max(1.0, abs(ref))


@pytest.mark.parametrize("K,group", [(1, 4), (2, 5)])
def test_local_energy_against_fock(K, group):
    cp = en.Couplings(t=0.7, mu=0.3, m=0.45, kb=-0.8, ke=1.3)
    lat, an, fk = _pair(2, 1, K, group)
    rng = np.random.default_rng(41)
    for _ in range(3):
        k = rng.integers(0, group, lat.n_links)
        a = en.local_energy(an, k, cp)
        b = fock_local_energy(fk, k, cp, en.eta, an.c)
        assert abs(a - b) <= 1e-11 * max(1.0, abs(b))


def test_z4_chain_matches_enumeration():
    """1 chain x 20000 sweeps on the 1x1 Z4 lattice (2 links, 16 configurations) vs exact averages."""
    lat, an, _ = _pair(1, 1, 1, 4)
    ws, plaq, dens = [], [], []
    for k in itertools.product(range(4), repeat=lat.n_links):
        k = np.array(k)
        ws.append(an.weight(k))
        plaq.append(an.plaquette(k))
        dens.append(an.density_from(an.gamma_out(np.linalg.inv(an.assemble_M(k)))).real)
    ws = np.array(ws) / np.sum(ws)
    exact = [ws @ np.array(plaq), ws @ np.array(dens)]
    w = WoodburyChain(an, synth.SEED_CHAIN, 0, refresh_every=1024)
    n_sweeps, burn = 20000, 500
    series = np.zeros((n_sweeps, 2))
    for s in range(n_sweeps):
        w.sweep()
        series[s, 0] = an.plaquette(w.k)
        series[s, 1] = an.density_from(an.gamma_out(w.G)).real
    series = series[burn:]
    for j in range(2):
        tau, _, _ = stats.tau_int(series[:, j])
        err = np.std(series[:, j]) * np.sqrt(2 * tau / len(series))
        assert abs(series[:, j].mean() - exact[j]) < 4 * err + 1e-12
