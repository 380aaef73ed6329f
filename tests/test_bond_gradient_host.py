"""The library's host combination of the bond-state gradient (ggf_bond_gradient) against the oracle.

Rows are built by the oracle for every configuration of a small lattice: the energy rows (rho / S,
rho h / S, Re E_loc) and the bond rows (patch set S, link values, the contraction R of the energy's
linear part with G[S, :], and G_SS) as ggf_measure_energy and ggf_measure_bond_rows lay them out.
The library's gradient over those rows must equal the oracle's definitional gradient over the same
configurations (equal weights), for every bond and generator.  Host code only: runs without a GPU.
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
CPD = dict(t=CP.t, mu=CP.mu, m=CP.m, kb=CP.kb, ke=CP.ke)
E_STRIDE = 1 + 4 * 4 * 4
B_STRIDE = 2 + 12 + 4 + 3 * 12 * 12


def _spec(lat, K, group):
    spec = synth.make_tensor(max(lat.Lx, 2), K=K, group=group)
    links, gk = synth.patch_bonds(lat.n_links, K)
    spec.patch_link, spec.gamma_bond_k = links, gk
    return spec


def oracle_rows(an, links, L):
    rho, rh = en.pair_matrices(an, links, CP)
    c = an.c
    S = np.conj(c) @ rho @ c
    erow = np.zeros(E_STRIDE)
    erow[0] = ((np.conj(c) @ rh @ c) / S).real
    K = an.K
    for p in range(K * K):
        i, j = divmod(p, K)
        erow[1 + 4 * p:5 + 4 * p] = [(rho[i, j] / S).real, (rho[i, j] / S).imag,
                                     (rh[i, j] / S).real, (rh[i, j] / S).imag]
    G = np.linalg.inv(an.assemble_M(links))
    R = bd.coefficient_contraction(an, links, CP, G)
    Sidx = an.S
    s = len(Sidx)
    brow = np.zeros(B_STRIDE)
    brow[0], brow[1] = s, L
    brow[2:2 + s] = Sidx
    for k in range(1, K):
        brow[14 + k] = links[int(an.patch_link[k])]
    for a in range(s):
        for b in range(s):
            brow[18 + 2 * (12 * a + b)] = R[a, b].real
            brow[19 + 2 * (12 * a + b)] = R[a, b].imag
            brow[306 + 12 * a + b] = G[Sidx[a], Sidx[b]]
    return erow, brow


@pytest.mark.parametrize("K,group", [(2, 2), (3, 3)])
def test_bond_gradient_matches_oracle(K, group):
    from paper_2412_01737_amd.ggf import bond_gradient
    lat = Lattice(2, 2)
    spec = _spec(lat, K, group)
    an = Ansatz(lat, spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k, spec.c)
    rng = np.random.default_rng(91 + K)
    configs = [synth.random_links(rng, lat.n_links, group) for _ in range(6)]
    erows, brows = zip(*[oracle_rows(an, k, 2) for k in configs])
    g = bond_gradient(spec, CPD, np.array(erows), np.array(brows))
    for k in range(1, K):
        for gi, pair in enumerate(bd.bond_pairs()):
            E = bd.bond_generator(*pair)
            es, des, dns = zip(*[bd.bond_sensitivities(an, links, CP, k, E) for links in configs])
            ref = bd.bond_gradient_from_samples(es, des, dns)
            assert abs(g[k - 1, gi] - ref) <= 1e-9 * max(1.0, abs(ref)), (k, pair, g[k - 1, gi], ref)


def test_bond_gradient_refuses_single_gaussian():
    from paper_2412_01737_amd.ggf import GGFError, bond_gradient
    lat = Lattice(2, 2)
    spec = _spec(lat, 2, 2)
    spec1 = synth.make_tensor(2, K=1)
    spec1.patch_link, spec1.gamma_bond_k = spec.patch_link[:1], spec.gamma_bond_k[:1]
    with pytest.raises((GGFError, ValueError)):
        bond_gradient(spec1, CPD, np.zeros((1, E_STRIDE)), np.zeros((1, B_STRIDE)))
