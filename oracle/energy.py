"""Local energy of the gauged Hamiltonian and the linear variational step for lambda.

Test infrastructure (the oracle): plain NumPy float64, written from the paper.

Hamiltonian (Sec. 2, free staggered fermions; Sec. 2.2 gauging; Sec. 2.3 plaquette
and electric terms), one fermion mode per site, Z_N links in the fundamental
representation D(g) = w^g, w = exp(2 pi i / N):

    H = t  sum_{x, mu} [ i eta_mu(x) psi_x^+ D(g_{x,mu}) psi_{x+mu} + h.c. ]
      + mu sum_x psi_x^+ psi_x  +  m sum_x (-1)^(x1+x2) psi_x^+ psi_x
      + kb sum_x [ U_sq(x) + U_sq(x)^* ]  +  ke sum_l J^2_l

eta is the pi-flux choice the paper gives as an example: -1 on the horizontal
links of odd rows, +1 elsewhere.  The couplings are free and signed: the paper
prints the plaquette term with a positive prefactor and relates kb to ke
through g_qft.  J^2 has eigenvalue 0 on the trivial irrep and 1 on the others,
as in the electric-field observable of ``model``.

Local energy (Sec. 5.2 combined with Sec. 5.3): with
rho_nm(G) = N_nm(G) / W(G) = <B_m|B_n> r_nm(G) and
h_nm(G) = the transition expectation of H in (n, m) (G-diagonal terms by Wick's
theorem from M_nm^-1, the electric term through the mixed occupation X_nm),

    E_loc(G) = sum_nm lambda_n^* lambda_m rho_nm h_nm / S(G),  S = sum_nm lambda_n^* lambda_m rho_nm,

and <H> = E_p[E_loc].  Linear method for lambda: with configurations drawn from
p for some lambda, the K x K matrices Hb = E_p[rho h / S] and Nb = E_p[rho / S]
give <H>(lambda') = lambda'^+ Hb lambda' / lambda'^+ Nb lambda' for every
lambda' (reweighting), so the best lambda' is the lowest generalised eigenvector
of (Hb, Nb).  This is the optimisation of the lambda_n among the variational
parameters (the outlook of Sec. 6.3 asks for gradient descent on all of them).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .model import Ansatz, link_phase


@dataclass
class Couplings:
    t: float = 1.0
    mu: float = 0.0
    m: float = 0.0
    kb: float = 0.0
    ke: float = 0.0


def eta(lat, x: int, mu: int) -> float:
    """pi-flux phases: -1 on horizontal links (mu = 0) whose row x2 is odd."""
    return -1.0 if (mu == 0 and lat.coords(x)[1] % 2 == 1) else 1.0


def bilinear(gout: np.ndarray, x: int, y: int) -> complex:
    """<phi_x^+ phi_y> with phi = (c_0 + i c_1)/2 and <c_a c_b> = delta_ab - i Gamma_ab."""
    def cc(a, b):
        return (1.0 if a == b else 0.0) - 1j * gout[a, b]
    return 0.25 * (cc(2 * x, 2 * y) + 1j * cc(2 * x, 2 * y + 1)
                   - 1j * cc(2 * x + 1, 2 * y) + cc(2 * x + 1, 2 * y + 1))


def plaquette_sum(an: Ansatz, links_k) -> float:
    """sum_x [U_sq(x) + U_sq(x)^*] (Sec. 2.3)."""
    lat, N = an.lat, an.group
    tot = 0.0
    for x in range(lat.V):
        l1, l2, l3, l4 = lat.plaquette_links(x)
        z = (link_phase(links_k[l1], N) * link_phase(links_k[l2], N)
             * np.conj(link_phase(links_k[l3], N)) * np.conj(link_phase(links_k[l4], N)))
        tot += 2.0 * z.real
    return tot


def pair_energy(an: Ansatz, links_k, ginv: np.ndarray, n: int, m: int, cp: Couplings) -> complex:
    """h_nm(G): transition expectation of H in the pair (n, m), ginv = M_nm^-1."""
    lat, N = an.lat, an.group
    gout = an.A + an.B @ ginv @ an.B.T
    hop = dens = stag = 0.0 + 0j
    for x in range(lat.V):
        d = bilinear(gout, x, x)
        dens += d
        x1, x2 = lat.coords(x)
        stag += (-1) ** (x1 + x2) * d
        for mu in range(2):
            y = lat.shift(x, 1, 0) if mu == 0 else lat.shift(x, 0, 1)
            D = link_phase(links_k[lat.link(x, mu)], N)
            e = eta(lat, x, mu)
            hop += 1j * e * D * bilinear(gout, x, y) - 1j * e * np.conj(D) * bilinear(gout, y, x)
    elec = 0.0 + 0j
    if cp.ke != 0.0:
        for ell in range(lat.n_links):
            u = lat.link_majoranas(ell)
            elec += an.mixed_occupation_patch(ginv[np.ix_(u, u)], links_k, ell, n, m)
    return cp.t * hop + cp.mu * dens + cp.m * stag + cp.kb * plaquette_sum(an, links_k) + cp.ke * elec


def pair_matrices(an: Ansatz, links_k, cp: Couplings):
    """(rho, rho * h): K x K complex, rho_nm = <B_m|B_n> r_nm (r by full Pfaffians)."""
    K = an.K
    rho = an.bond_overlaps() * an.cross_ratio_def(links_k) if K > 1 else np.ones((1, 1), complex)
    rh = np.zeros((K, K), complex)
    for n in range(K):
        for m in range(K):
            ginv = np.linalg.inv(an.assemble_M(links_k, n, m))
            rh[n, m] = rho[n, m] * pair_energy(an, links_k, ginv, n, m, cp)
    return rho, rh


def local_energy(an: Ansatz, links_k, cp: Couplings, c=None) -> complex:
    """E_loc(G) for amplitudes c (default: the ansatz's lambda)."""
    c = an.c if c is None else np.asarray(c, complex)
    rho, rh = pair_matrices(an, links_k, cp)
    return (np.conj(c) @ rh @ c) / (np.conj(c) @ rho @ c)


def linear_method(Hb: np.ndarray, Nb: np.ndarray):
    """Lowest generalised eigenpair of the Hermitian parts of (Hb, Nb): (energy, lambda),
    lambda normalised to lambda^+ Nb lambda = 1 with lambda_0 real and positive."""
    H = 0.5 * (Hb + Hb.conj().T)
    S = 0.5 * (Nb + Nb.conj().T)
    L = np.linalg.cholesky(S)
    Li = np.linalg.inv(L)
    w, v = np.linalg.eigh(Li @ H @ Li.conj().T)
    lam = Li.conj().T @ v[:, 0]
    lam = lam * (abs(lam[0]) / lam[0]) if abs(lam[0]) > 0 else lam
    return float(w[0]), lam
