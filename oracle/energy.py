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

Gradient with respect to Gamma_A (any K): Gamma_A(theta) = exp(theta E) Gamma_A
exp(-theta E) for antisymmetric generators E keeps the on-site state pure and
even.  With Delta = [E, Gamma_A],
    d<H> = E_p[d e] + E_p[(e - <H>) d log N],
where d e(G) = tr(Delta S_e(G)) and d log N(G) = tr(Delta S_N(G)) for 10 x 10
sensitivity matrices of the configuration.
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


# ----- gradient with respect to Gamma_A -----
def rotated_gamma_loc(gamma_loc: np.ndarray, X: np.ndarray) -> np.ndarray:
    """exp(X) Gamma_A exp(-X) for a real antisymmetric 10 x 10 generator X (stays pure and even)."""
    from scipy.linalg import expm
    R = expm(X)
    return R @ gamma_loc @ R.T


def generator(k: int, l: int) -> np.ndarray:
    E = np.zeros((10, 10))
    E[k, l] = 1.0
    E[l, k] = -1.0
    return E


def energy_coefficients(an: Ansatz, links_k, cp: Couplings) -> np.ndarray:
    """C[p, q]: the coefficient of Gamma_out[p, q] in the fermion part of the local energy
    (by linearity; <phi_x^+ phi_y> = 1/4 [cc(x0,y0) + i cc(x0,y1) - i cc(x1,y0) + cc(x1,y1)],
    cc(a, b) = delta_ab - i Gamma_out[a, b])."""
    lat, N, V = an.lat, an.group, an.lat.V
    C = np.zeros((2 * V, 2 * V), complex)

    def add_bilinear(coef, x, y):
        for (a, b, w) in ((0, 0, 1.0), (0, 1, 1j), (1, 0, -1j), (1, 1, 1.0)):
            C[2 * x + a, 2 * y + b] += coef * 0.25 * w * (-1j)

    for x in range(V):
        x1, x2 = lat.coords(x)
        add_bilinear(cp.mu + cp.m * (-1) ** (x1 + x2), x, x)
        for mu in range(2):
            y = lat.shift(x, 1, 0) if mu == 0 else lat.shift(x, 0, 1)
            D = link_phase(links_k[lat.link(x, mu)], N)
            e_ = eta(lat, x, mu)
            add_bilinear(cp.t * 1j * e_ * D, x, y)
            add_bilinear(-cp.t * 1j * e_ * np.conj(D), y, x)
    return C


def pair_sensitivities(an: Ansatz, links_k, cp: Couplings, G: np.ndarray, n: int = 0, m: int = 0):
    """(S_e, S_N) of the pair (n, m) from G = M_nm^-1: d h_nm = tr(Delta S_e) and
    (1/2) tr(G dM) = tr(Delta S_N) for Delta = [E, Gamma_A], tr(Delta S) = sum_ij Delta_ij S_ji.

    Gamma_out = A + B G B^T gives d Gamma_out = dA + dB G B^T + B G dB^T + P dM P^T with
    P = B G (G antisymmetric, dG = -G dM G); the electric term X = en + (1/2) tr(G_UU R) of
    the pair gives dX = -(1/2) tr((G dM G)_UU R); dM = (+)_x Delta_d on every site."""
    lat, V = an.lat, an.lat.V
    C = energy_coefficients(an, links_k, cp)
    Sa = np.zeros((2, 2), complex)
    Sb = np.zeros((2, 8), complex)
    Sd = np.zeros((8, 8), complex)
    GBt = G @ an.B.T                       # n x 2V
    P = an.B @ G                           # 2V x n
    for x in range(V):
        rows = slice(2 * x, 2 * x + 2)
        cols8 = slice(8 * x, 8 * x + 8)
        # dA: Gamma_out[2x+a, 2x+b] += Delta_a[a, b]
        Sa += C[rows, rows].T
        # dB G B^T: Gamma_out[2x+a, q] += sum_i Delta_b[a, i] (G B^T)[8x+i, q]
        Sb += (GBt[cols8, :] @ C[rows, :].T).T
        # B G dB^T: Gamma_out[p, 2x+b] += sum_i (B G)[p, 8x+i] Delta_b[b, i]
        Sb += (P[:, cols8].T @ C[:, rows]).T
    # P dM P^T: sum_pq C[p,q] (P dM P^T)[p,q] = sum_z tr(Delta_d (P^T C P)[z, z])
    Q = P.T @ C @ P
    for z in range(V):
        blk = slice(8 * z, 8 * z + 8)
        Sd += Q[blk, blk].T
    if cp.ke != 0.0:
        # X_l is affine in the antisymmetric G_UU: its slope along e_ij - e_ji (i < j) is read
        # off the oracle's own X at unit steps (exact for an affine function), and
        # d G_UU = -(G dM G)_UU with (G dM G)[a, b] = sum_z tr(Delta_d outer(G[z-block, b], G[a, z-block]))
        for ell in range(lat.n_links):
            u = lat.link_majoranas(ell)
            g_uu = G[np.ix_(u, u)]
            x0 = an.mixed_occupation_patch(g_uu, links_k, ell, n, m)
            for i in range(4):
                for j in range(i + 1, 4):
                    step = np.zeros((4, 4))
                    step[i, j], step[j, i] = 1.0, -1.0
                    slope = an.mixed_occupation_patch(g_uu + step, links_k, ell, n, m) - x0
                    for z in range(V):
                        blk = slice(8 * z, 8 * z + 8)
                        Sd += -cp.ke * slope * np.outer(G[blk, u[j]], G[u[i], blk])
    S_e = np.zeros((10, 10), complex)
    S_e[0:2, 0:2] = Sa
    S_e[2:10, 0:2] = Sb.T
    S_e[2:10, 2:10] = Sd
    S_N = np.zeros((10, 10), complex)
    for x in range(V):
        blk = slice(8 * x, 8 * x + 8)
        S_N[2:10, 2:10] += 0.5 * G[blk, blk]
    return S_e, S_N


def sensitivities(an: Ansatz, links_k, cp: Couplings):
    """(e, S_e, S_N) of one configuration: for every antisymmetric generator E,
    d e(G) = tr(Delta S_e) and d log N(G) = tr(Delta S_N) with Delta = [E, Gamma_A] the
    change of the on-site covariance (the same on every site); e(G) is the local energy.

    K = 1: N(G) = W(G) = 2^-4V sqrt(det M), d log N = (1/2) tr(G dM).  K > 1: with
    om_ab = lambda_a^* lambda_b rho_ab, S = sum om, E = sum om h / S and
    d log r_ab = (1/2) tr(M_ab^-1 dM) - (1/2) tr(G dM) (the cross terms' Delta_ab do not depend on
    Gamma_A),
        d log N = sum_ab (om_ab / S) (1/2) tr(M_ab^-1 dM),
        d E     = sum_ab (om_ab / S) [d h_ab + (h_ab - E) (1/2) tr(M_ab^-1 dM)]
    (the (1/2) tr(G dM) terms cancel since sum om / S = 1)."""
    K = an.K
    if K == 1:
        G = np.linalg.inv(an.assemble_M(links_k))
        S_e, S_N = pair_sensitivities(an, links_k, cp, G)
        return local_energy(an, links_k, cp), S_e, S_N.real
    rho, rh = pair_matrices(an, links_k, cp)
    om = np.conj(an.c)[:, None] * an.c[None, :] * rho
    S = om.sum()
    h = rh / rho
    E = (om * h).sum() / S
    S_e = np.zeros((10, 10), complex)
    S_N = np.zeros((10, 10), complex)
    for a in range(K):
        for b in range(K):
            Gab = np.linalg.inv(an.assemble_M(links_k, a, b))
            se, sn = pair_sensitivities(an, links_k, cp, Gab, a, b)
            S_e += om[a, b] / S * (se + (h[a, b] - E) * sn)
            S_N += om[a, b] / S * sn
    return E, S_e, S_N


def gradient_from_samples(gamma_loc: np.ndarray, es, S_es, S_Ns, weights=None):
    """d<H>/d theta_kl for the generators E_kl (k < l) from per-configuration (e, S_e, S_N)
    drawn from p(G) (or weighted by p(G) when weights are given):
    mean[tr(Delta S_e)] + mean[(e - mean e) tr(Delta S_N)], real part, from
    <H> = sum_G N(G) e(G) / sum_G N(G).  Returned as the antisymmetric 10 x 10 matrix g with
    g[k, l] = d<H>/d theta_kl."""
    es = np.asarray(es)
    w = np.full(len(es), 1.0 / len(es)) if weights is None else np.asarray(weights) / np.sum(weights)
    ebar = np.sum(w * es)
    Sbar = (np.tensordot(w, np.asarray(S_es), axes=1)
            + np.tensordot(w * (es - ebar), np.asarray(S_Ns), axes=1))
    # tr([E, Gamma] S) = tr(E (Gamma S - S Gamma)); for E_kl: Y[l, k] - Y[k, l]
    Y = gamma_loc @ Sbar - Sbar @ gamma_loc
    g = (Y.T - Y).real
    return g
