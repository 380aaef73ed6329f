"""Gradient of <H> with respect to the patch bond states Gamma_{B_n} (K > 1).

Test infrastructure (the oracle): plain NumPy float64, written from the paper.

The outlook of Sec. 6.3 asks for gradient descent on the variational
parameters; for a superposed ansatz (Sec. 5) these include the bond states
b_k (k >= 1) that B_k places on its patch link.  A bond is a pure even state
of the link's two virtual modes; rotations of its covariance,
    Gamma_{b_k}(theta) = exp(theta E) Gamma_{b_k} exp(-theta E),
E real antisymmetric 4 x 4 on the link's Majoranas (out 0, out 1, in 0, in 1),
keep it pure and even, and the phase convention <b_0|b_k> > 0 of the ansatz
fixes the state vector.  Only the (n, m) pairs that involve bond k depend on
theta, through the link's transition covariance and overlap; W(G) does not.

Per configuration, with om_nm = c_n^* c_m rho_nm, rho_nm = <B_m|B_n> r_nm,
S = sum om, e = sum om h / S:
    d log N = sum_nm (om_nm / S) d log rho_nm,   d log rho = d log <B_m|B_n> + d log r_nm,
    d e     = sum_nm (om_nm / S) [d h_nm + (h_nm - e) d log rho_nm],
    d log r_nm = (1/2) tr(M_nm^-1 dM_nm)          (r = Pf(M_nm) / Pf(M_00)),
and d h_nm has two parts: h_nm is affine in M_nm^-1 (Wick's theorem for the
fermion terms, the mixed occupation for the electric term), so the change
through dM_nm^-1 = -M_nm^-1 dM_nm M_nm^-1 is h_nm(dM^-1) - h_nm(0); and the
electric term of the patch link also depends on the bond's transition
directly.  Then d<H>/d theta = E_p[Re d e] + E_p[(Re e - <H>) d log N].

Two routes: ``bond_sensitivities`` from the definition (dense inverses of
every M_nm); ``bond_sensitivities_patch`` from G = M_00^-1 alone (G_SS and the
contraction R of the energy's coefficients with the rows G[S, :]), the form a
kernel evaluates; the tests pin the second to the first and the first to
central differences of exactly enumerated <H>.
"""
from __future__ import annotations

import numpy as np

from . import gaussian
from .energy import Couplings, energy_coefficients, pair_energy
from .model import THETA_REGULAR, Ansatz


def bond_generator(a: int, b: int) -> np.ndarray:
    E = np.zeros((4, 4))
    E[a, b], E[b, a] = 1.0, -1.0
    return E


def bond_pairs():
    """The six generators (a, b), a < b, in the order the library reports them."""
    return [(a, b) for a in range(4) for b in range(a + 1, 4)]


def rotated_bond(gamma4: np.ndarray, E: np.ndarray, theta: float) -> np.ndarray:
    from scipy.linalg import expm
    R = expm(theta * E)
    return R @ gamma4 @ R.T


def _quadratic(gamma: np.ndarray, cs) -> np.ndarray:
    """H(Gamma) = -(i/4) sum_ab Gamma_ab c_a c_b, whose ground state has covariance Gamma."""
    h = np.zeros_like(cs[0])
    for a in range(4):
        for b in range(4):
            if gamma[a, b] != 0:
                h = h + (-0.25j) * gamma[a, b] * (cs[a] @ cs[b])
    return h


def bond_state_derivative(an: Ansatz, k: int, E: np.ndarray) -> np.ndarray:
    """d b_k / d theta: the ground state of H(Gamma_k(theta)) moves by first-order
    perturbation theory (the exact derivative, in the gauge <b|db> = 0), then the phase
    convention <b_0|b_k> > 0 adds i v times minus the change of arg <b_0|b_k>."""
    cs = an._cs2
    v = an.bstate[k]
    g = gaussian.covariance_of_state(v, 2, cs).real
    dg = E @ g - g @ E
    h = _quadratic(g, cs)
    dh = _quadratic(dg, cs)
    w, vec = np.linalg.eigh(0.5 * (h + h.conj().T))
    dv = np.zeros(4, complex)
    for j in range(1, 4):
        dv -= vec[:, j] * (np.vdot(vec[:, j], dh @ v) / (w[j] - w[0]))
    v0 = an.bstate[0]
    ov = np.vdot(v0, v)
    return dv - 1j * np.imag(np.vdot(v0, dv) / ov) * v


def _transition_derivative(bra, ket, dbra, dket, cs):
    """(dGamma, d<bra|ket>) of the transition covariance (i/2)<bra|[c_a,c_b]|ket>/<bra|ket>."""
    ov = np.vdot(bra, ket)
    dov = np.vdot(dbra, ket) + np.vdot(bra, dket)
    g = gaussian.transition_covariance(bra, ket, 2, cs)
    dg = np.zeros((4, 4), complex)
    for a in range(4):
        for b in range(4):
            if a != b:
                comm = cs[a] @ cs[b] - cs[b] @ cs[a]
                dg[a, b] = 0.5j * (np.vdot(dbra, comm @ ket) + np.vdot(bra, comm @ dket)) / ov
    return dg - g * (dov / ov), dov


def _bond_vector_derivs(an: Ansatz, ell: int, n: int, m: int, k: int, db: np.ndarray):
    """(dket, dbra) of link ell's bond vectors in the transition |B_n><B_m|."""
    z = np.zeros(4, complex)
    on = int(an.patch_link[k]) == ell
    dket = db if (on and n == k) else z
    dbra = db if (on and m == k) else z
    return dket, dbra


def link_transition_derivative(an: Ansatz, ell: int, n: int, m: int, k: int, db: np.ndarray):
    ket, bra = an.bond_vectors(ell, n, m)
    dket, dbra = _bond_vector_derivs(an, ell, n, m, k, db)
    return _transition_derivative(bra, ket, dbra, dket, an._cs2)


def mixed_occupation_derivative(an: Ansatz, ginv_uu: np.ndarray, links_k, ell: int, n: int, m: int,
                                k: int, db: np.ndarray) -> complex:
    """d X_nm(ell) / d theta at fixed M_nm^-1 (the bond's own change), from the patch-lemma form of
    ``Ansatz.mixed_occupation_patch``: ratio = (ot / o0) Pf(blk), blk = [[G_UU, 1], [-1, ct - c0]],
    d log Pf(blk) = (1/2) tr(blk^-1 dblk)."""
    cs = an._cs2
    ket, bra = an.bond_vectors(ell, n, m)
    dket, dbra = _bond_vector_derivs(an, ell, n, m, k, db)
    u = an.out_phase(2 * np.pi * (int(links_k[ell]) % an.group) / an.group).conj()
    parts = []
    for theta in (0.0, THETA_REGULAR):
        sh = an.out_phase(-theta)
        b, kt, dbr, dkt = u @ sh @ bra, u @ ket, u @ sh @ dbra, u @ dket
        c = gaussian.transition_covariance(b, kt, 2, cs)
        dc, dov = _transition_derivative(b, kt, dbr, dkt, cs)
        parts.append((c, np.vdot(b, kt), dc, dov))
    (c0, o0, dc0, do0), (ct, ot, dct, dot) = parts
    blk = np.zeros((8, 8), complex)
    blk[:4, :4] = ginv_uu
    blk[:4, 4:] = np.eye(4)
    blk[4:, :4] = -np.eye(4)
    blk[4:, 4:] = ct - c0
    dblk = np.zeros((8, 8), complex)
    dblk[4:, 4:] = dct - dc0
    pf = gaussian.pfaffian(blk)
    ratio = (ot / o0) * pf
    dratio = ratio * (dot / ot - do0 / o0) + (ot / o0) * pf * 0.5 * np.trace(np.linalg.solve(blk, dblk))
    return dratio / (np.exp(1j * THETA_REGULAR) - 1.0)


def _pair_derivatives(an: Ansatz, links_k, cp: Couplings, n: int, m: int, k: int, db: np.ndarray, minv):
    """(d log rho_nm, d h_nm) of one pair involving bond k, from the dense M_nm^-1."""
    ell = int(an.patch_link[k])
    u = an.lat.link_majoranas(ell)
    dg, dov_link = link_transition_derivative(an, ell, n, m, k, db)
    ov_link = an.link_transition(ell, n, m)[1]
    dM = np.zeros_like(minv)
    dM[np.ix_(u, u)] = an._rot_block(dg, links_k[ell])
    dlogr = 0.5 * np.trace(minv @ dM)
    dlogrho = dov_link / ov_link + dlogr
    dminv = -minv @ dM @ minv
    dh = pair_energy(an, links_k, dminv, n, m, cp) - pair_energy(an, links_k, np.zeros_like(minv), n, m, cp)
    if cp.ke != 0.0:
        dh += cp.ke * mixed_occupation_derivative(an, minv[np.ix_(u, u)], links_k, ell, n, m, k, db)
    return dlogrho, dh


def _combine(an, rho, h, dlogrho):
    om = np.conj(an.c)[:, None] * an.c[None, :] * rho
    S = om.sum()
    e = (om * h).sum() / S
    dlogN = (om * dlogrho).sum() / S
    de = (om * (dlogrho * (h - e))).sum() / S
    return e, de, dlogN


def bond_sensitivities(an: Ansatz, links_k, cp: Couplings, k: int, E: np.ndarray):
    """(e, d e, d log N) of one configuration along generator E of bond k (definitional route:
    full Pfaffians for rho, dense inverses of every M_nm)."""
    K = an.K
    db = bond_state_derivative(an, k, E)
    rho = an.bond_overlaps() * an.cross_ratio_def(links_k)
    h = np.zeros((K, K), complex)
    dlogrho = np.zeros((K, K), complex)
    dh = np.zeros((K, K), complex)
    for n in range(K):
        for m in range(K):
            minv = np.linalg.inv(an.assemble_M(links_k, n, m))
            h[n, m] = pair_energy(an, links_k, minv, n, m, cp)
            if k in (n, m):
                dlogrho[n, m], dh[n, m] = _pair_derivatives(an, links_k, cp, n, m, k, db, minv)
    e, de, dlogN = _combine(an, rho, h, dlogrho)
    om = np.conj(an.c)[:, None] * an.c[None, :] * rho
    de += (om * dh).sum() / om.sum()
    return e, de, dlogN.real


def bond_gradient_from_samples(es, des, dlogNs, weights=None) -> float:
    """d<H>/d theta = mean[Re d e] + mean[(Re e - <H>) d log N] over samples of p(G)
    (or weighted by p(G))."""
    es = np.asarray(es).real
    w = np.full(len(es), 1.0 / len(es)) if weights is None else np.asarray(weights) / np.sum(weights)
    ebar = np.sum(w * es)
    return float(np.sum(w * np.asarray(des).real) + np.sum(w * (es - ebar) * np.asarray(dlogNs).real))


# ----- patch route: from G = M_00^-1 alone -----
def coefficient_contraction(an: Ansatz, links_k, cp: Couplings, G: np.ndarray) -> np.ndarray:
    """R[a, b] = sum_ij C_ij G[i, S_a] G[S_b, j] for the linear part of h in M^-1 with the reference
    bond's electric response on every link: C = B^T C_out B for the fermion terms (C_out the
    coefficients of Gamma_out) plus, per link, the slopes of X_l in (M^-1)_UU (read off the oracle's
    own affine X at unit steps)."""
    S = an.S
    Cout = energy_coefficients(an, links_k, cp)
    C = an.B.T @ Cout @ an.B
    if cp.ke != 0.0:
        for ell in range(an.lat.n_links):
            u = an.lat.link_majoranas(ell)
            x0 = an.mixed_occupation_patch(np.zeros((4, 4)), links_k, ell, 0, 0)
            for i in range(4):
                for j in range(i + 1, 4):
                    step = np.zeros((4, 4))
                    step[i, j], step[j, i] = 1.0, -1.0
                    C[u[i], u[j]] += cp.ke * (an.mixed_occupation_patch(step, links_k, ell, 0, 0) - x0)
    return G[:, S].T @ C @ G[S, :].T


def bond_sensitivities_patch(an: Ansatz, links_k, cp: Couplings, k: int, E: np.ndarray, G: np.ndarray,
                             h: np.ndarray, rho: np.ndarray, R: np.ndarray):
    """The same as ``bond_sensitivities`` from G, the pair energies h and weights rho and the
    contraction R: with M_nm^-1 = G - G_S Y G_S^T, Y = Delta (1 + G_SS Delta)^-1,
    dY = (1 - Y G_SS) dDelta (1 + G_SS Delta)^-1 and dM^-1 = -G_S dY G_S^T,
        d h_nm = -tr(dY R_nm^T) + ke dX_nm(patch link, explicit),
    R_nm = R + the change of the electric slopes on the pair's patch links (from G_SS)."""
    S = an.S
    pos = {int(v): i for i, v in enumerate(S)}
    s = len(S)
    gss = G[np.ix_(S, S)]
    db = bond_state_derivative(an, k, E)
    K = an.K
    ell_k = int(an.patch_link[k])
    uk = [pos[int(v)] for v in an.lat.link_majoranas(ell_k)]
    dlogrho = np.zeros((K, K), complex)
    dh = np.zeros((K, K), complex)
    for n in range(K):
        for m in range(K):
            if k not in (n, m):
                continue
            dl = an.delta_patch(links_k, n, m)
            A = np.eye(s) + gss @ dl
            Y = dl @ np.linalg.inv(A)
            minv_ss = gss - gss @ Y @ gss
            dg, dov_link = link_transition_derivative(an, ell_k, n, m, k, db)
            ddl = np.zeros((s, s), complex)
            ddl[np.ix_(uk, uk)] = an._rot_block(dg, links_k[ell_k])
            dlogr = 0.5 * np.trace(minv_ss @ ddl)
            dlogrho[n, m] = dov_link / an.link_transition(ell_k, n, m)[1] + dlogr
            dY = (np.eye(s) - Y @ gss) @ ddl @ np.linalg.inv(A)
            Rnm = R.copy()
            if cp.ke != 0.0:
                for ell in set(int(an.patch_link[q]) for q in (n, m) if q > 0):
                    u = [pos[int(v)] for v in an.lat.link_majoranas(ell)]
                    x0r = an.mixed_occupation_patch(np.zeros((4, 4)), links_k, ell, 0, 0)
                    x0p = an.mixed_occupation_patch(np.zeros((4, 4)), links_k, ell, n, m)
                    for i in range(4):
                        for j in range(i + 1, 4):
                            step = np.zeros((4, 4))
                            step[i, j], step[j, i] = 1.0, -1.0
                            dslope = ((an.mixed_occupation_patch(step, links_k, ell, n, m) - x0p)
                                      - (an.mixed_occupation_patch(step, links_k, ell, 0, 0) - x0r))
                            # C[u_i, u_j] changes by ke dslope: R += ke dslope G[u_i, S]^T G[S, u_j]^T
                            Rnm += cp.ke * dslope * np.outer(gss[u[i], :], gss[:, u[j]])
            dh[n, m] = -np.sum(dY * Rnm)
            if cp.ke != 0.0:
                dh[n, m] += cp.ke * mixed_occupation_derivative(an, minv_ss[np.ix_(uk, uk)], links_k, ell_k,
                                                                n, m, k, db)
    e, de, dlogN = _combine(an, rho, h, dlogrho)
    om = np.conj(an.c)[:, None] * an.c[None, :] * rho
    de += (om * dh).sum() / om.sum()
    return e, de, dlogN.real
