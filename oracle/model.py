"""Weights, cross terms and observables in covariance form (Sec. 3.2, 5, 5.1, 5.2).

Notation.  Gamma_loc (10x10) splits into the physical block a (2x2), the
physical-virtual block b (2x8) and the virtual block d (8x8).  Over the lattice
A = (+)_x a, B = (+)_x b, D = (+)_x d.  The gauge field rotates the two
Majoranas of the outgoing leg of each link by R(theta) = [[cos, sin], [-sin, cos]],
theta = 2 pi k / N: this is how exp(i theta n) acts on (c_0, c_1), and Sec. 5
writes the gauged tensor as Gamma_A(G) = O^T Gamma_A O.  Moving O onto the
bonds gives the virtual matrix
    M(G) = D + O(G) Gamma_B O(G)^T          (n x n, n = 8V, real antisymmetric).

* weight (Sec. 3.2, PEPS norm; Sec. 5 with n = m):
    W(G) = tr(rho_A(G) (rho_B x 1)) = sqrt(det(M/2)) = 2^-4V sqrt(det M),
  i.e. log W = (1/2) log det M - 4 V ln 2.  The physical block drops out
  because the projected state is pure (its covariance has determinant 1).
* physical covariance of the normalised projected state:
    Gamma_out = A + B M^-1 B^T.
* cross terms (Sec. 5):
    N_nm(G) = <psi_n(G)|psi_m(G)> = W(G) <B_m|B_n> Pf(M_nm) / Pf(M_00),
  with M_nm = D + O Gamma_nm O^T and Gamma_nm the covariance of the transition
  operator |B_n><B_m| / <B_m|B_n>; N(G) = sum_nm c_n^* c_m N_nm(G).
* observables: plaquette (Sec. 2.3), Wilson loops (Sec. 5.1), and fermionic
  two-point functions by Wick's theorem, <c_a c_b> = -i Gamma_out_ab (Sec. 3.2;
  the printed exponent of (-i) is read as w/2), combined over cross terms as
  in Sec. 5.2.
* electric field (Sec. 2.2, the H_E term; Sec. 5.3):
    f_E(G) = sum_g' <g|J^2|g'> sum_nm c_n^* c_m <psi_n(G)|psi_m(g'; G)> / N(G),
  g = g_ell, with psi_m(g'; G) the state of G with link ell set to g'.  For Z_N the
  Casimir is read as diagonal on the irreps j (eigenvalue e_j), irrep basis
  |j> = N^-1/2 sum_g w^(j g) |g>, w = exp(2 pi i / N).  The overlaps are Gaussian
  traces with the bond operator of link ell taken between U(g)^+ b_n and
  U(g')^+ b_m.  For Z2 with a maximally entangled bond that bond overlap is zero
  and the transition covariance does not exist, so the overlaps are evaluated
  through exp(i theta n_out) = 1 + (e^(i theta) - 1) n_out (n_out^2 = n_out): an
  overlap is affine in e^(i theta), and its slope is read at the regular angle
  THETA_REGULAR.
"""
from __future__ import annotations

import numpy as np

from . import gaussian
from .lattice import Lattice

NOBS = 21           # observable slots: plaq, wilson2x2, density, logN, meson r=1..16, electric
OBS_PLAQ, OBS_WILSON, OBS_DENSITY, OBS_LOGN, OBS_MESON0 = 0, 1, 2, 3, 4
OBS_ELECTRIC = 20
MAX_MESON = 16
THETA_REGULAR = np.pi / 2   # phase angle at which the mixed occupation is read off (Sec. 5.3)


def rotation(theta: float) -> np.ndarray:
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[c, s], [-s, c]])


def link_phase(k: int, group: int) -> complex:
    return np.exp(2j * np.pi * (int(k) % group) / group)


class Ansatz:
    """Covariance-form evaluator of one (superposed) ansatz on a lattice."""

    def __init__(self, lat: Lattice, gamma_loc, gamma_bond, group: int = 2,
                 patch_link=None, gamma_bond_k=None, c=None):
        self.lat = lat
        self.group = group
        g = np.asarray(gamma_loc, float)
        self.a, self.b, self.d = g[0:2, 0:2], g[0:2, 2:10], g[2:10, 2:10]
        V, n = lat.V, lat.n
        self.D = np.zeros((n, n))
        self.A = np.zeros((2 * V, 2 * V))
        self.B = np.zeros((2 * V, n))
        for x in range(V):
            self.D[8 * x:8 * x + 8, 8 * x:8 * x + 8] = self.d
            self.A[2 * x:2 * x + 2, 2 * x:2 * x + 2] = self.a
            self.B[2 * x:2 * x + 2, 8 * x:8 * x + 8] = self.b
        self.gamma_bond = np.asarray(gamma_bond, float)
        self.K = 1 if patch_link is None else len(patch_link)
        self.patch_link = np.array([-1] if patch_link is None else patch_link)
        self.c = np.ones(1, complex) if c is None else np.asarray(c, complex)
        self._link_states(gamma_bond_k)

    # ----- superposed bonds (Sec. 5: reference bond B_0 and <B_n|B_0> real) -----
    def _link_states(self, gamma_bond_k):
        cs2 = gaussian.majorana_matrices(2)
        self._cs2 = cs2
        self._trans_cache = {}
        v0 = gaussian.state_of_covariance(self.gamma_bond, 2, cs2)
        self.bstate = [v0]
        for k in range(1, self.K):
            vk = gaussian.state_of_covariance(np.asarray(gamma_bond_k[k]), 2, cs2)
            ov = np.vdot(v0, vk)
            self.bstate.append(vk * (abs(ov) / ov))         # <b_0|b_k> > 0
        S = []
        for k in range(1, self.K):
            S.extend(self.lat.link_majoranas(int(self.patch_link[k])).tolist())
        self.S = np.array(sorted(set(S)), int)

    def link_transition(self, ell: int, n: int, m: int):
        """(covariance, overlap <bra|ket>) of link ell in the transition |B_n><B_m|."""
        key = (int(ell), int(n), int(m))
        if key not in self._trans_cache:
            self._trans_cache[key] = self._link_transition(*key)
        return self._trans_cache[key]

    def bond_vectors(self, ell: int, n: int, m: int):
        """(ket, bra): two-mode bond states of link ell in the transition |B_n><B_m|."""
        ket = self.bstate[n] if (n > 0 and self.patch_link[n] == ell) else self.bstate[0]
        bra = self.bstate[m] if (m > 0 and self.patch_link[m] == ell) else self.bstate[0]
        return ket, bra

    def _link_transition(self, ell: int, n: int, m: int):
        ket, bra = self.bond_vectors(ell, n, m)
        ov = np.vdot(bra, ket)
        if ket is bra:
            cov = gaussian.covariance_of_state(ket, 2, self._cs2)
        else:
            cov = gaussian.transition_covariance(bra, ket, 2, self._cs2)
        return cov, ov

    def bond_overlap(self, n: int, m: int) -> complex:
        """<B_m|B_n>: product over links of the link overlaps."""
        ov = 1.0 + 0j
        for ell in set(int(self.patch_link[k]) for k in (n, m) if k > 0):
            ov *= self.link_transition(ell, n, m)[1]
        return ov

    # ----- virtual matrices -----
    def _rot_block(self, gamma4, k: int):
        o = np.eye(4)
        o[0:2, 0:2] = rotation(2 * np.pi * (int(k) % self.group) / self.group)
        return o @ gamma4 @ o.T

    def assemble_M(self, links_k, n: int = 0, m: int = 0) -> np.ndarray:
        """M_nm(G) = D + O(G) Gamma_nm O(G)^T (n = m = 0: the reference bond)."""
        lat = self.lat
        patch = set(int(self.patch_link[k]) for k in (n, m) if k > 0)
        cplx = bool(patch)
        M = self.D.astype(complex) if cplx else self.D.copy()
        for ell in range(lat.n_links):
            u = lat.link_majoranas(ell)
            g4 = self.link_transition(ell, n, m)[0] if ell in patch else self.gamma_bond
            M[np.ix_(u, u)] += self._rot_block(g4, links_k[ell])
        return M

    def log_weight(self, links_k) -> float:
        sign, ld = np.linalg.slogdet(self.assemble_M(links_k))
        if sign <= 0:
            return -np.inf
        return 0.5 * ld - 4 * self.lat.V * np.log(2.0)

    def weight(self, links_k) -> float:
        return float(np.exp(self.log_weight(links_k)))

    def gamma_out(self, Ginv: np.ndarray) -> np.ndarray:
        return self.A + self.B @ Ginv @ self.B.T

    def cross_ratio_def(self, links_k) -> np.ndarray:
        """r_nm(G) = Pf(M_nm) / Pf(M_00) by full Pfaffians (the definitional route)."""
        pf0 = gaussian.pfaffian(self.assemble_M(links_k))
        r = np.zeros((self.K, self.K), complex)
        for n in range(self.K):
            for m in range(self.K):
                r[n, m] = gaussian.pfaffian(self.assemble_M(links_k, n, m)) / pf0
        return r

    def bond_overlaps(self) -> np.ndarray:
        """ov[n, m] = <B_m|B_n>."""
        if not hasattr(self, "_ov"):
            self._ov = np.array([[self.bond_overlap(n, m) for m in range(self.K)]
                                 for n in range(self.K)])
        return self._ov

    def cross_terms(self, links_k) -> np.ndarray:
        """N_nm(G) = W(G) <B_m|B_n> Pf(M_nm)/Pf(M_00)."""
        return self.weight(links_k) * self.bond_overlaps() * self.cross_ratio_def(links_k)

    def norm(self, links_k) -> float:
        """N(G) = sum_nm c_n^* c_m N_nm(G)."""
        N = self.cross_terms(links_k)
        return float(np.real(np.conj(self.c) @ N @ self.c))

    def s_factor_def(self, links_k) -> complex:
        """S(G) = N(G)/W(G) = sum_nm c_n^* c_m <B_m|B_n> r_nm(G)."""
        return np.conj(self.c) @ (self.bond_overlaps() * self.cross_ratio_def(links_k)) @ self.c

    # ----- patch route (Woodbury-friendly): only G restricted to the patch Majoranas -----
    def delta_patch(self, links_k, n: int, m: int) -> np.ndarray:
        """Delta^nm = (M_nm - M_00) restricted to the patch Majoranas S."""
        S = self.S
        pos = {int(v): i for i, v in enumerate(S)}
        dl = np.zeros((len(S), len(S)), complex)
        for ell in set(int(self.patch_link[k]) for k in (n, m) if k > 0):
            u = self.lat.link_majoranas(ell)
            g4 = self.link_transition(ell, n, m)[0] - self.gamma_bond
            blk = self._rot_block(g4, links_k[ell])
            iu = [pos[int(v)] for v in u]
            dl[np.ix_(iu, iu)] += blk
        return dl

    def cross_ratio_patch(self, G_SS: np.ndarray, links_k) -> np.ndarray:
        """r_nm = Pf(M_00 + Delta)/Pf(M_00) = (-1)^(s/2) Pf([[G_SS, I], [-I, Delta_SS]])."""
        s = len(self.S)
        r = np.ones((self.K, self.K), complex)
        for n in range(self.K):
            for m in range(self.K):
                if n == 0 and m == 0:
                    continue
                blk = np.zeros((2 * s, 2 * s), complex)
                blk[:s, :s] = G_SS
                blk[:s, s:] = np.eye(s)
                blk[s:, :s] = -np.eye(s)
                blk[s:, s:] = self.delta_patch(links_k, n, m)
                r[n, m] = (-1) ** (s // 2) * gaussian.pfaffian(blk)
        return r

    def s_factor_patch(self, G_SS, links_k) -> complex:
        return np.conj(self.c) @ (self.bond_overlaps() * self.cross_ratio_patch(G_SS, links_k)) @ self.c

    # ----- electric field (Sec. 2.2 electric term, Sec. 5.3) -----
    def casimir_kernel(self, spectrum) -> np.ndarray:
        """kappa[D] = <g|J^2|g'> for g - g' = D (mod N): (1/N) sum_j e_j w^(j D)."""
        N = self.group
        e = np.asarray(spectrum, complex)
        return np.array([sum(e[j] * np.exp(2j * np.pi * j * D / N) for j in range(N)) / N
                         for D in range(N)])

    @staticmethod
    def out_phase(theta: float) -> np.ndarray:
        """exp(i theta n_out) on a link's two-mode space (mode 0 = out, the high bit)."""
        e = np.exp(1j * theta)
        return np.diag([1.0, 1.0, e, e])

    def shifted_transition(self, links_k, ell: int, theta: float, n: int, m: int):
        """(covariance, overlap <bra|ket>) of link ell's bond operator in
        <psi_n(G)|psi_m(G; theta)>, psi_m(G; theta) = <B_m|U(G) exp(i theta n_out)|A>:
        ket U(g)^+ b_n, bra U(g)^+ exp(-i theta n_out) b_m."""
        ket, bra = self.bond_vectors(ell, n, m)
        u = self.out_phase(2 * np.pi * (int(links_k[ell]) % self.group) / self.group).conj()
        ket = u @ ket
        bra = u @ self.out_phase(-theta) @ bra
        cov = gaussian.transition_covariance(bra, ket, 2, self._cs2)
        return cov, np.vdot(bra, ket)

    def shifted_overlap_def(self, links_k, ell: int, theta: float, n: int, m: int) -> complex:
        """<psi_n(G)|psi_m(G; theta)> by full Pfaffians (theta = 2 pi d / N: link ell set to g + d)."""
        M = self.assemble_M(links_k, n, m).astype(complex)
        u = self.lat.link_majoranas(ell)
        cov, ov = self.shifted_transition(links_k, ell, theta, n, m)
        M[np.ix_(u, u)] = self.D[np.ix_(u, u)] + cov
        for l2 in set(int(self.patch_link[k]) for k in (n, m) if k > 0):
            if l2 != ell:
                ov *= self.link_transition(l2, n, m)[1]
        pf0 = gaussian.pfaffian(self.assemble_M(links_k))
        return self.weight(links_k) * ov * gaussian.pfaffian(M) / pf0

    def electric_def(self, links_k, ell: int, spectrum) -> complex:
        """f_E(G) on link ell from its definition: the sum over g' of <g|J^2|g'> times the
        superposed overlaps, divided by N(G)."""
        N, g = self.group, int(links_k[ell]) % self.group
        kap = self.casimir_kernel(spectrum)
        e0 = np.exp(1j * THETA_REGULAR) - 1.0
        num = den = 0.0 + 0j
        for n in range(self.K):
            for m in range(self.K):
                w = np.conj(self.c[n]) * self.c[m]
                o0 = self.shifted_overlap_def(links_k, ell, 0.0, n, m)
                slope = (self.shifted_overlap_def(links_k, ell, THETA_REGULAR, n, m) - o0) / e0
                for gp in range(N):
                    ov = o0 + (np.exp(2j * np.pi * (gp - g) / N) - 1.0) * slope
                    num += w * kap[(g - gp) % N] * ov
                den += w * o0
        return num / den

    def mixed_occupation_patch(self, ginv_uu: np.ndarray, links_k, ell: int, n: int, m: int) -> complex:
        """X_nm = <psi_n(G)|psi_m(G; theta)> slope / <psi_n|psi_m>, from the 4x4 block of
        M_nm^-1 on link ell: the patch lemma gives the ratio of the theta overlap to the
        theta = 0 one as [ov(theta)/ov(0)] Pf([[G_UU, 1], [-1, Delta]]), Delta the change of
        the link block."""
        c0, o0 = self.shifted_transition(links_k, ell, 0.0, n, m)
        ct, ot = self.shifted_transition(links_k, ell, THETA_REGULAR, n, m)
        blk = np.zeros((8, 8), complex)
        blk[:4, :4] = ginv_uu
        blk[:4, 4:] = np.eye(4)
        blk[4:, :4] = -np.eye(4)
        blk[4:, 4:] = ct - c0
        ratio = (ot / o0) * gaussian.pfaffian(blk)
        return (ratio - 1.0) / (np.exp(1j * THETA_REGULAR) - 1.0)

    def electric_patch(self, links_k, ell: int, spectrum, ginv, wts) -> complex:
        """f_E(G) on link ell from M_nm^-1 (ginv[n][m], full n x n) and the cross weights
        wts[n, m] = c_n^* c_m <B_m|B_n> r_nm (K = 1: [[1]])."""
        N, g = self.group, int(links_k[ell]) % self.group
        kap = self.casimir_kernel(spectrum)
        u = self.lat.link_majoranas(ell)
        num = 0.0 + 0j
        for n in range(self.K):
            for m in range(self.K):
                x = self.mixed_occupation_patch(ginv[n][m][np.ix_(u, u)], links_k, ell, n, m)
                for gp in range(N):
                    num += wts[n, m] * kap[(g - gp) % N] * (1.0 + (np.exp(2j * np.pi * (gp - g) / N) - 1.0) * x)
        return num / np.sum(wts)

    def electric_mean(self, links_k, ginv, wts) -> float:
        """Lattice mean over links of Re f_E with e_0 = 0 and e_j = 1 otherwise (the flux
        carried by the link in units of the Casimir of the non-trivial irreps)."""
        spec = np.ones(self.group)
        spec[0] = 0.0
        tot = sum(self.electric_patch(links_k, ell, spec, ginv, wts).real for ell in range(self.lat.n_links))
        return tot / self.lat.n_links

    # ----- observables -----
    def plaquette_value(self, links_k, x: int) -> complex:
        """U(x,e1) U(x+e1,e2) U(x+e2,e1)^* U(x,e2)^* (Sec. 2.3), the plaquette with lower-left corner x."""
        N = self.group
        l1, l2, l3, l4 = self.lat.plaquette_links(x)
        return (link_phase(links_k[l1], N) * link_phase(links_k[l2], N)
                * np.conj(link_phase(links_k[l3], N)) * np.conj(link_phase(links_k[l4], N)))

    def plaquette(self, links_k) -> float:
        """Lattice mean of Re of the plaquette (Sec. 2.3)."""
        return sum(self.plaquette_value(links_k, x).real for x in range(self.lat.V)) / self.lat.V

    def wilson2x2_value(self, links_k, x: int) -> complex:
        """Oriented product of the 8 links around the 2x2 square with lower-left corner x (Sec. 5.1)."""
        lat, N = self.lat, self.group
        z = 1.0 + 0j
        p = x
        for _ in range(2):                   # along +e1
            z *= link_phase(links_k[lat.link(p, 0)], N)
            p = lat.shift(p, 1, 0)
        for _ in range(2):                   # along +e2
            z *= link_phase(links_k[lat.link(p, 1)], N)
            p = lat.shift(p, 0, 1)
        for _ in range(2):                   # along -e1
            p = lat.shift(p, -1, 0)
            z *= np.conj(link_phase(links_k[lat.link(p, 0)], N))
        for _ in range(2):                   # along -e2
            p = lat.shift(p, 0, -1)
            z *= np.conj(link_phase(links_k[lat.link(p, 1)], N))
        return z

    def wilson2x2(self, links_k) -> float:
        """Lattice mean of Re of the 2x2 Wilson loop."""
        return sum(self.wilson2x2_value(links_k, x).real for x in range(self.lat.V)) / self.lat.V

    def density_from(self, gout: np.ndarray) -> complex:
        """Lattice mean of <psi_p^+ psi_p> = (1 + Gamma_out[2x, 2x+1]) / 2."""
        V = self.lat.V
        return np.mean([(1.0 + gout[2 * x, 2 * x + 1]) / 2.0 for x in range(V)])

    def meson_from(self, gout: np.ndarray, links_k, r: int) -> complex:
        """(1/V) sum_x 2 Re-part-to-be of [prod_j<r U(x+j e1, e1)] <phi_x^+ phi_{x+r e1}>.

        <phi_x^+ phi_y> = (1/4)[<c_x0 c_y0> + i<c_x0 c_y1> - i<c_x1 c_y0> + <c_x1 c_y1>]
        with phi = (c_0 + i c_1)/2 and <c_a c_b> = -i Gamma_out_ab.  Returns the
        (complex, for transition covariances) mean of 2 x (line x bilinear).
        """
        lat, N = self.lat, self.group
        tot = 0.0 + 0j
        for x in range(lat.V):
            y = x
            line = 1.0 + 0j
            for _ in range(r):
                line *= link_phase(links_k[lat.link(y, 0)], N)
                y = lat.shift(y, 1, 0)
            cc = lambda a, b: -1j * gout[a, b]
            bil = 0.25 * (cc(2 * x, 2 * y) + 1j * cc(2 * x, 2 * y + 1)
                          - 1j * cc(2 * x + 1, 2 * y) + cc(2 * x + 1, 2 * y + 1))
            tot += 2.0 * line * bil
        return tot / lat.V

    def fermion_obs(self, gout, links_k) -> np.ndarray:
        out = np.zeros(NOBS, complex)
        out[OBS_DENSITY] = self.density_from(gout)
        for r in range(1, min(self.lat.Lx // 2, MAX_MESON) + 1):
            out[OBS_MESON0 + r - 1] = self.meson_from(gout, links_k, r)
        return out

    def observables(self, links_k, Ginv=None) -> np.ndarray:
        """All observable slots for one configuration (Sec. 5.1, 5.2, 5.3), real parts."""
        if Ginv is None:
            Ginv = np.linalg.inv(self.assemble_M(links_k))
        out = np.zeros(NOBS)
        out[OBS_PLAQ] = self.plaquette(links_k)
        out[OBS_WILSON] = self.wilson2x2(links_k)
        lw = self.log_weight(links_k)
        if self.K == 1:
            f = self.fermion_obs(self.gamma_out(Ginv), links_k)
            out[OBS_LOGN] = lw
            out[OBS_ELECTRIC] = self.electric_mean(links_k, [[Ginv]], np.ones((1, 1)))
        else:
            ov = self.bond_overlaps()
            r = self.cross_ratio_def(links_k)
            wts = np.conj(self.c)[:, None] * self.c[None, :] * ov * r
            S = wts.sum()
            f = np.zeros(NOBS, complex)
            ginv = [[None] * self.K for _ in range(self.K)]
            for n in range(self.K):
                for m in range(self.K):
                    ginv[n][m] = np.linalg.inv(self.assemble_M(links_k, n, m))
                    gnm = self.A + self.B @ ginv[n][m] @ self.B.T
                    f += wts[n, m] / S * self.fermion_obs(gnm, links_k)
            out[OBS_LOGN] = lw + np.log(S.real)
            out[OBS_ELECTRIC] = self.electric_mean(links_k, ginv, wts)
        keep = [OBS_DENSITY] + [OBS_MESON0 + i for i in range(MAX_MESON)]
        out[keep] = f[keep].real
        return out

    def transition_inverse_factor(self, G: np.ndarray, links_k, n: int, m: int) -> np.ndarray:
        """Y_nm with M_nm^-1 = G - G[:,S] Y_nm G[S,:]: M_nm = M_00 + Delta, Delta nonzero only on the
        patch Majoranas S, so by the Woodbury identity Y = Delta_SS (1 + G_SS Delta_SS)^-1 (this form
        needs no inverse of Delta, which is singular on the patch links a pair does not involve)."""
        S = self.S
        dl = self.delta_patch(links_k, n, m)
        return dl @ np.linalg.inv(np.eye(len(S)) + G[np.ix_(S, S)] @ dl)

    def observables_from_inverse(self, links_k, G: np.ndarray, logw=None) -> np.ndarray:
        """The observable slots of ``observables`` from G = M(G)^-1 alone (a maintained inverse, or a
        fresh one of a lattice too large for the full Pfaffians and inverses of every M_nm): the cross
        ratios by the patch lemma on G_SS, and M_nm^-1 by the Woodbury correction of
        ``transition_inverse_factor``; log W from a fresh determinant unless given."""
        G = np.asarray(G, float)
        out = np.zeros(NOBS)
        out[OBS_PLAQ] = self.plaquette(links_k)
        out[OBS_WILSON] = self.wilson2x2(links_k)
        lw = self.log_weight(links_k) if logw is None else logw
        gbb = self.B @ G @ self.B.T
        if self.K == 1:
            f = self.fermion_obs(self.A + gbb, links_k)
            out[OBS_LOGN] = lw
            out[OBS_ELECTRIC] = self.electric_mean(links_k, [[G]], np.ones((1, 1)))
        else:
            S = self.S
            r = self.cross_ratio_patch(G[np.ix_(S, S)], links_k)
            wts = np.conj(self.c)[:, None] * self.c[None, :] * self.bond_overlaps() * r
            Stot = wts.sum()
            f = np.zeros(NOBS, complex)
            blocks = [[None] * self.K for _ in range(self.K)]
            bgs = self.B @ G[:, S]
            gsb = G[S, :] @ self.B.T
            for n in range(self.K):
                for m in range(self.K):
                    Y = self.transition_inverse_factor(G, links_k, n, m)
                    f += wts[n, m] / Stot * self.fermion_obs(self.A + gbb - bgs @ Y @ gsb, links_k)
                    blocks[n][m] = _WoodburyBlocks(G, S, Y)
            out[OBS_LOGN] = lw + np.log(Stot.real)
            out[OBS_ELECTRIC] = self.electric_mean(links_k, blocks, wts)
        keep = [OBS_DENSITY] + [OBS_MESON0 + i for i in range(MAX_MESON)]
        out[keep] = f[keep].real
        return out


class _WoodburyBlocks:
    """Index access M_nm^-1[np.ix_(u, v)] = G[u,v] - G[u,S] Y G[S,v] without forming M_nm^-1."""

    def __init__(self, G, S, Y):
        self.G, self.S, self.Y = G, S, Y

    def __getitem__(self, idx):
        u, v = idx
        u, v = np.ravel(u), np.ravel(v)
        return self.G[np.ix_(u, v)] - self.G[np.ix_(u, self.S)] @ self.Y @ self.G[np.ix_(self.S, v)]

