"""Brute-force Fock-space contraction of the gauged (superposed) PEPS (Sec. 3, 3.1, 4).

For a gauge configuration G the physical state of bond superposition n is
  psi_n(G) = <B_n| U(G) |A>,
with |A> the product of on-site Gaussian states, U(G) = prod_links exp(i theta_l n_out(l))
acting on the outgoing virtual leg of each link, and <B_n| the product of
bond states (Sec. 3.1, gauged PEPS; Sec. 4, the superposed ansatz).  Each
bond state is an even 2-mode state (alpha + beta psi_out^+ psi_in^+)|0>, so
the partial contraction is the product over links of the even operators
  |0><b|_l = (1 - n_out)(1 - n_in)(conj(alpha) + conj(beta) psi_in psi_out),
applied to U(G)|A>; afterwards every virtual mode is empty and the surviving
amplitudes are those of psi_n(G) on the V physical modes.

The vector is kept sparse (index, amplitude), which keeps 2x2 lattices (20 modes,
2^20 basis states) cheap.  Everything here is exact linear algebra in the
Jordan-Wigner basis of ``gaussian``; nothing uses covariance-matrix formulas.
"""
from __future__ import annotations

import numpy as np

from . import gaussian
from .lattice import Lattice, SLOT_P


def _parity_before(idx: np.ndarray, mode: int, n_modes: int) -> np.ndarray:
    """(-1)^(number of occupied modes with index < mode) for each basis index."""
    full = (1 << n_modes) - 1
    mask = full ^ ((1 << (n_modes - mode)) - 1)
    cnt = np.bitwise_count(idx & np.int64(mask))
    return 1 - 2 * (cnt & 1).astype(np.int64)


def product_state(v_loc: np.ndarray, n_sites: int, tol: float = 1e-13):
    """Sparse |A> = prod over sites (in site order) of a 5-mode local state."""
    nz = np.nonzero(np.abs(v_loc) > tol)[0]
    idx = np.zeros(1, np.int64)
    amp = np.ones(1, complex)
    for _ in range(n_sites):
        idx = (idx[:, None] << 5 | nz[None, :]).reshape(-1)
        amp = (amp[:, None] * v_loc[nz][None, :]).reshape(-1)
    return idx, amp


def _merge(idx: np.ndarray, amp: np.ndarray):
    u, inv = np.unique(idx, return_inverse=True)
    re = np.bincount(inv, weights=amp.real, minlength=len(u))
    im = np.bincount(inv, weights=amp.imag, minlength=len(u))
    return u, re + 1j * im


def contract_bond(idx, amp, mode_out, mode_in, alpha, beta, n_modes):
    """Apply |0><b| on modes (out, in) for |b> = (alpha + beta psi_out^+ psi_in^+)|0>."""
    bo = np.int64(1 << (n_modes - 1 - mode_out))
    bi = np.int64(1 << (n_modes - 1 - mode_in))
    occ_o = (idx & bo) != 0
    occ_i = (idx & bi) != 0
    s00 = ~occ_o & ~occ_i
    s11 = occ_o & occ_i
    idx0, amp0 = idx[s00], amp[s00] * np.conj(alpha)
    i11 = idx[s11]
    sgn = _parity_before(i11, mode_out, n_modes)          # psi_out acts first
    i11b = i11 ^ bo
    sgn = sgn * _parity_before(i11b, mode_in, n_modes)    # then psi_in
    idx1 = i11b ^ bi
    amp1 = amp[s11] * np.conj(beta) * sgn
    return _merge(np.concatenate([idx0, idx1]), np.concatenate([amp0, amp1]))


def link_state_amplitudes(gamma4: np.ndarray):
    """(alpha, beta) of the even 2-mode state with covariance gamma4 (order out0,out1,in0,in1).

    Global phase fixed so that the amplitude of largest modulus is real positive;
    callers fix relative phases of superposed bonds themselves.
    """
    v = gaussian.state_of_covariance(gamma4, 2)
    # basis |n_out n_in>: index 0 = |00>, 3 = |11> = psi_out^+ psi_in^+|0>
    if abs(v[1]) > 1e-10 or abs(v[2]) > 1e-10:
        raise ValueError("bond state is not even")
    a, b = v[0], v[3]
    ph = a / abs(a) if abs(a) >= abs(b) else b / abs(b)
    return a / ph, b / ph


def physical_state(lat: Lattice, v_loc: np.ndarray, links_k: np.ndarray, group: int,
                   bond_ab: np.ndarray) -> np.ndarray:
    """psi(G) = <B|U(G)|A> as a dense vector over the V physical modes.

    bond_ab: (n_links, 2) complex amplitudes (alpha, beta) of each link's bond state.
    """
    V = lat.V
    n_modes = 5 * V
    idx, amp = product_state(v_loc, V)
    # U(G): phase exp(i theta) on states with the outgoing virtual mode occupied
    for ell in range(lat.n_links):
        kl = int(links_k[ell]) % group
        if kl == 0:
            continue
        mo, _ = lat.link_modes(ell)
        occ = (idx >> np.int64(n_modes - 1 - mo)) & 1
        amp = amp * np.where(occ == 1, np.exp(2j * np.pi * kl / group), 1.0)
    for ell in range(lat.n_links):
        mo, mi = lat.link_modes(ell)
        idx, amp = contract_bond(idx, amp, mo, mi, bond_ab[ell, 0], bond_ab[ell, 1], n_modes)
    # surviving basis states have empty virtual modes; read the physical bits
    phys = np.zeros(len(idx), np.int64)
    for x in range(V):
        bit = (idx >> np.int64(n_modes - 1 - (5 * x + SLOT_P))) & 1
        phys |= bit << np.int64(V - 1 - x)
    out = np.zeros(2 ** V, complex)
    np.add.at(out, phys, amp)
    return out


class FockPEPS:
    """Brute-force evaluator for one ansatz on a small lattice."""

    def __init__(self, lat: Lattice, gamma_loc: np.ndarray, gamma_bond: np.ndarray,
                 group: int = 2, patch_link=None, gamma_bond_k=None):
        self.lat = lat
        self.group = group
        self.v_loc = gaussian.state_of_covariance(gamma_loc, 5)
        a0, b0 = link_state_amplitudes(gamma_bond)
        self.bond0 = np.array([a0, b0])
        self.K = 1 if patch_link is None else len(patch_link)
        self.patch_link = [-1] if patch_link is None else list(patch_link)
        self.bond_k = [self.bond0]
        for k in range(1, self.K):
            a, b = link_state_amplitudes(gamma_bond_k[k])
            ov = np.conj(a0) * a + np.conj(b0) * b          # <b_0|b_k>
            ph = ov / abs(ov)                                # phase convention <b_0|b_k> > 0
            self.bond_k.append(np.array([a, b]) / ph)
        self._cs = None

    def bonds_for(self, k: int) -> np.ndarray:
        ab = np.tile(self.bond0, (self.lat.n_links, 1)).astype(complex)
        if k > 0:
            ab[self.patch_link[k]] = self.bond_k[k]
        return ab

    def states(self, links_k) -> list[np.ndarray]:
        return [physical_state(self.lat, self.v_loc, links_k, self.group, self.bonds_for(k))
                for k in range(self.K)]

    def weight(self, links_k) -> float:
        """W(G) = <psi(G)|psi(G)> for the reference bond (K = 1 weight)."""
        phi = physical_state(self.lat, self.v_loc, links_k, self.group, self.bonds_for(0))
        return float(np.vdot(phi, phi).real)

    def cross_terms(self, links_k) -> np.ndarray:
        """N_nm(G) = <psi_n(G)|psi_m(G)> (Sec. 5, norm of the superposed state)."""
        ph = self.states(links_k)
        return np.array([[np.vdot(ph[n], ph[m]) for m in range(self.K)] for n in range(self.K)])

    def majoranas(self):
        if self._cs is None:
            self._cs = gaussian.majorana_matrices(self.lat.V)
        return self._cs

    def covariance_out(self, links_k, n: int = 0, m: int = 0) -> np.ndarray:
        """Physical (transition) covariance (i/2)<psi_n|[c_a,c_b]|psi_m>/<psi_n|psi_m>."""
        ph = self.states(links_k) if self.K > 1 else [
            physical_state(self.lat, self.v_loc, links_k, self.group, self.bonds_for(0))]
        return gaussian.transition_covariance(ph[n], ph[m], self.lat.V, self.majoranas())

    def expect(self, links_k, op: np.ndarray, c=None) -> complex:
        """sum_nm c_n^* c_m <psi_n|op|psi_m> / N(G) for a dense physical operator."""
        ph = self.states(links_k)
        c = np.ones(1) if c is None else np.asarray(c)
        psi = sum(c[k] * ph[k] for k in range(self.K))
        return np.vdot(psi, op @ psi) / np.vdot(psi, psi)

    def electric(self, links_k, ell: int, spectrum, c=None) -> complex:
        """f_E(G) on link ell (Sec. 5.3) from dense states: J^2 is built in the group basis as
        F diag(e) F^+ with the irrep columns F[g, j] = N^-1/2 w^(j g), and every overlap
        <psi_n(G)|psi_m(g'; G)> is an inner product of contracted vectors."""
        N = self.group
        w = np.exp(2j * np.pi / N)
        F = np.array([[w ** (j * g) for j in range(N)] for g in range(N)]) / np.sqrt(N)
        J2 = F @ np.diag(np.asarray(spectrum, complex)) @ F.conj().T
        c = np.ones(1) if c is None else np.asarray(c)
        k = np.asarray(links_k).copy()
        g = int(k[ell]) % N
        ph = self.states(k)
        psi = sum(c[n] * ph[n] for n in range(self.K))
        num = 0.0 + 0j
        for gp in range(N):
            k2 = k.copy()
            k2[ell] = gp
            ph2 = self.states(k2)
            psi2 = sum(c[m] * ph2[m] for m in range(self.K))
            num += J2[g, gp] * np.vdot(psi, psi2)
        return num / np.vdot(psi, psi)



# ----- Hamiltonian (Sec. 2, 2.2, 2.3) on dense vectors -----
def annihilators(n_modes: int) -> list[np.ndarray]:
    """psi_j = (prod_{k<j} Z_k) |0><1|_j, mode 0 the highest bit (the basis of ``gaussian``)."""
    Z = np.diag([1.0, -1.0]).astype(complex)
    lower = np.array([[0.0, 1.0], [0.0, 0.0]], complex)
    I2 = np.eye(2, dtype=complex)
    ops = []
    for j in range(n_modes):
        m = np.eye(1, dtype=complex)
        for k in range(n_modes):
            m = np.kron(m, Z if k < j else (lower if k == j else I2))
        ops.append(m)
    return ops


def fermion_hamiltonian(lat: Lattice, links_k, group: int, cp, eta, ann) -> np.ndarray:
    """<G|H|G> on the physical modes: hopping with D(g) = w^g and the pi-flux phases eta,
    chemical and staggered mass terms, and the plaquette term times the identity."""
    V = lat.V
    w = np.exp(2j * np.pi / group)
    H = np.zeros((2 ** V, 2 ** V), complex)
    for x in range(V):
        nx = ann[x].conj().T @ ann[x]
        x1, x2 = lat.coords(x)
        H += cp.mu * nx + cp.m * (-1) ** (x1 + x2) * nx
        for mu in range(2):
            y = lat.shift(x, 1, 0) if mu == 0 else lat.shift(x, 0, 1)
            T = 1j * eta(lat, x, mu) * w ** int(links_k[lat.link(x, mu)]) * (ann[x].conj().T @ ann[y])
            H += cp.t * (T + T.conj().T)
        l1, l2, l3, l4 = lat.plaquette_links(x)
        z = w ** int(links_k[l1] + links_k[l2] - links_k[l3] - links_k[l4])
        H += cp.kb * (z + np.conj(z)) * np.eye(2 ** V)
    return H


def _unit_casimir(group: int) -> np.ndarray:
    """J^2 on one link in the group basis: 0 on the trivial irrep, 1 on the others."""
    w = np.exp(2j * np.pi / group)
    F = np.array([[w ** (j * g) for j in range(group)] for g in range(group)]) / np.sqrt(group)
    e = np.ones(group)
    e[0] = 0.0
    return F @ np.diag(e) @ F.conj().T


def fock_local_energy(fk: "FockPEPS", links_k, cp, eta, c) -> complex:
    """E_loc(G) = [<psi(G)|H(G)|psi(G)> + ke sum_l sum_g' <g|J^2|g'> <psi(G)|psi(g'; G)>] / <psi|psi>."""
    k = np.asarray(links_k)
    ph = fk.states(k)
    psi = sum(c[n] * ph[n] for n in range(fk.K))
    Hf = fermion_hamiltonian(fk.lat, k, fk.group, cp, eta, annihilators(fk.lat.V))
    den = np.vdot(psi, psi)
    num = np.vdot(psi, Hf @ psi)
    if cp.ke != 0.0:
        spec = np.ones(fk.group)
        spec[0] = 0.0
        for ell in range(fk.lat.n_links):
            num += cp.ke * fk.electric(k, ell, spec, c) * den
    return num / den


def subspace_matrices(fk: "FockPEPS", cp, eta):
    """<Psi_n|H|Psi_m> and <Psi_n|Psi_m> for Psi_n = sum_G |G> (x) psi_n(G) on the full
    gauge (x) fermion space; the electric term acts as J^2 on each link's axis."""
    import itertools
    lat, N, V, K = fk.lat, fk.group, fk.lat.V, fk.K
    nl = lat.n_links
    shape = [N] * nl + [2 ** V]
    Psi = [np.zeros(shape, complex) for _ in range(K)]
    HPsi = [np.zeros(shape, complex) for _ in range(K)]
    ann = annihilators(V)
    for G in itertools.product(range(N), repeat=nl):
        k = np.array(G)
        ph = fk.states(k)
        Hf = fermion_hamiltonian(lat, k, N, cp, eta, ann)
        for n in range(K):
            Psi[n][G] = ph[n]
            HPsi[n][G] = Hf @ ph[n]
    if cp.ke != 0.0:
        J2 = _unit_casimir(N)
        for n in range(K):
            for ell in range(nl):
                HPsi[n] += cp.ke * np.moveaxis(np.tensordot(J2, Psi[n], axes=([1], [ell])), 0, ell)
    Hm = np.array([[np.vdot(Psi[a], HPsi[b]) for b in range(K)] for a in range(K)])
    Nm = np.array([[np.vdot(Psi[a], Psi[b]) for b in range(K)] for a in range(K)])
    return Hm, Nm
