"""Non-abelian link groups on multi-mode virtual legs: weights in covariance form (Sec. 2.1, 3.2, 5).

TEST INFRASTRUCTURE ONLY (see the package header): nothing in the product path imports this module.
Parity unpinned parts: none; the weight is pinned against the Fock-space contraction below
(tests/test_oracle_nonabelian.py).  No GPU kernel implements this model yet.

Sec. 2.1 gives the link Hilbert space of a compact (or finite) group G: a link configuration is a group
element g per link, and a matter or virtual index transforming in an irrep j picks up the unitary
D^j(g).  Here every virtual leg carries d fermionic modes (psi_1 .. psi_d) on which the link's element
acts by the d-dimensional irrep D(g), psi^+_b -> sum_a D(g)_ab psi^+_a, through the Gaussian unitary
V(D) = exp(i psi^+ H psi) with D = exp(iH).  On the leg's 2d Majoranas (c_2k = psi_k + psi_k^+,
c_2k+1 = -i (psi_k - psi_k^+), Sec. 3.2) V c_b V^+ = sum_a O_ab c_a with, for D = X + iY,
    O[2k][2j] = X_kj,  O[2k+1][2j] = Y_kj,  O[2k][2j+1] = -Y_kj,  O[2k+1][2j+1] = X_kj,
an orthogonal matrix and a representation of G (O(D D') = O(D) O(D')).

Layout of a site (the Z_N model of `model` with d modes per leg): n_phys physical modes, then the
legs +e1 (out), +e2 (out), -e1 (in), -e2 (in), d modes each; Gamma_loc is the site's pure covariance
over those 2 (n_phys + 4d) Majoranas, its virtual block d_site the last 8d rows and columns.  Each link
(x -> x + e_mu) carries a pure bond state b on its 4d Majoranas (out leg of x, then in leg of x + e_mu);
the link element rotates the out leg: Gamma_b(g) = (O(D(g)) (+) 1) Gamma_b (O(D(g)) (+) 1)^T.  As for Z_N
(Sec. 3.2 PEPS norm, the gauge rotation of Sec. 5 moved onto the bonds),
    M(G) = D + Gamma_B(G)  (n x n, n = 8 d V),   W(G) = <psi(G)|psi(G)> = sqrt(det(M / 2)).
A link change g -> g' changes M on the link's 4d Majoranas U only, so
    W(G') / W(G) = sqrt(det(1 + M^-1_UU dM_UU))     (matrix determinant lemma).
"""
from __future__ import annotations

import numpy as np


def quaternion_group() -> list[np.ndarray]:
    """The quaternion group Q8 in its faithful 2-dimensional irrep: +-1, +-i sigma_x, +-i sigma_y,
    +-i sigma_z (a finite non-abelian subgroup of SU(2), the group of the paper's SU(2) examples)."""
    one = np.eye(2, dtype=complex)
    sx = np.array([[0, 1], [1, 0]], complex)
    sy = np.array([[0, -1j], [1j, 0]], complex)
    sz = np.array([[1, 0], [0, -1]], complex)
    return [s * m for s in (1, -1) for m in (one, 1j * sx, 1j * sy, 1j * sz)]


def majorana_rotation(u: np.ndarray) -> np.ndarray:
    """O with V(u) c_b V(u)^+ = sum_a O_ab c_a for the mode rotation psi^+_b -> sum_a u_ab psi^+_a."""
    d = u.shape[0]
    x, y = u.real, u.imag
    o = np.zeros((2 * d, 2 * d))
    o[0::2, 0::2] = x
    o[1::2, 0::2] = y
    o[0::2, 1::2] = -y
    o[1::2, 1::2] = x
    return o


class NonAbelianAnsatz:
    """Gauged Gaussian PEPS on an Lx x Ly torus with d-mode legs carrying the irrep `elements`."""

    def __init__(self, lx: int, ly: int, gamma_loc: np.ndarray, gamma_bond: np.ndarray,
                 elements: list[np.ndarray], n_phys: int):
        self.lx, self.ly = lx, ly
        self.elements = [np.asarray(e, complex) for e in elements]
        self.d = self.elements[0].shape[0]
        self.n_phys = n_phys
        self.nv = 8 * self.d                                   # virtual Majoranas per site
        assert gamma_loc.shape == (2 * n_phys + self.nv,) * 2
        assert gamma_bond.shape == (4 * self.d,) * 2
        self.gamma_loc = np.asarray(gamma_loc, float)
        self.gamma_bond = np.asarray(gamma_bond, float)
        self.rot = [majorana_rotation(e) for e in self.elements]

    @property
    def V(self) -> int:
        return self.lx * self.ly

    @property
    def n_links(self) -> int:
        return 2 * self.V

    def site(self, x1: int, x2: int) -> int:
        return (x2 % self.ly) * self.lx + (x1 % self.lx)

    def link_sites(self, ell: int):
        """Link ell = 2 i + mu joins site i (its out leg mu) to i + e_mu (its in leg 2 + mu)."""
        i, mu = divmod(ell, 2)
        x1, x2 = i % self.lx, i // self.lx
        j = self.site(x1 + 1, x2) if mu == 0 else self.site(x1, x2 + 1)
        return i, mu, j, 2 + mu

    def leg_majoranas(self, site: int, leg: int) -> list[int]:
        base = self.nv * site + 2 * self.d * leg
        return list(range(base, base + 2 * self.d))

    def link_majoranas(self, ell: int) -> list[int]:
        i, lo, j, li = self.link_sites(ell)
        return self.leg_majoranas(i, lo) + self.leg_majoranas(j, li)

    def bond_block(self, k: int) -> np.ndarray:
        """Gamma_b(g_k): the bond covariance with the out leg rotated by element k."""
        o = np.eye(4 * self.d)
        o[:2 * self.d, :2 * self.d] = self.rot[k]
        return o @ self.gamma_bond @ o.T

    def assemble_M(self, links: np.ndarray) -> np.ndarray:
        n = self.nv * self.V
        dsite = self.gamma_loc[2 * self.n_phys:, 2 * self.n_phys:]
        m = np.zeros((n, n))
        for s in range(self.V):
            m[s * self.nv:(s + 1) * self.nv, s * self.nv:(s + 1) * self.nv] = dsite
        for ell in range(self.n_links):
            u = self.link_majoranas(ell)
            m[np.ix_(u, u)] += self.bond_block(int(links[ell]))
        return m

    def log_weight(self, links: np.ndarray) -> float:
        """log W(G) = (1/2) log det(M / 2)."""
        sign, ld = np.linalg.slogdet(self.assemble_M(links) / 2.0)
        if sign <= 0:
            raise ValueError("det M <= 0: the configuration has zero weight")
        return 0.5 * ld

    def element_index(self, u: np.ndarray) -> int:
        return min(range(len(self.elements)), key=lambda k: np.abs(self.elements[k] - u).max())

    def plaquette_trace(self, links: np.ndarray, i: int) -> complex:
        """(1/d) tr D(g_{x,x+e1} g_{x+e1,x+e1+e2} g_{x+e2,x+e1+e2}^-1 g_{x,x+e2}^-1) at site x = i
        (the plaquette operator's expectation in a configuration, Sec. 2.3)."""
        x1, x2 = i % self.lx, i // self.lx
        a = self.site(x1 + 1, x2)
        b = self.site(x1, x2 + 1)
        e = self.elements
        u = (e[int(links[2 * i])] @ e[int(links[2 * a + 1])] @ e[int(links[2 * b])].conj().T
             @ e[int(links[2 * i + 1])].conj().T)
        return complex(np.trace(u)) / self.d

    def gauge_transform(self, links: np.ndarray, h: np.ndarray) -> np.ndarray:
        """g_{x -> y} -> h_x g h_y^-1 for site elements h (indices), the link field's gauge action."""
        out = links.copy()
        for ell in range(self.n_links):
            i, _, j, _ = self.link_sites(ell)
            u = self.elements[int(h[i])] @ self.elements[int(links[ell])] @ self.elements[int(h[j])].conj().T
            out[ell] = self.element_index(u)
        return out

    def link_ratio(self, ginv: np.ndarray, links: np.ndarray, ell: int, k_new: int) -> float:
        """W(G with g_ell -> element k_new) / W(G) from M^-1 on the link's 4d Majoranas."""
        u = self.link_majoranas(ell)
        dm = self.bond_block(k_new) - self.bond_block(int(links[ell]))
        return float(np.sqrt(np.linalg.det(np.eye(len(u)) + ginv[np.ix_(u, u)] @ dm)))


# ---- Fock-space brute force (the pin): <psi(G)|psi(G)> by explicit contraction ----

def majoranas_sparse(n_modes: int):
    """c_0 .. c_{2N-1} as sparse matrices in the Jordan-Wigner basis of `gaussian` (mode 0 leftmost)."""
    import scipy.sparse as sp
    dim = 2 ** n_modes
    s = np.arange(dim)
    ops = []
    par = np.zeros(dim, int)
    for j in range(n_modes):
        bit = (s >> (n_modes - 1 - j)) & 1
        sign = (1 - 2 * par).astype(complex)
        t = s ^ (1 << (n_modes - 1 - j))
        ops.append(sp.csr_matrix((sign, (t, s)), shape=(dim, dim)))
        ops.append(sp.csr_matrix((sign * 1j * (1 - 2 * bit), (t, s)), shape=(dim, dim)))
        par = par ^ bit
    return ops


def pure_state(gamma: np.ndarray, n_modes: int, cs=None) -> np.ndarray:
    """Ground state of H = -(i/4) sum Gamma_ab c_a c_b, the pure state of covariance gamma (Sec. 3.2)."""
    import scipy.sparse as sp
    cs = majoranas_sparse(n_modes) if cs is None else cs
    h = sp.csr_matrix((2 ** n_modes, 2 ** n_modes), dtype=complex)
    for a in range(2 * n_modes):
        for b in range(2 * n_modes):
            if gamma[a, b] != 0:
                h = h + (-0.25j * gamma[a, b]) * (cs[a] @ cs[b])
    h = h.toarray()
    w, v = np.linalg.eigh(0.5 * (h + h.conj().T))
    if w[1] - w[0] < 1e-8:
        raise ValueError("covariance is not pure")
    return v[:, 0]


def mode_unitary(u: np.ndarray) -> np.ndarray:
    """V(u) = exp(i psi^+ H psi), u = exp(iH), as a 2^d x 2^d matrix (Jordan-Wigner on d modes)."""
    from scipy.linalg import expm, logm
    d = u.shape[0]
    h = -1j * logm(u)
    h = 0.5 * (h + h.conj().T)
    cs = majoranas_sparse(d)
    psi = [0.5 * (cs[2 * j] + 1j * cs[2 * j + 1]).toarray() for j in range(d)]
    gen = sum(h[a, b] * psi[a].conj().T @ psi[b] for a in range(d) for b in range(d))
    return expm(1j * gen)


def reorder_modes(vec: np.ndarray, order: list[int], n_modes: int) -> np.ndarray:
    """The state with its modes put in the new order (position p holds old mode order[p]), with the
    fermionic sign of the reordering (one factor -1 per pair of occupied modes whose order flips)."""
    dim = 2 ** n_modes
    s = np.arange(dim)
    occ = [(s >> (n_modes - 1 - j)) & 1 for j in range(n_modes)]
    t = np.zeros(dim, int)
    for p in range(n_modes):
        t |= occ[order[p]] << (n_modes - 1 - p)
    flip = np.zeros(dim, int)
    for p in range(n_modes):
        for q in range(p + 1, n_modes):
            if order[p] > order[q]:
                flip ^= occ[order[p]] & occ[order[q]]
    out = np.zeros(dim, complex)
    out[t] = vec * (1 - 2 * flip)
    return out


def fock_weight(an: NonAbelianAnsatz, links: np.ndarray, site_state: np.ndarray,
                bond_state: np.ndarray) -> float:
    """<psi(G)|psi(G)> with psi(G) = (x)_links <b(g_l)| (x)_sites |A>, contracted in the Fock space of all
    sites' modes (even site and bond states, so the products need no reordering signs), the virtual
    modes moved behind the physical ones and projected on the rotated bond states."""
    npm, d, ns = an.n_phys, an.d, an.n_phys + 4 * an.d
    nsites = an.V
    full = np.ones(1, complex)
    for _ in range(nsites):
        full = np.kron(full, site_state)
    nm = nsites * ns
    phys = [s * ns + k for s in range(nsites) for k in range(npm)]
    virt = [s * ns + npm + k for s in range(nsites) for k in range(4 * d)]
    full = reorder_modes(full, phys + virt, nm)
    # bond states in link order (out leg modes, then in leg modes), each rotated on its out leg
    rots = [mode_unitary(e) for e in an.elements]
    bonds = np.ones(1, complex)
    lmodes = []
    for ell in range(an.n_links):
        i, lo, j, li = an.link_sites(ell)
        bonds = np.kron(bonds, np.kron(rots[int(links[ell])], np.eye(2 ** d)) @ bond_state)
        lmodes += [4 * d * i + d * lo + a for a in range(d)] + [4 * d * j + d * li + a for a in range(d)]
    nvm = len(lmodes)
    pos = [0] * nvm                                   # global virtual mode -> its position in link order
    for k, gm in enumerate(lmodes):
        pos[gm] = k
    bonds = reorder_modes(bonds, pos, nvm)
    out = full.reshape(2 ** (nsites * npm), 2 ** nvm) @ bonds.conj()
    return float(np.vdot(out, out).real)
