"""Gaussian fermionic toolkit (Sec. 3.2): Majoranas, covariance matrices, Pfaffians.

Conventions (Sec. 3.2, definition of the Majorana modes and of Gamma):
  c_{2j} = psi_j + psi_j^+,  c_{2j+1} = -i (psi_j - psi_j^+),
  Gamma_ab = (i/2) <[c_a, c_b]>.
With these, the empty mode has Gamma = [[0,-1],[1,0]] and the filled mode
[[0,1],[-1,0]].

Jordan-Wigner: mode 0 is the leftmost tensor factor; basis index
s = sum_j n_j 2^(N-1-j); psi_j = Z x ... x Z x sigma^- x 1 x ... (sigma^- = |0><1|),
so c_{2j} = Z..Z X_j and c_{2j+1} = Z..Z Y_j.
"""
from __future__ import annotations

import itertools

import numpy as np

_X = np.array([[0, 1], [1, 0]], complex)
_Y = np.array([[0, -1j], [1j, 0]], complex)
_Z = np.array([[1, 0], [0, -1]], complex)
_I = np.eye(2, dtype=complex)


def majorana_matrices(n_modes: int) -> list[np.ndarray]:
    """Dense 2^N x 2^N Majorana operators c_0 .. c_{2N-1} (small N only)."""
    ops = []
    for j in range(n_modes):
        for single in (_X, _Y):
            m = np.eye(1, dtype=complex)
            for k in range(n_modes):
                f = _Z if k < j else (single if k == j else _I)
                m = np.kron(m, f)
            ops.append(m)
    return ops


def number_matrices(n_modes: int) -> list[np.ndarray]:
    """Dense occupation operators n_j = psi_j^+ psi_j."""
    dim = 2 ** n_modes
    s = np.arange(dim)
    return [np.diag(((s >> (n_modes - 1 - j)) & 1).astype(complex)) for j in range(n_modes)]


def covariance_of_state(v: np.ndarray, n_modes: int, cs=None) -> np.ndarray:
    """Gamma_ab = (i/2) <v|[c_a,c_b]|v> / <v|v> from a state vector (Sec. 3.2)."""
    cs = majorana_matrices(n_modes) if cs is None else cs
    nrm = np.vdot(v, v)
    m = 2 * n_modes
    g = np.zeros((m, m), complex)
    cv = [c @ v for c in cs]
    for a in range(m):
        for b in range(m):
            if a != b:
                g[a, b] = 0.5j * (np.vdot(v, cs[a] @ cv[b]) - np.vdot(v, cs[b] @ cv[a])) / nrm
    return g


def transition_covariance(bra: np.ndarray, ket: np.ndarray, n_modes: int, cs=None) -> np.ndarray:
    """Covariance of the operator |ket><bra| / <bra|ket>: (i/2)<bra|[c_a,c_b]|ket>/<bra|ket>."""
    cs = majorana_matrices(n_modes) if cs is None else cs
    ov = np.vdot(bra, ket)
    m = 2 * n_modes
    g = np.zeros((m, m), complex)
    for a in range(m):
        for b in range(m):
            if a != b:
                comm = cs[a] @ cs[b] - cs[b] @ cs[a]
                g[a, b] = 0.5j * np.vdot(bra, comm @ ket) / ov
    return g


def state_of_covariance(gamma: np.ndarray, n_modes: int, cs=None) -> np.ndarray:
    """Pure Gaussian state with covariance gamma: ground state of H = -(i/4) sum Gamma_ab c_a c_b.

    For a single mode with Gamma = [[0,-1],[1,0]], H = n - 1/2, whose ground
    state is the empty mode, matching the convention above.  The returned
    vector has unit norm and an arbitrary global phase.
    """
    cs = majorana_matrices(n_modes) if cs is None else cs
    m = 2 * n_modes
    h = np.zeros_like(cs[0])
    for a in range(m):
        for b in range(m):
            if gamma[a, b] != 0:
                h = h + (-0.25j) * gamma[a, b] * (cs[a] @ cs[b])
    w, vecs = np.linalg.eigh(0.5 * (h + h.conj().T))
    if w[1] - w[0] < 1e-8:
        raise ValueError("covariance is not pure (degenerate ground state)")
    return vecs[:, 0]


def pfaffian(a: np.ndarray) -> complex:
    """Pfaffian by skew-symmetric Gaussian elimination with pivoting.

    At each pair step the largest entry of column k below row k is moved to
    row/column k+1 (each swap flips the sign), the Pfaffian collects
    A[k, k+1], and a congruence with unit determinant clears row/column k
    beyond k+1:  A_trail += tau v^T - v tau^T with tau = A[k, k+2:]/A[k, k+1]
    and v = A[k+2:, k+1].  (The same elimination is described by Wimmer,
    ACM TOMS 38 (2012), as the Parlett-Reid tridiagonalisation.)
    """
    a = np.array(a, dtype=complex if np.iscomplexobj(a) else float, copy=True)
    n = a.shape[0]
    if n % 2:
        return 0.0
    pf = 1.0
    for k in range(0, n - 1, 2):
        kp = k + 1 + int(np.argmax(np.abs(a[k + 1:, k])))
        if kp != k + 1:
            a[[k + 1, kp], :] = a[[kp, k + 1], :]
            a[:, [k + 1, kp]] = a[:, [kp, k + 1]]
            pf = -pf
        piv = a[k, k + 1]
        if piv == 0:
            return 0.0 * pf
        pf = pf * piv
        if k + 2 < n:
            tau = a[k, k + 2:] / piv
            v = a[k + 2:, k + 1].copy()
            a[k + 2:, k + 2:] += np.outer(tau, v) - np.outer(v, tau)
    return pf


def pfaffian_bruteforce(a: np.ndarray) -> complex:
    """Pfaffian from its definition as a signed sum over perfect matchings (n <= 10).

    Expansion along the first row: Pf(A) = sum_j (-1)^(j+1) A[0, j] Pf(A without rows/cols 0, j)
    (0-based j >= 1).
    """
    n = a.shape[0]
    if n == 0:
        return 1.0
    if n % 2:
        return 0.0
    total = 0.0
    for j in range(1, n):
        keep = [k for k in range(n) if k not in (0, j)]
        sub = a[np.ix_(keep, keep)]
        total = total + (-1) ** (j + 1) * a[0, j] * pfaffian_bruteforce(sub)
    return total


def pfaffian_matchings(a: np.ndarray) -> complex:
    """Pfaffian by explicit enumeration of perfect matchings and the permutation sign (n <= 8)."""
    n = a.shape[0]
    total = 0.0
    for perm in itertools.permutations(range(n)):
        ok = all(perm[2 * i] < perm[2 * i + 1] for i in range(n // 2)) and \
            all(perm[2 * i] < perm[2 * i + 2] for i in range(n // 2 - 1))
        if not ok:
            continue
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        term = (-1) ** inv
        for i in range(n // 2):
            term = term * a[perm[2 * i], perm[2 * i + 1]]
        total = total + term
    return total


def vacuum_covariance(n_modes: int) -> np.ndarray:
    g = np.zeros((2 * n_modes, 2 * n_modes))
    for j in range(n_modes):
        g[2 * j, 2 * j + 1] = -1.0
        g[2 * j + 1, 2 * j] = 1.0
    return g


def overlap_pure(g1: np.ndarray, g2: np.ndarray) -> float:
    """tr(rho1 rho2) = 2^-N sqrt(det(Gamma1 + Gamma2)) for Gaussian states on N modes.

    Sec. 3.2 states the overlap as Pf((Gamma1+Gamma2)/2); that form is only
    right up to sign, so the square root of the determinant is used, as the
    same section recommends for real non-negative results.
    """
    n = g1.shape[0] // 2
    d = np.linalg.det(g1 + g2)
    return float(2.0 ** (-n) * np.sqrt(max(d.real, 0.0)))
