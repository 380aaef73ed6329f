"""Seeded synthetic inputs for gauged (superposed) Gaussian fermionic PEPS.

This module is the only code shared by the CPU oracle and the HIP path.  It
produces the *inputs* of the method -- the variational parameters of the
ansatz (Sec. 4: amplitudes lambda_n, on-site covariance Gamma_A and bond
covariances Gamma_{B_n}) and the lattice/chain mix of a batch -- and holds none
of the method's arithmetic (no weights, overlaps, Pfaffians or updates).

Workload recipe (the paper measures nothing, so every input is synthetic):

* on-site tensor: Gamma_loc = O J O^T on 5 modes (1 physical + 4 virtual legs,
  leg order p,l,u,r,d of the on-site tensor of Sec. 3), J = (+)_5 [[0,1],[-1,0]],
  O Haar-orthogonal from a seeded QR of an N(0,1) 10x10 matrix with the
  sign(diag R) correction; the last column of O is negated when det O = +1 so
  that the local state has even fermion parity;
* reference bond: the maximally entangled pair (1 + psi_out^+ psi_in^+)|0>/sqrt2
  on every link (the bond state of Sec. 3), as a fixed 4x4 covariance in
  Majorana order (out0, out1, in0, in1);
* superposed bonds (K > 1): bond k >= 1 equals the reference bond except on one
  seeded link l_k, where its covariance is R_k Gamma_b0 R_k^T with
  R_k = expm(eps * A_k), A_k a seeded antisymmetric 4x4 generator of unit
  Frobenius norm and eps = 0.1 (a perturbation localised on the 2-site patch
  that the link joins);
* amplitudes: lambda_k = x_k + i y_k with x, y ~ N(0, 1);
* mixed batches: per chain L ~ U{6,8,12,16,20}, K ~ U{1,2,4}, group ~ U{Z2,Z3}.

Seeds: tensor 1, patches 2, amplitudes 3, chain key 4, batch mix 5.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

SEED_TENSOR = 1
SEED_PATCH = 2
SEED_AMPLITUDE = 3
SEED_CHAIN = 4
SEED_MIX = 5

# Covariance of (1 + psi_out^+ psi_in^+)|0>/sqrt(2) in Majorana order
# (out0, out1, in0, in1), with c_{2j} = psi_j + psi_j^+, c_{2j+1} = -i(psi_j - psi_j^+)
# and Gamma_ab = (i/2) <[c_a, c_b]>.  An input constant (the reference bond);
# the oracle derives it independently from the state vector in its tests.
GAMMA_BOND0 = np.array(
    [[0.0, 0.0, 0.0, -1.0],
     [0.0, 0.0, -1.0, 0.0],
     [0.0, 1.0, 0.0, 0.0],
     [1.0, 0.0, 0.0, 0.0]])


def haar_orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-distributed O(n) matrix: QR of a Gaussian matrix, R's diagonal signs folded into Q."""
    z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    return q * np.sign(np.diag(r))[None, :]


def local_gamma(seed: int = SEED_TENSOR) -> np.ndarray:
    """10x10 on-site covariance O J O^T (even parity), Majorana order (p,l,u,r,d) x (0,1)."""
    rng = np.random.default_rng(seed)
    o = haar_orthogonal(rng, 10)
    if np.linalg.det(o) > 0:
        o[:, 9] = -o[:, 9]
    j = np.zeros((10, 10))
    for m in range(5):
        j[2 * m, 2 * m + 1] = 1.0
        j[2 * m + 1, 2 * m] = -1.0
    g = o @ j @ o.T
    return 0.5 * (g - g.T)


@dataclass
class TensorSpec:
    """Inputs of one superposed ansatz: what ggf_set_tensor receives."""
    group: int                      # 2 = Z2, 3 = Z3
    gamma_loc: np.ndarray           # (10, 10) float64
    gamma_bond: np.ndarray          # (4, 4) float64, reference bond b_0
    K: int = 1
    patch_link: np.ndarray = field(default_factory=lambda: np.array([-1], np.int32))
    gamma_bond_k: np.ndarray = field(default_factory=lambda: np.zeros((1, 4, 4)))
    c: np.ndarray = field(default_factory=lambda: np.ones(1, complex))


def patch_bonds(n_links: int, K: int, seed: int = SEED_PATCH, eps: float = 0.1):
    """K-1 distinct seeded patch links and their perturbed bond covariances (k = 0 is the reference)."""
    rng = np.random.default_rng(seed)
    links = np.full(K, -1, np.int32)
    gk = np.zeros((K, 4, 4))
    gk[0] = GAMMA_BOND0
    if K > 1:
        if K - 1 > n_links:
            raise ValueError("more patches than links")
        links[1:] = rng.choice(n_links, size=K - 1, replace=False)
        for k in range(1, K):
            x = rng.standard_normal((4, 4))
            a = x - x.T
            a /= np.linalg.norm(a)
            r = scipy.linalg.expm(eps * a)
            g = r @ GAMMA_BOND0 @ r.T
            gk[k] = 0.5 * (g - g.T)
    return links, gk


def amplitudes(K: int, seed: int = SEED_AMPLITUDE) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(K)
    y = rng.standard_normal(K)
    return x + 1j * y


def make_tensor(L: int, K: int = 1, group: int = 2, seed_tensor: int = SEED_TENSOR,
                seed_patch: int = SEED_PATCH, seed_amp: int = SEED_AMPLITUDE,
                eps: float = 0.1) -> TensorSpec:
    """The standard synthetic ansatz for an L x L periodic lattice."""
    links, gk = patch_bonds(2 * L * L, K, seed_patch, eps)
    c = amplitudes(K, seed_amp) if K > 1 else np.ones(1, complex)
    return TensorSpec(group=group, gamma_loc=local_gamma(seed_tensor),
                      gamma_bond=GAMMA_BOND0.copy(), K=K, patch_link=links,
                      gamma_bond_k=gk, c=c)


MIX_L = (6, 8, 12, 16, 20)
MIX_K = (1, 2, 4)
MIX_GROUP = (2, 3)


def mixed_batch(n_chains: int, seed: int = SEED_MIX, Ls=MIX_L, Ks=MIX_K, groups=MIX_GROUP):
    """Per-chain (L, K, group) for an uneven batch, each drawn uniformly from its set."""
    rng = np.random.default_rng(seed)
    L = rng.choice(np.asarray(Ls), size=n_chains)
    K = rng.choice(np.asarray(Ks), size=n_chains)
    g = rng.choice(np.asarray(groups), size=n_chains)
    return L.astype(np.int32), K.astype(np.int32), g.astype(np.int32)


def random_links(rng: np.random.Generator, n_links: int, group: int) -> np.ndarray:
    """A uniformly random gauge configuration (link values k in Z_N), as int8."""
    return rng.integers(0, group, size=n_links).astype(np.int8)
