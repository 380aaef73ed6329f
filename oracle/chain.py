"""Metropolis chains over gauge configurations (Sec. 5.1: <W> = sum_G p(G) W(G),
p(G) = N(G)/N, sampled without a sign problem).

The paper names no sampler; the reading used here is single-link Metropolis:
a sweep visits links 0 .. 2V-1 in order; Z_N proposes k -> (k + 1 + (x2 mod (N-1))) mod N
(Z2: k -> 1-k; Z3: k -> (k + 1 + (x2 & 1)) mod 3); the proposal is accepted iff u < N(G')/N(G)
(strict), with (u, x2) from Philox at counter (chain, sweep, link, 0).
A cold start has every k = 0; a hot start takes k = x0 mod N from Philox at
counter (chain, 0xffffffff, link, 1).

Near ties.  A decision with |u - R| < 1e-9 R could flip under a rounding
change of R (the HIP path evaluates R through other, equally exact routes), so
every chain counts them in ``ties``; parity tests compare decisions and report
these counts instead of assuming them away.

Two evaluators of the ratio:
* ``DefinitionChain``: fresh log-determinant (and, for K > 1, full Pfaffians of
  every M_nm) of the current and proposed configuration -- the definition;
* ``WoodburyChain``: maintains G = M^-1, log W and S = N/W; the ratio is
  det(1 + G_UU dM_UU)^(1/2) S'/S by the matrix determinant lemma, and an
  accepted flip applies the Woodbury identity
  G' = G - G[:,U] (dM^-1 + G_UU)^-1 G[U,:].  Every ``refresh_every``
  accepted flips (checked at the end of a sweep) G, log W and S are recomputed
  from the link field and the drift of log W is recorded.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import philox
from .model import Ansatz, rotation

HOT_SWEEP = 0xFFFFFFFF
TIE_REL = 1e-9


def near_tie(u: float, R: float) -> bool:
    """|u - R| < 1e-9 R: a decision that rounding of R could change."""
    return abs(float(u) - R) < TIE_REL * R


def hot_links(seed: int, chain: int, n_links: int, group: int) -> np.ndarray:
    x0, _, _, _ = philox.philox_vec(chain, HOT_SWEEP, np.arange(n_links), 1,
                                    seed & 0xFFFFFFFF, seed >> 32)
    return (x0 % np.uint64(group)).astype(np.int8)


def propose(k: int, step: int, group: int) -> int:
    return (k + step) % group


def delta_uu(an: Ansatz, k_old: int, k_new: int) -> np.ndarray:
    """Change of M(G) on the link Majoranas (out0,out1,in0,in1) when the link changes k_old -> k_new."""
    x0 = an.gamma_bond[0:2, 2:4]
    th = 2 * np.pi / an.group
    x = (rotation(th * k_new) - rotation(th * k_old)) @ x0
    d = np.zeros((4, 4))
    d[0:2, 2:4] = x
    d[2:4, 0:2] = -x.T
    return d


class DefinitionChain:
    """Metropolis with N(G')/N(G) from scratch for every proposal."""

    def __init__(self, an: Ansatz, seed: int, chain: int, links0=None):
        self.an, self.seed, self.chain = an, seed, chain
        self.k = np.zeros(an.lat.n_links, np.int8) if links0 is None else np.array(links0, np.int8)
        self.sweep_idx = 0
        self.logn = self._logn(self.k)
        self.accepts = 0
        self.ties = 0

    def _logn(self, k) -> float:
        lw = self.an.log_weight(k)
        if self.an.K == 1:
            return lw
        return lw + np.log(self.an.s_factor_def(k).real)

    def sweep(self):
        an = self.an
        for ell in range(an.lat.n_links):
            u, step = philox.draw(self.seed, self.chain, self.sweep_idx, ell, an.group)
            knew = self.k.copy()
            knew[ell] = propose(int(self.k[ell]), int(step), an.group)
            ln_new = self._logn(knew)
            R = np.exp(ln_new - self.logn)
            self.ties += near_tie(u, R)
            if float(u) < R:
                self.k, self.logn = knew, ln_new
                self.accepts += 1
        self.sweep_idx += 1


class WoodburyChain:
    """Metropolis with a maintained inverse G = M(G)^-1, rank-4 Woodbury updates."""

    def __init__(self, an: Ansatz, seed: int, chain: int, links0=None, refresh_every: int = 0):
        self.an, self.seed, self.chain = an, seed, chain
        self.k = np.zeros(an.lat.n_links, np.int8) if links0 is None else np.array(links0, np.int8)
        self.refresh_every = refresh_every
        self.sweep_idx = 0
        self.accepts = 0
        self.proposals = 0
        self.since_refresh = 0
        self.ties = 0
        self.drifts = []
        self.refresh()

    def refresh(self):
        an = self.an
        M = an.assemble_M(self.k)
        sign, ld = np.linalg.slogdet(M)
        self.G = np.linalg.inv(M)
        self.logw = 0.5 * ld - 4 * an.lat.V * np.log(2.0)
        self.S = 1.0 + 0j
        if an.K > 1:
            S = an.S
            self.S = an.s_factor_patch(self.G[np.ix_(S, S)], self.k)
        self.since_refresh = 0

    def ratio(self, ell: int, k_new: int):
        """(R, rho, S', dM) for changing link ell to k_new."""
        an = self.an
        u = an.lat.link_majoranas(ell)
        dm = delta_uu(an, int(self.k[ell]), k_new)
        guu = self.G[np.ix_(u, u)]
        rho = float(np.linalg.det(np.eye(4) + guu @ dm))
        s_new = 1.0 + 0j
        if an.K > 1:
            S = an.S
            kw = np.linalg.inv(np.linalg.inv(dm) + guu)
            gss = self.G[np.ix_(S, S)] - self.G[np.ix_(S, u)] @ kw @ self.G[np.ix_(u, S)]
            knew = self.k.copy()
            knew[ell] = k_new
            s_new = an.s_factor_patch(gss, knew)
        R = np.sqrt(max(rho, 0.0)) * (s_new.real / self.S.real)
        return R, rho, s_new, dm

    def accept(self, ell: int, k_new: int, rho: float, s_new, dm):
        u = self.an.lat.link_majoranas(ell)
        guu = self.G[np.ix_(u, u)]
        kw = np.linalg.inv(np.linalg.inv(dm) + guu)
        self.G = self.G - self.G[:, u] @ kw @ self.G[u, :]
        self.logw += 0.5 * np.log(rho)
        self.S = s_new
        self.k[ell] = k_new
        self.accepts += 1
        self.since_refresh += 1

    @property
    def logn(self) -> float:
        return self.logw + (np.log(self.S.real) if self.an.K > 1 else 0.0)

    def sweep(self):
        an = self.an
        for ell in range(an.lat.n_links):
            u, step = philox.draw(self.seed, self.chain, self.sweep_idx, ell, an.group)
            k_new = propose(int(self.k[ell]), int(step), an.group)
            R, rho, s_new, dm = self.ratio(ell, k_new)
            self.proposals += 1
            self.ties += near_tie(u, R)
            if float(u) < R:
                self.accept(ell, k_new, rho, s_new, dm)
        self.sweep_idx += 1
        if self.refresh_every > 0 and self.since_refresh >= self.refresh_every:
            lw_acc = self.logw
            self.refresh()
            self.drifts.append(abs(lw_acc - self.logw))

    def observables(self) -> np.ndarray:
        return self.an.observables(self.k)


def block_move(ch: "WoodburyChain", params, P: int, patch: int, route: str = "def", rho: float = 1.0):
    """One Metropolis-Hastings block move on a P x P patch (Z2), learned proposal.

    The proposal resamples the patch links from the network's factorised
    Bernoulli q(.|context) (logits from the float32 forward pass, uniforms
    from Philox at (chain, sweep, patch, 3 + j)); it is accepted iff
    u < N(G') q(x|ctx) / (N(G) q(x'|ctx)) with u from (chain, sweep, patch, 2).
    With a move rate rho < 1 each patch link keeps its value with probability
    1 - rho and is otherwise drawn from q(.|context) (link j becomes 1 iff its
    uniform is below (1 - rho) x_j + rho sigmoid(z_j)), and the ratio uses the
    proposal densities q(x|x', ctx) / q(x'|x, ctx) by their definition.  The
    context masks the patch, so q does not depend on the patch links.
    N is evaluated from scratch for both configurations: W from a fresh
    determinant and, for K > 1, N/W = sum_nm c_n^* c_m <B_m|B_n> Pf(M_nm)/Pf(M_00)
    (Sec. 5) -- with ``route="def"`` from full Pfaffians of every M_nm (the
    definition), with ``route="patch"`` from a fresh inverse by the patch lemma
    (Pfaffians of order <= 16; for lattices where full Pfaffians are out of reach,
    and pinned to the definition on every case both can run).  An accepted move
    refactorises G.  Returns (proposed, accepted, changed links).
    """
    from . import nn
    an = ch.an
    if an.group != 2:
        raise ValueError("block moves are defined for Z2")
    if route not in ("def", "patch"):
        raise ValueError("route is 'def' or 'patch'")
    L = an.lat.Lx
    pl = nn.patch_links(L, P, patch)
    z, _ = nn.forward(params, nn.window(ch.k, L, P, patch), np.float32)
    zl = nn.logits_patch_order(z).astype(np.float64)
    u_acc, u = nn.draw_block(ch.seed, ch.chain, ch.sweep_idx, patch, len(pl))
    y_old = ch.k[pl].astype(np.float64)
    y_new = (u < nn.propose_p1(zl, y_old, rho)).astype(np.float64)
    m = int(np.sum(y_new != y_old))
    if m == 0:
        return False, False, 0
    k_new = ch.k.copy()
    k_new[pl] = y_new.astype(np.int8)

    def log_n(k):
        M = an.assemble_M(k)
        if an.K == 1 or route == "def":
            sign, ld = np.linalg.slogdet(M)
            lw = 0.5 * ld - 4 * an.lat.V * np.log(2.0)
            return lw if an.K == 1 else lw + np.log(an.s_factor_def(k).real)
        # one LU factorisation gives det M and the patch block (M^-1)_SS (columns S of the inverse)
        lu, piv = scipy.linalg.lu_factor(M)
        lw = 0.5 * np.sum(np.log(np.abs(np.diag(lu)))) - 4 * an.lat.V * np.log(2.0)
        E = np.zeros((M.shape[0], len(an.S)))
        E[an.S, np.arange(len(an.S))] = 1.0
        g_ss = scipy.linalg.lu_solve((lu, piv), E)[an.S, :]
        return lw + np.log(an.s_factor_patch(g_ss, k).real)

    if rho == 1.0:
        log_qr = nn.log_q(zl, y_old) - nn.log_q(zl, y_new)
    else:
        log_qr = nn.log_q_move(zl, y_old, y_new, rho) - nn.log_q_move(zl, y_new, y_old, rho)
    R = np.exp(log_n(k_new) - log_n(ch.k) + log_qr)
    ch.ties += near_tie(u_acc, R)
    if u_acc < R:
        ch.k = k_new
        ch.refresh()
        return True, True, m
    return True, False, m


def block_sweep(ch: "WoodburyChain", params, P: int, route: str = "def", rho: float = 1.0):
    """Block moves on every patch in order, then the sweep counter advances (shared with link sweeps)."""
    L = ch.an.lat.Lx
    stats = [0, 0]
    for p in range((L // P) ** 2):
        prop, acc, _ = block_move(ch, params, P, p, route, rho)
        stats[0] += prop
        stats[1] += acc
    ch.sweep_idx += 1
    return stats
