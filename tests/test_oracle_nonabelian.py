"""The non-abelian oracle (oracle/nonabelian.py) against what fixes it independently (CPU only).

* Q8 in its 2-dimensional irrep is a group (closure, unitarity) and is non-abelian;
* the Majorana rotation of a leg is the action of the Gaussian unitary V(u) on the Majorana operators,
  computed here with dense Fock-space operators, and a representation of the group;
* the covariance weight W(G) = sqrt(det(M(G) / 2)) equals the explicit Fock-space contraction
  <psi(G)|psi(G)> of the PEPS on a 2 x 1 torus with 2-mode legs (20 fermionic modes), for random
  link configurations of Q8 elements (Sec. 3.2, 5; the link space of Sec. 2.1);
* a link change's weight ratio from M^-1 on the link's Majoranas (determinant lemma) equals the ratio
  of fresh determinants;
* the plaquette trace is invariant under gauge transformations of the link field (which fixes the
  orientation of its four links) and is not a class function of any single link.
"""
import numpy as np

from oracle import gaussian as ga
from oracle import nonabelian as na


def _random_pure_even(n_maj: int, rng) -> np.ndarray:
    """O J O^T with O in SO(n_maj): a pure covariance of an even-parity state."""
    q, r = np.linalg.qr(rng.standard_normal((n_maj, n_maj)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    j = np.kron(np.eye(n_maj // 2), np.array([[0.0, 1.0], [-1.0, 0.0]]))
    return q @ j @ q.T


def _bond_state(d: int) -> np.ndarray:
    """prod_a (1 + psi^+_{out a} psi^+_{in a}) / sqrt2 |0> on the modes (out 1..d, in 1..d)."""
    cs = ga.majorana_matrices(2 * d)
    psi = [0.5 * (cs[2 * k] + 1j * cs[2 * k + 1]) for k in range(2 * d)]
    v = np.zeros(2 ** (2 * d), complex)
    v[0] = 1.0
    for a in range(d):
        v = (np.eye(len(v)) + psi[a].conj().T @ psi[d + a].conj().T) @ v / np.sqrt(2.0)
    return v


def test_quaternion_group_is_a_nonabelian_group():
    g = na.quaternion_group()
    assert len(g) == 8
    for a in g:
        assert np.abs(a @ a.conj().T - np.eye(2)).max() < 1e-15
        assert abs(np.linalg.det(a) - 1.0) < 1e-15
        for b in g:
            assert min(np.abs(a @ b - c).max() for c in g) < 1e-15        # closure
    assert any(np.abs(a @ b - b @ a).max() > 0.5 for a in g for b in g)


def test_majorana_rotation_is_the_mode_rotation_and_a_representation():
    g = na.quaternion_group()
    cs = ga.majorana_matrices(2)
    # the module's sparse Majoranas are those of the dense Jordan-Wigner construction
    for a, b in zip(na.majoranas_sparse(3), ga.majorana_matrices(3)):
        assert np.abs(a.toarray() - b).max() == 0.0
    # a generic unitary as well (product of a group element and a real rotation by 0.3 with a phase)
    c, s = np.cos(0.3), np.sin(0.3)
    extra = g[2] @ np.array([[c, s], [-s, c]]) * np.exp(0.7j)
    for u in g + [extra]:
        o = na.majorana_rotation(u)
        assert np.abs(o @ o.T - np.eye(4)).max() < 1e-14
        v = na.mode_unitary(u)
        for b in range(4):
            lhs = v @ cs[b] @ v.conj().T
            rhs = sum(o[a, b] * cs[a] for a in range(4))
            assert np.abs(lhs - rhs).max() < 1e-12
    for a in g:
        for b in g:
            assert np.abs(na.majorana_rotation(a @ b) - na.majorana_rotation(a) @ na.majorana_rotation(b)).max() < 1e-14


def test_weight_formula_equals_fock_contraction():
    rng = np.random.default_rng(11)
    d, n_phys = 2, 2
    n_maj = 2 * (n_phys + 4 * d)
    gl = _random_pure_even(n_maj, rng)
    bond = _bond_state(d)
    gb = ga.covariance_of_state(bond, 2 * d).real
    an = na.NonAbelianAnsatz(2, 1, gl, gb, na.quaternion_group(), n_phys)
    site = na.pure_state(gl, n_phys + 4 * d)
    for _ in range(5):
        links = rng.integers(0, 8, size=an.n_links)
        w_fock = na.fock_weight(an, links, site, bond)
        w_cov = np.exp(an.log_weight(links))
        assert abs(w_cov - w_fock) <= 1e-10 * w_fock, (links, w_cov, w_fock)


def test_link_ratio_by_determinant_lemma():
    rng = np.random.default_rng(12)
    d, n_phys = 2, 2
    gl = _random_pure_even(2 * (n_phys + 4 * d), rng)
    gb = ga.covariance_of_state(_bond_state(d), 2 * d).real
    an = na.NonAbelianAnsatz(3, 2, gl, gb, na.quaternion_group(), n_phys)
    links = rng.integers(0, 8, size=an.n_links)
    ginv = np.linalg.inv(an.assemble_M(links))
    lw = an.log_weight(links)
    for ell in range(an.n_links):
        k_new = (int(links[ell]) + 1 + int(rng.integers(0, 7))) % 8
        new = links.copy()
        new[ell] = k_new
        ref = np.exp(an.log_weight(new) - lw)
        assert abs(an.link_ratio(ginv, links, ell, k_new) - ref) <= 1e-10 * ref


def test_plaquette_trace_is_gauge_invariant():
    rng = np.random.default_rng(13)
    gl = _random_pure_even(2 * (2 + 8), rng)
    gb = ga.covariance_of_state(_bond_state(2), 4).real
    an = na.NonAbelianAnsatz(3, 3, gl, gb, na.quaternion_group(), 2)
    for _ in range(5):
        links = rng.integers(0, 8, size=an.n_links)
        h = rng.integers(0, 8, size=an.V)
        moved = an.gauge_transform(links, h)
        for i in range(an.V):
            assert abs(an.plaquette_trace(moved, i) - an.plaquette_trace(links, i)) < 1e-14
    # a wrong orientation (one link not inverted) is not invariant for this non-abelian group: on a
    # configuration whose wrong loop has a nonzero trace, some gauge transformation flips its sign
    e = an.elements

    def wrong(lk, i):
        x1, x2 = i % an.lx, i // an.lx
        a, b = an.site(x1 + 1, x2), an.site(x1, x2 + 1)
        u = e[int(lk[2 * i])] @ e[int(lk[2 * a + 1])] @ e[int(lk[2 * b])] @ e[int(lk[2 * i + 1])].conj().T
        return np.trace(u) / 2
    links = rng.integers(0, 8, size=an.n_links)
    while abs(wrong(links, 0)) < 0.5:
        links = rng.integers(0, 8, size=an.n_links)
    diffs = [abs(wrong(an.gauge_transform(links, rng.integers(0, 8, size=an.V)), 0) - wrong(links, 0))
             for _ in range(40)]
    assert max(diffs) > 0.5
