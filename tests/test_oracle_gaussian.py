"""Pins of the oracle's Gaussian toolkit against hand values, closed forms and brute force.

Covers the Majorana/covariance conventions (Sec. 3.2), the Pfaffian, the
overlap formula (Sec. 3.2, with the sign reading for Pf((G1+G2)/2)), the bond
state, the worked contraction of the appendix on graphical Gaussian calculus,
and the Philox generator (published known-answer vectors).
"""
import os

import numpy as np
import pytest

import synth
from oracle import gaussian, philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_skew(rng, n, cplx=False):
    a = rng.standard_normal((n, n))
    if cplx:
        a = a + 1j * rng.standard_normal((n, n))
    return a - a.T


def _rand_pure_cov(rng, modes):
    o = synth.haar_orthogonal(rng, 2 * modes)
    j = -gaussian.vacuum_covariance(modes)
    return o @ j @ o.T


def test_single_mode_hand_values():
    """Empty mode -> [[0,-1],[1,0]], filled -> [[0,1],[-1,0]] under c0 = psi+psi^+, c1 = -i(psi-psi^+)."""
    vac = np.array([1, 0], complex)
    occ = np.array([0, 1], complex)
    assert np.allclose(gaussian.covariance_of_state(vac, 1), [[0, -1], [1, 0]])
    assert np.allclose(gaussian.covariance_of_state(occ, 1), [[0, 1], [-1, 0]])
    gv = gaussian.vacuum_covariance(1)
    assert gaussian.overlap_pure(gv, gv) == pytest.approx(1.0)          # tr(rho^2) = 1
    assert gaussian.overlap_pure(gv, -gv) == pytest.approx(0.0)         # orthogonal
    assert gaussian.overlap_pure(gv, np.zeros((2, 2))) == pytest.approx(0.5)  # with 1/2


def test_state_of_covariance_roundtrip():
    rng = np.random.default_rng(7)
    for modes in (1, 2, 3, 5):
        g = _rand_pure_cov(rng, modes)
        v = gaussian.state_of_covariance(g, modes)
        assert np.abs(gaussian.covariance_of_state(v, modes) - g).max() < 1e-12


@pytest.mark.parametrize("cplx", [False, True])
def test_pfaffian_matches_definition(cplx):
    rng = np.random.default_rng(11)
    for n in (2, 4, 6, 8):
        a = _rand_skew(rng, n, cplx)
        ref = gaussian.pfaffian_matchings(a)
        assert abs(gaussian.pfaffian(a) - ref) < 1e-11 * max(1, abs(ref))
        assert abs(gaussian.pfaffian_bruteforce(a) - ref) < 1e-11 * max(1, abs(ref))


def test_pfaffian_identities():
    rng = np.random.default_rng(12)
    for n in (10, 16, 24):
        a = _rand_skew(rng, n, True)
        pf = gaussian.pfaffian(a)
        det = np.linalg.det(a)
        assert abs(pf * pf - det) < 1e-9 * abs(det)
        # congruence: Pf(B A B^T) = det(B) Pf(A)
        b = rng.standard_normal((n, n))
        assert abs(gaussian.pfaffian(b @ a @ b.T) - np.linalg.det(b) * pf) < 1e-8 * abs(np.linalg.det(b) * pf)
    blk = np.zeros((6, 6))
    for i, v in enumerate((2.0, -3.0, 0.5)):
        blk[2 * i, 2 * i + 1], blk[2 * i + 1, 2 * i] = v, -v
    assert gaussian.pfaffian(blk) == pytest.approx(-3.0)
    assert gaussian.pfaffian(np.zeros((4, 4))) == 0


def test_overlap_formula_and_printed_sign():
    """tr(rho1 rho2) = 2^-N sqrt det(G1+G2); the printed Pf((G1+G2)/2) is right only up to sign."""
    rng = np.random.default_rng(3)
    cs = gaussian.majorana_matrices(3)
    signs = set()
    for _ in range(12):
        g1, g2 = _rand_pure_cov(rng, 3), _rand_pure_cov(rng, 3)
        v1 = gaussian.state_of_covariance(g1, 3, cs)
        v2 = gaussian.state_of_covariance(g2, 3, cs)
        tr = abs(np.vdot(v1, v2)) ** 2
        assert gaussian.overlap_pure(g1, g2) == pytest.approx(tr, abs=1e-13)
        pf = gaussian.pfaffian((g1 + g2) / 2)
        assert abs(abs(pf) - tr) < 1e-12
        if tr > 1e-6:
            signs.add(np.sign(pf.real))
    assert -1.0 in signs       # the printed identity fails in sign for some pairs


def test_reference_bond_covariance():
    """GAMMA_BOND0 is the covariance of (1 + psi_out^+ psi_in^+)|0>/sqrt2 (out mode first)."""
    v = np.zeros(4, complex)
    v[0] = v[3] = 1 / np.sqrt(2)        # |00> + |11>, |11> = psi_0^+ psi_1^+|0>
    g = gaussian.covariance_of_state(v, 2)
    assert np.abs(g - synth.GAMMA_BOND0).max() < 1e-15


def _fermion_ops(n_modes):
    """Dense psi_j^+ from the Majoranas: psi^+ = (c_2j - i c_2j+1)/2."""
    cs = gaussian.majorana_matrices(n_modes)
    return [(cs[2 * j] - 1j * cs[2 * j + 1]) / 2 for j in range(n_modes)]


def test_appendix_worked_contraction():
    """<B|T> for 2 virtual + 2 physical modes (appendix on graphical Gaussian calculus).

    Fock contraction gives (1 + B12 T12)|00> + (T34 + B12 Pf(T))|11> with
    Pf(T) = T12 T34 - T13 T24 + T14 T23; the printed +B12 T13 T24 is read as a
    sign typo, and this test shows the printed form disagrees.
    """
    import scipy.linalg
    rng = np.random.default_rng(5)
    cd = _fermion_ops(4)
    vac = np.zeros(16, complex)
    vac[0] = 1
    for _ in range(5):
        t = _rand_skew(rng, 4)
        b12 = rng.standard_normal()
        gen = sum(0.5 * t[i, j] * cd[i] @ cd[j] for i in range(4) for j in range(4))
        ket = scipy.linalg.expm(gen) @ vac
        bra = (np.eye(16) + b12 * cd[0] @ cd[1]) @ vac
        # <B| acts on modes 0,1 (first in JW order); project them back to the vacuum
        bra_op = (np.eye(16) + b12 * (cd[0] @ cd[1]).conj().T)
        w = bra_op @ ket
        amp00 = w[0b0000]
        amp11 = w[0b0011] * 1.0     # |11> on modes 2,3 = psi_2^+ psi_3^+|0>
        check = np.vdot(bra, ket)   # sanity: the |00> amplitude is the full overlap with B
        pf = t[0, 1] * t[2, 3] - t[0, 2] * t[1, 3] + t[0, 3] * t[1, 2]
        assert abs(amp00 - (1 + b12 * t[0, 1])) < 1e-12
        assert abs(check - amp00) < 1e-12
        assert abs(amp11 - (t[2, 3] + b12 * pf)) < 1e-12
        printed = t[2, 3] + b12 * t[0, 1] * t[2, 3] + b12 * t[0, 2] * t[1, 3] + b12 * t[0, 3] * t[1, 2]
        assert abs(amp11 - printed) > 1e-6


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert philox.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])
        vec = philox.philox_vec(*[np.array([x], np.uint64) for x in v[0:4]], v[4], v[5])
        assert tuple(int(x[0]) for x in vec) == tuple(v[6:10])


def test_philox_uniform_and_step():
    u, step = philox.draw(4, np.arange(1000), 3, 7)
    assert np.all((u >= 0) & (u < 1))
    assert set(np.unique(step)) == {1, 2}
    assert abs(u.mean() - 0.5) < 0.05
    x0, x1, x2, _ = philox.philox4x32_10((5, 3, 7, 0), (4, 0))
    u1, s1 = philox.draw(4, 5, 3, 7)
    assert float(u1) == (((x1 << 32) | x0) >> 11) * 2.0 ** -53
    assert int(s1) == 1 + (x2 & 1)
