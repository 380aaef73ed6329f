"""Pins of the oracle's gauge observables -- the plaquette (Sec. 2.3) and the 2x2
Wilson loop (Sec. 5.1) -- and of the meson strings at separation r >= 2 (Sec. 5.2).

The gauge observables are fixed by facts of lattice geometry and gauge theory
that do not restate the oracle's formulas: a gauge transformation at any site
leaves every loop unchanged (this fixes the orientation of each link in each
loop), one changed link changes exactly the loops whose boundary contains it
(two plaquettes, four 2x2 loops), a 2x2 loop of an abelian field is the product
of the four plaquettes it encloses, and the cold configuration gives 1.  The
meson strings are compared with a dense Fock-space expectation of
phi_x^+ phi_{x+r e1} on a 4x1 ring, the smallest lattice with r = 2.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import gaussian
from oracle.fock import FockPEPS
from oracle.lattice import Lattice
from oracle.model import Ansatz, OBS_MESON0


def _ansatz(Lx, Ly, group, K=1):
    lat = Lattice(Lx, Ly)
    spec = synth.make_tensor(2, K=K, group=group)
    if K > 1:
        links, gk = synth.patch_bonds(lat.n_links, K)
        spec.patch_link, spec.gamma_bond_k = links, gk
    return lat, spec, Ansatz(lat, spec.gamma_loc, spec.gamma_bond, group, spec.patch_link,
                             spec.gamma_bond_k, spec.c)


def _values(an, k):
    V = an.lat.V
    return (np.array([an.plaquette_value(k, x) for x in range(V)]),
            np.array([an.wilson2x2_value(k, x) for x in range(V)]))


@pytest.mark.parametrize("group", [2, 3, 5])
def test_cold_configuration_gives_one(group):
    lat, _, an = _ansatz(4, 6, group)
    k = np.zeros(lat.n_links, np.int64)
    assert an.plaquette(k) == 1.0 and an.wilson2x2(k) == 1.0


@pytest.mark.parametrize("Lx,Ly,group", [(4, 4, 3), (6, 4, 5), (4, 6, 3), (4, 4, 7)])
def test_gauge_transformation_leaves_every_loop_unchanged(Lx, Ly, group):
    """g_x = w^q at one site: U(x, mu) -> w^q U(x, mu) on the two links leaving x and
    U(y, mu) -> U(y, mu) w^-q on the two links entering it.  Every plaquette and 2x2 loop
    (complex values, not only their real parts) must be unchanged; a loop that took any of
    its links with the wrong orientation would pick up a phase w^(+-2q)."""
    lat, _, an = _ansatz(Lx, Ly, group)
    rng = np.random.default_rng(3)
    for _ in range(3):
        k = rng.integers(0, group, lat.n_links)
        p0, w0 = _values(an, k)
        for x in range(lat.V):
            q = int(rng.integers(1, group))
            k2 = k.copy()
            x1, x2 = lat.coords(x)
            k2[2 * x + 0] += q                           # x -> x + e1 leaves x
            k2[2 * x + 1] += q                           # x -> x + e2 leaves x
            k2[2 * lat.site(x1 - 1, x2) + 0] -= q        # x - e1 -> x enters x
            k2[2 * lat.site(x1, x2 - 1) + 1] -= q        # x - e2 -> x enters x
            k2 %= group
            p1, w1 = _values(an, k2)
            assert np.abs(p1 - p0).max() < 1e-13, (x, q)
            assert np.abs(w1 - w0).max() < 1e-13, (x, q)


@pytest.mark.parametrize("Lx,Ly,group", [(4, 4, 2), (4, 4, 3), (6, 4, 5)])
def test_one_link_changes_two_plaquettes_and_four_wilson_loops(Lx, Ly, group):
    """Link (x, e1) bounds the plaquettes at x and x - e2 and the 2x2 loops at x, x - e1,
    x - 2e2, x - e1 - 2e2; link (x, e2) the plaquettes at x and x - e1 and the 2x2 loops at
    x, x - e2, x - 2e1, x - 2e1 - e2.  Raising the link by one multiplies one plaquette by w
    and the other by w^-1 (the link runs forward along one and backward along the other)."""
    lat, _, an = _ansatz(Lx, Ly, group)
    w = np.exp(2j * np.pi / group)
    rng = np.random.default_rng(5)
    k = rng.integers(0, group, lat.n_links)
    p0, w0 = _values(an, k)
    for ell in range(lat.n_links):
        x, mu = divmod(ell, 2)
        x1, x2 = lat.coords(x)
        if mu == 0:
            want_p = {x, lat.site(x1, x2 - 1)}
            want_w = {x, lat.site(x1 - 1, x2), lat.site(x1, x2 - 2), lat.site(x1 - 1, x2 - 2)}
        else:
            want_p = {x, lat.site(x1 - 1, x2)}
            want_w = {x, lat.site(x1, x2 - 1), lat.site(x1 - 2, x2), lat.site(x1 - 2, x2 - 1)}
        k2 = k.copy()
        k2[ell] = (k2[ell] + 1) % group
        p1, w1 = _values(an, k2)
        changed_p = set(np.flatnonzero(np.abs(p1 - p0) > 1e-12).tolist())
        changed_w = set(np.flatnonzero(np.abs(w1 - w0) > 1e-12).tolist())
        assert changed_p == want_p, ell
        assert changed_w == want_w, ell
        ratios = sorted([p1[s] / p0[s] for s in want_p], key=lambda z: np.angle(z))
        assert abs(ratios[0] * ratios[1] - 1.0) < 1e-13
        assert min(abs(ratios[0] - w), abs(ratios[0] - 1 / w)) < 1e-13


@pytest.mark.parametrize("Lx,Ly,group", [(4, 4, 2), (4, 6, 3), (6, 6, 5)])
def test_wilson2x2_is_the_product_of_its_four_plaquettes(Lx, Ly, group):
    """For an abelian field each interior link of the 2x2 square is traversed once in each
    direction by the four plaquettes it encloses, so W(x) = P(x) P(x+e1) P(x+e2) P(x+e1+e2)."""
    lat, _, an = _ansatz(Lx, Ly, group)
    rng = np.random.default_rng(7)
    for _ in range(4):
        k = rng.integers(0, group, lat.n_links)
        p, w = _values(an, k)
        for x in range(lat.V):
            x1, x2 = lat.coords(x)
            prod = p[x] * p[lat.site(x1 + 1, x2)] * p[lat.site(x1, x2 + 1)] * p[lat.site(x1 + 1, x2 + 1)]
            assert abs(w[x] - prod) < 1e-13
        assert abs(an.wilson2x2(k) - np.mean(w).real) < 1e-14
        assert abs(an.plaquette(k) - np.mean(p).real) < 1e-14


def test_z2_single_flip_means():
    """Z2, one link flipped from the cold configuration: two plaquettes and four 2x2 loops are -1."""
    lat, _, an = _ansatz(6, 4, 2)
    for ell in range(lat.n_links):
        k = np.zeros(lat.n_links, np.int64)
        k[ell] = 1
        assert abs(an.plaquette(k) - (1 - 4 / lat.V)) < 1e-14
        assert abs(an.wilson2x2(k) - (1 - 8 / lat.V)) < 1e-14


@pytest.mark.parametrize("K,group", [(1, 2), (1, 3), (2, 2), (2, 3)])
def test_meson_strings_r1_r2_against_fock(K, group):
    """M_r = (1/V) sum_x 2 Re[prod_{j<r} U(x + j e1, e1) <phi_x^+ phi_{x+r e1}>] for r = 1, 2 on a
    4x1 ring (20 modes) against the dense expectation of phi_x^+ phi_y, phi = (c_0 + i c_1)/2."""
    lat, spec, an = _ansatz(4, 1, group, K)
    fk = FockPEPS(lat, spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k)
    V = lat.V
    cs = gaussian.majorana_matrices(V)
    phi = [(cs[2 * x] + 1j * cs[2 * x + 1]) / 2 for x in range(V)]
    c = spec.c if K > 1 else None
    rng = np.random.default_rng(11)
    configs = [rng.integers(0, group, lat.n_links) for _ in range(3)]
    configs.append(np.array([0, 1, 1, 0, 0, 0, 1, 1]) % group)
    for k in configs:
        obs = an.observables(k)
        for r in (1, 2):
            tot = 0.0
            for x in range(V):
                x1, x2 = lat.coords(x)
                y = lat.site(x1 + r, x2)
                line = np.prod([np.exp(2j * np.pi * (k[2 * lat.site(x1 + j, x2)] % group) / group)
                                for j in range(r)])
                tot += 2 * line * fk.expect(k, phi[x].conj().T @ phi[y], c)
            assert abs(obs[OBS_MESON0 + r - 1] - (tot / V).real) < 1e-12, (r, k)


@pytest.mark.parametrize("L,K,group", [(2, 1, 2), (4, 1, 3), (2, 2, 2), (4, 3, 3), (4, 2, 2), (6, 4, 2)])
def test_observables_from_inverse_equal_the_definition(L, K, group):
    """Every observable slot from the maintained-inverse route (patch-lemma cross ratios, Woodbury
    transition inverses) equals the definition (full Pfaffians and inverses of every M_nm)."""
    lat = Lattice(L, L)
    spec = synth.make_tensor(L, K=K, group=group)
    an = Ansatz(lat, spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k, spec.c)
    rng = np.random.default_rng(31)
    for _ in range(2 if L < 6 else 1):
        k = rng.integers(0, group, lat.n_links)
        ref = an.observables(k)
        got = an.observables_from_inverse(k, np.linalg.inv(an.assemble_M(k)))
        assert np.abs(got - ref).max() < 1e-10, np.abs(got - ref).max()
