"""Pins of the learned-proposal oracle (masked-patch convolutional conditional, block MH).

* the valid 3x3 convolution equals an explicit sum over its definition;
* gradients equal central finite differences of the loss;
* the mask: patch links do not reach the logits, links beyond the 4-site halo
  do not either, window links do;
* bf16 rounding and the Adam step against closed forms;
* exact stationarity of the block-MH transition matrix on the 2x2 lattice
  (p(G) from exhaustive enumeration is invariant under one patch move), also
  with a move rate rho < 1, whose draw rule is checked against its density;
* a long block-move chain reproduces exhaustive enumeration (rho = 1 and 1/2).
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import nn
from oracle.chain import WoodburyChain, block_move, block_sweep
from oracle.lattice import Lattice
from oracle.model import Ansatz


def test_conv_matches_definition():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 6, 7))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = nn.conv(x, w, b)
    ref = np.zeros((4, 4, 5))
    for o in range(4):
        for y in range(4):
            for xx in range(5):
                ref[o, y, xx] = b[o] + sum(w[o, c, dy, dx] * x[c, y + dy, xx + dx]
                                           for c in range(3) for dy in range(3) for dx in range(3))
    assert np.abs(out - ref).max() < 1e-12


def test_parameter_count_and_split():
    p = np.arange(nn.n_params(), dtype=np.float32)
    assert nn.n_params() == 2 * 32 * 9 + 32 + 2 * (32 * 32 * 9 + 32) + 32 * 2 * 9 + 2
    parts = nn.split(p)
    assert parts[0][0].shape == (32, 2, 3, 3) and parts[3][0].shape == (2, 32, 3, 3)
    assert parts[3][1][-1] == nn.n_params() - 1


@pytest.mark.parametrize("P", [1, 2, 4])
def test_gradient_matches_finite_differences(P):
    rng = np.random.default_rng(P)
    L = max(4, 2 * P)
    params = (nn.init_params(7) + 0.05 * rng.standard_normal(nn.n_params())).astype(np.float32)
    params[nn.n_params() - 2:] = [0.3, -0.2]
    links = rng.integers(0, 2, 2 * L * L)
    ex = [(nn.window(links, L, P, p), links[nn.patch_links(L, P, p)].astype(float)) for p in range((L // P) ** 2)][:3]
    _, g = nn.loss_and_grad(params, ex, round_bf16=False)
    idx = rng.choice(nn.n_params(), 40, replace=False)
    idx = np.concatenate([idx, [0, 575, 576, nn.n_params() - 1]])
    for i in idx:
        h = 1e-3
        pp = params.astype(np.float64).copy()
        pm = pp.copy()
        pp[i] += h
        pm[i] -= h

        def loss(q):
            tot = 0.0
            for x, y in ex:
                z, _ = nn.forward(q, x, np.float64, round_bf16=False)
                tot += nn.bce_loss(nn.logits_patch_order(z), y)
            return tot / len(ex)

        fd = (loss(pp) - loss(pm)) / (2 * h)
        assert abs(fd - g[i]) < 1e-4 * max(1.0, abs(fd)), (i, fd, g[i])


def test_mask_and_receptive_field():
    rng = np.random.default_rng(3)
    L, P, p = 16, 4, 5
    params = nn.init_params(11)
    links = rng.integers(0, 2, 2 * L * L)
    z0, _ = nn.forward(params, nn.window(links, L, P, p))
    pl = nn.patch_links(L, P, p)
    l2 = links.copy()
    l2[pl] = 1 - l2[pl]                         # patch links are masked
    z1, _ = nn.forward(params, nn.window(l2, L, P, p))
    assert np.array_equal(z0, z1)
    ox, oy = nn.patch_origin(L, P, p)
    far = ((oy + 10) % L) * L + (ox + 10) % L     # beyond the 4-site halo
    l3 = links.copy()
    l3[2 * far] ^= 1
    assert np.array_equal(nn.forward(params, nn.window(l3, L, P, p))[0], z0)
    near = ((oy - 2) % L) * L + (ox + 1) % L      # inside the window
    l4 = links.copy()
    l4[2 * near + 1] ^= 1
    assert not np.array_equal(nn.forward(params, nn.window(l4, L, P, p))[0], z0)


def test_bf16_rounding_and_bce():
    x = np.array([1.0, 1.00390625, 1.005859375, -2.5, 3.14159265], np.float32)
    r = nn.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0            # tie rounds to even
    assert r[2] == np.float32(1.0078125)
    assert r[3] == -2.5
    assert abs(r[4] - 3.140625) < 1e-7
    assert nn.bce_loss(np.zeros(6), np.array([0, 1, 0, 1, 1, 0])) == pytest.approx(6 * np.log(2))


def test_adam_first_step():
    p = np.array([1.0, -2.0, 0.5], np.float32)
    g = np.array([0.3, -1e-3, 0.0])
    m = np.zeros(3, np.float32)
    v = np.zeros(3, np.float32)
    p1, m1, v1 = nn.adam_step(p, g, m, v, 1, 0.01)
    expect = p - 0.01 * g / (np.abs(g) + 1e-8)
    assert np.abs(p1 - expect).max() < 1e-6


def _exact_transition_rho(an, params, P, patch, weights, rho):
    """Transition matrix of one block move with move rate rho, its proposal probabilities taken from
    the oracle's draw rule (link l becomes 1 with probability propose_p1) and its acceptance from the
    oracle's proposal densities log_q_move; also checks that the two agree."""
    L = an.lat.Lx
    n_links = an.lat.n_links
    states = list(itertools.product(range(2), repeat=n_links))
    index = {s: i for i, s in enumerate(states)}
    T = np.zeros((len(states), len(states)))
    pl = nn.patch_links(L, P, patch)
    for i, s in enumerate(states):
        k = np.array(s, np.int8)
        z, _ = nn.forward(params, nn.window(k, L, P, patch), np.float32)
        zl = nn.logits_patch_order(z).astype(np.float64)
        y_old = k[pl].astype(float)
        p1 = nn.propose_p1(zl, y_old, rho)
        stay = 1.0
        for ynew in itertools.product(range(2), repeat=len(pl)):
            ynew = np.array(ynew, float)
            q = float(np.prod(np.where(ynew == 1.0, p1, 1.0 - p1)))
            assert abs(q - np.exp(nn.log_q_move(zl, ynew, y_old, rho))) < 1e-14
            if np.array_equal(ynew, y_old):
                continue
            k2 = k.copy()
            k2[pl] = ynew.astype(np.int8)
            j = index[tuple(k2)]
            back = np.exp(nn.log_q_move(zl, y_old, ynew, rho))
            a = min(1.0, weights[j] * back / (weights[i] * q))
            T[i, j] = q * a
            stay -= q * a
        T[i, i] = stay
    return T


def _exact_transition(an, params, P, patch, weights):
    """Transition matrix of one block move on `patch` over all configurations (Z2, small lattice)."""
    L = an.lat.Lx
    n_links = an.lat.n_links
    states = list(itertools.product(range(2), repeat=n_links))
    index = {s: i for i, s in enumerate(states)}
    T = np.zeros((len(states), len(states)))
    pl = nn.patch_links(L, P, patch)
    for i, s in enumerate(states):
        k = np.array(s, np.int8)
        z, _ = nn.forward(params, nn.window(k, L, P, patch), np.float32)
        zl = nn.logits_patch_order(z).astype(np.float64)
        y_old = k[pl].astype(float)
        stay = 1.0
        for ynew in itertools.product(range(2), repeat=len(pl)):
            ynew = np.array(ynew, float)
            if np.array_equal(ynew, y_old):
                continue
            q = np.exp(nn.log_q(zl, ynew))
            k2 = k.copy()
            k2[pl] = ynew.astype(np.int8)
            j = index[tuple(k2)]
            a = min(1.0, weights[j] * np.exp(nn.log_q(zl, y_old)) / (weights[i] * q))
            T[i, j] = q * a
            stay -= q * a
        T[i, i] = stay
    return T


def test_block_move_exact_stationarity_2x2():
    lat = Lattice(2, 2)
    spec = synth.make_tensor(2)
    an = Ansatz(lat, spec.gamma_loc, spec.gamma_bond, 2)
    w = np.array([an.weight(np.array(s, np.int8)) for s in itertools.product(range(2), repeat=8)])
    pi = w / w.sum()
    params = nn.init_params(5)
    params[-2:] = [0.4, -0.7]
    for patch in range(4):
        T = _exact_transition(an, params, 1, patch, w)
        assert np.abs(T.sum(1) - 1).max() < 1e-12
        assert np.abs(pi @ T - pi).max() < 1e-14


@pytest.mark.parametrize("rho", [0.5, 0.125])
def test_block_move_rate_exact_stationarity_2x2(rho):
    """Move rate rho < 1 (each patch link kept with probability 1 - rho): the oracle's draw rule
    and its proposal density agree, and the block-MH transition matrix leaves p(G) invariant, on
    2x2 with P = 1 (one link per patch) and P = 2 (every link of the lattice in one patch)."""
    lat = Lattice(2, 2)
    spec = synth.make_tensor(2)
    an = Ansatz(lat, spec.gamma_loc, spec.gamma_bond, 2)
    w = np.array([an.weight(np.array(s, np.int8)) for s in itertools.product(range(2), repeat=8)])
    pi = w / w.sum()
    params = nn.init_params(5)
    params[-2:] = [0.4, -0.7]
    for P, patches in ((1, range(4)), (2, range(1))):
        for patch in patches:
            T = _exact_transition_rho(an, params, P, patch, w, rho)
            assert np.abs(T.sum(1) - 1).max() < 1e-12
            assert np.abs(pi @ T - pi).max() < 1e-14


def test_block_move_rate_one_is_the_factorised_proposal():
    rng = np.random.default_rng(3)
    z = rng.standard_normal(32)
    y0 = (rng.random(32) < 0.5).astype(float)
    y1 = (rng.random(32) < 0.5).astype(float)
    assert np.array_equal(nn.propose_p1(z, y0, 1.0), nn.sigmoid(z))
    a = nn.log_q_move(z, y0, y1, 1.0) - nn.log_q_move(z, y1, y0, 1.0)
    assert abs(a - (nn.log_q(z, y0) - nn.log_q(z, y1))) < 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("rho", [1.0, 0.5])
def test_block_chain_matches_enumeration_2x2(rho):
    lat = Lattice(2, 2)
    spec = synth.make_tensor(2)
    an = Ansatz(lat, spec.gamma_loc, spec.gamma_bond, 2)
    states = [np.array(s, np.int8) for s in itertools.product(range(2), repeat=8)]
    w = np.array([an.weight(s) for s in states])
    exact = sum(wi * an.plaquette(s) for wi, s in zip(w, states)) / w.sum()
    params = nn.init_params(5)
    ch = WoodburyChain(an, synth.SEED_CHAIN, 0)
    series = []
    acc = [0, 0]
    for _ in range(3000):
        st = block_sweep(ch, params, 1, rho=rho)
        acc[0] += st[0]
        acc[1] += st[1]
        series.append(an.plaquette(ch.k))
    series = np.array(series[300:])
    from oracle import stats
    tau, _, _ = stats.tau_int(series)
    err = np.std(series) * np.sqrt(2 * tau / len(series))
    assert acc[1] > 0.1 * acc[0]
    assert abs(series.mean() - exact) < 4 * err


def _route_params(seed, bias):
    rng = np.random.default_rng(seed)
    p = (nn.init_params(seed) + 0.02 * rng.standard_normal(nn.n_params())).astype(np.float32)
    p[-2:] = bias
    return p


@pytest.mark.parametrize("L,P,K,bias,sweeps", [
    (4, 2, 2, 0.0, 3),    # K = 2 on a 4x4 lattice: proposals change about half of the 8 patch links
    (4, 2, 3, -1.0, 3),
    (4, 4, 4, -1.5, 2),   # one patch covering the lattice, every patch link of the superposition inside
    (8, 4, 2, -3.0, 2),   # the shape of the GPU bit-exact block-move case with K = 2
])
def test_block_move_routes_agree(L, P, K, bias, sweeps):
    """The K > 1 block-move weight by full Pfaffians of every M_nm (the definition) and by the
    patch lemma on a fresh inverse take identical decisions and give N(G) within 1e-10: the
    patch route is used only where full Pfaffians are out of reach (lattices above 8 x 8)."""
    spec = synth.make_tensor(2, K=K)
    lat = Lattice(L, L)
    links, gk = synth.patch_bonds(lat.n_links, K)
    an = Ansatz(lat, spec.gamma_loc, spec.gamma_bond, 2, links, gk, spec.c)
    params = _route_params(13, bias)
    chains = {r: WoodburyChain(an, synth.SEED_CHAIN, 0) for r in ("def", "patch")}
    moves = 0
    for _ in range(sweeps):
        for p in range((L // P) ** 2):
            out = {r: block_move(ch, params, P, p, r) for r, ch in chains.items()}
            assert out["def"] == out["patch"]
            moves += out["def"][0]
            assert np.array_equal(chains["def"].k, chains["patch"].k)
        for ch in chains.values():
            ch.sweep_idx += 1
    assert moves > 0
    assert chains["def"].ties == chains["patch"].ties == 0
    k = chains["def"].k
    s_def, s_patch = an.s_factor_def(k), an.s_factor_patch(np.linalg.inv(an.assemble_M(k))[np.ix_(an.S, an.S)], k)
    assert abs(s_def - s_patch) < 1e-10 * abs(s_def)
