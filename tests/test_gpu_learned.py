"""GPU parity of the learned block proposal against the oracle (through the C ABI).

* network logits within 2e-5 of the oracle's float32 forward (same bf16 weights);
* gradients of the mean cross-entropy within 1e-3 relative of the oracle's
  float64 back-propagation;
* one Adam step against the closed form;
* block Metropolis-Hastings moves: link fields bit-exact against the oracle's
  definitional block move (fresh determinants, full Pfaffians of every M_nm for
  K > 1) after every sweep, mixed with single-link sweeps; log W and G within
  float64 tolerance; K = 1 and K = 2.
"""
import numpy as np
import pytest

import synth
from gpu_common import ansatz_for, gpu_context, oracle_chain, say, spec_for
from oracle import nn
from oracle.chain import block_sweep

pytestmark = pytest.mark.gpu


def _params(seed, scale=0.05):
    rng = np.random.default_rng(seed)
    p = (nn.init_params(seed) + scale * rng.standard_normal(nn.n_params())).astype(np.float32)
    p[-2:] = [0.3, -0.4]
    return p


@pytest.mark.parametrize("L,P", [(8, 4), (4, 2), (2, 1), (16, 4)])
def test_forward_matches_oracle(L, P):
    say(f"nn forward L={L} P={P}")
    spec = spec_for(L)
    ctx = gpu_context([spec], [L] * 3, init=1)
    ctx.nn_init(P, 11)
    params = ctx.nn_params(_params(3))
    npatch = (L // P) ** 2
    ch = [0, 1, 2, 1]
    pa = [0, npatch - 1, npatch // 2, 1 % npatch]
    z = ctx.nn_forward(ch, pa)
    for e in range(len(ch)):
        links, _ = ctx.get_state(ch[e])
        zr, _ = nn.forward(params, nn.window(links, L, P, pa[e]), np.float32)
        assert np.abs(z[e] - nn.logits_patch_order(zr)).max() < 2e-5


def test_init_matches_oracle():
    spec = spec_for(8)
    ctx = gpu_context([spec], [8])
    ctx.nn_init(4, 1234)
    assert np.array_equal(ctx.nn_params(), nn.init_params(1234))


@pytest.mark.parametrize("P", [4, 2])
def test_gradient_matches_oracle(P):
    say(f"nn grad P={P}")
    L = 8
    spec = spec_for(L)
    ctx = gpu_context([spec], [L] * 4, init=1)
    ctx.nn_init(P, 5)
    params = ctx.nn_params(_params(7))
    rng = np.random.default_rng(1)
    ch = rng.integers(0, 4, 24)
    pa = rng.integers(0, (L // P) ** 2, 24)
    loss, g = ctx.nn_grad(ch, pa)
    ex = []
    for c, p in zip(ch, pa):
        links, _ = ctx.get_state(int(c))
        ex.append((nn.window(links, L, P, int(p)), links[nn.patch_links(L, P, int(p))].astype(float)))
    lref, gref = nn.loss_and_grad(params, ex)
    assert abs(loss - lref) < 1e-4 * abs(lref)
    assert np.linalg.norm(g - gref) < 1e-3 * np.linalg.norm(gref)
    big = np.abs(gref) > 1e-2 * np.abs(gref).max()
    assert np.abs(g[big] - gref[big]).max() < 1e-3 * np.abs(gref).max()


def test_adam_step_matches_closed_form():
    L, P = 8, 4
    ctx = gpu_context([spec_for(L)], [L] * 2, init=1)
    ctx.nn_init(P, 9)
    p0 = ctx.nn_params()
    ctx.nn_train(1, 16, 1e-2, 77)
    p1 = ctx.nn_params()
    # first Adam step moves a parameter by lr * g / (|g| + eps): never more than lr,
    # and lr to within 1e-4 relative wherever |g| >> eps
    d = np.abs(p0 - p1).astype(np.float64)
    assert d.max() <= 1e-2 * (1 + 1e-5)
    assert np.mean(np.abs(d - 1e-2) < 1e-6) > 0.9


@pytest.mark.parametrize("L,P,K,mix,bias,init", [
    (8, 4, 1, False, -1.5, 0),    # about 6 of 32 links proposed to change: ranks up to ~40
    (8, 4, 2, True, -3.0, 0),
    (4, 2, 1, True, 0.0, 1),
    (8, 2, 1, False, -0.5, 1),
    (6, 2, 1, False, -1.0, 1),    # n = 288: ragged 64 x 128 update tiles
])
def test_block_moves_bit_exact(L, P, K, mix, bias, init):
    say(f"block moves L={L} P={P} K={K} mix={mix} bias={bias}")
    spec = synth.make_tensor(2, K=K)
    ctx = gpu_context([spec], [L] * 2, init=init)
    ctx.nn_init(P, 21)
    p = _params(13, 0.02)
    p[-2:] = bias
    params = ctx.nn_params(p)
    orc = [oracle_chain(spec, L, c, init=init)[1] for c in range(2)]
    for s in range(4):
        if mix and s % 2 == 1:
            ctx.sweep(1)
            for oc in orc:
                oc.sweep()
        else:
            ctx.block_sweep(1)
            for oc in orc:
                block_sweep(oc, params, P)
        for c, oc in enumerate(orc):
            links, info = ctx.get_state(c)
            assert np.array_equal(links, oc.k), (s, c)
            assert info["sweeps"] == oc.sweep_idx
    an = ansatz_for(spec, L)
    for c, oc in enumerate(orc):
        links, info = ctx.get_state(c)
        assert abs(info["logw"] - an.log_weight(links)) < 1e-9 * abs(info["logw"])
        G = ctx.get_inverse(c)
        Gt = np.linalg.inv(an.assemble_M(links))
        assert np.abs(G - Gt).max() < 1e-9 * np.abs(Gt).max()
        if K > 1:
            assert abs(info["s_re"] - an.s_factor_def(links).real) < 1e-8 * abs(info["s_re"])
    props = sum(ctx.block_stats(c)[0] for c in range(2))
    accs = sum(ctx.block_stats(c)[1] for c in range(2))
    assert props > 0 and accs > 0


@pytest.mark.parametrize("L,P,K,bias,pend,init", [
    (8, 4, 2, 0.0, 128, 1),   # about 16 of 32 links change: pairs of moves merge or overflow the capacity
    (8, 4, 1, -1.5, 128, 0),  # ranks ~24: several moves per update of G
    (8, 2, 1, -0.5, 24, 1),   # capacity below some single moves
    (6, 2, 2, 0.0, 64, 1),    # n = 288: ragged update tiles
    (4, 2, 4, 0.0, 128, 1),   # K = 4: twelve patch Majoranas in the pending correction
])
def test_block_moves_delayed_equal_immediate(L, P, K, bias, pend, init):
    """Delayed block moves (pending moves combined into one update of G, each decision on G_cur)
    against immediate ones and the oracle's definitional moves: the same decisions after every
    sweep, log W, S and G within float64 tolerance of each other and of the definitions, and
    fewer updates of G than accepted moves."""
    say(f"delayed block moves L={L} P={P} K={K} bias={bias} block_pend={pend}")
    spec = synth.make_tensor(2, K=K)
    ctxs = []
    for pv in (0, pend):
        ctx = gpu_context([spec], [L] * 3, init=init)
        ctx.set_option("block_pend", pv)
        ctx.nn_init(P, 21)
        p = _params(13, 0.02)
        p[-2:] = bias
        params = ctx.nn_params(p)
        ctxs.append(ctx)
    orc = [oracle_chain(spec, L, c, init=init)[1] for c in range(3)]
    for s in range(3):
        for ctx in ctxs:
            ctx.block_sweep(1)
        for oc in orc:
            # K > 1: the patch-lemma weight (decisions equal the definition's, test_block_move_routes_agree)
            block_sweep(oc, params, P, route="patch" if K > 1 else "def")
        for c, oc in enumerate(orc):
            for ctx in ctxs:
                assert np.array_equal(ctx.get_state(c)[0], oc.k), (s, c)
    an = ansatz_for(spec, L)
    imm, dly = ctxs
    for c in range(3):
        links, info = dly.get_state(c)
        info0 = imm.get_state(c)[1]
        assert abs(info["logw"] - an.log_weight(links)) < 1e-9 * abs(info["logw"])
        assert abs(info["logw"] - info0["logw"]) < 1e-10 * abs(info["logw"])
        Gt = np.linalg.inv(an.assemble_M(links))
        G1 = dly.get_inverse(c)
        assert np.abs(G1 - Gt).max() < 1e-9 * np.abs(Gt).max()
        assert np.abs(G1 - imm.get_inverse(c)).max() < 1e-10 * np.abs(Gt).max()
        if K > 1:
            assert abs(info["s_re"] - an.s_factor_def(links).real) < 1e-8 * abs(info["s_re"])
            assert abs(info["s_re"] - info0["s_re"]) < 1e-10 * abs(info["s_re"])
    st0 = np.array([imm.block_stats(c) for c in range(3)])
    st1 = np.array([dly.block_stats(c) for c in range(3)])
    assert np.array_equal(st0[:, :3], st1[:, :3])
    assert np.array_equal(st0[:, 3], st0[:, 1])              # immediate: one update per accepted move
    assert st1[:, 1].sum() > 0 and st1[:, 3].sum() < st1[:, 1].sum()
    say(f"accepted moves {st1[:, 1].tolist()}, updates of G {st1[:, 3].tolist()}")


@pytest.mark.parametrize("L,P,K,bias,rho,pend,init", [
    (8, 4, 1, 0.0, 0.25, 128, 0),     # about 4 of 32 patch links redrawn per move, delayed moves
    (8, 2, 2, 0.0, 0.5, 128, 1),
    (6, 2, 1, 0.5, 0.125, 0, 1),      # n = 288 (ragged tiles), each move applied at once
])
def test_block_moves_move_rate_bit_exact(L, P, K, bias, rho, pend, init):
    """Move rate rho < 1 (option block_rho): decisions against the oracle's block moves with the same
    rate after every sweep; log W, S and G within float64 tolerance of the definitions."""
    say(f"block moves with move rate {rho}: L={L} P={P} K={K} bias={bias} block_pend={pend}")
    spec = synth.make_tensor(2, K=K)
    ctx = gpu_context([spec], [L] * 2, init=init)
    ctx.set_option("block_pend", pend)
    ctx.set_option("block_rho", int(rho * 65536))
    ctx.nn_init(P, 21)
    p = _params(13, 0.02)
    p[-2:] = bias
    params = ctx.nn_params(p)
    orc = [oracle_chain(spec, L, c, init=init)[1] for c in range(2)]
    for s in range(3):
        ctx.block_sweep(1)
        for oc in orc:
            block_sweep(oc, params, P, route="patch" if K > 1 else "def", rho=rho)
        for c, oc in enumerate(orc):
            links, info = ctx.get_state(c)
            assert np.array_equal(links, oc.k), (s, c)
            assert info["sweeps"] == oc.sweep_idx
    an = ansatz_for(spec, L)
    for c in range(2):
        links, info = ctx.get_state(c)
        assert abs(info["logw"] - an.log_weight(links)) < 1e-9 * abs(info["logw"])
        Gt = np.linalg.inv(an.assemble_M(links))
        assert np.abs(ctx.get_inverse(c) - Gt).max() < 1e-9 * np.abs(Gt).max()
        if K > 1:
            assert abs(info["s_re"] - an.s_factor_def(links).real) < 1e-8 * abs(info["s_re"])
    st = np.array([ctx.block_stats(c) for c in range(2)])
    say(f"proposed {st[:, 0].tolist()}, accepted {st[:, 1].tolist()}, links changed {st[:, 2].tolist()}")
    assert st[:, 1].sum() > 0


def test_block_moves_fp32_with_refresh():
    """Float32 inverse, matrix-core float32 block updates, float64 refactorisation every 8 changed links."""
    say("block moves fp32 L=12 P=4 K=2")
    L, P, K = 12, 4, 2
    spec = synth.make_tensor(2, K=K)
    ctx = gpu_context([spec], [L] * 2, init=0, precision=32, refresh_every=8)
    ctx.nn_init(P, 21)
    p = _params(13, 0.02)
    p[-2:] = -1.5
    params = ctx.nn_params(p)
    orc = [oracle_chain(spec, L, c, init=0)[1] for c in range(2)]
    for s in range(3):
        ctx.block_sweep(1)
        for oc in orc:
            # full Pfaffians of order 1152 are out of reach here: the patch-lemma weight, whose
            # decisions equal the definition's on every case both run (test_block_move_routes_agree)
            block_sweep(oc, params, P, route="patch")
        for c, oc in enumerate(orc):
            assert np.array_equal(ctx.get_state(c)[0], oc.k), (s, c)
    an = ansatz_for(spec, L)
    for c in range(2):
        links, info = ctx.get_state(c)
        assert info["refreshes"] >= 1
        assert abs(info["logw"] - an.log_weight(links)) < 1e-5 * abs(info["logw"])
        Gt = np.linalg.inv(an.assemble_M(links))
        assert np.abs(ctx.get_inverse(c) - Gt).max() < 1e-4 * np.abs(Gt).max()
    assert sum(ctx.block_stats(c)[1] for c in range(2)) > 0


def test_training_learns_the_conditional_and_moves_blocks():
    """Online training on samples the plain sampler generates lowers the cross-entropy of the
    patch conditional; the trained network's block moves are accepted and change several links
    per accepted rank-4m update (one pass over G for m links, where single-link moves need m)."""
    say("training L=8 P=2")
    L, P, nc = 8, 2, 64
    ctx = gpu_context([spec_for(L)], [L] * nc, init=1)
    ctx.sweep(5)
    ctx.nn_init(P, 3)

    def block_rates():
        p0 = np.array([ctx.block_stats(c) for c in range(nc)])
        ctx.block_sweep(2)
        d = np.array([ctx.block_stats(c) for c in range(nc)]) - p0
        return d[:, 1].sum() / max(1, d[:, 0].sum()), d[:, 2].sum() / max(1, d[:, 1].sum())

    acc0, links0 = block_rates()
    loss0 = ctx.nn_grad(list(range(nc)), [0] * nc)[0]
    for _ in range(6):
        ctx.sweep(2)
        ctx.nn_train(40, 256, 3e-3, 99)
    loss1 = ctx.nn_grad(list(range(nc)), [0] * nc)[0]
    acc1, links1 = block_rates()
    say(f"cross-entropy {loss0:.3f} -> {loss1:.3f} nats/patch; block acceptance untrained {acc0:.3f} "
        f"({links0:.2f} links/accept), trained {acc1:.3f} ({links1:.2f} links/accept)")
    assert loss1 < 0.8 * loss0
    assert acc1 > 0.05 and links1 > 1.5


def _ess_between_chains(x):
    x = np.asarray(x, np.float64)
    se2 = x.mean(axis=0).var(ddof=1) / x.shape[1]
    return x.var(ddof=1) / se2


@pytest.mark.parametrize("L,K,tensor_seed,precision", [
    (8, 1, 16, 64),     # a tensor whose single-link acceptance is about 0.75: a conditional worth learning
    (16, 2, 1, 32),     # the 32x32 workload's ansatz (single-link acceptance 0.99) on a 16x16 lattice
])
def test_trained_network_gain_over_untrained(L, K, tensor_seed, precision):
    """What the trained network gains over the same block moves with an untrained (uniform) proposal, at
    equal patch size and chain count: acceptance, links changed per accepted move and effective samples
    of the plaquette per block sweep (spread of the chain means), for the trained network as trained
    (output scale 1) and with its output layer scaled by the beta in {0, 1/4, 1/2, 3/4, 1} that changes
    the most links per block sweep on the training chains, then the move rate rho in {1, 1/2, 1/4, 1/8}
    chosen the same way (adapted during burn-in, then frozen; beta = 0 is the uniform proposal, which is
    also run with its own best rate).  The gain is measured and reported; the test asserts that training
    lowered the cross-entropy of the patch conditional, that each chosen setting changes at least as many
    links per sweep on the training chains as the one it was chosen over, and that every sampler moves."""
    from oracle.stats import tau_int_chains
    P, nc, sweeps, n_last = 4, 128, 24, 2 * 32 * 9 + 2
    spec = synth.make_tensor(L, K=K, seed_tensor=tensor_seed)
    from paper_2412_01737_amd.ggf import OBS_LINK
    tr = gpu_context([spec], [L] * 64, init=1, precision=precision, refresh_every=4096)
    tr.nn_init(P, 3)
    loss0 = tr.nn_grad(list(range(64)), [0] * 64)[0]
    for s in range(8):
        tr.sweep(1)
        tr.nn_train(40, 256, 3e-3, 99 + s)
    loss1 = tr.nn_grad(list(range(64)), [0] * 64)[0]
    trained = tr.nn_params()
    def links_per_sweep(params, rho):
        tr.nn_params(params)
        tr.set_option("block_rho", int(rho * 65536))
        st0 = np.array([tr.block_stats(c) for c in range(64)])
        tr.block_sweep(2)
        return (np.array([tr.block_stats(c) for c in range(64)]) - st0)[:, 2].sum() / 128.0

    def scaled(beta):
        p = trained.copy()
        p[-n_last:] *= beta
        return p

    trials = {beta: links_per_sweep(scaled(beta), 1.0) for beta in (0.0, 0.25, 0.5, 0.75, 1.0)}
    beta = max(trials, key=trials.get)
    rates = {1.0: trials[beta]}
    rates.update({rho: links_per_sweep(scaled(beta), rho) for rho in (0.5, 0.25, 0.125)})
    rho = max(rates, key=rates.get)
    urates = {1.0: trials[0.0]}
    urates.update({r: links_per_sweep(scaled(0.0), r) for r in (0.5, 0.25, 0.125)})
    urho = max(urates, key=urates.get)
    tr.close()
    res = {}
    for name, params, r in (("trained", trained, 1.0), ("tuned", scaled(beta), rho),
                            ("uniform tuned", scaled(0.0), urho), ("untrained", scaled(0.0), 1.0)):
        ctx = gpu_context([spec], [L] * nc, init=1, precision=precision, refresh_every=4096)
        ctx.set_option("block_rho", int(r * 65536))
        ctx.nn_init(P, 3)
        ctx.nn_params(params)
        ctx.block_sweep(2)
        st0 = np.array([ctx.block_stats(c) for c in range(nc)])
        plaq = []
        for _ in range(sweeps):
            ctx.block_sweep(1)
            plaq.append(ctx.measure(OBS_LINK)[:, 0])
        st = np.array([ctx.block_stats(c) for c in range(nc)]) - st0
        plaq = np.array(plaq)
        res[name] = dict(acceptance=st[:, 1].sum() / max(1, st[:, 0].sum()),
                         links_per_move=st[:, 2].sum() / max(1, st[:, 1].sum()),
                         ess_per_sweep=_ess_between_chains(plaq) / sweeps,
                         tau=tau_int_chains(plaq)[0])
        ctx.close()
    u = res["untrained"]
    msg = [f"L={L} K={K} tensor seed {tensor_seed}: cross-entropy {loss0:.3f} -> {loss1:.3f} nats/patch; "
           f"links per sweep on the training chains by beta {dict((b, round(v, 2)) for b, v in trials.items())}, "
           f"chosen beta {beta}; by move rate at that beta {dict((q, round(v, 2)) for q, v in rates.items())}, "
           f"chosen {rho}; uniform proposal by move rate {dict((q, round(v, 2)) for q, v in urates.items())}, "
           f"chosen {urho}"]
    for name, r in res.items():
        msg.append(f"{name}: acceptance {r['acceptance']:.3f}, {r['links_per_move']:.2f} links/move, "
                   f"{r['ess_per_sweep']:.1f} ESS/sweep, tau {r['tau']:.2f}, "
                   f"gain x{r['ess_per_sweep'] / u['ess_per_sweep']:.2f}")
    say("; ".join(msg))
    assert loss1 < loss0
    assert trials[beta] >= trials[0.0] and rates[rho] >= trials[beta] and urates[urho] >= trials[0.0]
    for r in res.values():
        assert r["acceptance"] > 0 and np.isfinite(r["ess_per_sweep"])
