"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Bars: accept/reject decisions bit-exact on shared Philox streams (compared as
the link field after every sweep: each link is visited once per sweep and a
proposal always changes it); float64 log-weights within 1e-10 relative; the
maintained inverse within 1e-10 of max|G|; observables within 1e-10 absolute
(float64).  Sizes span several Gauss-Jordan panels and update tiles, with a
ragged last panel (n = 8 L^2 is not a multiple of the panel width for L = 6).
"""
import numpy as np
import pytest

import synth
from gpu_common import ansatz_for, gpu_context, oracle_chain, say, spec_for

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,K,group,init", [(2, 1, 2, 0), (4, 1, 3, 1), (6, 1, 2, 1), (4, 2, 2, 0),
                                            (4, 3, 3, 1), (6, 4, 2, 0)])
def test_init_weight_inverse_and_cross_terms(L, K, group, init):
    say(f"init L={L} K={K} group={group} init={init}")
    spec = spec_for(L, K, group)
    ctx = gpu_context([spec], [L] * 3, init=init)
    for c in range(3):
        an, oc = oracle_chain(spec, L, c, init=init)
        links, info = ctx.get_state(c)
        assert np.array_equal(links, oc.k)
        assert abs(info["logw"] - oc.logw) <= 1e-10 * abs(oc.logw)
        G = ctx.get_inverse(c)
        assert np.abs(G - oc.G).max() <= 1e-10 * np.abs(oc.G).max()
        if K > 1:
            assert abs(info["s_re"] - oc.S.real) <= 1e-10 * abs(oc.S.real)


@pytest.mark.parametrize("L,K,group,init,sweeps,chains", [
    (2, 1, 2, 0, 200, 1),     # 2x2, the exhaustive-enumeration lattice
    (4, 1, 3, 1, 10, 3),
    (8, 1, 2, 0, 4, 4),       # 8x8 chains at their real shape
    (4, 2, 2, 1, 6, 2),
    (4, 3, 3, 0, 5, 2),
    (6, 4, 2, 1, 3, 2),
])
def test_accept_reject_bit_exact(L, K, group, init, sweeps, chains):
    say(f"chain parity L={L} K={K} group={group} init={init} sweeps={sweeps} chains={chains}")
    spec = spec_for(L, K, group)
    ctx = gpu_context([spec], [L] * chains, init=init)
    orc = [oracle_chain(spec, L, c, init=init)[1] for c in range(chains)]
    for s in range(sweeps):
        ctx.sweep(1)
        for c, oc in enumerate(orc):
            oc.sweep()
            links, info = ctx.get_state(c)
            assert np.array_equal(links, oc.k), f"chain {c} sweep {s}"
    for c, oc in enumerate(orc):
        _, info = ctx.get_state(c)
        assert info["accepts"] == oc.accepts
        assert info["proposals"] == sweeps * 2 * L * L
        assert abs(info["logw"] - oc.logw) <= 1e-10 * abs(oc.logw)
        if K > 1:
            assert abs(info["s_re"] - oc.S.real) <= 1e-9 * abs(oc.S.real)
        G = ctx.get_inverse(c)
        assert np.abs(G - oc.G).max() <= 1e-9 * np.abs(oc.G).max()


@pytest.mark.parametrize("L,K,group", [(2, 1, 2), (4, 1, 3), (6, 1, 2), (4, 2, 2), (4, 3, 3)])
def test_observables(L, K, group):
    say(f"observables L={L} K={K} group={group}")
    spec = spec_for(L, K, group)
    ctx = gpu_context([spec], [L] * 2, init=1)
    an = ansatz_for(spec, L)
    for _ in range(2):
        obs = ctx.measure()
        for c in range(2):
            links, _ = ctx.get_state(c)
            ref = an.observables(links)
            assert np.abs(obs[c] - ref).max() < 1e-10, (c, obs[c], ref)
        ctx.sweep(1)


def test_refresh_drift_fp64():
    say("refresh drift fp64 L=6")
    spec = spec_for(6)
    ctx = gpu_context([spec], [6] * 2, refresh_every=16)
    orc = [oracle_chain(spec, 6, c, refresh_every=16)[1] for c in range(2)]
    for _ in range(3):
        ctx.sweep(1)
        for c, oc in enumerate(orc):
            oc.sweep()
            assert np.array_equal(ctx.get_state(c)[0], oc.k)
    for c in range(2):
        info = ctx.get_state(c)[1]
        assert info["refreshes"] == 3
        assert info["max_drift"] < 1e-10


def test_fp32_updates_with_fp64_refresh():
    """Float32 inverse and updates, float64 refactorisation every 64 accepted flips."""
    say("fp32 L=6 K=2")
    spec = spec_for(6, K=2)
    ctx = gpu_context([spec], [6] * 2, precision=32, refresh_every=64)
    orc = [oracle_chain(spec, 6, c)[1] for c in range(2)]
    mismatch = 0
    for _ in range(4):
        ctx.sweep(1)
        for c, oc in enumerate(orc):
            oc.sweep()
            links, info = ctx.get_state(c)
            mismatch += int(not np.array_equal(links, oc.k))
    assert mismatch == 0
    for c, oc in enumerate(orc):
        info = ctx.get_state(c)[1]
        assert info["refreshes"] >= 1
        assert abs(info["logw"] - oc.logw) < 1e-4 * abs(oc.logw)
        assert info["max_drift"] < 1e-3


@pytest.mark.parametrize("nb", [8, 64, 128, 256])
def test_refactorisation_panel_widths(nb):
    """Blocked Gauss-Jordan with every panel width (recursive base panels, matrix-core update) at n = 2048."""
    say(f"refactorisation nb={nb} L=16")
    L = 16
    spec = spec_for(L)
    from paper_2412_01737_amd.ggf import Context
    ctx = Context(0)
    ctx.set_option("gj_nb", nb)
    tid = ctx.set_tensor_spec(spec)
    ctx.init_chains([L], tid, synth.SEED_CHAIN, init=1, precision=64)
    an = ansatz_for(spec, L)
    links, info = ctx.get_state(0)
    M = an.assemble_M(links)
    Gt = np.linalg.inv(M)
    assert abs(info["logw"] - an.log_weight(links)) < 1e-10 * abs(info["logw"])
    assert np.abs(ctx.get_inverse(0) - Gt).max() < 1e-10 * np.abs(Gt).max()


def test_checkpoint_resume_bit_exact():
    say("checkpoint resume L=4 Z3")
    spec = spec_for(4, 1, 3)
    a = gpu_context([spec], [4] * 2, init=1)
    a.sweep(6)
    b = gpu_context([spec], [4] * 2, init=1)
    b.sweep(3)
    saved = [b.get_state(c) for c in range(2)]
    b.close()
    c2 = gpu_context([spec], [4] * 2, init=0)
    for c, (links, info) in enumerate(saved):
        c2.set_state(c, links, info["sweeps"])
    c2.sweep(3)
    for c in range(2):
        la, ia = a.get_state(c)
        lc, ic = c2.get_state(c)
        assert np.array_equal(la, lc)
        assert ia["sweeps"] == ic["sweeps"] == 6
        assert abs(ia["logw"] - ic["logw"]) < 1e-10 * abs(ia["logw"])


def test_recovery_from_corrupted_inverse():
    say("recovery L=4")
    spec = spec_for(4)
    ctx = gpu_context([spec], [4] * 2)
    G = ctx.get_inverse(1)
    G[:] = np.nan
    ctx.set_inverse(1, G)
    ctx.sweep(1)
    links, info = ctx.get_state(1)
    assert info["recoveries"] == 1
    an = ansatz_for(spec, 4)
    assert abs(info["logw"] - an.log_weight(links)) < 1e-10 * abs(info["logw"])
    np.testing.assert_allclose(ctx.get_inverse(1), np.linalg.inv(an.assemble_M(links)), atol=1e-10)
    assert ctx.get_state(0)[1]["recoveries"] == 0


@pytest.mark.parametrize("delay", [0, 8, 24, 32])
def test_delayed_update_windows(delay):
    """Flips applied in windows of `delay` link steps (one rank-4 pass per accepted flip when 0) on 6x6 Z3 K=2:
    72 link steps give full and partial windows; decisions, log W, S and G against the oracle's one-flip-at-a-time
    Woodbury chain."""
    L, K, group, chains, sweeps = 6, 2, 3, 3, 3
    say(f"delayed updates window={delay} L={L} K={K} Z{group}")
    spec = spec_for(L, K, group)
    ctx = gpu_context([spec], [L] * chains, init=1, delay=delay)
    orc = [oracle_chain(spec, L, c, init=1)[1] for c in range(chains)]
    for s in range(sweeps):
        ctx.sweep(1)
        for c, oc in enumerate(orc):
            oc.sweep()
            assert np.array_equal(ctx.get_state(c)[0], oc.k), f"chain {c} sweep {s}"
    for c, oc in enumerate(orc):
        _, info = ctx.get_state(c)
        assert abs(info["logw"] - oc.logw) <= 1e-10 * abs(oc.logw)
        assert abs(info["s_re"] - oc.S.real) <= 1e-9 * abs(oc.S.real)
        G = ctx.get_inverse(c)
        assert np.abs(G - oc.G).max() <= 1e-9 * np.abs(oc.G).max()


@pytest.mark.parametrize("L,precision", [(8, 64), (6, 64), (2, 64), (8, 32)])
def test_window_flush_antisymmetric(L, precision):
    """G = M^-1 is antisymmetric (Sec. 3.2: M is); the window flush updates the 64 x 64 tiles on and above the
    diagonal and writes each tile below as the negated transpose of its mirror.  After a sweep the stored
    inverse is exactly antisymmetric with a zero diagonal, for full tiles (8x8: n = 512) and ragged ones
    (6x6: n = 288; 2x2: n = 32, one partial tile), and matches the oracle's one-flip-at-a-time inverse."""
    say(f"antisymmetric flush L={L} float{precision}")
    spec = spec_for(L, 1, 2)
    ctx = gpu_context([spec], [L] * 2, init=1, precision=precision, delay=16)
    orc = [oracle_chain(spec, L, c, init=1)[1] for c in range(2)]
    ctx.sweep(1)
    for c, oc in enumerate(orc):
        oc.sweep()
        assert np.array_equal(ctx.get_state(c)[0], oc.k), f"chain {c}"
        G = ctx.get_inverse(c)
        assert np.array_equal(G, -G.T), f"chain {c}: max |G + G^T| = {np.abs(G + G.T).max()}"
        tol = 1e-9 if precision == 64 else 1e-4
        assert np.abs(G - oc.G).max() <= tol * np.abs(oc.G).max()


def test_delay_window_changes_between_sweeps():
    """The window may change between sweeps (nothing is pending at a sweep's end)."""
    say("delay window changes")
    L = 4
    spec = spec_for(L, 2, 2)
    ctx = gpu_context([spec], [L] * 2, init=1, delay=8)
    orc = [oracle_chain(spec, L, c, init=1)[1] for c in range(2)]
    for s, d in enumerate([8, 32, 0, 16]):
        ctx.set_option("delay", d)
        ctx.sweep(1)
        for c, oc in enumerate(orc):
            oc.sweep()
            assert np.array_equal(ctx.get_state(c)[0], oc.k), f"chain {c} sweep {s} window {d}"
    G = ctx.get_inverse(1)
    assert np.abs(G - orc[1].G).max() <= 1e-9 * np.abs(orc[1].G).max()


@pytest.mark.parametrize("delay", [0, 8])
def test_uneven_batch_mixed_lattices(delay):
    """One context, chains of different L, K and group, lock-step over the longest sweep."""
    say(f"uneven batch window={delay}")
    # patch links drawn on the 2x2 lattice exist on every lattice of the batch
    specs = [spec_for(2, 1, 2), spec_for(2, 2, 3), spec_for(2, 3, 2)]
    Ls = [2, 4, 6, 4, 6, 2]
    tids = [0, 1, 2, 0, 1, 2]
    ctx = gpu_context(specs, Ls, tensor_ids=tids, init=1, delay=delay)
    orc = [oracle_chain(specs[t], L, c, init=1)[1] for c, (L, t) in enumerate(zip(Ls, tids))]
    for _ in range(3):
        ctx.sweep(1)
        for c, oc in enumerate(orc):
            oc.sweep()
            assert np.array_equal(ctx.get_state(c)[0], oc.k), c


def test_graph_replay_matches_direct_launches():
    say("graph replay")
    spec = spec_for(4, 2, 3)
    a = gpu_context([spec], [4] * 3, init=1)
    b = gpu_context([spec], [4] * 3, init=1)
    b.set_option("graph", 1)
    for _ in range(4):
        a.sweep(1)
        b.sweep(1)
        oa, ob = a.measure(), b.measure()     # eager work between replays
        assert np.array_equal(oa, ob)
        for c in range(3):
            assert np.array_equal(a.get_state(c)[0], b.get_state(c)[0])


def test_invalid_inputs_rejected():
    from paper_2412_01737_amd.ggf import Context, GGFError, GGF_EINVAL, GGF_ESTATE
    ctx = Context(0)
    spec = spec_for(4)
    with pytest.raises(GGFError) as e:
        ctx.sweep(1)
    assert e.value.status == GGF_ESTATE
    bad = spec.gamma_loc.copy()
    bad[0, 1] += 0.1
    with pytest.raises(GGFError) as e:
        ctx.set_tensor(2, bad, spec.gamma_bond)
    assert e.value.status == GGF_EINVAL
    for bad_group in (1, 65):                   # Z_N with 2 <= N <= 64
        with pytest.raises(GGFError):
            ctx.set_tensor(bad_group, spec.gamma_loc, spec.gamma_bond)
    tid = ctx.set_tensor_spec(spec)
    for L in (3, 0, 34):
        with pytest.raises(GGFError):
            ctx.init_chains([L], [tid], 1)
    with pytest.raises(GGFError):
        ctx.init_chains([4], [tid + 7], 1)
    for bad_delay in (12, 40, -2):
        with pytest.raises(GGFError):
            ctx.set_option("delay", bad_delay)
    for key, bad in (("block_pend", 129), ("block_rho", 0), ("block_rho", 65537), ("no_such_option", 1)):
        with pytest.raises(GGFError) as e:
            ctx.set_option(key, bad)
        assert e.value.status == GGF_EINVAL
    ctx.set_option("block_pend", 0)
    ctx.set_option("block_rho", 65536)
    ctx.init_chains([2], [tid], 1)
    ctx.sweep(0)
    with pytest.raises(GGFError):
        ctx.set_state(0, np.full(8, 2, np.int8), 0)
