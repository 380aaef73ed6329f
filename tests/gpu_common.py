"""Shared helpers for the GPU parity tests (HIP library through the C ABI vs the oracle)."""
import sys

import numpy as np

import synth
from oracle.chain import WoodburyChain, hot_links
from oracle.lattice import Lattice
from oracle.model import Ansatz


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ansatz_for(spec, L):
    return Ansatz(Lattice(L, L), spec.gamma_loc, spec.gamma_bond, spec.group, spec.patch_link,
                  spec.gamma_bond_k, spec.c)


def spec_for(L, K=1, group=2):
    return synth.make_tensor(L, K=K, group=group)


def gpu_context(specs, Ls, seed=synth.SEED_CHAIN, init=0, precision=64, refresh_every=0, tensor_ids=None,
                delay=None):
    """Context with one chain per entry of Ls; specs: one spec per distinct tensor; delay: window of delayed
    updates in link steps (None = the library's default)."""
    from paper_2412_01737_amd.ggf import Context
    ctx = Context(0)
    if delay is not None:
        ctx.set_option("delay", delay)
    ids = [ctx.set_tensor_spec(s) for s in specs]
    tids = [ids[0]] * len(Ls) if tensor_ids is None else [ids[t] for t in tensor_ids]
    ctx.init_chains(Ls, tids, seed, init=init, precision=precision, refresh_every=refresh_every)
    return ctx


def oracle_chain(spec, L, chain, seed=synth.SEED_CHAIN, init=0, refresh_every=0):
    an = ansatz_for(spec, L)
    l0 = hot_links(seed, chain, an.lat.n_links, spec.group) if init == 1 else None
    return an, WoodburyChain(an, seed, chain, l0, refresh_every=refresh_every)
