"""Write the stored results of sampled chains of the 32x32 K=2 learned-proposal workload from the oracle.

Calls only ``oracle/`` (and ``synth`` for the seeded inputs).  Z2 on the 32x32
periodic lattice (n = 8192), K = 2 (one eps = 0.1 patch bond), hot start,
chains 0 and 255 of a 256-chain launch, one block sweep of learned
Metropolis-Hastings moves on the 64 4x4-site patches (Sec. 5.1 estimator with
the masked-patch proposal) with fixed network parameters: the seeded
Glorot-uniform initialisation (seed 13, float32) with both output biases
zero, so that every link is proposed with probability near 1/2 and most moves,
which change about 16 links, are accepted.  Each move's
weight N(G') / N(G) is taken from fresh LU factorisations of M(G') and M(G):
W from the determinant, N/W from the patch block of the inverse by the patch
lemma (full Pfaffians of order 8192 are out of reach; the patch route is pinned
to them on every case both can run).

Stored per chain: the link field after the hot start and after the block sweep
(one hex digit per link), the proposed and accepted moves, the near ties, log W
from a fresh determinant and the 21 observable slots from a fresh inverse
(maintained-inverse route of the oracle, pinned to the definition).

Usage: python tests/golden/make_c5.py   (about 30 minutes on 8 cores)
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

L, K, P = 32, 2, 4
CHAINS = (0, 255)
PARAM_SEED, BIAS = 13, 0.0


def params():
    from oracle import nn
    p = nn.init_params(PARAM_SEED).astype(np.float32)
    p[-2:] = BIAS
    return p


def run(chain):
    import threadpoolctl
    threadpoolctl.threadpool_limits(max(1, (os.cpu_count() or 2) // len(CHAINS)))
    import synth
    from oracle.chain import WoodburyChain, block_sweep, hot_links
    from oracle.lattice import Lattice
    from oracle.model import Ansatz
    spec = synth.make_tensor(L, K=K)
    an = Ansatz(Lattice(L, L), spec.gamma_loc, spec.gamma_bond, 2, spec.patch_link, spec.gamma_bond_k, spec.c)
    l0 = hot_links(synth.SEED_CHAIN, chain, an.lat.n_links, 2)
    ch = WoodburyChain(an, synth.SEED_CHAIN, chain, l0)
    prop, acc = block_sweep(ch, params(), P, route="patch")
    G = np.linalg.inv(an.assemble_M(ch.k))
    logw = an.log_weight(ch.k)
    obs = an.observables_from_inverse(ch.k, G, logw)
    return l0, ch.k.copy(), prop, acc, ch.ties, logw, obs


def main():
    import multiprocessing as mp
    with mp.get_context("fork").Pool(len(CHAINS)) as pool:
        results = pool.map(run, CHAINS)
    with open(os.path.join(HERE, "c5_block_sweep.txt"), "w") as f:
        f.write("# 32x32 Z2 K=2 (eps = 0.1 patch bond), hot start, seed key 4: one learned block sweep (4x4-site\n")
        f.write("# patches, network = oracle nn.init_params(13) as float32 with output biases 0), decisions\n")
        f.write("# from fresh LU factorisations (oracle block_move, patch route).  Written by\n")
        f.write("# tests/golden/make_c5.py (oracle only).  Per chain: header, link field after the hot start,\n")
        f.write("# link field after the sweep (one hex digit per link), then the 21 observable slots.\n")
        for c, (l0, k1, prop, acc, ties, logw, obs) in zip(CHAINS, results):
            f.write(f"chain {c} proposed {prop} accepted {acc} near_ties {ties} logw {float(logw)!r}\n")
            f.write("start " + "".join("%x" % int(v) for v in l0) + "\n")
            f.write("after " + "".join("%x" % int(v) for v in k1) + "\n")
            f.write("obs " + " ".join(repr(float(v)) for v in obs) + "\n")
            f.flush()


def load(path):
    out, cur = {}, None
    with open(path) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "chain":
                cur = {"proposed": int(t[3]), "accepted": int(t[5]), "near_ties": int(t[7]), "logw": float(t[9])}
                out[int(t[1])] = cur
            elif t[0] in ("start", "after"):
                cur[t[0]] = np.array([int(ch, 16) for ch in t[1]], np.int8)
            elif t[0] == "obs":
                cur["obs"] = np.array([float(v) for v in t[1:]])
    return out


if __name__ == "__main__":
    main()
