"""Write the stored decision sequences of sampled chains of an uneven batch from the oracle.

Calls only ``oracle/`` (and ``synth`` for the seeded inputs).  The batch is the
first 512 chains of the uneven workload's mix (synth.mixed_batch, seed 5: L in
{6, 8, 12, 16, 20}, K in {1, 2, 4}, Z2 or Z3 per chain), each (L, K, group)
with its own ansatz whose patch links are drawn on its own lattice
(synth.make_tensor(L, K, group)).  For the first chain of every (L, K, group)
present, hot start and two single-link Metropolis sweeps of the oracle's
Woodbury chain (Sec. 5.1; the Woodbury route is pinned to fresh determinants
and full Pfaffians on every lattice where those run).

Stored per chain: index, L, K, group, the link field after each sweep (one
hex digit per link), accepted flips, near ties and log W from a fresh
determinant.

Usage: python tests/golden/make_c4.py   (a few minutes on 8 cores)
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N_BATCH, SWEEPS = 512, 2


def sampled():
    """(chain, L, K, group) of the first chain of every (L, K, group) in the batch."""
    import synth
    Ls, Ks, gs = synth.mixed_batch(N_BATCH)
    seen, out = set(), []
    for c in range(N_BATCH):
        key = (int(Ls[c]), int(Ks[c]), int(gs[c]))
        if key not in seen:
            seen.add(key)
            out.append((c,) + key)
    return out


def run(c, L, K, group):
    import threadpoolctl
    threadpoolctl.threadpool_limits(1)
    import synth
    from oracle.chain import WoodburyChain, hot_links
    from oracle.lattice import Lattice
    from oracle.model import Ansatz
    spec = synth.make_tensor(L, K=K, group=group)
    an = Ansatz(Lattice(L, L), spec.gamma_loc, spec.gamma_bond, group, spec.patch_link, spec.gamma_bond_k, spec.c)
    ch = WoodburyChain(an, synth.SEED_CHAIN, c, hot_links(synth.SEED_CHAIN, c, an.lat.n_links, group))
    fields = []
    for _ in range(SWEEPS):
        ch.sweep()
        fields.append(ch.k.copy())
    return c, L, K, group, fields, ch.accepts, ch.ties, an.log_weight(ch.k)


def main():
    jobs = sampled()
    jobs.sort(key=lambda j: -j[1] ** 4 * j[2])          # largest first
    with mp.get_context("fork").Pool(os.cpu_count() or 1) as pool:
        res = pool.starmap(run, jobs)
    with open(os.path.join(HERE, "c4_uneven.txt"), "w") as f:
        f.write("# Uneven batch: first 512 chains of synth.mixed_batch (seed 5), one ansatz per (L, K, group) with\n")
        f.write("# patch links drawn on its own lattice, hot start, seed key 4; for the first chain of every\n")
        f.write("# (L, K, group): the link field after each of 2 single-link sweeps (oracle Woodbury chain,\n")
        f.write("# Sec. 5.1), one hex digit per link.  Written by tests/golden/make_c4.py (oracle only).\n")
        for c, L, K, group, fields, acc, ties, logw in sorted(res):
            f.write(f"chain {c} L {L} K {K} group {group} accepts {acc} near_ties {ties} logw {float(logw)!r}\n")
            for fl in fields:
                f.write("".join("%x" % int(v) for v in fl) + "\n")


def load(path):
    out, cur = {}, None
    with open(path) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "chain":
                cur = {"L": int(t[3]), "K": int(t[5]), "group": int(t[7]), "accepts": int(t[9]),
                       "near_ties": int(t[11]), "logw": float(t[13]), "fields": []}
                out[int(t[1])] = cur
            else:
                cur["fields"].append(np.array([int(ch, 16) for ch in t[0]], np.int8))
    return out


if __name__ == "__main__":
    main()
