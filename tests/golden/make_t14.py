"""Write the stored decision sequences of the long single-link chains (T14) from the oracle.

Calls only ``oracle/`` (and ``synth`` for the seeded inputs).  Two runs of the
Sec. 5.1 estimator's Metropolis chain, each decision taken from a fresh
log-determinant of M(G') (the definition, ``DefinitionChain``):

* ``t14_c1.txt``: Z2 on the 2x2 periodic lattice, K = 1, cold start, chain 0,
  10^4 sweeps; the link field after every sweep (8 links, bit l = k_l, two hex
  digits per sweep);
* ``t14_c2.txt``: Z2 on the 8x8 periodic lattice, K = 1, hot start, chains
  0..7 (and 2047, 4095, sampled chains of the 4096-chain launch), 1000 sweeps;
  per chain the CRC-32 of the link field (128 bytes, one per link) after every
  sweep and the final link field.

Each file also holds, per chain, the accepted flips, the near ties
(|u - R| < 1e-9 R) and the final log W from a fresh determinant.

Usage: python tests/golden/make_t14.py [c1|c2|all]   (c2 takes about 25 minutes on 8 cores)
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys
import zlib

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

C1 = dict(L=2, sweeps=10000, chains=1, init=0)
C2 = dict(L=8, sweeps=1000, chains=[0, 1, 2, 3, 4, 5, 6, 7, 2047, 4095], init=1)


def _run(L, sweeps, chain, init):
    import threadpoolctl
    threadpoolctl.threadpool_limits(1)
    import synth
    from oracle.chain import DefinitionChain, hot_links
    from oracle.lattice import Lattice
    from oracle.model import Ansatz
    spec = synth.make_tensor(L)
    an = Ansatz(Lattice(L, L), spec.gamma_loc, spec.gamma_bond, 2)
    l0 = hot_links(synth.SEED_CHAIN, chain, an.lat.n_links, 2) if init == 1 else None
    ch = DefinitionChain(an, synth.SEED_CHAIN, chain, l0)
    fields = []
    for _ in range(sweeps):
        ch.sweep()
        fields.append(ch.k.copy())
    return chain, fields, ch.accepts, ch.ties, an.log_weight(ch.k)


def c1():
    cfg = C1
    chain, fields, acc, ties, logw = _run(cfg["L"], cfg["sweeps"], 0, cfg["init"])
    codes = ["%02x" % int(sum(int(v) << i for i, v in enumerate(f))) for f in fields]
    with open(os.path.join(HERE, "t14_c1.txt"), "w") as f:
        f.write("# T14 C1: Z2 2x2 periodic, K=1, cold start, chain 0, seed key 4, 10000 sweeps, single-link\n")
        f.write("# Metropolis (Sec. 5.1), decisions from a fresh log-determinant per proposal (oracle DefinitionChain).\n")
        f.write("# Written by tests/golden/make_t14.py (oracle only).  Link field after each sweep: one byte,\n")
        f.write("# bit l = k_l, 2 hex digits per sweep, 100 sweeps per data line.\n")
        f.write(f"chain 0 accepts {acc} near_ties {ties} logw {float(logw)!r}\n")
        for i in range(0, len(codes), 100):
            f.write("".join(codes[i:i + 100]) + "\n")


def c2():
    cfg = C2
    with mp.get_context("fork").Pool(min(len(cfg["chains"]), os.cpu_count() or 1)) as pool:
        res = pool.starmap(_run, [(cfg["L"], cfg["sweeps"], c, cfg["init"]) for c in cfg["chains"]])
    with open(os.path.join(HERE, "t14_c2.txt"), "w") as f:
        f.write("# T14 C2: Z2 8x8 periodic, K=1, hot start, chains 0..7, 2047, 4095, seed key 4, 1000 sweeps,\n")
        f.write("# single-link\n")
        f.write("# Metropolis (Sec. 5.1), decisions from a fresh log-determinant per proposal (oracle DefinitionChain).\n")
        f.write("# Written by tests/golden/make_t14.py (oracle only).  Per chain: a header line, the final link\n")
        f.write("# field (one hex digit per link), then the CRC-32 of the link field (128 bytes, one per link)\n")
        f.write("# after each sweep, 8 hex digits per sweep, 16 sweeps per line.\n")
        for chain, fields, acc, ties, logw in sorted(res, key=lambda r: r[0]):
            crcs = ["%08x" % zlib.crc32(np.asarray(fl, np.uint8).tobytes()) for fl in fields]
            f.write(f"chain {chain} accepts {acc} near_ties {ties} logw {float(logw)!r}\n")
            f.write("final " + "".join("%x" % int(v) for v in fields[-1]) + "\n")
            for i in range(0, len(crcs), 16):
                f.write(" ".join(crcs[i:i + 16]) + "\n")


def load(path):
    """Parse a stored file: {chain: {"accepts", "near_ties", "logw", "lines": [data lines]}}."""
    out, cur = {}, None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("chain "):
                t = line.split()
                cur = {"accepts": int(t[3]), "near_ties": int(t[5]), "logw": float(t[7]), "lines": []}
                out[int(t[1])] = cur
            else:
                cur["lines"].append(line)
    return out


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("c1", "all"):
        c1()
    if which in ("c2", "all"):
        c2()
