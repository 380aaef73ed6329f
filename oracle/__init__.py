"""CPU FP64 oracle for gauged superposed Gaussian fermionic PEPS Monte Carlo.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything under ``oracle/``; only the test suite, the smoke check of
the package entry module and the CPU-baseline leg of the benchmark do.  The
oracle shares no code with the HIP library: it reads the seeded inputs from
``synth`` and computes everything else itself, in plain NumPy (library
primitives only: slogdet, inv, eigh, QR).

Modules (each function cites the passage of the paper it follows):

* ``philox``   -- Philox4x32-10 counter-based generator (Salmon et al., SC'11).
* ``gaussian`` -- Majorana conventions, covariance matrices, Pfaffians (Sec. 3.2).
* ``fock``     -- dense/sparse Jordan-Wigner Fock-space brute force of the
  gauged PEPS contraction <B|U(G)|A> (Sec. 3, 3.1, 4); the pin for everything.
* ``lattice``  -- geometry and index conventions.
* ``model``    -- weights, cross terms and observables in covariance form
  (Sec. 3.2, 5, 5.1, 5.2).
* ``chain``    -- the Metropolis chain over gauge configurations (Sec. 5.1),
  in a definitional mode (fresh determinant/Pfaffians per proposal) and an
  independent Woodbury mode.
* ``stats``    -- integrated autocorrelation time and effective sample size.
* ``nonabelian`` -- a non-abelian link group (Q8 in its 2-dimensional irrep) on
  2-mode virtual legs: weight and link ratio in covariance form, pinned by the
  Fock-space contraction on a 2 x 1 torus (Sec. 2.1, 3.2, 5; no kernel yet).
"""
