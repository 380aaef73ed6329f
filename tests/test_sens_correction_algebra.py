"""Algebra of the K > 1 sensitivities above n = 512, on the CPU in float64 (no GPU, no library).

For a pair (a, b) the library never forms M_ab^-1 = G + G_S Y_ab G_S^T: with A = G[:, S] and
AY = A Y_ab it reads M_ab^-1[r][c] = G[r][c] + sum_q AY[r][q] A[c][q], and the b-contracted blocks
sum_j M_ab^-1[r][8w + j] b[a][j] from G and Ab[2w + a][q] = sum_j b[a][j] A[8w + j][q].  Its electric
part expands the product of two rows of M_ab^-1,
  sum_l sum_{i<j} R_l[j][i] M[P][u_j] M[Q][u_i]
    = sum_l sum_{i<j} R_l[j][i] G[P][u_j] G[Q][u_i] + sum_q AY[Q][q] Xa[P][q] + sum_q AY[P][q] Xb[Q][q]
      + sum_{q,q'} AY[P][q] Z[q][q'] AY[Q][q'],
with Xa[P][q] = sum R[j][i] G[P][u_j] A[u_i][q], Xb[Q][q] = sum R[j][i] A[u_j][q] G[Q][u_i] and
Z[q][q'] = sum R[j][i] A[u_j][q] A[u_i][q'].  Each identity is checked against the matrix it replaces.
"""
import numpy as np


def _setup(seed, V=9, s=6):
    rng = np.random.default_rng(seed)
    n = 8 * V
    g = rng.standard_normal((n, n))
    G = g - g.T
    S = rng.choice(n, size=s, replace=False)
    y = rng.standard_normal((s, s)) + 1j * rng.standard_normal((s, s))
    Y = y - y.T
    A = G[:, S]
    AY = A @ Y
    M = G + A @ Y @ A.T
    return rng, n, G, A, AY, M


def test_entries_from_the_rank_s_correction():
    _, n, G, A, AY, M = _setup(1)
    assert np.abs(M - (G + AY @ A.T)).max() < 1e-12 * np.abs(M).max()
    assert np.abs(M + M.T).max() < 1e-12 * np.abs(M).max()      # M_ab^-1 stays antisymmetric


def test_b_contracted_blocks():
    rng, n, G, A, AY, M = _setup(2)
    b = rng.standard_normal((2, 8))
    V = n // 8
    Ab = np.einsum("aj,wjq->waq", b, A.reshape(V, 8, -1))          # Ab[w][a][q]
    for r in (0, 5, n - 1):
        for w in (0, 3, V - 1):
            ref = M[r, 8 * w:8 * w + 8] @ b.T                       # t_a = sum_j M[r][8w + j] b[a][j]
            got = G[r, 8 * w:8 * w + 8] @ b.T + AY[r] @ Ab[w].T
            assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_electric_expansion():
    rng, n, G, A, AY, M = _setup(3)
    nl = n // 4
    links = rng.permutation(n).reshape(nl, 4)                       # every Majorana on one link
    R = rng.standard_normal((nl, 4, 4)) + 1j * rng.standard_normal((nl, 4, 4))
    pairs = [(i, j) for i in range(4) for j in range(i + 1, 4)]
    Z = np.zeros((A.shape[1], A.shape[1]), complex)
    for ell in range(nl):
        u = links[ell]
        for i, j in pairs:
            Z += R[ell, j, i] * np.outer(A[u[j]], A[u[i]])
    for P, Q in ((0, 1), (7, 3), (n - 1, n - 2), (4, 4)):
        ref = 0.0
        gg = 0.0
        Xa = np.zeros(A.shape[1], complex)
        Xb = np.zeros(A.shape[1], complex)
        for ell in range(nl):
            u = links[ell]
            for i, j in pairs:
                r = R[ell, j, i]
                ref += r * M[P, u[j]] * M[Q, u[i]]
                gg += r * G[P, u[j]] * G[Q, u[i]]
                Xa += r * G[P, u[j]] * A[u[i]]
                Xb += r * A[u[j]] * G[Q, u[i]]
        got = gg + AY[Q] @ Xa + AY[P] @ Xb + AY[P] @ Z @ AY[Q]
        assert abs(got - ref) < 1e-11 * max(1.0, abs(ref)), (P, Q, got, ref)
