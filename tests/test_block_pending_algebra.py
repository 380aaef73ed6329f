"""Algebra of delayed block moves, on the CPU in float64 (no GPU, no library).

A block move on Majoranas U with the antisymmetric change dM_UU updates the
inverse G = M^-1 of the antisymmetric M by Woodbury: G' = G - G[:,U] W G[U,:],
W = dM (1 + G_UU dM)^-1.  The library keeps accepted moves pending and:

* forms the current inverse on a new move's rows and columns from the pending
  moves (U_p, W_p): G_cur[x][y] = G[x][y] + sum_a F[x][a] E[y][a], with
  E = G[U_x, U_p] and F = E W_p;
* joins an accepted move (U_n, W_n, formed on G_cur) to the pending ones:
  G - G[:,U] W_c G[U,:] on U = U_p + U_n with H = W_n F,
  W_c = [[W_p + F^T H, H^T], [-H, W_n]].

Both identities are checked against the definition: sequential Woodbury updates
and a fresh inverse of M + dM.  W is antisymmetric (W = (dM^-1 + G_UU)^-1), which
the combined form relies on; that is checked too.
"""
import numpy as np


def _antisym(rng, n, scale=1.0):
    a = rng.standard_normal((n, n)) * scale
    return a - a.T


def _block_change(rng, links):
    """dM on the 4 Majoranas of each link: [[0, X], [-X^T, 0]] with X 2x2 (a bond-state change)."""
    r = 4 * len(links)
    dm = np.zeros((r, r))
    for q in range(len(links)):
        x = rng.standard_normal((2, 2))
        dm[4 * q:4 * q + 2, 4 * q + 2:4 * q + 4] = x
        dm[4 * q + 2:4 * q + 4, 4 * q:4 * q + 2] = -x.T
    return dm


def _woodbury(G, U, dm):
    W = dm @ np.linalg.inv(np.eye(len(U)) + G[np.ix_(U, U)] @ dm)
    return G - G[:, U] @ W @ G[U, :], W


def _setup(seed, n=96):
    rng = np.random.default_rng(seed)
    M = _antisym(rng, n) + 6.0 * np.kron(np.eye(n // 2), np.array([[0.0, 1.0], [-1.0, 0.0]]))
    return rng, M, np.linalg.inv(M)


def test_w_is_antisymmetric():
    rng, M, G = _setup(1)
    U = list(range(8, 16))
    dm = _block_change(rng, [0, 1])
    _, W = _woodbury(G, U, dm)
    assert np.abs(W + W.T).max() < 1e-12 * np.abs(W).max()


def test_current_inverse_on_new_rows_from_pending_moves():
    rng, M, G = _setup(2)
    Up = list(range(0, 12))                       # three pending links
    Un = list(range(40, 48))                      # the next move's two links
    S = [60, 61, 62, 63]                          # patch Majoranas (K > 1)
    dmp = _block_change(rng, [0, 1, 2])
    Gcur, Wp = _woodbury(G, Up, dmp)
    rows = Un + S
    E = G[np.ix_(rows, Up)]
    F = E @ Wp
    Gc = G[np.ix_(rows, rows)] + F @ E.T
    assert np.abs(Gc - Gcur[np.ix_(rows, rows)]).max() < 1e-12 * np.abs(Gcur).max()
    # and it is the inverse of the changed M on those entries
    Mp = M.copy()
    Mp[np.ix_(Up, Up)] += dmp
    assert np.abs(Gc - np.linalg.inv(Mp)[np.ix_(rows, rows)]).max() < 1e-10 * np.abs(Gcur).max()


def test_combined_update_equals_sequential_moves():
    rng, M, G = _setup(3)
    Up = list(range(4, 20))                       # four pending links
    Un = list(range(52, 64))                      # three new links, disjoint from U_p
    dmp, dmn = _block_change(rng, range(4)), _block_change(rng, range(3))
    G1, Wp = _woodbury(G, Up, dmp)
    G2, Wn = _woodbury(G1, Un, dmn)               # W_n formed on G_cur = G1
    E = G[np.ix_(Un, Up)]
    F = E @ Wp
    H = Wn @ F
    rp, rn = len(Up), len(Un)
    Wc = np.zeros((rp + rn, rp + rn))
    Wc[:rp, :rp] = Wp + F.T @ H
    Wc[:rp, rp:] = H.T
    Wc[rp:, :rp] = -H
    Wc[rp:, rp:] = Wn
    U = Up + Un
    Gc = G - G[:, U] @ Wc @ G[U, :]
    assert np.abs(Gc - G2).max() < 1e-11 * np.abs(G2).max()
    Mp = M.copy()
    Mp[np.ix_(Up, Up)] += dmp
    Mp[np.ix_(Un, Un)] += dmn
    assert np.abs(Gc - np.linalg.inv(Mp)).max() < 1e-10 * np.abs(G2).max()
    # applied as the flush does, G + P^T W_c P with P = G[U,:] (G antisymmetric)
    P = G[U, :]
    assert np.abs(G + P.T @ Wc @ P - Gc).max() < 1e-11 * np.abs(G2).max()


def test_combined_update_chains_over_three_moves():
    """Merging repeatedly (pending set grows move by move) still equals the definition."""
    rng, M, G = _setup(4)
    moves = [list(range(0, 8)), list(range(24, 36)), list(range(72, 80))]
    Mp = M.copy()
    Gseq = G.copy()
    Up, Wp = [], np.zeros((0, 0))
    for U_n in moves:
        dmn = _block_change(rng, range(len(U_n) // 4))
        Gseq, Wn = _woodbury(Gseq, U_n, dmn)
        Mp[np.ix_(U_n, U_n)] += dmn
        if Up:
            F = G[np.ix_(U_n, Up)] @ Wp
            H = Wn @ F
            rp, rn = len(Up), len(U_n)
            Wc = np.zeros((rp + rn, rp + rn))
            Wc[:rp, :rp] = Wp + F.T @ H
            Wc[:rp, rp:] = H.T
            Wc[rp:, :rp] = -H
            Wc[rp:, rp:] = Wn
            Up, Wp = Up + U_n, Wc
        else:
            Up, Wp = list(U_n), Wn
    Gc = G - G[:, Up] @ Wp @ G[Up, :]
    assert np.abs(Gc - Gseq).max() < 1e-10 * np.abs(Gseq).max()
    assert np.abs(Gc - np.linalg.inv(Mp)).max() < 1e-9 * np.abs(Gseq).max()
    assert np.abs(Wp + Wp.T).max() < 1e-10 * np.abs(Wp).max()
