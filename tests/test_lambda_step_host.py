"""The library's host linear-method step (ggf_lambda_step) against the oracle's.

ggf_lambda_step averages rows of pair matrices, takes Hermitian parts, and
returns the lowest generalised eigenpair.  It uses a complex Cholesky factor
and a real Jacobi solver of the doubled real form.  The oracle uses NumPy's
Cholesky and eigh.  Host code only: runs without a GPU.
"""
import numpy as np
import pytest

from oracle.energy import linear_method

STRIDE = 1 + 4 * 4 * 4


def _rows(K, n, rng):
    rows = np.zeros((n, STRIDE))
    Hs, Ns = [], []
    for r in range(n):
        a = rng.standard_normal((K, K)) + 1j * rng.standard_normal((K, K))
        rho = a @ a.conj().T + 0.5 * np.eye(K) + 0.05 * (rng.standard_normal((K, K)) + 1j * rng.standard_normal((K, K)))
        rh = rng.standard_normal((K, K)) + 1j * rng.standard_normal((K, K))
        Hs.append(rh)
        Ns.append(rho)
        for p in range(K * K):
            i, j = divmod(p, K)
            rows[r, 1 + 4 * p:5 + 4 * p] = [rho[i, j].real, rho[i, j].imag, rh[i, j].real, rh[i, j].imag]
    return rows, np.mean(Hs, axis=0), np.mean(Ns, axis=0)


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_lambda_step_matches_oracle(K):
    from paper_2412_01737_amd.ggf import lambda_step
    rng = np.random.default_rng(70 + K)
    rows, Hb, Nb = _rows(K, 37, rng)
    e, lam = lambda_step(K, rows)
    e0, lam0 = linear_method(Hb, Nb)
    assert abs(e - e0) <= 1e-11 * max(1.0, abs(e0))
    assert np.abs(lam - lam0).max() <= 1e-9 * np.abs(lam0).max()
    S = 0.5 * (Nb + Nb.conj().T)
    assert abs(np.conj(lam) @ S @ lam - 1.0) < 1e-11
    assert abs(lam[0].imag) < 1e-14 and lam[0].real >= 0


def test_lambda_step_rejects_bad_input():
    from paper_2412_01737_amd.ggf import GGFError, lambda_step
    rows = np.zeros((3, STRIDE))
    rows[:, 1] = -1.0                      # rho_00 / S < 0: not positive definite
    with pytest.raises(GGFError):
        lambda_step(1, rows)
    rows[:, 1] = np.nan
    with pytest.raises(GGFError):
        lambda_step(1, rows)


def test_gamma_gradient_matches_oracle():
    """ggf_gamma_gradient (host) against the oracle's combination of per-sample sensitivities."""
    import synth
    from oracle.energy import gradient_from_samples
    from paper_2412_01737_amd.ggf import GGF_ENERGY_STRIDE, GGF_SENS_STRIDE, gamma_gradient
    rng = np.random.default_rng(90)
    n = 23
    g = synth.local_gamma()
    er = np.zeros((n, GGF_ENERGY_STRIDE))
    er[:, 0] = rng.standard_normal(n)
    sr = rng.standard_normal((n, GGF_SENS_STRIDE))
    out = gamma_gradient(g, er, sr)
    ref = gradient_from_samples(g, er[:, 0], sr[:, :100].reshape(n, 10, 10), sr[:, 100:].reshape(n, 10, 10))
    assert np.abs(out - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    assert np.abs(out + out.T).max() < 1e-14
