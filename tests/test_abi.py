"""The C-ABI library loads and exports every function include/ggf.h declares (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ggf.h")
LIB = os.path.join(ROOT, "paper_2412_01737_amd", "libggf.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ggf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("ggf_create", "ggf_set_tensor", "ggf_init_chains", "ggf_sweep", "ggf_measure",
              "ggf_get_state", "ggf_set_state", "ggf_last_error", "ggf_destroy"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libggf.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_2412_01737_amd import ggf
    assert set(ggf.EXPORTS) == set(declared())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libggf.so not built")
def test_host_only_entry_points():
    """ggf_autocorr_time runs on the host; the null-context paths return errors without a GPU."""
    import numpy as np
    from paper_2412_01737_amd import ggf
    lib = ggf.load()
    assert lib.ggf_sweep(None, 1, None) == ggf.GGF_EINVAL
    assert lib.ggf_last_error(None) == b"null context"
    lib.ggf_destroy(None)
    tau, err, w = ggf.autocorr_time(np.random.default_rng(1).standard_normal((4000, 3)))
    assert abs(tau - 0.5) < 0.1 and w >= 1
    with pytest.raises(ggf.GGFError):
        ggf.autocorr_time(np.zeros((1, 1)))


def _ar1(rng, phi, n_t, n_series):
    x = np.zeros((n_t, n_series))
    e = rng.standard_normal((n_t, n_series))
    x[0] = e[0] / np.sqrt(1 - phi * phi)
    for t in range(1, n_t):
        x[t] = phi * x[t - 1] + e[t]
    return x


@pytest.mark.skipif(not os.path.exists(LIB), reason="libggf.so not built")
def test_native_tau_int_equals_the_oracle():
    """ggf_autocorr_time (host code of the library) against oracle/stats on AR(1) series, an AR(1)
    ensemble and a recorded plaquette series of an oracle chain; the flags mark the clamp at 1/2 and
    series too short for the estimate."""
    from oracle import stats
    from oracle.chain import WoodburyChain
    from oracle.lattice import Lattice
    from oracle.model import Ansatz
    import synth
    from paper_2412_01737_amd import ggf
    rng = np.random.default_rng(17)
    for phi, n_t in ((0.9, 20000), (0.5, 5000), (0.0, 3000)):
        x = _ar1(rng, phi, n_t, 1)[:, 0]
        t0, e0, w0 = stats.tau_int(x)
        t1, e1, w1, fl = ggf.autocorr_time(x, with_flags=True)
        assert abs(t1 - t0) <= 1e-10 * t0 and abs(e1 - e0) <= 1e-10 * e0 and w1 == w0
        if phi > 0:
            assert fl == 0
    x = _ar1(rng, 0.8, 600, 64)
    t0, e0, w0 = stats.tau_int_chains(x)
    t1, e1, w1, fl = ggf.autocorr_time(x, with_flags=True)
    assert abs(t1 - t0) <= 1e-10 * t0 and abs(e1 - e0) <= 1e-10 * e0 and w1 == w0 and fl == 0
    spec = synth.make_tensor(2)
    an = Ansatz(Lattice(2, 2), spec.gamma_loc, spec.gamma_bond, 2)
    ch = WoodburyChain(an, synth.SEED_CHAIN, 0)
    series = []
    for _ in range(1500):
        ch.sweep()
        series.append(an.plaquette(ch.k))
    t0, e0, w0 = stats.tau_int(np.array(series))
    t1, e1, w1 = ggf.autocorr_time(np.array(series))
    assert abs(t1 - t0) <= 1e-10 * t0 and abs(e1 - e0) <= 1e-10 * e0 and w1 == w0
    # a short series of a slow AR(1) process (true tau 19.5): biased towards 1/2 and flagged
    t_short, _, _, fl = ggf.autocorr_time(_ar1(rng, 0.95, 8, 4), with_flags=True)
    assert fl & ggf.TAU_SHORT and t_short < 5
    _, _, _, fl = ggf.autocorr_time(np.array([1.0, -1.0, 1.0, -1.0, 1.0, -1.0]), with_flags=True)
    assert fl & ggf.TAU_FLOOR


def test_oracle_tau_int_chains_ar1_closed_form():
    """An ensemble of AR(1) series has tau_int = (1 + phi) / (2 (1 - phi)); one series reduces to tau_int."""
    from oracle import stats
    rng = np.random.default_rng(23)
    phi = 0.7
    x = _ar1(rng, phi, 4000, 32)
    tau, err, _ = stats.tau_int_chains(x)
    assert abs(tau - (1 + phi) / (2 * (1 - phi))) < 4 * err
    assert stats.tau_int_chains(x[:, :1]) == stats.tau_int(x[:, 0])


@pytest.mark.skipif(not os.path.exists(LIB), reason="libggf.so not built")
def test_library_was_built_from_these_sources():
    """The digest compiled into libggf.so equals the digest of the sources beside it (build() records it)."""
    from paper_2412_01737_amd import build
    from paper_2412_01737_amd.ggf import library_digest
    assert library_digest() == build.source_digest()
