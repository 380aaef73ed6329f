"""The C-ABI library loads and exports every function include/ggf.h declares (no GPU needed)."""
import ctypes
import os
import re

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
