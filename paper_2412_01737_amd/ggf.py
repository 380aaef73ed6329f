"""Thin ctypes binding of libggf.so (the C ABI declared in include/ggf.h).

Argument marshalling only: every step of the Monte Carlo path runs in the HIP
library.  Importing this module does not touch the GPU; ``load()`` raises if
the library has not been built, and nothing here falls back to a CPU path.
The same names as the C ABI are exported (``ggf_create``, ``ggf_set_tensor``,
...); ``Context`` wraps them with status checking.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libggf.so")

GGF_OK, GGF_EINVAL, GGF_ENOMEM, GGF_ESINGULAR, GGF_ENONFINITE, GGF_EDEVICE, GGF_ESTATE = 0, -1, -2, -3, -4, -5, -6
GGF_KMAX = 4
GGF_NOBS = 21
GGF_ENERGY_STRIDE = 1 + 4 * GGF_KMAX * GGF_KMAX
GGF_STAGE_MAX_CHAINS = 16384
GGF_SENS_STRIDE = 200
GGF_BOND_SMAX = 12
GGF_BOND_STRIDE = 2 + GGF_BOND_SMAX + GGF_KMAX + 3 * GGF_BOND_SMAX * GGF_BOND_SMAX
OBS_LINK, OBS_DENSITY, OBS_MESON, OBS_ELECTRIC = 1, 2, 4, 8
OBS_ALL = 15
_STATUS = {0: "GGF_OK", -1: "GGF_EINVAL", -2: "GGF_ENOMEM", -3: "GGF_ESINGULAR",
           -4: "GGF_ENONFINITE", -5: "GGF_EDEVICE", -6: "GGF_ESTATE"}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class TensorDesc(ctypes.Structure):
    _fields_ = [("group", ctypes.c_int32), ("gamma_loc", _dp), ("gamma_bond", _dp), ("K", ctypes.c_int32),
                ("patch_link", _ip), ("gamma_bond_k", _dp), ("c_re", _dp), ("c_im", _dp)]


class ChainInfo(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("n", ctypes.c_int32), ("tensor_id", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("logw", ctypes.c_double), ("s_re", ctypes.c_double),
                ("s_im", ctypes.c_double), ("sweeps", ctypes.c_uint64), ("accepts", ctypes.c_uint64),
                ("proposals", ctypes.c_uint64), ("refreshes", ctypes.c_uint64), ("recoveries", ctypes.c_uint64),
                ("max_drift", ctypes.c_double), ("near_ties", ctypes.c_uint64), ("link_cursor", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Couplings(ctypes.Structure):
    """ggf_couplings: H = t hopping + mu density + m staggered density + kb plaquettes + ke J^2."""
    _fields_ = [("t", ctypes.c_double), ("mu", ctypes.c_double), ("m", ctypes.c_double), ("kb", ctypes.c_double),
                ("ke", ctypes.c_double)]


EXPORTS = {
    "ggf_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]),
    "ggf_set_tensor": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(TensorDesc), ctypes.POINTER(ctypes.c_int32)]),
    "ggf_init_chains": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _ip, _ip, ctypes.c_uint64, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "ggf_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "ggf_measure": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "ggf_measure_staged": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, _dp, ctypes.c_void_p]),
    "ggf_measure_energy": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Couplings), ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_void_p]),
    "ggf_optimise_lambda": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Couplings), ctypes.c_int32,
                                           ctypes.c_int32, _dp, _dp, _dp, _dp, ctypes.c_void_p]),
    "ggf_measure_sensitivity": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Couplings), ctypes.c_void_p,
                                               ctypes.c_int32, ctypes.c_void_p]),
    "ggf_gamma_gradient": (ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp, ctypes.c_int64, _dp]),
    "ggf_set_bond": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, _dp, ctypes.c_void_p]),
    "ggf_measure_bond_rows": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Couplings), ctypes.c_void_p,
                                             ctypes.c_int32, ctypes.c_void_p]),
    "ggf_bond_gradient": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(TensorDesc), ctypes.POINTER(Couplings), _dp,
                                         _dp, ctypes.c_int64, _dp]),
    "ggf_set_gamma_loc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp, ctypes.c_void_p]),
    "ggf_optimise_gamma": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Couplings), ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_double, _dp, _dp, _dp, ctypes.c_void_p]),
    "ggf_set_lambda": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp, _dp, ctypes.c_void_p]),
    "ggf_lambda_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp, ctypes.c_int64, _dp, _dp, _dp]),
    "ggf_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ChainInfo)]),
    "ggf_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_uint64]),
    "ggf_get_inverse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp]),
    "ggf_set_inverse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _dp]),
    "ggf_refresh_all": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "ggf_set_option": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int64]),
    "ggf_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.c_void_p]),
    "ggf_update_timing": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64)]),
    "ggf_ratio_timing": (ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.POINTER(ctypes.c_int64)]),
    "ggf_autocorr_time": (ctypes.c_int, [_dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_double, _dp, _dp,
                                         ctypes.POINTER(ctypes.c_int64), _ip]),
    "ggf_nn_nparams": (ctypes.c_int32, []),
    "ggf_nn_init": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64]),
    "ggf_nn_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "ggf_nn_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _ip, _ip, ctypes.POINTER(ctypes.c_float)]),
    "ggf_nn_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _ip, _ip, ctypes.POINTER(ctypes.c_float), _dp]),
    "ggf_nn_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_uint64,
                                    _dp, ctypes.c_void_p]),
    "ggf_block_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "ggf_block_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_uint64)]),
    "ggf_stream_probe": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_int32, ctypes.c_void_p]),
    "ggf_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "ggf_source_digest": (ctypes.c_char_p, []),
    "ggf_destroy": (None, [ctypes.c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libggf.so and declare every exported symbol; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2412_01737_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def __getattr__(name):
    if name in EXPORTS:
        return getattr(load(), name)
    raise AttributeError(name)


class GGFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def _stream_ptr(stream) -> int | None:
    """Raw hipStream_t from None (legacy default stream), an int, or a torch stream."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Context:
    """One ggf_ctx on a device; methods mirror the C ABI and raise GGFError on failure."""

    def __init__(self, device: int = 0):
        self._lib = load()
        h = ctypes.c_void_p()
        st = self._lib.ggf_create(ctypes.byref(h), device)
        if st != GGF_OK:
            raise GGFError(st, f"ggf_create(device={device}) failed")
        self.h = h
        self.n_chains = 0

    def _check(self, st: int):
        if st != GGF_OK:
            raise GGFError(st, self._lib.ggf_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self._lib.ggf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tensor(self, group, gamma_loc, gamma_bond, K=1, patch_link=None, gamma_bond_k=None, c=None) -> int:
        gl, gb = _f64(gamma_loc), _f64(gamma_bond)
        keep = [gl, gb]
        d = TensorDesc()
        d.group, d.K = int(group), int(K)
        d.gamma_loc = gl.ctypes.data_as(_dp)
        d.gamma_bond = gb.ctypes.data_as(_dp)
        if K > 1:
            pl = np.ascontiguousarray(np.asarray(patch_link, np.int32))
            gk = _f64(gamma_bond_k)
            cc = np.asarray(c, complex)
            cre, cim = _f64(cc.real), _f64(cc.imag)
            keep += [pl, gk, cre, cim]
            d.patch_link = pl.ctypes.data_as(_ip)
            d.gamma_bond_k = gk.ctypes.data_as(_dp)
            d.c_re = cre.ctypes.data_as(_dp)
            d.c_im = cim.ctypes.data_as(_dp)
        tid = ctypes.c_int32()
        self._check(self._lib.ggf_set_tensor(self.h, ctypes.byref(d), ctypes.byref(tid)))
        del keep
        return tid.value

    def set_tensor_spec(self, spec) -> int:
        """Register a synth.TensorSpec-like object (group, gamma_loc, gamma_bond, K, ...)."""
        return self.set_tensor(spec.group, spec.gamma_loc, spec.gamma_bond, spec.K, spec.patch_link,
                               spec.gamma_bond_k, spec.c)

    def init_chains(self, L, tensor_id, seed: int, init: int = 0, precision: int = 64,
                    refresh_every: int = 0, stream=None):
        L = np.ascontiguousarray(np.asarray(L, np.int32).reshape(-1))
        tid = np.ascontiguousarray(np.broadcast_to(np.asarray(tensor_id, np.int32), L.shape))
        self._check(self._lib.ggf_init_chains(self.h, len(L), L.ctypes.data_as(_ip), tid.ctypes.data_as(_ip),
                                              int(seed), int(init), int(precision), int(refresh_every),
                                              _stream_ptr(stream)))
        self.n_chains = len(L)
        self.L = L

    def sweep(self, n_sweeps: int = 1, stream=None):
        self._check(self._lib.ggf_sweep(self.h, int(n_sweeps), _stream_ptr(stream)))

    def measure(self, mask: int = OBS_ALL, out=None, stream=None):
        """Observables [n_chains, GGF_NOBS]: into a device tensor `out` (async) or a new numpy array."""
        if out is None:
            host = np.zeros((self.n_chains, GGF_NOBS))
            self._check(self._lib.ggf_measure(self.h, int(mask), host.ctypes.data_as(ctypes.c_void_p), 0,
                                              _stream_ptr(stream)))
            return host
        ptr = out.data_ptr() if hasattr(out, "data_ptr") else int(out)
        self._check(self._lib.ggf_measure(self.h, int(mask), ctypes.c_void_p(ptr), 1, _stream_ptr(stream)))
        return out

    def measure_staged(self, mask: int = OBS_ALL, stream=None) -> np.ndarray:
        """Observables [n_chains, GGF_NOBS] into a new host array through ggf_measure_staged (no device
        allocation; at most GGF_STAGE_MAX_CHAINS chains)."""
        host = np.zeros((self.n_chains, GGF_NOBS))
        self._check(self._lib.ggf_measure_staged(self.h, int(mask), host.ctypes.data_as(_dp), _stream_ptr(stream)))
        return host

    def measure_energy(self, couplings, out=None, stream=None):
        """Local-energy rows [n_chains, GGF_ENERGY_STRIDE] (ggf_measure_energy); couplings is a
        Couplings or a mapping with keys t, mu, m, kb, ke."""
        cp = couplings if isinstance(couplings, Couplings) else Couplings(**dict(couplings))
        if out is None:
            host = np.zeros((self.n_chains, GGF_ENERGY_STRIDE))
            self._check(self._lib.ggf_measure_energy(self.h, ctypes.byref(cp), host.ctypes.data_as(ctypes.c_void_p),
                                                     0, _stream_ptr(stream)))
            return host
        ptr = out.data_ptr() if hasattr(out, "data_ptr") else int(out)
        self._check(self._lib.ggf_measure_energy(self.h, ctypes.byref(cp), ctypes.c_void_p(ptr), 1,
                                                 _stream_ptr(stream)))
        return out

    def measure_sensitivity(self, couplings, out=None, stream=None):
        """Sensitivity rows [n_chains, GGF_SENS_STRIDE] (ggf_measure_sensitivity)."""
        cp = couplings if isinstance(couplings, Couplings) else Couplings(**dict(couplings))
        if out is None:
            host = np.zeros((self.n_chains, GGF_SENS_STRIDE))
            self._check(self._lib.ggf_measure_sensitivity(self.h, ctypes.byref(cp),
                                                          host.ctypes.data_as(ctypes.c_void_p), 0,
                                                          _stream_ptr(stream)))
            return host
        ptr = out.data_ptr() if hasattr(out, "data_ptr") else int(out)
        self._check(self._lib.ggf_measure_sensitivity(self.h, ctypes.byref(cp), ctypes.c_void_p(ptr), 1,
                                                      _stream_ptr(stream)))
        return out

    def set_bond(self, tensor_id: int, k: int, gamma_bond_k, stream=None):
        """ggf_set_bond: new bond state of B_k on its patch link; the chains' S(G) are recomputed."""
        g = np.ascontiguousarray(np.asarray(gamma_bond_k, np.float64).reshape(4, 4))
        self._check(self._lib.ggf_set_bond(self.h, int(tensor_id), int(k), g.ctypes.data_as(_dp),
                                           _stream_ptr(stream)))

    def measure_bond_rows(self, couplings, out=None, stream=None):
        """Rows [n_chains, GGF_BOND_STRIDE] for the gradient with respect to the patch bond states
        (ggf_measure_bond_rows)."""
        cp = couplings if isinstance(couplings, Couplings) else Couplings(**dict(couplings))
        if out is None:
            host = np.zeros((self.n_chains, GGF_BOND_STRIDE))
            self._check(self._lib.ggf_measure_bond_rows(self.h, ctypes.byref(cp), host.ctypes.data_as(ctypes.c_void_p),
                                                        0, _stream_ptr(stream)))
            return host
        ptr = out.data_ptr() if hasattr(out, "data_ptr") else int(out)
        self._check(self._lib.ggf_measure_bond_rows(self.h, ctypes.byref(cp), ctypes.c_void_p(ptr), 1,
                                                    _stream_ptr(stream)))
        return out

    def set_gamma_loc(self, tensor_id: int, gamma_loc, stream=None):
        """ggf_set_gamma_loc: new on-site covariance for a tensor; its chains are refactorised."""
        g = np.ascontiguousarray(np.asarray(gamma_loc, np.float64).reshape(10, 10))
        self._check(self._lib.ggf_set_gamma_loc(self.h, int(tensor_id), g.ctypes.data_as(_dp), _stream_ptr(stream)))

    def optimise_gamma(self, tensor_id: int, couplings, n_iters: int, n_sweeps: int, step: float, stream=None):
        """ggf_optimise_gamma: (energies [n_iters], grad_norms [n_iters], final Gamma_A 10 x 10)."""
        cp = couplings if isinstance(couplings, Couplings) else Couplings(**dict(couplings))
        en = np.zeros(n_iters)
        gn = np.zeros(n_iters)
        g = np.zeros((10, 10))
        self._check(self._lib.ggf_optimise_gamma(self.h, int(tensor_id), ctypes.byref(cp), int(n_iters), int(n_sweeps),
                                                 float(step), en.ctypes.data_as(_dp), gn.ctypes.data_as(_dp),
                                                 g.ctypes.data_as(_dp), _stream_ptr(stream)))
        return en, gn, g

    def set_lambda(self, tensor_id: int, c, stream=None):
        """ggf_set_lambda: new amplitudes lambda_n (complex [K]) for a tensor; S(G) recomputed."""
        c = np.asarray(c, complex)
        re = np.ascontiguousarray(c.real, np.float64)
        im = np.ascontiguousarray(c.imag, np.float64)
        self._check(self._lib.ggf_set_lambda(self.h, int(tensor_id), re.ctypes.data_as(_dp), im.ctypes.data_as(_dp),
                                             _stream_ptr(stream)))

    def optimise_lambda(self, tensor_id: int, couplings, n_iters: int, n_sweeps: int, K: int, stream=None):
        """ggf_optimise_lambda: (energies [n_iters], e_opt [n_iters], final lambda complex [K])."""
        cp = couplings if isinstance(couplings, Couplings) else Couplings(**dict(couplings))
        en = np.zeros(n_iters)
        eo = np.zeros(n_iters)
        lr = np.zeros(K)
        li = np.zeros(K)
        self._check(self._lib.ggf_optimise_lambda(self.h, int(tensor_id), ctypes.byref(cp), int(n_iters),
                                                  int(n_sweeps), en.ctypes.data_as(_dp), eo.ctypes.data_as(_dp),
                                                  lr.ctypes.data_as(_dp), li.ctypes.data_as(_dp),
                                                  _stream_ptr(stream)))
        return en, eo, lr + 1j * li

    def get_state(self, chain: int):
        info = ChainInfo()
        self._check(self._lib.ggf_get_state(self.h, int(chain), None, ctypes.byref(info)))
        links = np.zeros(2 * info.L * info.L, np.int8)
        self._check(self._lib.ggf_get_state(self.h, int(chain), links.ctypes.data_as(ctypes.c_void_p), None))
        return links, info.as_dict()

    def set_state(self, chain: int, links, sweeps: int):
        lk = np.ascontiguousarray(np.asarray(links, np.int8))
        self._check(self._lib.ggf_set_state(self.h, int(chain), lk.ctypes.data_as(ctypes.c_void_p), int(sweeps)))

    def get_inverse(self, chain: int) -> np.ndarray:
        L = int(self.L[chain])
        n = 8 * L * L
        out = np.zeros((n, n))
        self._check(self._lib.ggf_get_inverse(self.h, int(chain), out.ctypes.data_as(_dp)))
        return out

    def set_inverse(self, chain: int, G):
        g = _f64(G)
        self._check(self._lib.ggf_set_inverse(self.h, int(chain), g.ctypes.data_as(_dp)))

    def refresh_all(self, stream=None):
        self._check(self._lib.ggf_refresh_all(self.h, _stream_ptr(stream)))

    def set_option(self, key: str, value: int):
        self._check(self._lib.ggf_set_option(self.h, key.encode(), int(value)))

    # ---- learned block proposal ----
    def nn_init(self, patch: int, seed: int):
        self._check(self._lib.ggf_nn_init(self.h, int(patch), int(seed)))
        self.patch = int(patch)

    def nn_params(self, set_params=None) -> np.ndarray:
        out = np.zeros(self._lib.ggf_nn_nparams(), np.float32)
        sp = None
        if set_params is not None:
            sp = np.ascontiguousarray(np.asarray(set_params, np.float32))
        self._check(self._lib.ggf_nn_params(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                            None if sp is None else sp.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        if sp is not None:
            return sp.copy()
        return out

    def _examples(self, chains, patches):
        c = np.ascontiguousarray(np.asarray(chains, np.int32))
        p = np.ascontiguousarray(np.asarray(patches, np.int32))
        return c, p

    def nn_forward(self, chains, patches) -> np.ndarray:
        c, p = self._examples(chains, patches)
        out = np.zeros((len(c), 2 * self.patch * self.patch), np.float32)
        self._check(self._lib.ggf_nn_forward(self.h, len(c), c.ctypes.data_as(_ip), p.ctypes.data_as(_ip),
                                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def nn_grad(self, chains, patches):
        c, p = self._examples(chains, patches)
        g = np.zeros(self._lib.ggf_nn_nparams(), np.float32)
        loss = ctypes.c_double()
        self._check(self._lib.ggf_nn_grad(self.h, len(c), c.ctypes.data_as(_ip), p.ctypes.data_as(_ip),
                                          g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss)))
        return loss.value, g

    def nn_train(self, steps: int, batch: int, lr: float, seed: int, stream=None) -> float:
        loss = ctypes.c_double()
        self._check(self._lib.ggf_nn_train(self.h, int(steps), int(batch), float(lr), int(seed), ctypes.byref(loss),
                                           _stream_ptr(stream)))
        return loss.value

    def block_sweep(self, n_sweeps: int = 1, stream=None):
        self._check(self._lib.ggf_block_sweep(self.h, int(n_sweeps), _stream_ptr(stream)))

    def block_stats(self, chain: int):
        """(proposed, accepted, links changed by accepted moves, updates of G) of one chain's block moves."""
        p, a, m, u = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        self._check(self._lib.ggf_block_stats(self.h, int(chain), ctypes.byref(p), ctypes.byref(a), ctypes.byref(m),
                                              ctypes.byref(u)))
        return p.value, a.value, m.value, u.value

    def autotune(self, sweeps_per_candidate: int = 1, cache_path: str | None = None, stream=None):
        """Choose the launch shapes of the path that runs on live sweeps: (flush_grid, window, 0) with
        delayed updates, (update_grid, update_tiles, non_temporal) with delay 0."""
        best = (ctypes.c_int64 * 3)()
        self._check(self._lib.ggf_autotune(self.h, int(sweeps_per_candidate),
                                           None if cache_path is None else cache_path.encode(), best,
                                           _stream_ptr(stream)))
        return tuple(best)

    def ratio_timing(self):
        """(ms, launches) of the ratio / decision kernels of the last timed sweep call."""
        ms = ctypes.c_double()
        la = ctypes.c_int64()
        self._check(self._lib.ggf_ratio_timing(self.h, ctypes.byref(ms), ctypes.byref(la)))
        return ms.value, la.value

    def update_timing(self):
        ms = ctypes.c_double()
        la = ctypes.c_int64()
        fl = ctypes.c_int64()
        self._check(self._lib.ggf_update_timing(self.h, ctypes.byref(ms), ctypes.byref(la), ctypes.byref(fl)))
        return ms.value, la.value, fl.value


def library_digest() -> str:
    """The source digest compiled into the loaded libggf.so."""
    return load().ggf_source_digest().decode()


TAU_FLOOR, TAU_SHORT = 1, 2


def autocorr_time(series, c: float = 5.0, with_flags: bool = False):
    """(tau, tau_err, window) of series[t, s] (time-major) via ggf_autocorr_time; with
    with_flags also the flags (TAU_FLOOR: clamped at 1/2; TAU_SHORT: series too short)."""
    x = np.ascontiguousarray(np.asarray(series, np.float64))
    if x.ndim == 1:
        x = x[:, None]
    tau, err, w, fl = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64(), ctypes.c_int32()
    st = load().ggf_autocorr_time(x.ctypes.data_as(_dp), x.shape[0], x.shape[1], float(c), ctypes.byref(tau),
                                  ctypes.byref(err), ctypes.byref(w), ctypes.byref(fl))
    if st != GGF_OK:
        raise GGFError(st, "ggf_autocorr_time: bad arguments")
    if with_flags:
        return tau.value, err.value, w.value, fl.value
    return tau.value, err.value, w.value


def lambda_step(K: int, rows):
    """ggf_lambda_step on host rows [n, GGF_ENERGY_STRIDE]: (energy, lambda as a complex array)."""
    lib = load()
    r = np.ascontiguousarray(np.asarray(rows, np.float64).reshape(-1, GGF_ENERGY_STRIDE))
    e = ctypes.c_double()
    lr = np.zeros(K)
    li = np.zeros(K)
    st = lib.ggf_lambda_step(None, int(K), r.ctypes.data_as(_dp), r.shape[0], ctypes.byref(e),
                             lr.ctypes.data_as(_dp), li.ctypes.data_as(_dp))
    if st != GGF_OK:
        raise GGFError(st, f"ggf_lambda_step failed ({_STATUS.get(st, st)})")
    return e.value, lr + 1j * li


def bond_gradient(spec, couplings, energy_rows, bond_rows):
    """ggf_bond_gradient on host rows of chains of the ansatz `spec` (group, gamma_loc, gamma_bond, K,
    patch_link, gamma_bond_k, c): d<H>/d theta for bonds k = 1 .. K-1 and the six generators, shape
    [K - 1, 6]."""
    lib = load()
    cp = couplings if isinstance(couplings, Couplings) else Couplings(**dict(couplings))
    gl, gb = _f64(spec.gamma_loc), _f64(spec.gamma_bond)
    pl = np.ascontiguousarray(np.asarray(spec.patch_link, np.int32))
    gk = _f64(spec.gamma_bond_k)
    cc = np.asarray(spec.c, complex)
    cre, cim = _f64(cc.real), _f64(cc.imag)
    d = TensorDesc()
    d.group, d.K = int(spec.group), int(spec.K)
    d.gamma_loc, d.gamma_bond = gl.ctypes.data_as(_dp), gb.ctypes.data_as(_dp)
    d.patch_link, d.gamma_bond_k = pl.ctypes.data_as(_ip), gk.ctypes.data_as(_dp)
    d.c_re, d.c_im = cre.ctypes.data_as(_dp), cim.ctypes.data_as(_dp)
    er = np.ascontiguousarray(np.asarray(energy_rows, np.float64).reshape(-1, GGF_ENERGY_STRIDE))
    br = np.ascontiguousarray(np.asarray(bond_rows, np.float64).reshape(-1, GGF_BOND_STRIDE))
    if er.shape[0] != br.shape[0]:
        raise ValueError("energy and bond rows must describe the same samples")
    out = np.zeros((int(spec.K) - 1, 6))
    st = lib.ggf_bond_gradient(None, ctypes.byref(d), ctypes.byref(cp), er.ctypes.data_as(_dp), br.ctypes.data_as(_dp),
                               er.shape[0], out.ctypes.data_as(_dp))
    if st != GGF_OK:
        raise GGFError(st, f"ggf_bond_gradient failed ({_STATUS.get(st, st)})")
    return out


def gamma_gradient(gamma_loc, energy_rows, sens_rows):
    """ggf_gamma_gradient on host rows: the antisymmetric 10 x 10 gradient of <H>."""
    lib = load()
    g = np.ascontiguousarray(np.asarray(gamma_loc, np.float64).reshape(10, 10))
    er = np.ascontiguousarray(np.asarray(energy_rows, np.float64).reshape(-1, GGF_ENERGY_STRIDE))
    sr = np.ascontiguousarray(np.asarray(sens_rows, np.float64).reshape(-1, GGF_SENS_STRIDE))
    if er.shape[0] != sr.shape[0]:
        raise ValueError("energy and sensitivity rows must describe the same samples")
    out = np.zeros((10, 10))
    st = lib.ggf_gamma_gradient(None, g.ctypes.data_as(_dp), er.ctypes.data_as(_dp), sr.ctypes.data_as(_dp),
                                er.shape[0], out.ctypes.data_as(_dp))
    if st != GGF_OK:
        raise GGFError(st, f"ggf_gamma_gradient failed ({_STATUS.get(st, st)})")
    return out

