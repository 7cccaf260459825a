"""ctypes binding of libptebd (argument marshalling only; every step runs in the library).

The library must have been built (``paper_2312_02667_amd.build.build()``); loading fails
loudly otherwise.

HIP runtime: libptebd links the system ROCm HIP runtime (``libamdhip64.so.7``).  The PyTorch
wheel of this image bundles a HIP runtime of its own, a separate instance in the same
process, so torch's stream handles and device pointers mean nothing to the library and the
binding never passes them.  The library allocates its own device memory; streams, when a
caller wants one other than the null stream, come from the library's runtime (``Stream``),
and ``device_synchronize`` waits for that runtime's work.
"""

from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libptebd.so")

OK = 0
EINVAL = -1
EOVERLAP = -2
ENOMEM = -3
EDEVICE = -4
ENONFINITE = -5
EANNIHILATED = -6
WNOCONV = 1

FP64 = 0
FP32 = 1
BF16X3 = 2  # declared by the header, not built: the library rejects it with EINVAL
FLAG_NO_STABILIZE = 1
FLAG_RELATIVE_EPS = 2
FLAG_COMPLEMENT_EPS = 4
FP32_CUTOFF_FLOOR = 1.9073486328125e-06  # 2^-19, PTEBD_FP32_CUTOFF_FLOOR
EPS_FLAGS = {"literal": 0, "relative": FLAG_RELATIVE_EPS, "complement": FLAG_COMPLEMENT_EPS}

PRECISIONS = {"fp64": FP64, "fp32": FP32}

_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)


class LayerStats(ctypes.Structure):
    _fields_ = [
        ("k", _i32p), ("rank", _i32p), ("eps", _dp), ("nu", _dp), ("sweeps", _i32p),
        ("triggered", ctypes.c_int32), ("ptsu_done", ctypes.c_int32),
        ("max_sweeps", ctypes.c_int32), ("n_unconverged", ctypes.c_int32),
        ("device_ms", ctypes.c_double),
    ]


class SvdParams(ctypes.Structure):
    _fields_ = [("max_sweeps", ctypes.c_int), ("tol_factor", ctypes.c_double),
                ("inner_sweeps", ctypes.c_int), ("inner_repeat", ctypes.c_double),
                ("sort_pairs", ctypes.c_int), ("precondition", ctypes.c_int),
                ("streams", ctypes.c_int), ("block_cols", ctypes.c_int),
                ("graphs", ctypes.c_int)]


class KernelStats(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double), ("launches", ctypes.c_int64),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


KERNELS = {"theta": 0, "jacobi": 1, "finalize": 2, "writeback": 3, "sample": 4, "precond": 5}


class PtebdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ptebd error {code}: {msg}")
        self.code = code


_LIB = None

# name -> (restype, argtypes)
_SIGS = {
    "ptebd_version": (ctypes.c_char_p, []),
    "ptebd_last_error": (ctypes.c_char_p, []),
    "ptebd_mps_create": (ctypes.c_int, [ctypes.c_int, _i32p, _i32p, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "ptebd_mps_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ptebd_get_svd_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SvdParams)]),
    "ptebd_set_svd_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SvdParams)]),
    "ptebd_apply_layer": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _i32p, _i32p, _dp,
                                          ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_int, ctypes.POINTER(LayerStats)]),
    "ptebd_ptsu": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double]),
    "ptebd_canonicalize": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _dp]),
    "ptebd_sample": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp,
                                     ctypes.POINTER(ctypes.c_uint8)]),
    "ptebd_norm": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp]),
    "ptebd_overlap": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_int, _dp, _dp]),
    "ptebd_expect_z": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp]),
    "ptebd_canon_distance": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp]),
    "ptebd_norm_estimate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp]),
    "ptebd_fidelity_estimate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp]),
    "ptebd_bond_dims": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _i32p, ctypes.c_int]),
    "ptebd_get_lambda": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp,
                                         ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "ptebd_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_size_t, _dp,
                                     ctypes.c_size_t]),
    "ptebd_import": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _i32p, _dp, _dp]),
    "ptebd_export_site": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp,
                                          ctypes.c_size_t, _i32p]),
    "ptebd_debug_theta": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp, _dp]),
    "ptebd_set_profiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "ptebd_get_kernel_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                               ctypes.POINTER(KernelStats)]),
    "ptebd_svd_batched": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          _dp, _dp, _dp, _dp, _i32p, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_void_p]),
    "ptebd_svd_batched_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_int, _dp, _dp, _dp, _dp, _i32p,
                                                  ctypes.c_int, ctypes.c_double,
                                                  ctypes.c_void_p]),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load libptebd.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2312_02667_amd.build.build()")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = handle
    return _LIB


def _check(code: int, allow_warn: bool = True) -> int:
    if code < 0 or (code > 0 and not allow_warn):
        raise PtebdError(code, lib().ptebd_last_error().decode())
    return code


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


_HIP = None


def hip():
    """The HIP runtime instance libptebd uses (loaded by the library itself; same soname)."""
    global _HIP
    if _HIP is None:
        lib()
        h = ctypes.CDLL("libamdhip64.so.7")
        h.hipDeviceSynchronize.restype = ctypes.c_int
        h.hipSetDevice.argtypes = [ctypes.c_int]
        h.hipSetDevice.restype = ctypes.c_int
        h.hipStreamCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        h.hipStreamCreateWithFlags.restype = ctypes.c_int
        h.hipStreamDestroy.argtypes = [ctypes.c_void_p]
        h.hipStreamDestroy.restype = ctypes.c_int
        h.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
        h.hipStreamSynchronize.restype = ctypes.c_int
        _HIP = h
    return _HIP


def _hip_check(code: int, what: str):
    if code != 0:
        raise RuntimeError(f"{what} failed with HIP error {code}")


def set_device(index: int = 0):
    _hip_check(hip().hipSetDevice(int(index)), "hipSetDevice")


def device_synchronize():
    """Wait for all work of the library's HIP runtime on the current device."""
    _hip_check(hip().hipDeviceSynchronize(), "hipDeviceSynchronize")


class Stream:
    """A HIP stream of the library's runtime (default priority; non-blocking with respect to
    the null stream).  ``handle`` is what ``MPS(stream=...)`` takes."""

    def __init__(self):
        self.handle = ctypes.c_void_p()
        _hip_check(hip().hipStreamCreateWithFlags(ctypes.byref(self.handle), 1),
                   "hipStreamCreateWithFlags")

    def synchronize(self):
        _hip_check(hip().hipStreamSynchronize(self.handle), "hipStreamSynchronize")

    def close(self):
        if self.handle:
            hip().hipStreamSynchronize(self.handle)
            hip().hipStreamDestroy(self.handle)
            self.handle = ctypes.c_void_p()


def default_stream():
    """The null stream of the library's runtime (None)."""
    return None


def _gates_array(gates) -> np.ndarray:
    g = np.ascontiguousarray(np.asarray(gates, dtype=np.complex128).reshape(-1, 4, 4))
    return g.view(np.float64).reshape(-1, 32)


class MPS:
    """A batch of MPS on the device (one handle of libptebd)."""

    def __init__(self, n_sites, chi_cap, precision: str = "fp64", stream=None):
        n_sites = np.atleast_1d(np.asarray(n_sites, dtype=np.int32))
        chi_cap = np.broadcast_to(np.asarray(chi_cap, dtype=np.int32), n_sites.shape).copy()
        self.n_sites = [int(x) for x in n_sites]
        self.chi_cap = [int(x) for x in chi_cap]
        self.precision = precision
        if isinstance(stream, Stream):
            stream = stream.handle.value
        self.stream = default_stream() if stream is None else stream
        self._h = ctypes.c_void_p()
        _check(lib().ptebd_mps_create(len(n_sites), _ptr(n_sites, ctypes.c_int32),
                                      _ptr(chi_cap, ctypes.c_int32), 2, PRECISIONS[precision],
                                      ctypes.c_void_p(self.stream), ctypes.byref(self._h)))

    def close(self):
        if self._h:
            lib().ptebd_mps_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def svd_params(self) -> dict:
        p = SvdParams()
        _check(lib().ptebd_get_svd_params(self._h, ctypes.byref(p)))
        return {name: getattr(p, name) for name, _ in SvdParams._fields_}

    def set_svd_params(self, **changes):
        """Change some SVD controls (max_sweeps, tol_factor, inner_sweeps, inner_repeat,
        sort_pairs, precondition); the others keep their current values."""
        p = SvdParams()
        _check(lib().ptebd_get_svd_params(self._h, ctypes.byref(p)))
        for name, value in changes.items():
            if name not in dict(SvdParams._fields_):
                raise TypeError(f"unknown SVD control {name!r}")
            setattr(p, name, type(getattr(p, name))(value))
        _check(lib().ptebd_set_svd_params(self._h, ctypes.byref(p)))

    def apply_layer(self, bonds, gates, chi_max: int, cutoff: float = 1e-12, ptsu_steps: int = 0,
                    stabilize: bool = True, state_idx=None, eps_reading: str = "literal") -> dict:
        """One circuit layer; ``eps_reading`` is "literal" (discarded sigma^2), "relative"
        (that over sum sigma^2) or "complement" (1 - kept sigma^2)."""
        if eps_reading not in EPS_FLAGS:
            raise ValueError(f"eps_reading must be one of {tuple(EPS_FLAGS)}")
        bonds = np.ascontiguousarray(bonds, dtype=np.int32)
        g = _gates_array(gates)
        n = len(bonds)
        if g.shape[0] != n:
            raise ValueError("one gate per bond")
        k = np.zeros(n, np.int32)
        rank = np.zeros(n, np.int32)
        eps = np.zeros(n, np.float64)
        nu = np.zeros(n, np.float64)
        sweeps = np.zeros(n, np.int32)
        st = LayerStats(_ptr(k, ctypes.c_int32), _ptr(rank, ctypes.c_int32),
                        _ptr(eps, ctypes.c_double), _ptr(nu, ctypes.c_double),
                        _ptr(sweeps, ctypes.c_int32), 0, 0, 0, 0, 0.0)
        sidx = None
        if state_idx is not None:
            sidx = np.ascontiguousarray(state_idx, dtype=np.int32)
        code = _check(lib().ptebd_apply_layer(
            self._h, n, _ptr(sidx, ctypes.c_int32) if sidx is not None else None,
            _ptr(bonds, ctypes.c_int32), _ptr(g, ctypes.c_double), int(chi_max), float(cutoff),
            int(ptsu_steps),
            (0 if stabilize else FLAG_NO_STABILIZE) | EPS_FLAGS[eps_reading],
            ctypes.byref(st)))
        return {"k": k, "rank": rank, "eps": eps, "nu": nu, "sweeps": sweeps,
                "triggered": bool(st.triggered), "ptsu_done": st.ptsu_done,
                "max_sweeps": st.max_sweeps, "n_unconverged": st.n_unconverged,
                "device_ms": st.device_ms, "status": code}

    def set_profiling(self, enable: bool = True):
        _check(lib().ptebd_set_profiling(self._h, 1 if enable else 0))

    def kernel_stats(self) -> dict:
        out = {}
        for name, kind in KERNELS.items():
            st = KernelStats()
            _check(lib().ptebd_get_kernel_stats(self._h, kind, ctypes.byref(st)))
            out[name] = {"total_ms": st.total_ms, "launches": int(st.launches),
                         "flops": st.flops, "bytes": st.bytes}
        return out

    def ptsu(self, steps: int, cutoff: float = 1e-12, s: int = 0):
        return _check(lib().ptebd_ptsu(self._h, s, int(steps), float(cutoff)))

    def canonicalize(self, cutoff: float = 1e-12, s: int = 0) -> float:
        """Canonical form with unit norm (in place); returns the norm before normalizing."""
        out = ctypes.c_double()
        _check(lib().ptebd_canonicalize(self._h, s, float(cutoff), ctypes.byref(out)))
        return out.value

    def sample(self, uniforms, s: int = 0) -> np.ndarray:
        """Perfect sampling from a canonical state: one bit string (uint8 row) per row of
        ``uniforms`` (shape (n_samples, N), values in [0, 1))."""
        u = np.ascontiguousarray(uniforms, dtype=np.float64)
        if u.ndim != 2 or u.shape[1] != self.n_sites[s]:
            raise ValueError("uniforms must have shape (n_samples, n_sites)")
        bits = np.zeros(u.shape, np.uint8)
        _check(lib().ptebd_sample(self._h, s, int(u.shape[0]), _ptr(u, ctypes.c_double),
                                  _ptr(bits, ctypes.c_uint8)), allow_warn=False)
        return bits

    def _scalar(self, fn, s):
        out = ctypes.c_double()
        _check(fn(self._h, s, ctypes.byref(out)))
        return out.value

    def norm(self, s: int = 0) -> float:
        return self._scalar(lib().ptebd_norm, s)

    def norm_estimate(self, s: int = 0) -> float:
        return self._scalar(lib().ptebd_norm_estimate, s)

    def fidelity_estimate(self, s: int = 0) -> float:
        return self._scalar(lib().ptebd_fidelity_estimate, s)

    def canon_distance(self, s: int = 0) -> float:
        return self._scalar(lib().ptebd_canon_distance, s)

    def overlap(self, other: "MPS", s: int = 0, s_other: int = 0) -> complex:
        """<self_s | other_s_other>."""
        re, im = ctypes.c_double(), ctypes.c_double()
        _check(lib().ptebd_overlap(self._h, s, other._h, s_other, ctypes.byref(re), ctypes.byref(im)))
        return complex(re.value, im.value)

    def expect_z(self, s: int = 0) -> np.ndarray:
        out = np.zeros(self.n_sites[s], np.float64)
        _check(lib().ptebd_expect_z(self._h, s, _ptr(out, ctypes.c_double)))
        return out

    def bond_dims(self, s: int = 0) -> list:
        out = np.zeros(self.n_sites[s] + 1, np.int32)
        _check(lib().ptebd_bond_dims(self._h, s, _ptr(out, ctypes.c_int32), len(out)))
        return [int(x) for x in out]

    def get_lambda(self, bond: int, s: int = 0) -> np.ndarray:
        cap = max(self.chi_cap[s], 1)
        out = np.zeros(cap, np.float64)
        ln = ctypes.c_int()
        _check(lib().ptebd_get_lambda(self._h, s, int(bond), _ptr(out, ctypes.c_double), cap,
                                      ctypes.byref(ln)))
        return out[: ln.value].copy()

    def export(self, s: int = 0):
        """(gammas, lambdas): lists of complex128 (chi_q, 2, chi_{q+1}) and float64 arrays."""
        dims = self.bond_dims(s)
        n = self.n_sites[s]
        ng = sum(4 * dims[q] * dims[q + 1] for q in range(n))
        nl = sum(dims)
        g = np.zeros(ng, np.float64)
        lam = np.zeros(nl, np.float64)
        _check(lib().ptebd_export(self._h, s, _ptr(g, ctypes.c_double), ng,
                                  _ptr(lam, ctypes.c_double), nl))
        gc = g.view(np.complex128)
        gammas, lambdas = [], []
        off = 0
        for q in range(n):
            cnt = 2 * dims[q] * dims[q + 1]
            gammas.append(gc[off:off + cnt].reshape(dims[q], 2, dims[q + 1]).copy())
            off += cnt
        off = 0
        for i in range(n + 1):
            lambdas.append(lam[off:off + dims[i]].copy())
            off += dims[i]
        return gammas, lambdas

    def export_site(self, q: int, s: int = 0) -> np.ndarray:
        """Gamma[q] of state s as a complex128 (chi_q, 2, chi_{q+1}) array."""
        dims = self.bond_dims(s)
        n = 4 * dims[q] * dims[q + 1]
        g = np.zeros(n, np.float64)
        d = np.zeros(2, np.int32)
        _check(lib().ptebd_export_site(self._h, s, int(q), _ptr(g, ctypes.c_double), n,
                                       _ptr(d, ctypes.c_int32)))
        return g.view(np.complex128).reshape(int(d[0]), 2, int(d[1])).copy()

    def import_state(self, gammas, lambdas, s: int = 0):
        dims = np.array([len(x) for x in lambdas], np.int32)
        g = np.ascontiguousarray(np.concatenate([np.asarray(x, np.complex128).reshape(-1)
                                                 for x in gammas])).view(np.float64)
        lam = np.ascontiguousarray(np.concatenate([np.asarray(x, np.float64) for x in lambdas]))
        _check(lib().ptebd_import(self._h, s, _ptr(dims, ctypes.c_int32),
                                  _ptr(g, ctypes.c_double), _ptr(lam, ctypes.c_double)))

    def debug_theta(self, q: int, gate=None, s: int = 0) -> np.ndarray:
        dims = self.bond_dims(s)
        m, n = 2 * dims[q], 2 * dims[q + 2]
        out = np.zeros(2 * m * n, np.float64)
        gp = None
        if gate is not None:
            garr = _gates_array(gate)[0].copy()
            gp = _ptr(garr, ctypes.c_double)
        _check(lib().ptebd_debug_theta(self._h, s, int(q), gp, _ptr(out, ctypes.c_double)))
        return out.view(np.complex128).reshape(m, n)


NOALLOC_SCRATCH_BYTES = 32 << 20  # PTEBD_NOALLOC_SCRATCH_BYTES


def svd_batched(a, precision: str = "fp64", max_sweeps: int = 30, tol_factor: float = 4.0,
                stream=None, noalloc: bool = False):
    """Batched SVD of complex matrices a[b] (m x n) on the device: (s, u, vh, sweeps, status).
    ``noalloc`` calls the entry point that allocates no device memory (fixed scratch array)."""
    a = np.ascontiguousarray(np.asarray(a, np.complex128))
    if a.ndim == 2:
        a = a[None]
    batch, m, n = a.shape
    k = min(m, n)
    s = np.zeros((batch, k), np.float64)
    u = np.zeros((batch, m, k), np.complex128)
    vh = np.zeros((batch, k, n), np.complex128)
    sw = np.zeros(batch, np.int32)
    stream = default_stream() if stream is None else stream
    fn = lib().ptebd_svd_batched_noalloc if noalloc else lib().ptebd_svd_batched
    code = _check(fn(
        PRECISIONS[precision], batch, m, n, _ptr(a.view(np.float64), ctypes.c_double),
        _ptr(s, ctypes.c_double), _ptr(u.view(np.float64), ctypes.c_double),
        _ptr(vh.view(np.float64), ctypes.c_double), _ptr(sw, ctypes.c_int32), int(max_sweeps),
        float(tol_factor), ctypes.c_void_p(stream)))
    return s, u, vh, sw, code
