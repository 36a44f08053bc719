"""FP64 CPU oracle for multi-rate SPIIR filtering — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg
may import this package.  The HIP library and its Python binding never do; the
two implementations share no code (only the seeded input generators in
``paper_1702_02256_amd.workloads`` feed both).

The arithmetic lives in ``spiir_oracle.c`` (plain double-complex loops, OpenMP
over templates); this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spiir_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, as the paper's CPU counterpart)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle()
        lib = C.CDLL(_LIB)
        dp, ip, i64 = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int64
        lib.oracle_create.restype = C.c_void_p
        lib.oracle_create.argtypes = [C.c_int, C.c_int, ip, dp, dp, ip, C.c_int, dp, C.c_int, dp]
        lib.oracle_destroy.argtypes = [C.c_void_p]
        lib.oracle_process.restype = C.c_int
        lib.oracle_process.argtypes = [C.c_void_p, dp, i64, dp]
        lib.oracle_process_range.restype = C.c_int
        lib.oracle_process_range.argtypes = [C.c_void_p, dp, i64, dp, C.c_int, C.c_int]
        lib.oracle_samples_done.restype = i64
        lib.oracle_samples_done.argtypes = [C.c_void_p]
        lib.oracle_filter_one.argtypes = [dp, dp, C.c_int32, dp, dp, i64, dp]
        lib.oracle_threads.restype = C.c_int
        lib.oracle_threads.argtypes = [C.c_int]
        lib.oracle_downsample.argtypes = [dp, C.c_int, dp, i64, dp]
        lib.oracle_upsample_add.argtypes = [dp, C.c_int, dp, i64, dp, dp]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _cplx_pairs(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.view(np.float64)


class OracleBank:
    """Streaming FP64 bank: ``process(x)`` consumes the next block of the stream."""

    def __init__(self, tables):
        lib = _load()
        self._keep = []
        nf = np.ascontiguousarray(tables.n_filters.reshape(-1), dtype=np.int32)
        a1 = _cplx_pairs(tables.a1)
        b0 = _cplx_pairs(tables.b0)
        d = np.ascontiguousarray(tables.delay, dtype=np.int32)
        hd = np.ascontiguousarray(tables.h_down, dtype=np.float64)
        hu = np.ascontiguousarray(tables.h_up, dtype=np.float64)
        self._keep += [nf, a1, b0, d, hd, hu]
        self.T, self.H = int(tables.n_templates), int(tables.n_bands)
        self._h = lib.oracle_create(self.T, self.H, _ip(nf), _dp(a1), _dp(b0), _ip(d),
                                    len(hd), _dp(hd), len(hu), _dp(hu))
        if not self._h:
            raise ValueError("oracle_create rejected the tables")
        self._lib = lib

    def process(self, x, t_lo: int = 0, t_hi: int | None = None) -> np.ndarray:
        """Next len(x) samples -> complex128 z[T, len(x)] (rows outside [t_lo, t_hi) are 0)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        n = len(x)
        z = np.zeros((self.T, n), np.complex128)
        hi = self.T if t_hi is None else t_hi
        rc = self._lib.oracle_process_range(self._h, _dp(x), n, _dp(z.view(np.float64)), t_lo, hi)
        if rc != 0:
            raise ValueError("block length must be a multiple of 2^(H-1)")
        return z

    @property
    def samples_done(self) -> int:
        return int(self._lib.oracle_samples_done(self._h))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def run_stream(tables, x, block: int | None = None) -> np.ndarray:
    """Whole stream through a fresh bank, in blocks of ``block`` samples (default: one)."""
    bank = OracleBank(tables)
    x = np.asarray(x, dtype=np.float64)
    if block is None or block >= len(x):
        out = bank.process(x)
    else:
        parts = [bank.process(x[i:i + block]) for i in range(0, len(x), block)]
        out = np.concatenate(parts, axis=1)
    bank.close()
    return out


def filter_one(a1: complex, b0: complex, d: int, x) -> np.ndarray:
    """One filter of Eq. (7) from zero state over a real or complex input."""
    lib = _load()
    x = np.asarray(x)
    xr = np.ascontiguousarray(x.real, dtype=np.float64)
    xi = np.ascontiguousarray(x.imag if np.iscomplexobj(x) else np.zeros(len(x)), dtype=np.float64)
    a = np.array([a1.real, a1.imag], np.float64)
    b = np.array([b0.real, b0.imag], np.float64)
    y = np.zeros(len(x), np.complex128)
    lib.oracle_filter_one(_dp(a), _dp(b), int(d), _dp(xr), _dp(xi), len(x), _dp(y.view(np.float64)))
    return y


def downsample(h_down, x) -> np.ndarray:
    """One /2 stage from zero history: out[m] = sum_j h[j] x[2m - j]."""
    lib = _load()
    h = np.ascontiguousarray(h_down, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(len(x) // 2, np.float64)
    lib.oracle_downsample(_dp(h), len(h), _dp(x), len(x), _dp(out))
    return out


def upsample_add(h_up, low, z) -> np.ndarray:
    """One x2 upsample-and-add stage from zero history (complex)."""
    lib = _load()
    h = np.ascontiguousarray(h_up, dtype=np.float64)
    low = np.ascontiguousarray(low, dtype=np.complex128)
    z = np.ascontiguousarray(z, dtype=np.complex128)
    assert len(z) == 2 * len(low)
    acc = np.zeros(len(z), np.complex128)
    lib.oracle_upsample_add(_dp(h), len(h), _dp(low.view(np.float64)), len(low),
                            _dp(z.view(np.float64)), _dp(acc.view(np.float64)))
    return acc


def set_threads(n: int = 0) -> int:
    """Threads of the template loop for timing (0 = all); returns the count in use."""
    return int(_load().oracle_threads(int(n)))
