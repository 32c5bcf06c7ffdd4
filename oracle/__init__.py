"""FP64 CPU oracle for the 1D complex-to-complex DFT (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it, and it
never imports the GPU library: the two share no code.

The C routines live in ``oracle.c``; this module builds them with gcc into
``liboracle.so`` next to the source (``build()``) and wraps them for numpy.
Conventions (paper section 3, Eq. 1; sign and scaling as the FFTW comparison
in section 4 implies): forward uses exp(-2 pi i k n / N), inverse uses
exp(+2 pi i k n / N), neither is scaled.

Parity status: every routine here is pinned by ``tests/test_oracle.py``
(closed forms, Eq. 1 built from Kronecker products, numpy's pocketfft,
invariants, brute-force sums and finite differences).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

FORWARD = -1
INVERSE = +1


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, no hand vectorisation) into liboracle.so."""
    global _lib
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    compile_source(_SRC, tmp)
    os.replace(tmp, _LIB)
    _lib = None
    return _LIB


def load_library(path: str):
    """Open a compiled copy of oracle.c and declare its C signatures."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.oracle_dft.argtypes = [i64, ctypes.c_int, dp, dp, dp, dp]
    lib.oracle_fft_r2.argtypes = [i64, ctypes.c_int, dp, dp, dp, dp]
    lib.oracle_fft_r2_batch.argtypes = [i64, i64, ctypes.c_int, dp, dp, dp, dp, ctypes.c_int]
    lib.oracle_wpower_loss.argtypes = [i64, dp, dp, dp, dp]
    lib.oracle_wpower_grad.argtypes = [i64, dp, dp, dp, dp, dp]
    lib.oracle_rfft_batch.argtypes = [i64, i64, dp, dp, dp, ctypes.c_int]
    lib.oracle_irfft_batch.argtypes = [i64, i64, dp, dp, dp, ctypes.c_int]
    for f in (lib.oracle_dft, lib.oracle_fft_r2, lib.oracle_fft_r2_batch,
              lib.oracle_wpower_loss, lib.oracle_wpower_grad, lib.oracle_rfft_batch,
              lib.oracle_irfft_batch):
        f.restype = ctypes.c_int
    return lib


def compile_source(src: str, out: str) -> str:
    """gcc -O2 build of an oracle source file into a shared library at `out`."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", out, src, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    _lib = load_library(_LIB)
    return _lib


def use_library(path: str | None) -> None:
    """Point the module-level functions at another compiled oracle (None = default)."""
    global _lib
    _lib = None if path is None else load_library(path)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _split(x) -> tuple[np.ndarray, np.ndarray]:
    """Real and imaginary parts as contiguous float64 (exact widening)."""
    x = np.asarray(x)
    if np.iscomplexobj(x):
        return (np.ascontiguousarray(x.real, dtype=np.float64),
                np.ascontiguousarray(x.imag, dtype=np.float64))
    return np.ascontiguousarray(x, dtype=np.float64), np.zeros(x.shape, np.float64)


def _check(rc: int, what: str):
    if rc == -1:
        raise ValueError(f"oracle {what}: invalid argument")
    if rc != 0:
        raise MemoryError(f"oracle {what}: allocation failed")


def dft(x, sign: int = FORWARD) -> np.ndarray:
    """O(N^2) DFT of the last axis, straight from the definition."""
    xr, xi = _split(x)
    n = xr.shape[-1]
    rows_r = xr.reshape(-1, n)
    rows_i = xi.reshape(-1, n)
    yr = np.empty_like(rows_r)
    yi = np.empty_like(rows_i)
    lib = _load()
    for b in range(rows_r.shape[0]):
        ar, ai = np.ascontiguousarray(rows_r[b]), np.ascontiguousarray(rows_i[b])
        br, bi = np.empty(n), np.empty(n)
        _check(lib.oracle_dft(n, sign, _ptr(ar), _ptr(ai), _ptr(br), _ptr(bi)), "dft")
        yr[b], yi[b] = br, bi
    return (yr + 1j * yi).reshape(xr.shape)


def fft(x, sign: int = FORWARD, threads: int = 1) -> np.ndarray:
    """Recursive radix-2 FFT of the last axis (power-of-two length)."""
    xr, xi = _split(x)
    n = xr.shape[-1]
    batch = xr.size // n if n else 0
    yr = np.empty_like(xr)
    yi = np.empty_like(xi)
    rc = _load().oracle_fft_r2_batch(n, batch, sign, _ptr(xr), _ptr(xi), _ptr(yr), _ptr(yi), threads)
    _check(rc, "fft_r2")
    return yr + 1j * yi


def ifft_unnormalised(x, threads: int = 1) -> np.ndarray:
    """Inverse transform without the 1/N factor (the adjoint F^H)."""
    return fft(x, INVERSE, threads)


def fft_split_inplace_arrays(xr: np.ndarray, xi: np.ndarray, yr: np.ndarray, yi: np.ndarray,
                             sign: int = FORWARD, threads: int = 1) -> None:
    """Batch FFT on caller-provided contiguous float64 arrays (no copies)."""
    n = xr.shape[-1]
    batch = xr.size // n
    for a in (xr, xi, yr, yi):
        if a.dtype != np.float64 or not a.flags.c_contiguous:
            raise ValueError("contiguous float64 arrays required")
    rc = _load().oracle_fft_r2_batch(n, batch, sign, _ptr(xr), _ptr(xi), _ptr(yr), _ptr(yi), threads)
    _check(rc, "fft_r2")


def wpower_loss(x, w) -> float:
    """L = sum_k w_k |(F x)_k|^2 for one transform."""
    xr, xi = _split(x)
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros(1)
    _check(_load().oracle_wpower_loss(xr.shape[-1], _ptr(xr), _ptr(xi), _ptr(w), _ptr(out)), "loss")
    return float(out[0])


def wpower_grad(x, w) -> np.ndarray:
    """dL/dRe(x) + i dL/dIm(x) = 2 F^H (w .* F x) for one transform."""
    xr, xi = _split(x)
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = xr.shape[-1]
    gr, gi = np.empty(n), np.empty(n)
    _check(_load().oracle_wpower_grad(n, _ptr(xr), _ptr(xi), _ptr(w), _ptr(gr), _ptr(gi)), "grad")
    return gr + 1j * gi


def rfft(x, threads: int = 1) -> np.ndarray:
    """Real-to-complex: the forward DFT of each real row of length N (last
    axis), its non-redundant half k = 0 .. N/2 (N/2 + 1 values per row)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[-1]
    batch = x.size // n if n else 0
    h = n // 2 + 1
    yr = np.empty(x.shape[:-1] + (h,))
    yi = np.empty_like(yr)
    _check(_load().oracle_rfft_batch(n, batch, _ptr(x), _ptr(yr), _ptr(yi), threads), "rfft")
    return yr + 1j * yi


def irfft(x, n: int, threads: int = 1) -> np.ndarray:
    """Complex-to-real: rows of N/2 + 1 values (last axis) -> the real part of
    the unnormalised inverse DFT of their Hermitian extension, N reals per row
    (irfft(rfft(x), N) = N x)."""
    xr, xi = _split(x)
    h = n // 2 + 1
    if xr.shape[-1] != h:
        raise ValueError(f"expected rows of {h} values for n = {n}")
    batch = xr.size // h
    y = np.empty(xr.shape[:-1] + (n,))
    _check(_load().oracle_irfft_batch(n, batch, _ptr(xr), _ptr(xi), _ptr(y), threads), "irfft")
    return y


def fftn(x, ndim: int, sign: int = FORWARD, threads: int = 1) -> np.ndarray:
    """Multi-dimensional DFT over the last `ndim` axes,
        X[k_1..k_d] = sum_{n_1..n_d} x[n_1..n_d] exp(sign 2 pi i sum_j k_j n_j / N_j),
    evaluated one axis at a time with the 1D transform above (the exponential
    factorises over the axes, so the d-fold sum is d nested 1D sums)."""
    y = np.asarray(x, dtype=np.complex128)
    for ax in range(y.ndim - ndim, y.ndim):
        moved = np.moveaxis(y, ax, -1)
        y = np.moveaxis(fft(np.ascontiguousarray(moved), sign, threads), -1, ax)
    return y


def rel_l2(y, ref) -> float:
    """||y - ref||_2 / ||ref||_2 in float64 (0/0 is 0)."""
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    num = np.linalg.norm((y - ref).ravel())
    den = np.linalg.norm(ref.ravel())
    if den == 0.0:
        return float(num)
    return float(num / den)


def rel_l2_rows(y, ref) -> np.ndarray:
    """Per-row (per-transform) relative L2 error along the last axis."""
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    num = np.linalg.norm(y - ref, axis=-1)
    den = np.linalg.norm(ref, axis=-1)
    return np.where(den == 0.0, num, num / np.where(den == 0.0, 1.0, den))
