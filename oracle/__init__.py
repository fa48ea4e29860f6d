"""CPU reference ("the oracle") for the polyphase filter bank, FP64.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library. It shares no code with
the GPU path; its arithmetic lives in ``pfb_oracle.c`` (plain C, built with
gcc and OpenMP), and this module only marshals numpy arrays into it.

Functions and the passages they follow:
  fir            -- Sec. 3.2, Algorithm 1 (the FIR of Sec. 2, first step)
  dft            -- Sec. 2, Eq. (2); sign=+1 gives the unnormalised inverse
  dft_bins       -- Eq. (2) evaluated at listed output indices only
  pfb_forward    -- Sec. 2 two-step scheme: FIR, then DFT of each spectrum
  fir_adjoint_x  -- adjoint of Algorithm 1 in the samples
  fir_adjoint_h  -- adjoint of Algorithm 1 in the coefficients
  pfb_adjoint    -- adjoint of the two-step scheme (inverse DFT, then both)
  pfb_adjoint_h_channels -- its tap gradient at listed channels only
  pfb_adjoint_x_rows     -- its sample gradient at listed raw spectra only
  leakage_loss   -- out-of-channel power of the frequency spectra and its
                    gradient (a training objective built on the scheme)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pfb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_pfb.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP). Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER(ctypes.c_double)
    I = ctypes.c_int64
    lib.oracle_fir.argtypes = [P, P, I, I, I, I, P]
    lib.oracle_dft.argtypes = [P, I, I, ctypes.c_int, P]
    lib.oracle_pfb_forward.argtypes = [P, P, I, I, I, I, P, P]
    lib.oracle_fir_adjoint_x.argtypes = [P, P, I, I, I, I, P]
    lib.oracle_fir_adjoint_h.argtypes = [P, P, I, I, I, I, P]
    lib.oracle_pfb_adjoint.argtypes = [P, P, P, I, I, I, I, P, P]
    lib.oracle_dft_bins.argtypes = [P, I, I, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), I, P]
    lib.oracle_num_threads.argtypes = []
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    for f in ("oracle_fir", "oracle_dft", "oracle_dft_bins", "oracle_pfb_forward", "oracle_fir_adjoint_x",
              "oracle_fir_adjoint_h", "oracle_pfb_adjoint", "oracle_num_threads",
              "oracle_set_num_threads"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the following oracle calls from this thread."""
    _check(_load().oracle_set_num_threads(int(n)), "oracle_set_num_threads")


def _as_c128(a) -> np.ndarray:
    """Widen a complex array, or a stored (..., 2) pair array of any real type,
    to contiguous complex128 (exact for every input type used here)."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return np.ascontiguousarray(a, dtype=np.complex128)
    if a.shape[-1] != 2:
        raise ValueError("real input must carry a trailing (re, im) axis")
    f = a.astype(np.float64)
    return np.ascontiguousarray(f[..., 0] + 1j * f[..., 1])


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(st: int, name: str):
    if st != 0:
        raise RuntimeError(f"{name} failed with status {st}")


def _shape_fir(x, h):
    x = _as_c128(x)
    h = np.ascontiguousarray(np.asarray(h), dtype=np.float64)
    if x.ndim == 2:
        x = x[None]
    B, rows, C = x.shape
    T = h.shape[0]
    if h.shape != (T, C):
        raise ValueError(f"taps shape {h.shape} does not match C={C}")
    S = rows - T + 1
    if S < 0:
        raise ValueError("fewer raw spectra than taps - 1")
    return x, h, B, S, C, T


def fir(x, h) -> np.ndarray:
    """Filtered spectra y[B, S, C] (complex128) from x[B, S+T-1, C] and h[T, C]."""
    x, h, B, S, C, T = _shape_fir(x, h)
    y = np.empty((B, S, C), dtype=np.complex128)
    _check(_load().oracle_fir(_ptr(x), _ptr(h), B, S, C, T, _ptr(y)), "oracle_fir")
    return y


def dft(a, sign: int = -1) -> np.ndarray:
    """Direct DFT along the last axis (Eq. (2)); sign=+1 for the unnormalised
    inverse. Returns complex128 of the same shape."""
    a = _as_c128(a)
    C = a.shape[-1]
    out = np.empty_like(a)
    nrows = a.size // C if C else 0
    _check(_load().oracle_dft(_ptr(a), nrows, C, int(sign), _ptr(out)), "oracle_dft")
    return out


def dft_bins(a, bins, sign: int = -1) -> np.ndarray:
    """Eq. (2) along the last axis, evaluated only at the output indices
    `bins` (the plain definition at those indices). Returns complex128 of
    shape a.shape[:-1] + (len(bins),)."""
    a = _as_c128(a)
    C = a.shape[-1]
    b = np.ascontiguousarray(np.asarray(bins, dtype=np.int64))
    nrows = a.size // C if C else 0
    out = np.empty(a.shape[:-1] + (b.size,), dtype=np.complex128)
    _check(_load().oracle_dft_bins(_ptr(a), nrows, C, int(sign),
                                   b.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), b.size, _ptr(out)),
           "oracle_dft_bins")
    return out


def pfb_forward(x, h, want_y: bool = False):
    """Frequency spectra Y[B, S, C]; with want_y also the filtered spectra."""
    x, h, B, S, C, T = _shape_fir(x, h)
    Y = np.empty((B, S, C), dtype=np.complex128)
    y = np.empty((B, S, C), dtype=np.complex128) if want_y else None
    yp = _ptr(y) if want_y else None
    _check(_load().oracle_pfb_forward(_ptr(x), _ptr(h), B, S, C, T, yp, _ptr(Y)),
           "oracle_pfb_forward")
    return (Y, y) if want_y else Y


def fir_adjoint_x(gy, h) -> np.ndarray:
    gy = _as_c128(gy)
    if gy.ndim == 2:
        gy = gy[None]
    h = np.ascontiguousarray(np.asarray(h), dtype=np.float64)
    B, S, C = gy.shape
    T = h.shape[0]
    gx = np.empty((B, S + T - 1, C), dtype=np.complex128)
    _check(_load().oracle_fir_adjoint_x(_ptr(gy), _ptr(h), B, S, C, T, _ptr(gx)),
           "oracle_fir_adjoint_x")
    return gx


def fir_adjoint_h(gy, x, T: int) -> np.ndarray:
    gy = _as_c128(gy)
    x = _as_c128(x)
    if gy.ndim == 2:
        gy, x = gy[None], x[None]
    B, S, C = gy.shape
    if x.shape != (B, S + T - 1, C):
        raise ValueError("x shape does not match gy and T")
    gh = np.empty((T, C), dtype=np.float64)
    _check(_load().oracle_fir_adjoint_h(_ptr(gy), _ptr(x), B, S, C, T, _ptr(gh)),
           "oracle_fir_adjoint_h")
    return gh


def pfb_adjoint(x, h, gY):
    """(gx, gh) for a real loss with frequency-spectra gradient gY."""
    x, h, B, S, C, T = _shape_fir(x, h)
    gY = _as_c128(gY)
    if gY.ndim == 2:
        gY = gY[None]
    if gY.shape != (B, S, C):
        raise ValueError("gY shape mismatch")
    gx = np.empty((B, S + T - 1, C), dtype=np.complex128)
    gh = np.empty((T, C), dtype=np.float64)
    _check(_load().oracle_pfb_adjoint(_ptr(x), _ptr(h), _ptr(gY), B, S, C, T, _ptr(gx),
                                      _ptr(gh)), "oracle_pfb_adjoint")
    return gx, gh


def pfb_adjoint_h_channels(x, gY, T: int, channels) -> np.ndarray:
    """Tap gradient of the adjoint (as pfb_adjoint) at the listed channels
    only: gh[t, j] for channel channels[j], shape [T, len(channels)].
    The filtered-spectra gradient of channel c is the inverse DFT of gY
    (adjoint of Eq. (2)) evaluated at output index c, and the tap gradient of
    channel c depends on that channel alone (adjoint of Algorithm 1), so
    both steps restrict exactly to the listed channels."""
    ch = np.asarray(channels, dtype=np.int64)
    gy = dft_bins(gY, ch, +1)
    x = np.asarray(x)
    xs = x[:, :, ch] if np.iscomplexobj(x) else x[:, :, ch, :]
    return fir_adjoint_h(gy, xs, T)


def pfb_adjoint_x_rows(h, gY, rows) -> np.ndarray:
    """Sample gradient of the adjoint (as pfb_adjoint) at the listed raw
    spectra p only, shape [B, len(rows), C]. gx[p] depends on the filtered
    gradient rows p-T+1 .. p inside [0, S) (adjoint of Algorithm 1), each the
    inverse DFT of one gY row (adjoint of Eq. (2)); those rows alone are
    transformed and scattered back."""
    gY = _as_c128(gY)
    if gY.ndim == 2:
        gY = gY[None]
    h = np.ascontiguousarray(np.asarray(h), dtype=np.float64)
    B, S, C = gY.shape
    T = h.shape[0]
    out = np.empty((B, len(rows), C), dtype=np.complex128)
    for j, p in enumerate(rows):
        if not 0 <= p < S + T - 1:
            raise ValueError(f"row {p} outside [0, S+T-1)")
        s0, s1 = max(0, p - T + 1), min(S, p + 1)
        gy = dft(gY[:, s0:s1], +1)
        out[:, j] = fir_adjoint_x(gy, h)[:, p - s0]
    return out


def leakage_loss(Y, tone_bins):
    """Out-of-channel power: L = sum_b sum_s sum_{m != k_b} |Y[b, s, m]|^2 and its
    gradient in the convention dL/dRe + i dL/dIm, which is 2 * M * Y with M the
    mask that is 0 on each stream's tone bin and 1 elsewhere."""
    Y = _as_c128(Y)
    mask = np.ones(Y.shape, dtype=np.float64)
    for b, k in enumerate(np.asarray(tone_bins)):
        mask[b, :, int(k)] = 0.0
    L = float(np.sum(mask * (Y.real ** 2 + Y.imag ** 2)))
    return L, 2.0 * mask * Y

