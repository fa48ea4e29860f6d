"""Performance measures for the polyphase filter bank (host-side arithmetic).

effective_flops      Sec. 4.1, Eq. (3): 2*S*C*(2T-1) per pass (complex input,
                     one multiply and one add per tap, T-1 additions).
fft_flops            5*C*log2(C) per C-point complex FFT (the usual count; the
                     paper uses a library FFT and gives no count).
efficiency           Sec. 4.1: epsilon = B_w / B_r, ideal S/(S+T-1).
mean_reuse_per_tap   Sec. 4.1, Eq. (7): R_T = (N-n)/N, N = S_B+T-1, n = T-1.
msamples_per_s       Sec. 3 and Sec. 5.3: the sample rate a device sustains,
                     counted as new input samples B*S*C per second.
*_bytes              Algorithmic HBM bytes: what the method itself must read
                     and write once (inputs, taps, outputs), used as the
                     numerator of achieved bandwidth.
"""
from __future__ import annotations

import math

BYTES_PER_SAMPLE = {"c64": 8, "ci16": 4, "ci8": 2, "cf16": 4}
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 2.4 GHz x 64 FMA lanes x 2 (no packed FP32)


def effective_flops(S: int, C: int, T: int, seconds: float = 1.0) -> float:
    return 2.0 * S * C * (2 * T - 1) / seconds


def fft_flops(C: int, nffts: int) -> float:
    return 5.0 * C * math.log2(C) * nffts


def efficiency(S: int, T: int) -> float:
    return S / (S + T - 1)


def mean_reuse_per_tap(SB: int, T: int) -> float:
    N = SB + T - 1
    n = T - 1
    return (N - n) / N


def msamples_per_s(B: int, S: int, C: int, seconds: float) -> float:
    return B * S * C / seconds / 1e6


def fir_bytes(B, S, C, T, dtype="c64") -> int:
    """FIR alone: read x once, the taps once, write y once."""
    return B * (S + T - 1) * C * BYTES_PER_SAMPLE[dtype] + T * C * 4 + B * S * C * 8


def fft_bytes(B, S, C) -> int:
    """Stand-alone FFT pass: read y, write Y."""
    return 2 * B * S * C * 8


def pfb_fused_bytes(B, S, C, T, dtype="c64") -> int:
    """Whole forward filter bank with the filtered spectra kept on chip."""
    return fir_bytes(B, S, C, T, dtype)


def pfb_split_bytes(B, S, C, T, dtype="c64") -> int:
    return fir_bytes(B, S, C, T, dtype) + fft_bytes(B, S, C)


def backward_fused_bytes(B, S, C, T) -> int:
    """Adjoint with the inverse-transformed gradient kept on chip: read gY and
    x, write gx; read the taps, write the tap gradient."""
    rows = S + T - 1
    return B * S * C * 8 + 2 * B * rows * C * 8 + 2 * T * C * 4


def brute_force_reads(S: int, T: int, SB: int) -> tuple[int, int]:
    """Count, by walking blocks of S_B filtered spectra, how many raw spectra a
    blocked FIR reads (each block reads S_B+T-1) and how many it would read
    with no reuse at all (T per filtered spectrum)."""
    reads = 0
    s = 0
    while s < S:
        sb = min(SB, S - s)
        reads += sb + T - 1
        s += sb
    return reads, S * T
