"""Seeded synthetic inputs for the polyphase filter bank.

This module is shared by the CPU oracle's tests, the GPU parity tests and the
benchmark. It produces input arrays only (sample streams, filter taps, tone
parameters, beam descriptions) and contains none of the filter bank's own
arithmetic: no FIR, no DFT, no adjoint.

Layouts follow the paper's data model (Sec. 2 and Sec. 3.1): a stream of
complex samples split into spectra of C channels, contiguous in channels, so a
stream is ``x[row][channel]`` with ``row`` a raw-spectrum index. Complex values
are stored interleaved (re, im). Taps are C*T FP32 values, unique per channel
and tap (Sec. 3.1), laid out ``h[t*C + c]``.

Every generator takes an explicit integer seed and uses numpy's PCG64.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Input element types of the filter bank (Sec. 3.1: 32-, 16- and 8-bit input;
# the low-precision forms are signed complex integers here, plus half floats).
DTYPES = ("c64", "ci16", "ci8", "cf16")
BYTES_PER_SAMPLE = {"c64": 8, "ci16": 4, "ci8": 2, "cf16": 4}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# ----------------------------------------------------------------------------
# Filter taps
# ----------------------------------------------------------------------------

def hamming(n: int) -> np.ndarray:
    """Symmetric Hamming window of length n, in float64."""
    if n == 1:
        return np.ones(1)
    k = np.arange(n, dtype=np.float64)
    return 0.54 - 0.46 * np.cos(2.0 * np.pi * k / (n - 1))


def hann(n: int) -> np.ndarray:
    """Symmetric Hann ("Hanning") window of length n, in float64."""
    if n == 1:
        return np.ones(1)
    k = np.arange(n, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * k / (n - 1))


def windowed_sinc_taps(channels: int, taps: int, window: str = "hamming") -> np.ndarray:
    """Prototype filter of length N = taps*channels: a sinc of cutoff 1/C times
    a window (Sec. 2, Fig. 2). Returned as float32 with shape [taps, channels],
    so ``h[t, c]`` is element ``t*C + c`` of the flat prototype.

    h[k] = w[k] * sinc((k - (N-1)/2) / C), sinc(u) = sin(pi u)/(pi u), with no
    normalisation (the peak is about 1). Computed in float64 and rounded once,
    round-to-nearest-even, to float32.
    """
    n = channels * taps
    k = np.arange(n, dtype=np.float64)
    u = (k - (n - 1) / 2.0) / channels
    w = hamming(n) if window == "hamming" else hann(n)
    h = w * np.sinc(u)
    return h.astype(np.float32).reshape(taps, channels)


def random_taps(channels: int, taps: int, seed: int) -> np.ndarray:
    """Unstructured taps (no symmetry), uniform in [-1, 1), float32 [T, C]."""
    return rng(seed).uniform(-1.0, 1.0, size=(taps, channels)).astype(np.float32)


# ----------------------------------------------------------------------------
# Sample streams
# ----------------------------------------------------------------------------

def complex_gaussian(shape, seed: int, sigma: float = 1.0) -> np.ndarray:
    """Complex Gaussian noise, real and imaginary parts iid N(0, sigma^2/2),
    so E|x|^2 = sigma^2. Returned as complex128."""
    g = rng(seed)
    s = sigma / math.sqrt(2.0)
    re = g.standard_normal(size=shape, dtype=np.float64) * s
    im = g.standard_normal(size=shape, dtype=np.float64) * s
    return re + 1j * im


def complex_gaussian_c64(shape, seed: int) -> np.ndarray:
    """Unit-variance complex Gaussian noise generated directly in float32
    (cheaper for the large benchmark shapes). Returned as complex64."""
    g = rng(seed)
    s = np.float32(1.0 / math.sqrt(2.0))
    out = np.empty(tuple(shape) + (2,), dtype=np.float32)
    g.standard_normal(size=out.shape, dtype=np.float32, out=out)
    out *= s
    return out.view(np.complex64).reshape(shape)


def centre_tone(rows: int, channels: int, bin_index: int, amplitude: float = 1.0) -> np.ndarray:
    """Tone at the centre of channel `bin_index`: x[n] = A exp(+2 pi i k n / C)
    with n = row*C + c the global sample index. complex128 [rows, C]."""
    n = np.arange(rows * channels, dtype=np.int64)
    ph = (n * bin_index) % channels  # exact integer reduction of the phase
    return amplitude * np.exp(2j * np.pi * ph.astype(np.float64) / channels).reshape(rows, channels)


def offset_tone(rows: int, channels: int, freq_cycles_per_sample: float, phase: float) -> np.ndarray:
    """Unit tone at an arbitrary frequency f (cycles per sample):
    x[n] = exp(i (2 pi f n + phase)), n = row*C + c. complex128 [rows, C]."""
    n = np.arange(rows * channels, dtype=np.float64)
    return np.exp(1j * (2.0 * np.pi * freq_cycles_per_sample * n + phase)).reshape(rows, channels)


def quantise(xc: np.ndarray, dtype: str) -> np.ndarray:
    """Store a complex128 stream in one of the filter bank's input types.

    Returns an array with a trailing (re, im) axis of the storage type:
    ci8  -> int8,  round half to even, clip to [-127, 127];
    ci16 -> int16, round half to even, clip to [-32767, 32767];
    cf16 -> float16, round to nearest even;
    c64  -> float32, round to nearest even.
    """
    pair = np.stack([xc.real, xc.imag], axis=-1)
    if dtype == "ci8":
        return np.clip(np.rint(pair), -127, 127).astype(np.int8)
    if dtype == "ci16":
        return np.clip(np.rint(pair), -32767, 32767).astype(np.int16)
    if dtype == "cf16":
        return pair.astype(np.float16)
    if dtype == "c64":
        return pair.astype(np.float32)
    raise ValueError(f"unknown dtype {dtype!r}")


def stored_to_complex128(stored: np.ndarray) -> np.ndarray:
    """Exact widening of a stored (..., 2) array to complex128."""
    f = stored.astype(np.float64)
    return f[..., 0] + 1j * f[..., 1]


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Stream:
    """One filter-bank problem: x has shape [B, S+T-1, C] (+ trailing re/im
    axis in its storage type) and h has shape [T, C] float32."""
    x: np.ndarray
    h: np.ndarray
    dtype: str
    B: int
    S: int
    C: int
    T: int
    tone_bins: np.ndarray | None = None

    @property
    def rows(self) -> int:
        return self.S + self.T - 1


def seed_for(config: int, variant: int = 0) -> int:
    return 1511000 + 100 * config + variant


def small_stream(B=1, C=256, T=8, S=4096, seed=None, tone_bin=37) -> Stream:
    """Single stream, complex64: unit-variance complex Gaussian noise plus a
    unit tone at the centre of channel `tone_bin`; Hamming-windowed sinc taps."""
    seed = seed_for(1) if seed is None else seed
    rows = S + T - 1
    xc = complex_gaussian((B, rows, C), seed)
    if tone_bin is not None:
        xc = xc + centre_tone(rows, C, tone_bin)[None]
    return Stream(quantise(xc, "c64"), windowed_sinc_taps(C, T), "c64", B, S, C, T)


def noise_stream(B, C, T, S, seed, dtype="c64", fast=False) -> Stream:
    """Noise-only stream in the requested storage type. int8 uses sigma=16 and
    int16 sigma=2000 per real component; fp16 and c64 are unit variance."""
    rows = S + T - 1
    if dtype == "c64" and fast:
        xs = complex_gaussian_c64((B, rows, C), seed)
        x = xs.view(np.float32).reshape(B, rows, C, 2)
        return Stream(x, windowed_sinc_taps(C, T), dtype, B, S, C, T)
    if dtype == "ci8":
        xc = complex_gaussian((B, rows, C), seed, sigma=16.0 * math.sqrt(2.0))
    elif dtype == "ci16":
        xc = complex_gaussian((B, rows, C), seed, sigma=2000.0 * math.sqrt(2.0))
    else:
        xc = complex_gaussian((B, rows, C), seed)
    return Stream(quantise(xc, dtype), windowed_sinc_taps(C, T), dtype, B, S, C, T)


def device_noise(shape, seed: int, device):
    """Unit-variance complex64 Gaussian noise generated on the device with a
    seeded torch generator (for timing runs whose sizes make host generation
    slow; the values play no role in the timing)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return torch.randn(tuple(shape), dtype=torch.complex64, device=device, generator=g)


def device_quantised_noise(shape, dtype: str, seed: int, device):
    """Noise of the given storage type generated on the device (timing runs):
    the same distributions as noise_stream (sigma 16 for int8, 2000 for int16
    per real component, round half to even, symmetric clip; unit variance for
    float16 and complex64), as a tensor in the library's layout (complex64
    [shape], else [shape + (2,)] of the storage type)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    pair = torch.randn(tuple(shape) + (2,), dtype=torch.float32, device=device, generator=g)
    if dtype == "ci8":
        return torch.clamp(torch.round(pair * 16.0), -127, 127).to(torch.int8)
    if dtype == "ci16":
        return torch.clamp(torch.round(pair * 2000.0), -32767, 32767).to(torch.int16)
    pair *= 1.0 / math.sqrt(2.0)
    if dtype == "cf16":
        return pair.to(torch.float16)
    return torch.view_as_complex(pair)


def device_tone_streams(B, C, T, S, seed, device):
    """The differentiable workload's tone-only streams (tone_params, the
    offset_tone formula), evaluated on the device in float64 and rounded once
    to complex64 [B, S+T-1, C] (timing runs)."""
    import torch
    rows = S + T - 1
    k, d, ph = tone_params(B, C, seed)
    n = torch.arange(rows * C, dtype=torch.float64, device=device)
    out = torch.empty((B, rows, C), dtype=torch.complex64, device=device)
    for b in range(B):
        ang = 2.0 * math.pi * float((k[b] + d[b]) / C) * n + float(ph[b])
        out[b] = torch.polar(torch.ones_like(ang), ang).to(torch.complex64).reshape(rows, C)
    return out


def tone_params(B: int, C: int, seed: int):
    """Per-stream off-centre tones: bin k_b uniform in [0, C), offset delta_b
    uniform in +-[0.1, 0.4] bins, phase uniform in [0, 2 pi)."""
    g = rng(seed)
    k = g.integers(0, C, size=B)
    mag = g.uniform(0.1, 0.4, size=B)
    sign = np.where(g.integers(0, 2, size=B) == 0, -1.0, 1.0)
    phase = g.uniform(0.0, 2.0 * np.pi, size=B)
    return k.astype(np.int64), sign * mag, phase


def tone_streams(B=32, C=1024, T=16, S=8192, seed=None) -> Stream:
    """Differentiable workload: per stream a unit tone at (k_b + delta_b)/C
    cycles per sample, tone only, complex64 (generated per stream in float64
    and rounded once)."""
    seed = seed_for(5) if seed is None else seed
    rows = S + T - 1
    k, d, ph = tone_params(B, C, seed)
    x = np.empty((B, rows, C, 2), dtype=np.float32)
    for b in range(B):
        xb = offset_tone(rows, C, (k[b] + d[b]) / C, ph[b])
        x[b, ..., 0] = xb.real
        x[b, ..., 1] = xb.imag
    st = Stream(x, windowed_sinc_taps(C, T), "c64", B, S, C, T)
    st.tone_bins = k
    return st


@dataclasses.dataclass
class Beam:
    C: int
    T: int
    S: int
    seed: int


def beam_table(nbeams=64, seed=None, c_choices=(128, 256, 512, 1024, 2048, 4096, 8192),
               t_choices=(4, 8, 16, 32), s_range=(1024, 32768)) -> list[Beam]:
    """Uneven multi-beam workload: C, T drawn uniformly from the choices, S
    uniform in [lo, hi] inclusive (output spectra per beam)."""
    seed = seed_for(4) if seed is None else seed
    g = rng(seed)
    out = []
    for i in range(nbeams):
        C = int(g.choice(c_choices))
        T = int(g.choice(t_choices))
        S = int(g.integers(s_range[0], s_range[1] + 1))
        out.append(Beam(C, T, S, seed * 1000 + i))
    return out
