"""Pins for the CPU oracle: each test checks the oracle against something other
than itself (a library routine, a closed form, an exact special case, brute
force, or a printed value of the paper), so that a dropped term, a wrong sign
or index, or a transposed operand fails at least one of them.
"""
import json
import os

import numpy as np
import pytest
import scipy.signal

import oracle
from paper_1511_03599_amd import metrics, synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return d / n if n else d


def rand_stream(B, S, C, T, seed):
    x = synth.complex_gaussian((B, S + T - 1, C), seed)
    h = synth.random_taps(C, T, seed + 1).astype(np.float64)
    return x, h


# --- FIR (Algorithm 1) ---------------------------------------------------------

@pytest.mark.parametrize("C", [1, 2, 3, 8])
@pytest.mark.parametrize("T", [1, 2, 3, 5])
@pytest.mark.parametrize("S", [1, 2, 7])
def test_fir_matches_library_convolution(C, T, S):
    """Per channel, the FIR is a 'valid' convolution with the reversed taps."""
    x, h = rand_stream(2, S, C, T, 11 + C + 10 * T + 100 * S)
    y = oracle.fir(x, h)
    assert y.shape == (2, S, C)
    for b in range(2):
        for c in range(C):
            ref = np.convolve(x[b, :, c], h[::-1, c], mode="valid")
            assert rel(y[b, :, c], ref) <= 1e-14


def test_fir_single_channel_is_correlation():
    x, h = rand_stream(1, 40, 1, 6, 5)
    y = oracle.fir(x, h)
    ref = np.correlate(x[0, :, 0], h[:, 0].astype(np.complex128), mode="valid")
    assert rel(y[0, :, 0], ref) <= 1e-14


def test_fir_impulse_returns_reversed_taps_exactly():
    C, T, S = 16, 8, 12
    h = synth.random_taps(C, T, 3).astype(np.float64)
    x = np.zeros((1, S + T - 1, C), dtype=np.complex128)
    x[0, T - 1, :] = 1.0
    y = oracle.fir(x, h)
    for s in range(S):
        want = h[T - 1 - s] if s < T else np.zeros(C)
        assert np.array_equal(y[0, s].real, want)
        assert np.array_equal(y[0, s].imag, np.zeros(C))


def test_fir_linearity():
    x1, h1 = rand_stream(2, 9, 6, 4, 21)
    x2, h2 = rand_stream(2, 9, 6, 4, 22)
    a, b = 0.7 - 0.2j, -1.3 + 0.5j
    lhs = oracle.fir(a * x1 + b * x2, h1)
    rhs = a * oracle.fir(x1, h1) + b * oracle.fir(x2, h1)
    assert rel(lhs, rhs) <= 1e-12
    lhs = oracle.fir(x1, 0.3 * h1 - 2.0 * h2)
    rhs = 0.3 * oracle.fir(x1, h1) - 2.0 * oracle.fir(x1, h2)
    assert rel(lhs, rhs) <= 1e-12


def test_fir_shift_equivariance_exact():
    x, h = rand_stream(1, 20, 8, 5, 31)
    y = oracle.fir(x, h)
    y_shift = oracle.fir(x[:, 1:], h)
    assert np.array_equal(y_shift, y[:, 1:])


# --- DFT (Eq. (2)) ---------------------------------------------------------------

@pytest.mark.parametrize("C", [1, 2, 3, 8, 12, 64, 96, 105, 3072])
def test_single_tap_unit_filter_is_library_fft(C):
    """With T=1 and h=1 the filter bank is the DFT of each raw spectrum."""
    x = synth.complex_gaussian((2, 5, C), 41 + C)
    h = np.ones((1, C))
    Y = oracle.pfb_forward(x, h)
    assert rel(Y, np.fft.fft(x, axis=-1)) <= 1e-12


def test_inverse_sign_is_unnormalised_library_ifft():
    a = synth.complex_gaussian((3, 32), 51)
    assert rel(oracle.dft(a, +1), np.fft.ifft(a, axis=-1) * 32) <= 1e-12


def test_dft_of_delta_is_all_ones_and_parseval():
    C = 32
    d = np.zeros((1, C), dtype=np.complex128)
    d[0, 0] = 1.0
    assert np.allclose(oracle.dft(d), np.ones(C), atol=0, rtol=0)
    a = synth.complex_gaussian((4, C), 52)
    A = oracle.dft(a)
    lhs = np.sum(np.abs(A) ** 2, axis=-1)
    rhs = C * np.sum(np.abs(a) ** 2, axis=-1)
    assert np.max(np.abs(lhs / rhs - 1)) <= 1e-12


def test_dft_shifted_delta_is_pure_phase():
    C, n0 = 16, 3
    d = np.zeros((1, C), dtype=np.complex128)
    d[0, n0] = 1.0
    m = np.arange(C)
    want = np.cos(2 * np.pi * n0 * m / C) - 1j * np.sin(2 * np.pi * n0 * m / C)
    assert rel(oracle.dft(d)[0], want) <= 1e-14


# --- FIR + DFT ---------------------------------------------------------------------

def test_centre_tone_closed_form():
    """A tone at the centre of channel k0 gives y[s][c] = g[c] e^{2 pi i k0 c / C}
    with g[c] = sum_t h[t][c], hence Y[s][m] = G[(m - k0) mod C] for every s,
    with G the DFT of g; the peak Y[s][k0] = sum of all taps."""
    C, T, S, k0 = 256, 8, 6, 37
    h = synth.windowed_sinc_taps(C, T).astype(np.float64)
    x = synth.centre_tone(S + T - 1, C, k0)[None]
    Y = oracle.pfb_forward(x, h)
    G = np.fft.fft(h.sum(axis=0))
    want = np.roll(G, k0)
    for s in range(S):
        assert rel(Y[0, s], want) <= 1e-12
        assert int(np.argmax(np.abs(Y[0, s]))) == k0
    assert abs(Y[0, 0, k0].real - h.sum()) <= 1e-9 * abs(h.sum())
    # The windowed-sinc prototype of this size peaks at about 255.34.
    assert 255.0 < h.sum() < 255.7


def test_pfb_reduces_leakage_of_off_centre_tone():
    """Sec. 2 (Fig. 4): for a tone between bin centres, the filter bank puts a
    smaller fraction of the power outside the tone's channel than the plain DFT."""
    C, T, S = 64, 8, 16
    k, d = 10, 0.3
    x = synth.offset_tone(S + T - 1, C, (k + d) / C, 0.4)[None]
    h = synth.windowed_sinc_taps(C, T).astype(np.float64)
    Yp = oracle.pfb_forward(x, h)
    Yd = oracle.pfb_forward(x[:, T - 1:], np.ones((1, C)))

    def out_frac(Y):
        p = np.abs(Y) ** 2
        near = p[..., k] + p[..., k + 1]
        return 1 - near.sum() / p.sum()

    assert out_frac(Yp) < 0.1 * out_frac(Yd)


def test_tone_peak_in_right_bin_with_noise():
    st = synth.small_stream(S=64)
    Y = oracle.pfb_forward(st.x, st.h)
    assert np.all(np.argmax(np.abs(Y[0]), axis=-1) == 37)


# --- Adjoints ------------------------------------------------------------------------

def test_adjoint_dot_product_in_x():
    B, S, C, T = 2, 7, 8, 4
    x, h = rand_stream(B, S, C, T, 61)
    V = synth.complex_gaussian((B, S, C), 62)
    Ax = oracle.pfb_forward(x, h)
    gx, _ = oracle.pfb_adjoint(x, h, V)
    lhs = np.vdot(V, Ax).real
    rhs = np.vdot(gx, x).real
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_dot_product_in_taps():
    B, S, C, T = 2, 7, 8, 4
    x, h = rand_stream(B, S, C, T, 63)
    V = synth.complex_gaussian((B, S, C), 64)
    dh = synth.random_taps(C, T, 65).astype(np.float64)
    # Y is linear in h for fixed x, so <V, Y(dh)> = <gh, dh>.
    lhs = np.vdot(V, oracle.pfb_forward(x, dh)).real
    _, gh = oracle.pfb_adjoint(x, h, V)
    rhs = float(np.sum(gh * dh))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_fir_adjoints_against_explicit_matrix():
    """Build the FIR as an explicit real matrix acting on (re, im) and compare
    both adjoints with its transpose."""
    B, S, C, T = 1, 4, 3, 3
    x, h = rand_stream(B, S, C, T, 66)
    rows = S + T - 1
    n_in, n_out = rows * C, S * C
    M = np.zeros((n_out, n_in))
    for s in range(S):
        for c in range(C):
            for t in range(T):
                M[s * C + c, (s + t) * C + c] = h[t, c]
    gy = synth.complex_gaussian((B, S, C), 67)
    gx = oracle.fir_adjoint_x(gy, h)
    want = (M.T @ gy[0].ravel()).reshape(rows, C)
    assert rel(gx[0], want) <= 1e-14
    gh = oracle.fir_adjoint_h(gy, x, T)
    want_h = np.zeros((T, C))
    for t in range(T):
        for c in range(C):
            # d y[s][c] / d h[t][c] = x[s+t][c]
            col = np.array([x[0, s + t, c] for s in range(S)])
            want_h[t, c] = np.sum(np.conj(gy[0, :, c]) * col).real
    assert rel(gh, want_h) <= 1e-14


@pytest.mark.parametrize("C", [8, 12, 64])
def test_dft_at_listed_bins_matches_library_fft(C):
    """Eq. (2) at a few output indices equals the library FFT at those bins;
    the inverse sign equals C times the library inverse FFT there."""
    a = synth.complex_gaussian((5, C), 81 + C)
    bins = [0, C - 1, C // 2, 3, 3]
    assert rel(oracle.dft_bins(a, bins), np.fft.fft(a, axis=-1)[:, bins]) <= 1e-13
    assert rel(oracle.dft_bins(a, bins, +1), C * np.fft.ifft(a, axis=-1)[:, bins]) <= 1e-13


def test_restricted_adjoints_equal_the_pinned_full_adjoint():
    """The tap gradient at listed channels and the sample gradient at listed
    raw spectra, as used at sizes where the full adjoint is too slow, equal
    the corresponding entries of the full adjoint (itself pinned above by the
    dot-product identities, the explicit matrix and finite differences),
    including rows at both ends where fewer than T filtered rows contribute."""
    B, S, C, T = 3, 11, 16, 5
    x, h = rand_stream(B, S, C, T, 91)
    gY = synth.complex_gaussian((B, S, C), 92)
    gx, gh = oracle.pfb_adjoint(x, h, gY)
    ch = [0, 15, 7, 7, 3]
    assert rel(oracle.pfb_adjoint_h_channels(x, gY, T, ch), gh[:, ch]) <= 1e-13
    xs = synth.quantise(x, "c64")      # the stored (..., 2) form is accepted too
    gh32 = oracle.pfb_adjoint(xs, h, gY)[1]
    assert rel(oracle.pfb_adjoint_h_channels(xs, gY, T, ch), gh32[:, ch]) <= 1e-13
    rows = [0, 1, T - 1, S - 1, S, S + T - 2]
    assert rel(oracle.pfb_adjoint_x_rows(h, gY, rows), gx[:, rows]) <= 1e-13


def test_leakage_loss_gradient_finite_difference_small():
    """Central differences (step 1e-6) of the out-of-channel loss against the
    oracle adjoint, on every tap and on a set of samples. The loss is quadratic
    in h for fixed x and in x for fixed h, so the central difference is exact
    apart from rounding."""
    B, S, C, T = 2, 8, 16, 4
    x = synth.complex_gaussian((B, S + T - 1, C), 71)
    h = synth.random_taps(C, T, 72).astype(np.float64)
    bins = np.array([3, 11])

    def L(xx, hh):
        return oracle.leakage_loss(oracle.pfb_forward(xx, hh), bins)[0]

    _, gY = oracle.leakage_loss(oracle.pfb_forward(x, h), bins)
    gx, gh = oracle.pfb_adjoint(x, h, gY)
    eps = 1e-6
    fd = np.zeros_like(h)
    for t in range(T):
        for c in range(C):
            e = np.zeros_like(h)
            e[t, c] = eps
            fd[t, c] = (L(x, h + e) - L(x, h - e)) / (2 * eps)
    assert rel(gh, fd) <= 1e-7
    g = synth.rng(73)
    for _ in range(12):
        b, r, c = g.integers(0, B), g.integers(0, S + T - 1), g.integers(0, C)
        for part, unit in ((0, 1.0), (1, 1j)):
            e = np.zeros_like(x)
            e[b, r, c] = eps * unit
            fd_v = (L(x + e, h) - L(x - e, h)) / (2 * eps)
            an = gx[b, r, c].real if part == 0 else gx[b, r, c].imag
            assert abs(fd_v - an) <= 1e-6 * max(1.0, abs(an))


def test_loss_gradient_is_twice_masked_spectrum():
    Y = synth.complex_gaussian((2, 3, 8), 74)
    bins = [1, 5]
    L, gY = oracle.leakage_loss(Y, bins)
    eps = 1e-6
    for (b, s, m) in [(0, 0, 0), (0, 2, 1), (1, 1, 5), (1, 2, 7)]:
        for unit in (1.0, 1j):
            e = np.zeros_like(Y)
            e[b, s, m] = eps * unit
            fd = (oracle.leakage_loss(Y + e, bins)[0] - oracle.leakage_loss(Y - e, bins)[0]) / (2 * eps)
            an = gY[b, s, m].real if unit == 1.0 else gY[b, s, m].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


# --- Inputs and measures ---------------------------------------------------------------

@pytest.mark.parametrize("C,T", [(256, 8), (1024, 16), (64, 3)])
def test_taps_generator_matches_library_firwin(C, T):
    h = synth.windowed_sinc_taps(C, T).astype(np.float64).ravel()
    ref = scipy.signal.firwin(C * T, 1.0 / C, window="hamming", scale=False) * C
    assert np.max(np.abs(h - ref)) <= 1e-7 * np.max(np.abs(ref))
    assert np.array_equal(h, h[::-1])


def test_quantisers_clip_and_round():
    xc = np.array([[1.5, -2.5, 300.7 - 400.2j, -1e9 + 1e9j]])
    q8 = synth.quantise(xc, "ci8")
    assert q8.dtype == np.int8
    assert q8[0, :, 0].tolist() == [2, -2, 127, -127]
    assert q8[0, :, 1].tolist() == [0, 0, -127, 127]
    q16 = synth.quantise(xc, "ci16")
    assert q16[0, :, 0].tolist() == [2, -2, 301, -32767]


def test_eq3_worked_example_golden():
    with open(os.path.join(GOLDEN, "eq3_worked_example.json")) as f:
        g = json.load(f)
    assert metrics.effective_flops(g["S"], g["C"], g["T"], g["seconds"]) == g["effective_flops"]


@pytest.mark.parametrize("S,T,SB", [(1, 4, 1), (10, 3, 10), (37, 8, 5), (100, 16, 32)])
def test_efficiency_and_reuse_by_counting(S, T, SB):
    # one block of all S filtered spectra reads S+T-1 raw spectra
    reads, _ = metrics.brute_force_reads(S, T, S)
    assert metrics.efficiency(S, T) == pytest.approx(S / reads)
    # Eq. (7): mean reuse per column per tap over a block of N = SB+T-1 columns
    N = SB + T - 1
    uses = np.zeros(N)
    for s in range(SB):
        for t in range(T):
            uses[s + t] += 1
    assert metrics.mean_reuse_per_tap(SB, T) == pytest.approx(uses.mean() / T)
    # with no reuse each filtered spectrum would read T raw spectra: ratio 1/T
    _, naive = metrics.brute_force_reads(S, T, SB)
    assert S / naive == pytest.approx(1.0 / T)
