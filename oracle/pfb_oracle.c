/*
 * Polyphase filter bank: plain CPU reference ("the oracle"), FP64.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the correctness reference for the
 * GPU library. It is used by the tests, by the smoke check and by the
 * benchmark's CPU-baseline leg, and by nothing else; the library never calls
 * it, and it shares no code, header, table or helper with the GPU path.
 *
 * It is written for a reader checking it against the paper by eye:
 *   - no blocking, no fusion, no reordering of sums beyond the definitions;
 *   - every complex value is a pair of doubles (re, im), interleaved;
 *   - every sum runs in the index order the definition states.
 *
 * Data model (Sec. 2, Sec. 3.1): a stream of complex samples split into
 * spectra of C channels, contiguous in channels; x[b][r][c] is channel c of
 * raw spectrum r of stream b. There are S+T-1 raw spectra per stream and S
 * filtered spectra, i.e. the filter is applied in "valid" mode with no zero
 * padding (the block of S_B filtered spectra reads S_B+T-1 raw spectra,
 * Sec. 3.2 and Fig. 5; the efficiency S/(S+T-1) of Sec. 4.1 also counts
 * S+T-1 raw spectra for S filtered ones).
 *
 * Coefficients: C*T real values, unique per (tap, channel), h[t*C + c]
 * (Sec. 3.1). The FIR index convention is the serial algorithm of Sec. 3.2
 * (Algorithm 1): filtered[s][c] = sum over t of h[t*C+c] * raw[s+t][c]. The
 * printed Eq. (1) has no channel term in its coefficient index and reaches
 * one past the end of b, so Algorithm 1's indexing is the one implemented.
 *
 * Parity status: every function below is pinned by CPU tests against
 * independent facts (brute-force library convolution, library FFT, closed
 * forms for impulses and centred tones, Parseval, the dot-product identity
 * for the adjoints, and central finite differences).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define RE(p, i) ((p)[2 * (i)])
#define IM(p, i) ((p)[2 * (i) + 1])

/* Status codes returned by every entry point. */
enum { ORACLE_OK = 0, ORACLE_EINVAL = 1, ORACLE_ENOMEM = 2 };

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by the following calls from this host thread (n >= 1). */
int oracle_set_num_threads(int n)
{
    if (n < 1)
        return ORACLE_EINVAL;
#ifdef _OPENMP
    omp_set_num_threads(n);
#endif
    return ORACLE_OK;
}

/*
 * FIR step (Sec. 2, first step of the scheme; Sec. 3.2, Algorithm 1).
 *   y[b][s][c] = sum_{t=0}^{T-1} h[t*C + c] * x[b][s+t][c]
 * x: [B][S+T-1][C] complex, h: [T][C] real, y: [B][S][C] complex.
 * The coefficients are real, so each tap scales re and im alike.
 */
int oracle_fir(const double *x, const double *h, int64_t B, int64_t S,
               int64_t C, int64_t T, double *y)
{
    if (B < 0 || S < 0 || C < 1 || T < 1 || !x || !h || !y)
        return ORACLE_EINVAL;
    const int64_t rows = S + T - 1;
    int64_t n = B * S;
#pragma omp parallel for schedule(static)
    for (int64_t bs = 0; bs < n; ++bs) {
        int64_t b = bs / S, s = bs % S;
        for (int64_t c = 0; c < C; ++c) {
            double acc_re = 0.0, acc_im = 0.0;
            for (int64_t t = 0; t < T; ++t) {
                int64_t xi = (b * rows + s + t) * C + c;
                double coeff = h[t * C + c];
                acc_re += coeff * RE(x, xi);
                acc_im += coeff * IM(x, xi);
            }
            int64_t yi = (b * S + s) * C + c;
            RE(y, yi) = acc_re;
            IM(y, yi) = acc_im;
        }
    }
    return ORACLE_OK;
}

/*
 * Twiddle table w[k] = exp(sign * 2 pi i k / C), k = 0..C-1, in FP64.
 * The DFT below indexes it with (n*m) mod C computed in 64-bit integers,
 * so the angle is reduced exactly before any floating point is involved.
 */
static double *twiddles(int64_t C, int sign)
{
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)C);
    if (!w)
        return NULL;
    for (int64_t k = 0; k < C; ++k) {
        double a = 2.0 * M_PI * (double)k / (double)C;
        RE(w, k) = cos(a);
        IM(w, k) = sign * sin(a);
    }
    return w;
}

/*
 * DFT step (Sec. 2, Eq. (2)), applied to each row of C values:
 *   Y[m] = sum_{n=0}^{C-1} y[n] * exp(sign * 2 pi i n m / C)
 * sign = -1 is the forward transform of the paper; sign = +1 gives the
 * unnormalised inverse used by the adjoint. No scaling, bins in natural
 * order 0..C-1. Direct O(C^2) sum per row.
 */
int oracle_dft(const double *in, int64_t nrows, int64_t C, int sign, double *out)
{
    if (nrows < 0 || C < 1 || !in || !out || (sign != 1 && sign != -1))
        return ORACLE_EINVAL;
    double *w = twiddles(C, sign);
    if (!w)
        return ORACLE_ENOMEM;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        const double *row = in + 2 * r * C;
        double *dst = out + 2 * r * C;
        for (int64_t m = 0; m < C; ++m) {
            double acc_re = 0.0, acc_im = 0.0;
            for (int64_t n = 0; n < C; ++n) {
                int64_t k = (n * m) % C;
                double a = RE(row, n), bb = IM(row, n);
                double wr = RE(w, k), wi = IM(w, k);
                acc_re += a * wr - bb * wi;
                acc_im += a * wi + bb * wr;
            }
            RE(dst, m) = acc_re;
            IM(dst, m) = acc_im;
        }
    }
    free(w);
    return ORACLE_OK;
}

/*
 * The same DFT (Sec. 2, Eq. (2)) evaluated only at the listed output indices:
 *   out[r][j] = sum_{n=0}^{C-1} in[r][n] * exp(sign * 2 pi i n bins[j] / C)
 * for every row r and j < nbins (each bins[j] in [0, C)). This is the plain
 * definition at fewer indices, so a few bins of a very long set of rows cost
 * O(rows * C * nbins) instead of O(rows * C^2). out: [nrows][nbins] complex.
 */
int oracle_dft_bins(const double *in, int64_t nrows, int64_t C, int sign,
                    const int64_t *bins, int64_t nbins, double *out)
{
    if (nrows < 0 || C < 1 || nbins < 0 || !in || !out || (nbins > 0 && !bins) ||
        (sign != 1 && sign != -1))
        return ORACLE_EINVAL;
    for (int64_t j = 0; j < nbins; ++j)
        if (bins[j] < 0 || bins[j] >= C)
            return ORACLE_EINVAL;
    double *w = twiddles(C, sign);
    if (!w)
        return ORACLE_ENOMEM;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        const double *row = in + 2 * r * C;
        for (int64_t j = 0; j < nbins; ++j) {
            const int64_t m = bins[j];
            double acc_re = 0.0, acc_im = 0.0;
            for (int64_t n = 0; n < C; ++n) {
                int64_t k = (n * m) % C;
                double a = RE(row, n), bb = IM(row, n);
                double wr = RE(w, k), wi = IM(w, k);
                acc_re += a * wr - bb * wi;
                acc_im += a * wi + bb * wr;
            }
            RE(out, r * nbins + j) = acc_re;
            IM(out, r * nbins + j) = acc_im;
        }
    }
    free(w);
    return ORACLE_OK;
}

/*
 * Whole forward filter bank (Sec. 2 scheme): FIR, then the DFT of every
 * filtered spectrum. y may be NULL when only Y is wanted; Y may be NULL when
 * only the filtered spectra are wanted.
 */
int oracle_pfb_forward(const double *x, const double *h, int64_t B, int64_t S,
                       int64_t C, int64_t T, double *y, double *Y)
{
    if (B < 0 || S < 0 || C < 1 || T < 1)
        return ORACLE_EINVAL;
    double *tmp = y;
    if (!tmp) {
        tmp = (double *)malloc(sizeof(double) * 2 * (size_t)(B * S * C));
        if (!tmp && B * S * C > 0)
            return ORACLE_ENOMEM;
    }
    int st = oracle_fir(x, h, B, S, C, T, tmp);
    if (st == ORACLE_OK && Y)
        st = oracle_dft(tmp, B * S, C, -1, Y);
    if (tmp != y)
        free(tmp);
    return st;
}

/*
 * Adjoint of the FIR with respect to the input samples. The FIR is linear in
 * x with real coefficients, so its adjoint scatters each filtered sample back
 * onto the raw samples that produced it, with the same coefficient:
 *   gx[b][p][c] = sum over (s, t) with s + t = p, 0 <= s < S, 0 <= t < T of
 *                 h[t*C + c] * gy[b][s][c]
 * gy: [B][S][C] complex, gx: [B][S+T-1][C] complex (overwritten).
 */
int oracle_fir_adjoint_x(const double *gy, const double *h, int64_t B, int64_t S,
                         int64_t C, int64_t T, double *gx)
{
    if (B < 0 || S < 0 || C < 1 || T < 1 || !gy || !h || !gx)
        return ORACLE_EINVAL;
    const int64_t rows = S + T - 1;
    int64_t n = B * rows;
#pragma omp parallel for schedule(static)
    for (int64_t bp = 0; bp < n; ++bp) {
        int64_t b = bp / rows, p = bp % rows;
        for (int64_t c = 0; c < C; ++c) {
            double acc_re = 0.0, acc_im = 0.0;
            for (int64_t t = 0; t < T; ++t) {
                int64_t s = p - t;
                if (s < 0 || s >= S)
                    continue;
                int64_t gi = (b * S + s) * C + c;
                acc_re += h[t * C + c] * RE(gy, gi);
                acc_im += h[t * C + c] * IM(gy, gi);
            }
            int64_t xi = (b * rows + p) * C + c;
            RE(gx, xi) = acc_re;
            IM(gx, xi) = acc_im;
        }
    }
    return ORACLE_OK;
}

/*
 * Gradient of a real loss with respect to the (real) coefficients, given the
 * gradient gy of the filtered spectra (complex, convention d/dRe + i d/dIm):
 *   gh[t*C + c] = sum_b sum_s Re( conj(gy[b][s][c]) * x[b][s+t][c] )
 *               = sum_b sum_s ( gy_re * x_re + gy_im * x_im )
 * summed over every stream, written (not accumulated) into gh: [T][C].
 */
int oracle_fir_adjoint_h(const double *gy, const double *x, int64_t B, int64_t S,
                         int64_t C, int64_t T, double *gh)
{
    if (B < 0 || S < 0 || C < 1 || T < 1 || !gy || !x || !gh)
        return ORACLE_EINVAL;
    const int64_t rows = S + T - 1;
    int64_t n = T * C;
#pragma omp parallel for schedule(static)
    for (int64_t tc = 0; tc < n; ++tc) {
        int64_t t = tc / C, c = tc % C;
        double acc = 0.0;
        for (int64_t b = 0; b < B; ++b)
            for (int64_t s = 0; s < S; ++s) {
                int64_t gi = (b * S + s) * C + c;
                int64_t xi = (b * rows + s + t) * C + c;
                acc += RE(gy, gi) * RE(x, xi) + IM(gy, gi) * IM(x, xi);
            }
        gh[tc] = acc;
    }
    return ORACLE_OK;
}

/*
 * Whole adjoint (backward) of the forward filter bank, given gY, the
 * gradient of a real loss with respect to the frequency spectra:
 *   gy = unnormalised inverse DFT of gY (the adjoint of Eq. (2)),
 *   gx = FIR adjoint in x of gy, gh = FIR adjoint in h of gy.
 * gx or gh may be NULL to skip that output.
 */
int oracle_pfb_adjoint(const double *x, const double *h, const double *gY,
                       int64_t B, int64_t S, int64_t C, int64_t T,
                       double *gx, double *gh)
{
    if (B < 0 || S < 0 || C < 1 || T < 1 || !gY)
        return ORACLE_EINVAL;
    double *gy = (double *)malloc(sizeof(double) * 2 * (size_t)(B * S * C));
    if (!gy && B * S * C > 0)
        return ORACLE_ENOMEM;
    int st = oracle_dft(gY, B * S, C, +1, gy);
    if (st == ORACLE_OK && gx)
        st = oracle_fir_adjoint_x(gy, h, B, S, C, T, gx);
    if (st == ORACLE_OK && gh)
        st = oracle_fir_adjoint_h(gy, x, B, S, C, T, gh);
    free(gy);
    return st;
}
