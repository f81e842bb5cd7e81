/*
 * CPU oracle for the slab-decomposed 3D real FFT (Verma et al., "Scalable
 * Multi-node Fast Fourier Transform on GPUs").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference against which the GPU library is checked.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Everything is computed in FP64, whatever the precision of the data under
 * test.  Complex numbers are interleaved (re, im) pairs of doubles.
 *
 * What is computed (section 2, the forward and inverse DFT equations):
 *   forward  F(k) = sum_j f(j) exp(-2 pi i k.j / N)      (unnormalized)
 *   inverse  f(j) = sum_k F(k) exp(+2 pi i k.j / N)      (unnormalized)
 * The transforms are separable, so a 3D transform is a 1D transform along
 * each axis in turn; the composition over axes is done by the Python side.
 *
 * Two ways of evaluating a 1D transform are provided:
 *   method 0: the direct O(N^2) sum of the definition, any N >= 1;
 *   method 1: iterative radix-2 Cooley-Tukey (the fast algorithm named in
 *             section 2), N a power of two.
 * Both use one table W[m] = exp(-2 pi i m / N), m = 0..N-1, whose entries are
 * computed one by one from libm cos/sin after an exact integer reduction of
 * the angle to the first octant (never by a recurrence).  The direct sum
 * indexes it with (j*k) mod N in exact 64-bit integer arithmetic.
 *
 * Real input (section 2, Hermitian symmetry of the transform of a real
 * field): only kz = 0..N/2 is stored, K = N/2 + 1 values.  The complex to
 * real transform of an arbitrary half spectrum G is defined as
 *   f(j) = sum_{k=0}^{K-1} w(k) Re(G(k) exp(+2 pi i k j / N)),
 *   w(0) = w(N/2) = 1, w(k) = 2 otherwise,
 * which is the inverse DFT of the Hermitian extension of G (the reading
 * taken where the paper is silent about non-Hermitian input).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* exp(-2 pi i m / n) for 0 <= m < n, by exact reduction to angle
 * pi*a/(4n) in [0, pi/4] (a = 8m folded by the circle's symmetries). */
static void unit_root(int64_t m, int64_t n, double *re, double *im)
{
    int64_t a = 8 * m;          /* angle = 2 pi a / (8n) */
    int neg_sin = 0, neg_cos = 0, swap = 0;
    if (a > 4 * n) { a = 8 * n - a; neg_sin = 1; }       /* t -> 2pi - t   */
    if (a > 2 * n) { a = 4 * n - a; neg_cos = 1; }       /* t -> pi - t    */
    if (a > n)     { a = 2 * n - a; swap = 1; }          /* t -> pi/2 - t  */
    double t = (M_PI * (double)a) / (4.0 * (double)n);
    double c = cos(t), s = sin(t);
    if (swap) { double u = c; c = s; s = u; }
    if (neg_cos) c = -c;
    if (neg_sin) s = -s;
    /* exp(-i theta) = cos(theta) - i sin(theta) */
    *re = c;
    *im = -s;
}

/* W[m] = exp(-2 pi i m / n), interleaved. */
static double *root_table(int64_t n)
{
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    for (int64_t m = 0; m < n; ++m) unit_root(m, n, &w[2 * m], &w[2 * m + 1]);
    return w;
}

/* Direct DFT of one line: y[k] = sum_j x[j] W^{sign * j k}; sign = -1 is the
 * forward transform (W = exp(-2 pi i / n)), +1 the inverse. */
static void dft_direct(int64_t n, const double *x, double *y, int sign,
                       const double *w)
{
    for (int64_t k = 0; k < n; ++k) {
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            int64_t m = (j * k) % n;
            double wr = w[2 * m];
            double wi = sign < 0 ? w[2 * m + 1] : -w[2 * m + 1];
            double xr = x[2 * j], xi = x[2 * j + 1];
            sr += xr * wr - xi * wi;
            si += xr * wi + xi * wr;
        }
        y[2 * k] = sr;
        y[2 * k + 1] = si;
    }
}

/* Radix-2 decimation-in-time Cooley-Tukey: bit-reversed copy, then log2(n)
 * rounds of butterflies (u + w v, u - w v) over blocks of doubling length. */
static void dft_radix2(int64_t n, const double *x, double *y, int sign,
                       const double *w)
{
    int bits = 0;
    while (((int64_t)1 << bits) < n) ++bits;
    for (int64_t i = 0; i < n; ++i) {
        int64_t r = 0;
        for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
        y[2 * r] = x[2 * i];
        y[2 * r + 1] = x[2 * i + 1];
    }
    for (int64_t len = 2; len <= n; len <<= 1) {
        int64_t half = len / 2, step = n / len;
        for (int64_t base = 0; base < n; base += len) {
            for (int64_t k = 0; k < half; ++k) {
                int64_t m = k * step;
                double wr = w[2 * m];
                double wi = sign < 0 ? w[2 * m + 1] : -w[2 * m + 1];
                double *u = &y[2 * (base + k)];
                double *v = &y[2 * (base + k + half)];
                double vr = v[0] * wr - v[1] * wi;
                double vi = v[0] * wi + v[1] * wr;
                double ur = u[0], ui = u[1];
                u[0] = ur + vr; u[1] = ui + vi;
                v[0] = ur - vr; v[1] = ui - vi;
            }
        }
    }
}

static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

static void dft_line(int method, int64_t n, const double *x, double *y,
                     int sign, const double *w)
{
    if (method == 1) dft_radix2(n, x, y, sign, w);
    else dft_direct(n, x, y, sign, w);
}

/*
 * Complex-to-complex DFT along the middle axis of a [B][N][M] complex array
 * (one line per (b, m), elements N apart by M).  sign -1 forward, +1 inverse.
 * in and out may be the same buffer.  Returns 0, or -1 on bad arguments.
 */
int oracle_c2c_axis(int64_t B, int64_t N, int64_t M, const double *in,
                    double *out, int sign, int method)
{
    if (B < 0 || N < 1 || M < 0 || (sign != -1 && sign != 1)) return -1;
    if (method == 1 && !is_pow2(N)) return -1;
    if (method != 0 && method != 1) return -1;
    double *w = root_table(N);
    int64_t lines = B * M;
#pragma omp parallel
    {
        double *xl = (double *)malloc(sizeof(double) * 2 * (size_t)N);
        double *yl = (double *)malloc(sizeof(double) * 2 * (size_t)N);
#pragma omp for schedule(static)
        for (int64_t l = 0; l < lines; ++l) {
            int64_t b = l / M, m = l % M;
            const double *src = in + 2 * (b * N * M + m);
            for (int64_t j = 0; j < N; ++j) {
                xl[2 * j] = src[2 * j * M];
                xl[2 * j + 1] = src[2 * j * M + 1];
            }
            dft_line(method, N, xl, yl, sign, w);
            double *dst = out + 2 * (b * N * M + m);
            for (int64_t k = 0; k < N; ++k) {
                dst[2 * k * M] = yl[2 * k];
                dst[2 * k * M + 1] = yl[2 * k + 1];
            }
        }
        free(xl);
        free(yl);
    }
    free(w);
    return 0;
}

/*
 * Real-to-complex DFT along the last axis: rows of N reals -> rows of
 * K = N/2 + 1 complex values F[k] = sum_j x[j] exp(-2 pi i k j / N),
 * k = 0..N/2 (the stored half, section 2).  The full complex DFT of the row
 * is evaluated (real input promoted to complex) and its first K bins kept.
 */
int oracle_r2c_rows(int64_t rows, int64_t N, const double *in, double *out,
                    int method)
{
    if (rows < 0 || N < 1 || (method != 0 && method != 1)) return -1;
    if (method == 1 && !is_pow2(N)) return -1;
    int64_t K = N / 2 + 1;
    double *w = root_table(N);
#pragma omp parallel
    {
        double *xl = (double *)malloc(sizeof(double) * 2 * (size_t)N);
        double *yl = (double *)malloc(sizeof(double) * 2 * (size_t)N);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < rows; ++r) {
            for (int64_t j = 0; j < N; ++j) {
                xl[2 * j] = in[r * N + j];
                xl[2 * j + 1] = 0.0;
            }
            dft_line(method, N, xl, yl, -1, w);
            memcpy(out + 2 * r * K, yl, sizeof(double) * 2 * (size_t)K);
        }
        free(xl);
        free(yl);
    }
    free(w);
    return 0;
}

/*
 * Complex-to-real transform along the last axis: rows of K = N/2 + 1 complex
 * values G -> rows of N reals
 *   f[j] = sum_{k=0}^{K-1} w(k) Re(G[k] exp(+2 pi i k j / N)),
 *   w(k) = 1 for k = 0 and 2k = N, 2 otherwise.
 * method 0 evaluates this sum as written.  method 1 builds the Hermitian
 * extension H (H[0], H[N/2] real parts of G, H[k] = G[k], H[N-k] = conj G[k])
 * and takes the real part of its radix-2 inverse DFT, which is the same sum.
 */
int oracle_c2r_rows(int64_t rows, int64_t N, const double *in, double *out,
                    int method)
{
    if (rows < 0 || N < 1 || (method != 0 && method != 1)) return -1;
    if (method == 1 && !is_pow2(N)) return -1;
    int64_t K = N / 2 + 1;
    double *w = root_table(N);
#pragma omp parallel
    {
        double *xl = (double *)malloc(sizeof(double) * 2 * (size_t)N);
        double *yl = (double *)malloc(sizeof(double) * 2 * (size_t)N);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < rows; ++r) {
            const double *g = in + 2 * r * K;
            double *f = out + r * N;
            if (method == 0) {
                for (int64_t j = 0; j < N; ++j) {
                    double s = 0.0;
                    for (int64_t k = 0; k < K; ++k) {
                        double wk = (k == 0 || 2 * k == N) ? 1.0 : 2.0;
                        int64_t m = (k * j) % N;
                        /* exp(+i t) = conj(W[m]) = (W_re, -W_im) */
                        double er = w[2 * m], ei = -w[2 * m + 1];
                        s += wk * (g[2 * k] * er - g[2 * k + 1] * ei);
                    }
                    f[j] = s;
                }
            } else {
                for (int64_t k = 0; k < N; ++k) {
                    if (k < K) {
                        xl[2 * k] = g[2 * k];
                        xl[2 * k + 1] = (k == 0 || 2 * k == N) ? 0.0 : g[2 * k + 1];
                    } else {
                        xl[2 * k] = g[2 * (N - k)];
                        xl[2 * k + 1] = -g[2 * (N - k) + 1];
                    }
                }
                dft_line(1, N, xl, yl, +1, w);
                for (int64_t j = 0; j < N; ++j) f[j] = yl[2 * j];
            }
        }
        free(xl);
        free(yl);
    }
    free(w);
    return 0;
}

/*
 * Sum over the z axis for fixed wavenumbers: for each real row f[r][0..N-1]
 * and each requested kz, A[r][q] = sum_z f[r][z] exp(-2 pi i kz_q z / N).
 * This is the innermost sum of the forward equation, evaluated for a few kz
 * so that whole kz-planes of a large transform can be checked without the
 * full transform.
 */
int oracle_zsum_rows(int64_t rows, int64_t N, const double *in, int64_t nq,
                     const int64_t *kz, double *out)
{
    if (rows < 0 || N < 1 || nq < 0) return -1;
    for (int64_t q = 0; q < nq; ++q)
        if (kz[q] < 0 || kz[q] >= N) return -1;
    double *w = root_table(N);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; ++r) {
        const double *f = in + r * N;
        for (int64_t q = 0; q < nq; ++q) {
            double sr = 0.0, si = 0.0;
            for (int64_t z = 0; z < N; ++z) {
                int64_t m = (kz[q] * z) % N;
                sr += f[z] * w[2 * m];
                si += f[z] * w[2 * m + 1];
            }
            out[2 * (r * nq + q)] = sr;
            out[2 * (r * nq + q) + 1] = si;
        }
    }
    free(w);
    return 0;
}

/* Threads the OpenMP runtime will use (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
