/*
 * FP64 reference FFT for the oracle.  TEST INFRASTRUCTURE ONLY: nothing in the
 * product path links or calls this file.
 *
 * Textbook recursive mixed-radix Cooley-Tukey (decimation in time) for any
 * length n: split off the smallest prime factor p of n, transform the p
 * decimated subsequences of length m = n/p, and combine them with the direct
 * O(p^2) sum  X[k + m s] = sum_q W_n^{q (k + m s)} Y_q[k].  Lengths that are
 * prime fall through to the direct DFT.  Twiddles W_N^e = exp(sign 2 pi i e/N)
 * are evaluated with cos/sin in double.
 *
 * Convention: forward  X[k] = sum_j x[j] exp(-2 pi i j k / n);
 *             inverse  x[j] = (1/n) sum_k X[k] exp(+2 pi i j k / n).
 * The spectral derivative operator of the solver (Sec. II-A: derivatives by
 * FFT / IFFT) is built on these two transforms.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int smallest_factor(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* out[0..n) = DFT of in[0], in[istride], ..., with root table w (w[e*wstride] =
 * W_n^e for e < n). */
static void dft_rec(const double complex *in, long istride, double complex *out, int n,
                    const double complex *w, long wstride)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    int p = smallest_factor(n);
    int m = n / p;
    for (int q = 0; q < p; ++q)
        dft_rec(in + q * istride, istride * p, out + (long)q * m, m, w, wstride * p);
    double complex tstack[64];
    double complex *t = p <= 64 ? tstack : (double complex *)malloc(sizeof(double complex) * p);
    for (int k = 0; k < m; ++k) {
        for (int q = 0; q < p; ++q) t[q] = out[(long)q * m + k];
        for (int s = 0; s < p; ++s) {
            double complex acc = 0;
            long idx = k + (long)m * s;
            long e = 0; /* e = q * idx mod n, advanced without a division */
            for (int q = 0; q < p; ++q) {
                acc += w[e * wstride] * t[q];
                e += idx;
                if (e >= n) e -= n;
            }
            out[idx] = acc;
        }
    }
    if (t != tstack) free(t);
}

void offt_roots(int n, int sign, double complex *w)
{
    for (int e = 0; e < n; ++e) {
        double a = 2.0 * M_PI * (double)e / (double)n;
        w[e] = cos(a) + sign * I * sin(a);
    }
}

/* In-place transform of x[0], x[stride], ..., length n.  work: 2n scratch. */
void offt_strided(double complex *x, long stride, int n, int sign, const double complex *w,
                  double complex *work)
{
    double complex *in = work, *out = work + n;
    for (int j = 0; j < n; ++j) in[j] = x[j * stride];
    dft_rec(in, 1, out, n, w, 1);
    double scale = sign > 0 ? 1.0 / n : 1.0;
    for (int j = 0; j < n; ++j) x[j * stride] = out[j] * scale;
}

void offt_1d(double complex *x, int n, int sign)
{
    double complex *w = malloc(sizeof(double complex) * n);
    double complex *work = malloc(sizeof(double complex) * 2 * n);
    offt_roots(n, sign, w);
    offt_strided(x, 1, n, sign, w, work);
    free(w);
    free(work);
}

/* 3-D transform of a[nz][ny][nx] (x fastest), applied axis by axis. */
void offt_3d(double complex *a, int nx, int ny, int nz, int sign)
{
    double complex *wx = malloc(sizeof(double complex) * nx);
    double complex *wy = malloc(sizeof(double complex) * ny);
    double complex *wz = malloc(sizeof(double complex) * nz);
    offt_roots(nx, sign, wx);
    offt_roots(ny, sign, wy);
    offt_roots(nz, sign, wz);
    long sxy = (long)nx * ny;
#pragma omp parallel
    {
        int nmax = nx > ny ? nx : ny;
        if (nz > nmax) nmax = nz;
        double complex *work = malloc(sizeof(double complex) * 2 * nmax);
#pragma omp for schedule(static)
        for (long r = 0; r < (long)ny * nz; ++r)
            offt_strided(a + r * nx, 1, nx, sign, wx, work);
#pragma omp for schedule(static)
        for (long r = 0; r < (long)nx * nz; ++r) {
            long z = r / nx, x = r % nx;
            offt_strided(a + z * sxy + x, nx, ny, sign, wy, work);
        }
#pragma omp for schedule(static)
        for (long r = 0; r < sxy; ++r)
            offt_strided(a + r, sxy, nz, sign, wz, work);
        free(work);
    }
    free(wx);
    free(wy);
    free(wz);
}
