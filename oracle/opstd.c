/*
 * FP64 CPU oracle of the Fourier pseudo-spectral, staggered-grid, leapfrog
 * solver of the lossless 3-D elastic wave equation.  TEST INFRASTRUCTURE ONLY.
 *
 * What it follows:
 *  - eq. 2 (first-order stress-velocity system) with the viscosities set to
 *    zero (Sec. II-A, lossless case);
 *  - eq. 4 for the Lame parameters: mu = rho cs^2, lambda = rho cp^2 - 2 mu;
 *  - Sec. II-A: spatial derivatives in the wavenumber domain by FFT / IFFT,
 *    leapfrog in time on a grid staggered in space and time;
 *  - Sec. II-B: a perfectly matched layer of a given number of cells at the
 *    domain edges, and the CFL number of eq. 5 for stability;
 *  - eq. 3: the hydrophone pressure p = -(sxx + syy + szz) / 3;
 *  - eq. 6-7: point sources described by a symmetric stress (moment) tensor.
 *
 * Readings where the paper is silent (the same readings the GPU library takes):
 *  - derivative operators D_d^{+-} f = IFFT[ i k_d exp(+-i k_d h_d / 2) kappa FFT f ],
 *    with the k-space correction kappa = sinc(c_ref |k| dt / 2) (1 when off);
 *  - nodes: normal stresses, lambda, mu, p at cell centres; v_x at (+1/2,0,0),
 *    v_y at (0,+1/2,0), v_z at (0,0,+1/2); s_xy at (+1/2,+1/2,0), s_xz at
 *    (+1/2,0,+1/2), s_yz at (0,+1/2,+1/2);
 *  - rho at velocity nodes: arithmetic mean of the two neighbours (the upper
 *    neighbour clamped at the high edge); mu at shear nodes: harmonic mean of
 *    the four surrounding centres (clamped), 0 if any of them is 0;
 *  - split-field PML on all six faces, profile alpha = (A c_ref / h)(depth/L)^4,
 *    factor a = exp(-alpha dt / 2) applied before and after adding the update;
 *    multi-axial (M-PML): the split part along axis d is damped by alpha_d plus
 *    p times the profiles of the two other axes, all evaluated at the field's
 *    own node (p = 0 is the classical split PML);
 *  - a source adds -dt w[n] M_cd / dV to each stress component, split equally
 *    over the split parts; shear parts are spread 1/4 to each of the 4 shear
 *    nodes around the cell centre;
 *  - optional source smoothing (Sec. II-A: the delta is smoothed with a
 *    Blackman window in the spatial-frequency domain): the point source's
 *    delta is transformed, multiplied by W(k) = prod_d [0.42 + 0.5 cos(k_d h_d)
 *    + 0.08 cos(2 k_d h_d)] (a Blackman window over [-pi/h_d, pi/h_d] on each
 *    axis, zero at the edges) and transformed back; every cell of the result
 *    (up to round-off) then carries a point source of that weight;
 *  - v is recorded at time (n + 1/2) dt, p at (n + 1) dt.
 *
 * Everything is evaluated plainly: each derivative is a full complex 3-D FFT of
 * the summed field, one pointwise multiply and a full complex inverse 3-D FFT
 * whose real part is kept.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

struct ostate {
    int nx, ny, nz;
    long n;
    double h[3], dt;
    int kspace;
    double c_ref;
    /* materials */
    double *lam, *mu, *rinv[3], *mu_s[3]; /* mu_s: xy, xz, yz */
    /* PML factors a_d at integer / half nodes; b = a^p for the other axes */
    double *a_int[3], *a_half[3];
    double *b_int[3], *b_half[3];
    /* wavenumbers per axis, 1-D operator symbols i k exp(+-i k h/2), kappa(|k|) */
    double *k[3];
    double complex *sym[3][2];
    double *kappa;
    /* state: v[c][d] (9), sn[c][d] (9 normal), ss[p][2] (shear xy:(x,y) xz:(x,z) yz:(y,z)) */
    double *v[3][3], *sn[3][3], *ss[3][2];
    /* Kelvin-Voigt viscosity (eq. 1-2): chi, eta at centres, eta at the shear
     * nodes; ep: the nine velocity derivatives of the previous step (order
     * D-_x vx, D-_y vy, D-_z vz, then the shear pieces xy(x), xy(y), xz(x),
     * xz(z), yz(y), yz(z)); NULL when lossless */
    double *chi, *eta, *eta_s[3];
    double *ep[9];
    /* sources / receivers */
    int n_src, nt_w;
    int *src;
    double *m6, *wav;
    /* source smoothing (0 off, 1 Blackman window in k-space): per source the
     * cells [sm_ofs[q], sm_ofs[q+1]) of sm_ijk / sm_w carry weight sm_w */
    int smooth;
    int *sm_ofs, *sm_ijk;
    double *sm_w;
    int n_rec;
    int *rec;
    long step;
    /* scratch */
    double complex *A, *B;
    double *tmp[9];
};

static inline long IDX(const ostate *s, long i, long j, long k)
{
    return i + s->nx * (j + (long)s->ny * k);
}

static double pml_alpha(double pos, int n, int L, double A, double c, double h)
{
    if (L <= 0) return 0.0;
    double d1 = (double)L - pos;
    double d2 = pos - (double)(n - 1 - L);
    double d = d1 > d2 ? d1 : d2;
    if (d < 0) d = 0;
    if (d > L) d = L;
    double r = d / L;
    return A * c / h * r * r * r * r;
}

static int build_operator(ostate *s);

static void free_state(ostate *s)
{
    if (!s) return;
    free(s->lam);
    free(s->mu);
    for (int d = 0; d < 3; ++d) {
        free(s->rinv[d]);
        free(s->mu_s[d]);
        free(s->a_int[d]);
        free(s->a_half[d]);
        free(s->b_int[d]);
        free(s->b_half[d]);
        free(s->k[d]);
        free(s->sym[d][0]);
        free(s->sym[d][1]);
        for (int c = 0; c < 3; ++c) {
            free(s->v[c][d]);
            free(s->sn[c][d]);
        }
        free(s->ss[d][0]);
        free(s->ss[d][1]);
    }
    for (int t = 0; t < 9; ++t) free(s->tmp[t]);
    free(s->kappa);
    free(s->A);
    free(s->B);
    free(s->src);
    free(s->m6);
    free(s->wav);
    free(s->sm_ofs);
    free(s->sm_ijk);
    free(s->sm_w);
    free(s->chi);
    free(s->eta);
    for (int d = 0; d < 3; ++d) free(s->eta_s[d]);
    for (int t = 0; t < 9; ++t) free(s->ep[t]);
    free(s->rec);
    free(s);
}

void opstd_destroy(ostate *s) { free_state(s); }

long opstd_step_index(const ostate *s) { return s->step; }

/* threads the OpenMP loops of the oracle use */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void opstd_set_step(ostate *s, long step) { s->step = step; }

ostate *opstd_create(int nx, int ny, int nz, const double *vp, const double *vs,
                     const double *rho, double dx, double dy, double dz, double dt, int pml_n,
                     double pml_A, double pml_p, int kspace, double c_ref, int n_rec,
                     const int *rec_ijk, int *err)
{
    *err = ORC_EINVAL;
    if (!(pml_p >= 0 && pml_p <= 1)) return NULL;
    if (nx < 2 || ny < 2 || nz < 2 || !(dx > 0) || !(dy > 0) || !(dz > 0) || !(dt > 0)) return NULL;
    if (pml_n < 0 || 2 * pml_n > nx || 2 * pml_n > ny || 2 * pml_n > nz || pml_A < 0) return NULL;
    long n = (long)nx * ny * nz;
    double cmax = 0;
    for (long c = 0; c < n; ++c) {
        if (!(vp[c] > 0) || !(rho[c] > 0) || !(vs[c] >= 0) || !isfinite(vp[c]) ||
            !isfinite(vs[c]) || !isfinite(rho[c]))
            return NULL;
        if (3.0 * vp[c] * vp[c] <= 4.0 * vs[c] * vs[c]) return NULL; /* bulk modulus > 0 */
        if (vp[c] > cmax) cmax = vp[c];
    }
    for (int r = 0; r < n_rec; ++r) {
        const int *q = rec_ijk + 3 * r;
        if (q[0] < 0 || q[0] >= nx || q[1] < 0 || q[1] >= ny || q[2] < 0 || q[2] >= nz) return NULL;
    }
    if (c_ref <= 0) c_ref = cmax;
    /* stability (eq. 5 generalised to 3-D for the leapfrog PSTD scheme) */
    double sh = sqrt(1 / (dx * dx) + 1 / (dy * dy) + 1 / (dz * dz));
    if (!kspace) {
        if (cmax * dt * sh > 2.0 / M_PI) {
            *err = ORC_EUNSTABLE;
            return NULL;
        }
    } else if (c_ref < cmax) {
        double arg = c_ref * M_PI * sh * dt / 2;
        double smax = arg >= M_PI / 2 ? 1.0 : sin(arg);
        if (cmax / c_ref * smax > 1.0) {
            *err = ORC_EUNSTABLE;
            return NULL;
        }
    }

    *err = ORC_ENOMEM;
    ostate *s = calloc(1, sizeof(ostate));
    if (!s) return NULL;
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->n = n;
    s->h[0] = dx;
    s->h[1] = dy;
    s->h[2] = dz;
    s->dt = dt;
    s->kspace = kspace;
    s->c_ref = c_ref;
    int N[3] = {nx, ny, nz};

    s->lam = malloc(sizeof(double) * n);
    s->mu = malloc(sizeof(double) * n);
    for (int d = 0; d < 3; ++d) {
        s->rinv[d] = malloc(sizeof(double) * n);
        s->mu_s[d] = malloc(sizeof(double) * n);
        s->a_int[d] = malloc(sizeof(double) * N[d]);
        s->a_half[d] = malloc(sizeof(double) * N[d]);
        s->b_int[d] = malloc(sizeof(double) * N[d]);
        s->b_half[d] = malloc(sizeof(double) * N[d]);
        for (int c = 0; c < 3; ++c) {
            s->v[c][d] = calloc(n, sizeof(double));
            s->sn[c][d] = calloc(n, sizeof(double));
        }
        s->ss[d][0] = calloc(n, sizeof(double));
        s->ss[d][1] = calloc(n, sizeof(double));
    }
    for (int t = 0; t < 9; ++t) s->tmp[t] = malloc(sizeof(double) * n);
    s->A = malloc(sizeof(double complex) * n);
    s->B = malloc(sizeof(double complex) * n);
    s->rec = malloc(sizeof(int) * 3 * (n_rec > 0 ? n_rec : 1));
    if (!s->lam || !s->mu || !s->A || !s->B || !s->rec || !s->tmp[8] || !s->ss[2][1]) {
        free_state(s);
        return NULL;
    }
    s->n_rec = n_rec;
    if (n_rec) memcpy(s->rec, rec_ijk, sizeof(int) * 3 * n_rec);

    /* eq. 4 */
    for (long c = 0; c < n; ++c) {
        s->mu[c] = rho[c] * vs[c] * vs[c];
        s->lam[c] = rho[c] * vp[c] * vp[c] - 2.0 * s->mu[c];
    }
    /* staggered material values */
    for (int kk = 0; kk < nz; ++kk)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long c = IDX(s, i, j, kk);
                int ip = i + 1 < nx ? i + 1 : nx - 1;
                int jp = j + 1 < ny ? j + 1 : ny - 1;
                int kp = kk + 1 < nz ? kk + 1 : nz - 1;
                s->rinv[0][c] = 1.0 / (0.5 * (rho[c] + rho[IDX(s, ip, j, kk)]));
                s->rinv[1][c] = 1.0 / (0.5 * (rho[c] + rho[IDX(s, i, jp, kk)]));
                s->rinv[2][c] = 1.0 / (0.5 * (rho[c] + rho[IDX(s, i, j, kp)]));
                /* four centres around each shear node */
                long q[3][4] = {
                    {c, IDX(s, ip, j, kk), IDX(s, i, jp, kk), IDX(s, ip, jp, kk)},  /* xy */
                    {c, IDX(s, ip, j, kk), IDX(s, i, j, kp), IDX(s, ip, j, kp)},    /* xz */
                    {c, IDX(s, i, jp, kk), IDX(s, i, j, kp), IDX(s, i, jp, kp)}};   /* yz */
                for (int p = 0; p < 3; ++p) {
                    double inv = 0;
                    int fluid = 0;
                    for (int t = 0; t < 4; ++t) {
                        double m = s->mu[q[p][t]];
                        if (m == 0) fluid = 1;
                        else inv += 1.0 / m;
                    }
                    s->mu_s[p][c] = fluid ? 0.0 : 4.0 / inv;
                }
            }
    /* PML factors */
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i < N[d]; ++i) {
            double ai = pml_alpha(i, N[d], pml_n, pml_A, c_ref, s->h[d]);
            double ah = pml_alpha(i + 0.5, N[d], pml_n, pml_A, c_ref, s->h[d]);
            s->a_int[d][i] = exp(-ai * dt / 2);
            s->a_half[d][i] = exp(-ah * dt / 2);
            s->b_int[d][i] = exp(-pml_p * ai * dt / 2);
            s->b_half[d][i] = exp(-pml_p * ah * dt / 2);
        }
    if (build_operator(s) != ORC_OK) {
        free_state(s);
        return NULL;
    }
    *err = ORC_OK;
    return s;
}

/* Kelvin-Voigt viscosity (eq. 1-2): chi and eta per cell (host [n]); NULL
 * for both restores the lossless medium.  eta at the shear nodes is the
 * harmonic mean of the four surrounding centres, 0 if any of them is 0 (the
 * reading taken for mu).  The previous-step derivatives start at zero. */
int opstd_set_viscosity(ostate *s, const double *chi, const double *eta)
{
    free(s->chi);
    free(s->eta);
    s->chi = s->eta = NULL;
    for (int d = 0; d < 3; ++d) {
        free(s->eta_s[d]);
        s->eta_s[d] = NULL;
    }
    for (int t = 0; t < 9; ++t) {
        free(s->ep[t]);
        s->ep[t] = NULL;
    }
    if (!chi && !eta) return ORC_OK;
    if (!chi || !eta) return ORC_EINVAL;
    long n = s->n;
    for (long c = 0; c < n; ++c)
        if (!(chi[c] >= 0) || !(eta[c] >= 0) || !isfinite(chi[c]) || !isfinite(eta[c])) return ORC_EINVAL;
    s->chi = malloc(sizeof(double) * n);
    s->eta = malloc(sizeof(double) * n);
    for (int d = 0; d < 3; ++d) s->eta_s[d] = malloc(sizeof(double) * n);
    for (int t = 0; t < 9; ++t) s->ep[t] = calloc(n, sizeof(double));
    if (!s->chi || !s->eta || !s->eta_s[2] || !s->ep[8]) return ORC_ENOMEM;
    memcpy(s->chi, chi, sizeof(double) * n);
    memcpy(s->eta, eta, sizeof(double) * n);
    int nx = s->nx, ny = s->ny, nz = s->nz;
    for (int kk = 0; kk < nz; ++kk)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long c = IDX(s, i, j, kk);
                int ip = i + 1 < nx ? i + 1 : nx - 1;
                int jp = j + 1 < ny ? j + 1 : ny - 1;
                int kp = kk + 1 < nz ? kk + 1 : nz - 1;
                long q[3][4] = {
                    {c, IDX(s, ip, j, kk), IDX(s, i, jp, kk), IDX(s, ip, jp, kk)},
                    {c, IDX(s, ip, j, kk), IDX(s, i, j, kp), IDX(s, ip, j, kp)},
                    {c, IDX(s, i, jp, kk), IDX(s, i, j, kp), IDX(s, i, jp, kp)}};
                for (int p = 0; p < 3; ++p) {
                    double inv = 0;
                    int zero = 0;
                    for (int t = 0; t < 4; ++t) {
                        double m = eta[q[p][t]];
                        if (m == 0) zero = 1;
                        else inv += 1.0 / m;
                    }
                    s->eta_s[p][c] = zero ? 0.0 : 4.0 / inv;
                }
            }
    return ORC_OK;
}

int opstd_n_state(const ostate *s) { return s->chi ? 33 : 24; }

int opstd_set_source_smoothing(ostate *s, int window)
{
    if (window != 0 && window != 1) return ORC_EINVAL;
    s->smooth = window;
    return ORC_OK;
}

/* wavenumber of index m on an axis of n cells of size h */
static double kwave(int m, int n, double h)
{
    int mm = m <= n / 2 ? m : m - n;
    return 2.0 * M_PI * mm / (n * h);
}

/* Smoothed delta of every source: FFT of the delta, times the separable
 * Blackman window, inverse FFT; cells whose weight is round-off (below 1e-12)
 * are dropped. */
static int build_smoothing(ostate *s)
{
    free(s->sm_ofs);
    free(s->sm_ijk);
    free(s->sm_w);
    s->sm_ofs = NULL;
    s->sm_ijk = NULL;
    s->sm_w = NULL;
    if (!s->smooth) return ORC_OK;
    int nx = s->nx, ny = s->ny, nz = s->nz;
    long cap = 256, cnt = 0;
    s->sm_ofs = malloc(sizeof(int) * (s->n_src + 1));
    s->sm_ijk = malloc(sizeof(int) * 3 * cap);
    s->sm_w = malloc(sizeof(double) * cap);
    if (!s->sm_ofs || !s->sm_ijk || !s->sm_w) return ORC_ENOMEM;
    double *wx = malloc(sizeof(double) * nx), *wy = malloc(sizeof(double) * ny), *wz = malloc(sizeof(double) * nz);
    const int N[3] = {nx, ny, nz};
    double *W[3] = {wx, wy, wz};
    for (int d = 0; d < 3; ++d)
        for (int m = 0; m < N[d]; ++m) {
            double kh = kwave(m, N[d], s->h[d]) * s->h[d];
            W[d][m] = 0.42 + 0.5 * cos(kh) + 0.08 * cos(2.0 * kh);
        }
    for (int q = 0; q < s->n_src; ++q) {
        s->sm_ofs[q] = (int)cnt;
        const int *p = s->src + 3 * q;
        memset(s->A, 0, sizeof(double complex) * s->n);
        s->A[IDX(s, p[0], p[1], p[2])] = 1.0;
        offt_3d(s->A, nx, ny, nz, -1);
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) s->A[IDX(s, i, j, k)] *= wx[i] * wy[j] * wz[k];
        offt_3d(s->A, nx, ny, nz, +1);
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    double w = creal(s->A[IDX(s, i, j, k)]);
                    if (fabs(w) < 1e-12) continue;
                    if (cnt == cap) {
                        cap *= 2;
                        s->sm_ijk = realloc(s->sm_ijk, sizeof(int) * 3 * cap);
                        s->sm_w = realloc(s->sm_w, sizeof(double) * cap);
                        if (!s->sm_ijk || !s->sm_w) return ORC_ENOMEM;
                    }
                    s->sm_ijk[3 * cnt] = i;
                    s->sm_ijk[3 * cnt + 1] = j;
                    s->sm_ijk[3 * cnt + 2] = k;
                    s->sm_w[cnt] = w;
                    ++cnt;
                }
    }
    s->sm_ofs[s->n_src] = (int)cnt;
    free(wx);
    free(wy);
    free(wz);
    return ORC_OK;
}

int opstd_smoothed_source(ostate *s, int q, int max, int *ijk, double *w)
{
    if (!s->smooth || q < 0 || q >= s->n_src) return ORC_EINVAL;
    int n = s->sm_ofs[q + 1] - s->sm_ofs[q];
    for (int e = 0; e < n && e < max; ++e) {
        for (int a = 0; a < 3; ++a) ijk[3 * e + a] = s->sm_ijk[3 * (s->sm_ofs[q] + e) + a];
        w[e] = s->sm_w[s->sm_ofs[q] + e];
    }
    return n;
}

int opstd_set_sources(ostate *s, int n_src, const int *src_ijk, const double *m6,
                      const double *wavelet, int nt_w)
{
    for (int q = 0; q < n_src; ++q) {
        const int *p = src_ijk + 3 * q;
        if (p[0] < 0 || p[0] >= s->nx || p[1] < 0 || p[1] >= s->ny || p[2] < 0 || p[2] >= s->nz)
            return ORC_EINVAL;
    }
    if (nt_w < 0 || n_src < 0) return ORC_EINVAL;
    free(s->src);
    free(s->m6);
    free(s->wav);
    s->n_src = n_src;
    s->nt_w = nt_w;
    s->src = malloc(sizeof(int) * 3 * (n_src + 1));
    s->m6 = malloc(sizeof(double) * 6 * (n_src + 1));
    s->wav = malloc(sizeof(double) * ((long)n_src * nt_w + 1));
    if (n_src) {
        memcpy(s->src, src_ijk, sizeof(int) * 3 * n_src);
        memcpy(s->m6, m6, sizeof(double) * 6 * n_src);
        memcpy(s->wav, wavelet, sizeof(double) * (long)n_src * nt_w);
    }
    int rc = build_smoothing(s);
    if (rc != ORC_OK) return rc;
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
            memset(s->v[c][d], 0, sizeof(double) * s->n);
            memset(s->sn[c][d], 0, sizeof(double) * s->n);
        }
    for (int p = 0; p < 3; ++p) {
        memset(s->ss[p][0], 0, sizeof(double) * s->n);
        memset(s->ss[p][1], 0, sizeof(double) * s->n);
    }
    if (s->chi)
        for (int t = 0; t < 9; ++t) memset(s->ep[t], 0, sizeof(double) * s->n);
    s->step = 0;
    return ORC_OK;
}

/* wavenumbers, operator symbols and the k-space correction */
static int build_operator(ostate *s)
{
    int N[3] = {s->nx, s->ny, s->nz};
    for (int d = 0; d < 3; ++d) {
        s->k[d] = malloc(sizeof(double) * N[d]);
        s->sym[d][0] = malloc(sizeof(double complex) * N[d]);
        s->sym[d][1] = malloc(sizeof(double complex) * N[d]);
        if (!s->k[d] || !s->sym[d][0] || !s->sym[d][1]) return ORC_ENOMEM;
        for (int i = 0; i < N[d]; ++i) {
            int m = i <= N[d] / 2 ? i : i - N[d];
            double kd = 2.0 * M_PI * m / (N[d] * s->h[d]);
            s->k[d][i] = kd;
            s->sym[d][0][i] = I * kd * cexp(-I * kd * 0.5 * s->h[d]); /* D^- */
            s->sym[d][1][i] = I * kd * cexp(+I * kd * 0.5 * s->h[d]); /* D^+ */
        }
    }
    s->kappa = malloc(sizeof(double) * s->n);
    if (!s->kappa) return ORC_ENOMEM;
    for (int kk = 0; kk < s->nz; ++kk)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                double q = sqrt(s->k[0][i] * s->k[0][i] + s->k[1][j] * s->k[1][j] +
                                s->k[2][kk] * s->k[2][kk]);
                double x = 0.5 * q * s->c_ref * s->dt;
                s->kappa[IDX(s, i, j, kk)] = (s->kspace && x != 0) ? sin(x) / x : 1.0;
            }
    return ORC_OK;
}

/* Spectrum of a real field into s->A (forward 3-D FFT). */
static void forward(ostate *s, const double *f)
{
    for (long c = 0; c < s->n; ++c) s->A[c] = f[c];
    offt_3d(s->A, s->nx, s->ny, s->nz, -1);
}

/* out = Re IFFT[ i k_d exp(sign i k_d h_d/2) kappa(|k|) * A ] */
static void derivative(ostate *s, int axis, int sign, double *out)
{
    int nx = s->nx, ny = s->ny;
    const double complex *sym = s->sym[axis][sign > 0];
#pragma omp parallel for schedule(static)
    for (long c = 0; c < s->n; ++c) {
        long i = c % nx, j = (c / nx) % ny, kk = c / ((long)nx * ny);
        long m = axis == 0 ? i : (axis == 1 ? j : kk);
        s->B[c] = sym[m] * s->kappa[c] * s->A[c];
    }
    offt_3d(s->B, nx, ny, s->nz, +1);
    for (long c = 0; c < s->n; ++c) out[c] = creal(s->B[c]);
}

void opstd_deriv(int nx, int ny, int nz, double dx, double dy, double dz, const double *f,
                 int axis, int sign, int kspace, double c_ref, double dt, double *out)
{
    ostate s;
    memset(&s, 0, sizeof(s));
    s.nx = nx;
    s.ny = ny;
    s.nz = nz;
    s.n = (long)nx * ny * nz;
    s.h[0] = dx;
    s.h[1] = dy;
    s.h[2] = dz;
    s.dt = dt;
    s.kspace = kspace;
    s.c_ref = c_ref;
    build_operator(&s);
    s.A = malloc(sizeof(double complex) * s.n);
    s.B = malloc(sizeof(double complex) * s.n);
    forward(&s, f);
    derivative(&s, axis, sign, out);
    for (int d = 0; d < 3; ++d) {
        free(s.k[d]);
        free(s.sym[d][0]);
        free(s.sym[d][1]);
    }
    free(s.kappa);
    free(s.A);
    free(s.B);
}

static void sum3(const ostate *s, double *const p[3], double *out)
{
    for (long c = 0; c < s->n; ++c) out[c] = p[0][c] + p[1][c] + p[2][c];
}

static void sum2(const ostate *s, double *const p[2], double *out)
{
    for (long c = 0; c < s->n; ++c) out[c] = p[0][c] + p[1][c];
}

/* Damping factor of the split part along axis d of a field whose node is
 * half a cell up along the axes flagged in half[]: a_d times b_e of the two
 * other axes (multi-axial PML). */
static inline double afac(const ostate *s, int d, const int pos[3], const int half[3])
{
    double a = half[d] ? s->a_half[d][pos[d]] : s->a_int[d][pos[d]];
    for (int e = 0; e < 3; ++e)
        if (e != d) a *= half[e] ? s->b_half[e][pos[e]] : s->b_int[e][pos[e]];
    return a;
}

static void velocity_step(ostate *s)
{
    double *S = s->tmp[0];
    double *dv[3][3];
    /* nine derivatives of the summed stresses (eq. 2, second line) */
    dv[0][0] = s->tmp[1];
    dv[0][1] = s->tmp[2];
    dv[0][2] = s->tmp[3];
    dv[1][0] = s->tmp[4];
    dv[1][1] = s->tmp[5];
    dv[1][2] = s->tmp[6];
    dv[2][0] = s->tmp[7];
    dv[2][1] = s->tmp[8];
    dv[2][2] = NULL;
    double *dzz = malloc(sizeof(double) * s->n);
    dv[2][2] = dzz;

    sum3(s, s->sn[0], S);                 /* sxx */
    forward(s, S);
    derivative(s, 0, +1, dv[0][0]);
    sum3(s, s->sn[1], S);                 /* syy */
    forward(s, S);
    derivative(s, 1, +1, dv[1][1]);
    sum3(s, s->sn[2], S);                 /* szz */
    forward(s, S);
    derivative(s, 2, +1, dv[2][2]);
    sum2(s, s->ss[0], S);                 /* sxy */
    forward(s, S);
    derivative(s, 1, -1, dv[0][1]);
    derivative(s, 0, -1, dv[1][0]);
    sum2(s, s->ss[1], S);                 /* sxz */
    forward(s, S);
    derivative(s, 2, -1, dv[0][2]);
    derivative(s, 0, -1, dv[2][0]);
    sum2(s, s->ss[2], S);                 /* syz */
    forward(s, S);
    derivative(s, 2, -1, dv[1][2]);
    derivative(s, 1, -1, dv[2][1]);

    double dt = s->dt;
#pragma omp parallel for schedule(static)
    for (int kk = 0; kk < s->nz; ++kk)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                long c = IDX(s, i, j, kk);
                int pos[3] = {i, j, kk};
                for (int comp = 0; comp < 3; ++comp)
                    for (int d = 0; d < 3; ++d) {
                        int half[3] = {comp == 0, comp == 1, comp == 2};
                        double a = afac(s, d, pos, half);
                        double *f = s->v[comp][d];
                        f[c] = a * (a * f[c] + dt * s->rinv[comp][c] * dv[comp][d][c]);
                    }
            }
    free(dzz);
}

static void stress_step(ostate *s)
{
    double *V = s->tmp[0];
    double *e[3] = {s->tmp[1], s->tmp[2], s->tmp[3]};   /* D_d^- v_d */
    /* shear strain-rate pieces: g[p][0], g[p][1] for the two split parts of
     * pair p (xy: parts x,y; xz: parts x,z; yz: parts y,z) */
    double *g[3][2] = {{s->tmp[4], s->tmp[5]}, {s->tmp[6], s->tmp[7]}, {s->tmp[8], NULL}};
    double *g21 = malloc(sizeof(double) * s->n);
    g[2][1] = g21;

    sum3(s, s->v[0], V);                  /* vx */
    forward(s, V);
    derivative(s, 0, -1, e[0]);
    derivative(s, 1, +1, g[0][1]);        /* D_y^+ vx -> sxy part y */
    derivative(s, 2, +1, g[1][1]);        /* D_z^+ vx -> sxz part z */
    sum3(s, s->v[1], V);                  /* vy */
    forward(s, V);
    derivative(s, 1, -1, e[1]);
    derivative(s, 0, +1, g[0][0]);        /* D_x^+ vy -> sxy part x */
    derivative(s, 2, +1, g[2][1]);        /* D_z^+ vy -> syz part z */
    sum3(s, s->v[2], V);                  /* vz */
    forward(s, V);
    derivative(s, 2, -1, e[2]);
    derivative(s, 0, +1, g[1][0]);        /* D_x^+ vz -> sxz part x */
    derivative(s, 1, +1, g[2][0]);        /* D_y^+ vz -> syz part y */

    static const int pair_axes[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    double dt = s->dt;
#pragma omp parallel for schedule(static)
    for (int kk = 0; kk < s->nz; ++kk)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                long c = IDX(s, i, j, kk);
                int pos[3] = {i, j, kk};
                double lam = s->lam[c], mu = s->mu[c];
                static const int centre[3] = {0, 0, 0};
                for (int comp = 0; comp < 3; ++comp)
                    for (int d = 0; d < 3; ++d) {
                        double a = afac(s, d, pos, centre);
                        double coef = lam + (comp == d ? 2.0 * mu : 0.0);
                        double *f = s->sn[comp][d];
                        double rhs = dt * coef * e[d][c];
                        if (s->chi) {
                            /* chi delta_ij d/dt(dv_k/dx_k) + 2 eta d/dt(dv_i/dx_i):
                             * backward difference of the derivative over the step */
                            double vcoef = s->chi[c] + (comp == d ? 2.0 * s->eta[c] : 0.0);
                            rhs += vcoef * (e[d][c] - s->ep[d][c]);
                        }
                        f[c] = a * (a * f[c] + rhs);
                    }
                for (int p = 0; p < 3; ++p)
                    for (int t = 0; t < 2; ++t) {
                        int d = pair_axes[p][t];
                        int half[3] = {0, 0, 0};
                        half[pair_axes[p][0]] = 1;
                        half[pair_axes[p][1]] = 1;
                        double a = afac(s, d, pos, half);
                        double *f = s->ss[p][t];
                        double rhs = dt * s->mu_s[p][c] * g[p][t][c];
                        if (s->chi) rhs += s->eta_s[p][c] * (g[p][t][c] - s->ep[3 + 2 * p + t][c]);
                        f[c] = a * (a * f[c] + rhs);
                    }
            }
    if (s->chi) {
        for (int d = 0; d < 3; ++d) memcpy(s->ep[d], e[d], sizeof(double) * s->n);
        for (int p = 0; p < 3; ++p)
            for (int t = 0; t < 2; ++t) memcpy(s->ep[3 + 2 * p + t], g[p][t], sizeof(double) * s->n);
    }
    free(g21);
}

/* point source of moment weight * M at cell p */
static void inject_point(ostate *s, const int *p, const double *m, double weight, double w)
{
    double dv = s->h[0] * s->h[1] * s->h[2];
    int nx = s->nx, ny = s->ny, nz = s->nz;
    static const int pair_axes[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    long c = IDX(s, p[0], p[1], p[2]);
    for (int comp = 0; comp < 3; ++comp) {
        double val = -s->dt * w * weight * m[comp] / dv;
        for (int d = 0; d < 3; ++d) s->sn[comp][d][c] += val / 3.0;
    }
    /* shear pair p sits half a cell up along both of its axes: the four
     * nodes around the centre are offsets {-1, 0} along those two axes */
    for (int pr = 0; pr < 3; ++pr) {
        double val = -s->dt * w * weight * m[3 + pr] / dv;
        int a0 = pair_axes[pr][0], a1 = pair_axes[pr][1];
        for (int o0 = -1; o0 <= 0; ++o0)
            for (int o1 = -1; o1 <= 0; ++o1) {
                int ix[3] = {p[0], p[1], p[2]};
                int N[3] = {nx, ny, nz};
                ix[a0] = (ix[a0] + o0 + N[a0]) % N[a0];
                ix[a1] = (ix[a1] + o1 + N[a1]) % N[a1];
                long cc = IDX(s, ix[0], ix[1], ix[2]);
                s->ss[pr][0][cc] += val / 8.0;
                s->ss[pr][1][cc] += val / 8.0;
            }
    }
}

static void inject(ostate *s)
{
    if (s->step >= s->nt_w) return;
    for (int q = 0; q < s->n_src; ++q) {
        const double *m = s->m6 + 6 * q;
        double w = s->wav[(long)q * s->nt_w + s->step];
        if (!s->smooth) {
            inject_point(s, s->src + 3 * q, m, 1.0, w);
        } else {
            for (int e = s->sm_ofs[q]; e < s->sm_ofs[q + 1]; ++e) inject_point(s, s->sm_ijk + 3 * e, m, s->sm_w[e], w);
        }
    }
}

int opstd_run(ostate *s, int nt, double *traces)
{
    int nr = s->n_rec;
    for (int n = 0; n < nt; ++n) {
        velocity_step(s);
        for (int r = 0; r < nr; ++r) {
            const int *q = s->rec + 3 * r;
            long c = IDX(s, q[0], q[1], q[2]);
            for (int comp = 0; comp < 3; ++comp) {
                double v = s->v[comp][0][c] + s->v[comp][1][c] + s->v[comp][2][c];
                traces[((long)(1 + comp) * nr + r) * nt + n] = v;
            }
        }
        stress_step(s);
        inject(s);
        for (int r = 0; r < nr; ++r) {
            const int *q = s->rec + 3 * r;
            long c = IDX(s, q[0], q[1], q[2]);
            double tr = 0;
            for (int comp = 0; comp < 3; ++comp)
                tr += s->sn[comp][0][c] + s->sn[comp][1][c] + s->sn[comp][2][c];
            traces[(long)r * nt + n] = -tr / 3.0;
        }
        s->step++;
        /* instability guard: a non-finite value anywhere ends the run */
        if ((n & 63) == 63 || n == nt - 1) {
            for (long c = 0; c < s->n; ++c)
                if (!isfinite(s->v[0][0][c]) || !isfinite(s->sn[0][0][c])) return ORC_EUNSTABLE;
        }
    }
    return ORC_OK;
}

/* state order: v[c][d] (9), sn[c][d] (9), ss xy(x,y) xz(x,z) yz(y,z) (6), and
 * with viscosity the nine previous velocity derivatives (9) */
void opstd_get_state(const ostate *s, double *fields)
{
    long n = s->n;
    int f = 0;
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) memcpy(fields + n * f++, s->v[c][d], sizeof(double) * n);
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) memcpy(fields + n * f++, s->sn[c][d], sizeof(double) * n);
    for (int p = 0; p < 3; ++p)
        for (int t = 0; t < 2; ++t) memcpy(fields + n * f++, s->ss[p][t], sizeof(double) * n);
    if (s->chi)
        for (int t = 0; t < 9; ++t) memcpy(fields + n * f++, s->ep[t], sizeof(double) * n);
}

void opstd_set_state(ostate *s, const double *fields)
{
    long n = s->n;
    int f = 0;
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) memcpy(s->v[c][d], fields + n * f++, sizeof(double) * n);
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) memcpy(s->sn[c][d], fields + n * f++, sizeof(double) * n);
    for (int p = 0; p < 3; ++p)
        for (int t = 0; t < 2; ++t) memcpy(s->ss[p][t], fields + n * f++, sizeof(double) * n);
    if (s->chi)
        for (int t = 0; t < 9; ++t) memcpy(s->ep[t], fields + n * f++, sizeof(double) * n);
}
