/*
 * FP64 CPU oracle for the pseudo-spectral elastic solver, the trace
 * superposition and their pieces.  TEST INFRASTRUCTURE ONLY: it is called by
 * the tests, by the bench's CPU-baseline leg and by the smoke check, never by
 * the product path, and it shares no code with the GPU library.
 */
#ifndef PSTD_ORACLE_H
#define PSTD_ORACLE_H

#include <complex.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EUNSTABLE (-4)

/* FFT (offt.c) */
void offt_roots(int n, int sign, double complex *w);
void offt_strided(double complex *x, long stride, int n, int sign, const double complex *w,
                  double complex *work);
void offt_1d(double complex *x, int n, int sign);
void offt_3d(double complex *a, int nx, int ny, int nz, int sign);

/* solver (opstd.c) */
typedef struct ostate ostate;

ostate *opstd_create(int nx, int ny, int nz, const double *vp, const double *vs,
                     const double *rho, double dx, double dy, double dz, double dt, int pml_n,
                     double pml_A, double pml_p, int kspace, double c_ref, int n_rec,
                     const int *rec_ijk, int *err);
int opstd_set_sources(ostate *s, int n_src, const int *src_ijk, const double *m6,
                      const double *wavelet, int nt_w);
int opstd_run(ostate *s, int nt, double *traces);
/* Kelvin-Voigt viscosity chi, eta per cell (NULL, NULL: lossless); clears the state. */
int opstd_set_viscosity(ostate *s, const double *chi, const double *eta);
/* Fields in opstd_get_state / opstd_set_state: 24, or 33 with viscosity. */
int opstd_n_state(const ostate *s);
/* Source smoothing for the next opstd_set_sources: 0 off, 1 Blackman window in k-space. */
int opstd_set_source_smoothing(ostate *s, int window);
/* Cells (ijk, up to max) and weights of source q's smoothed delta; returns the count. */
int opstd_smoothed_source(ostate *s, int q, int max, int *ijk, double *w);
void opstd_get_state(const ostate *s, double *fields);
void opstd_set_state(ostate *s, const double *fields);
long opstd_step_index(const ostate *s);
int oracle_threads(void);
void opstd_set_step(ostate *s, long step);
void opstd_destroy(ostate *s);
void opstd_deriv(int nx, int ny, int nz, double dx, double dy, double dz, const double *f,
                 int axis, int sign, int kspace, double c_ref, double dt, double *out);

/* superposition (ocombine.c) */
int ocombine(const float *tr, int n_src, int n_rec, int nt_in, double dt_in, const double *t0,
             int n_ev, const int *src_idx, const double *amp, const double *t_origin, int nt_out,
             double dt_out, double *out);

#endif
