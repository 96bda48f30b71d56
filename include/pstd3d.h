/*
 * pstd3d — MI355X (gfx950) Fourier pseudo-spectral elastic wave solver and
 * trace superposition.  Plain C ABI: host or device pointers and sizes only.
 *
 * Physics (arXiv 1705.04874, Das, Chen & Hobson):
 *  - 3-D elastic first-order stress-velocity system (eq. 1-2, Sec. II-A),
 *    lossless by default, with optional Kelvin-Voigt viscosities chi, eta;
 *    Lame parameters from cp, cs, rho (eq. 4), hydrophone pressure
 *    p = -(sxx + syy + szz)/3 (eq. 3);
 *  - Fourier pseudo-spectral spatial derivatives, leapfrog time stepping on a
 *    grid staggered in space and time (Sec. II-A), with a k-space correction
 *    kappa = sinc(c_ref |k| dt / 2) on the derivative operator;
 *  - a split-field perfectly matched layer of `thickness` cells on all six
 *    faces (Sec. II-B), CFL number of eq. 5;
 *  - point sources given by a symmetric moment tensor (eq. 6-7) with a
 *    moment-rate wavelet; four-component seabed receivers (Sec. II-B);
 *  - superposition of single-event traces with amplitudes and origin times
 *    (Sec. IV, Cases 1-3).
 *
 * Conventions.
 *  - Arrays over the grid are [nz][ny][nx], x fastest, z = 0 at the top.
 *  - Moment tensors are 6 doubles (xx, yy, zz, xy, xz, yz) in N*m.
 *  - Traces are float [n_shots][4][n_rec][nt], components (p, vx, vy, vz).
 *    p of step n is sampled at time (n+1) dt at the cell centre; v of step n
 *    at (n+1/2) dt at the component's staggered node (vx at (i+1/2, j, k) ...).
 *  - Host inputs are copied during the call; device buffers passed in remain
 *    owned by the caller.  A context owns its tables and state (device memory
 *    allocated with hipMalloc) and is used from one stream at a time.
 *  - Every call returns PSTD_OK (0) or a negative error code; the message of
 *    the last error on the calling thread is returned by pstd3d_last_error().
 *    No C++ exception crosses the ABI.
 */
#ifndef PSTD3D_H
#define PSTD3D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSTD_OK 0
#define PSTD_EINVAL (-1)        /* bad argument or model value */
#define PSTD_ENOMEM (-2)        /* device allocation failed */
#define PSTD_EDEVICE (-3)       /* HIP runtime error */
#define PSTD_EUNSTABLE (-4)     /* CFL condition violated, or non-finite field */
#define PSTD_EUNSUPPORTED (-5)  /* grid length with a factor other than 2, 3, 5 or not built */

typedef struct pstd3d_ctx pstd3d_ctx;

/* Velocity model and receivers (Sec. II-B).  vp, vs (m/s) and rho (kg/m^3)
 * are host arrays [nz][ny][nx]; rec_ijk is a host array [n_rec][3] of cell
 * indices (i, j, k).  kspace: 1 applies the k-space correction (default), 0
 * gives the plain pseudo-spectral operator.  c_ref <= 0 selects max(vp); it
 * sets both the k-space correction and the PML profile. */
typedef struct {
    int nx, ny, nz;
    const double *vp, *vs, *rho;
    int n_rec;
    const int32_t *rec_ijk;
    int kspace;
    double c_ref;
} pstd3d_model;

/* Split-field PML (Sec. II-B): `thickness` cells inside the grid on each
 * face, absorption alpha_d = (A c_ref / h_d) (depth / thickness)^4 with A in
 * nepers per cell (2 is a good default).  mratio = p >= 0 makes it
 * multi-axial: the split part along axis d is damped by alpha_d + p times the
 * profiles of the two other axes (p = 0: the classical split PML). */
typedef struct {
    int thickness;
    double A;
    double mratio;
} pstd3d_pml;

/* Create a solver for one model.  d = (dx, dy, dz) metres, dt seconds.
 * Validates the model (finite, vp > 0, rho > 0, vs >= 0, positive bulk
 * modulus), the receivers (inside the grid), the grid lengths (2, 3, 5
 * factors, built lengths) and stability: with kspace = 0 it requires
 * c_max dt sqrt(sum 1/h^2) <= 2/pi (eq. 5 in 3-D for the leapfrog scheme);
 * with kspace = 1 and c_ref >= c_max any dt is stable.  The current HIP
 * device is the context's device.  On success *out holds the context. */
int pstd3d_create(const pstd3d_model *m, const double d[3], double dt, const pstd3d_pml *pml,
                  pstd3d_ctx **out);

/* Define the shots and reset every shot's state to zero at step 0.
 * Shot s owns the point sources [shot_ofs[s], shot_ofs[s+1]) (host int32
 * [n_shots+1]); source q has cell src_ijk[3q..3q+3), moment tensor
 * m6[6q..6q+6) and wavelet row wavelet[q*nt_w .. (q+1)*nt_w) (host doubles,
 * moment rate in 1/s, sample n applied during step n, zero beyond nt_w).
 * In step n each stress component c,d of the source cell receives
 * -dt * w[n] * M_cd / (dx dy dz), split equally over its split parts; shear
 * components go 1/4 to each of the four shear nodes around the cell centre
 * (eq. 6-7; Sec. II-A point sources).  The shots' state is allocated here
 * (hipMalloc), or placed in the workspace given to pstd3d_set_workspace; the
 * first call of a context also times the launch-shape candidates (see
 * pstd3d_set_tuning). */
int pstd3d_set_sources(pstd3d_ctx *c, int n_shots, const int32_t *shot_ofs, const int32_t *src_ijk,
                       const double *m6, const double *wavelet, int nt_w);

/* Source smoothing for the following pstd3d_set_sources calls (Sec. II-A: the
 * point source's delta is smoothed with a Blackman window in the
 * spatial-frequency domain to limit the oscillations a discrete delta causes
 * with Fourier derivatives).  PSTD_SMOOTH_BLACKMAN applies on every axis the
 * window W(k) = 0.42 + 0.5 cos(k h) + 0.08 cos(2 k h) over [-pi/h, pi/h]
 * (zero at the edges, W(0) = 1 so the moment is kept); in space it is the
 * separable stencil (0.04, 0.25, 0.42, 0.25, 0.04) around the source cell,
 * periodic at the grid edges: 125 point sources of weights summing to 1. */
#define PSTD_SMOOTH_NONE 0
#define PSTD_SMOOTH_BLACKMAN 1
int pstd3d_set_source_smoothing(pstd3d_ctx *c, int window);

/* Kelvin-Voigt viscosity (eq. 1-2): the stress rate gains
 * chi delta_ij d/dt(div v) + eta d/dt(dv_i/dx_j + dv_j/dx_i).  chi, eta (Pa s)
 * are host arrays [nz][ny][nx], finite and >= 0; eta at a shear node is the
 * harmonic mean of the four surrounding cells (0 if any is 0), as for mu.
 * Each time derivative is taken as the change of the velocity derivative over
 * one step (backward difference), so every shot carries the nine derivatives
 * of its previous step as 9 more state fields (33 in all); they start at zero.
 * NULL for both restores the lossless medium.  The explicit viscous term is
 * stable only while dt (pi/h)^2 (chi + 2 eta) / rho stays well below 1 on the
 * finest axis; this call does not check it (a run that blows up returns
 * PSTD_EUNSTABLE).  Clears the shots: call pstd3d_set_sources again (which
 * retunes the stress kernel for the viscous variant). */
int pstd3d_set_viscosity(pstd3d_ctx *c, const double *chi, const double *eta);

/* State fields per shot: 24 (lossless) or 33 (viscous). */
int pstd3d_state_fields(const pstd3d_ctx *c);

/* Advance every shot by nt steps on `hip_stream` (a hipStream_t, may be
 * NULL for the null stream) and write the receiver traces of those steps to
 * the caller-owned device buffer traces_dev [n_shots][4][n_rec][nt].
 * Stateful: a second call continues where the first stopped.  Returns
 * PSTD_EUNSTABLE if a non-finite value reached the receivers. */
int pstd3d_run(pstd3d_ctx *c, int nt, float *traces_dev, void *hip_stream);

/* Advance several contexts (uneven grids allowed) by nt steps as one HIP
 * graph per step: the per-context step sequences are captured on forked
 * streams so the graph runs them concurrently; traces[i] is context i's
 * device trace buffer.  All contexts must live on the current device. */
int pstd3d_run_many(pstd3d_ctx *const *ctxs, int n, int nt, float *const *traces, void *hip_stream);

/* Checkpoint: copy shot `shot`'s state (float, host [F][nz][ny][nx] with
 * F = pstd3d_state_fields: the 24 split fields in the order vx(x,y,z)
 * vy(x,y,z) vz(x,y,z) sxx(x,y,z) syy(x,y,z) szz(x,y,z) sxy(x,y) sxz(x,z)
 * syz(y,z), then with viscosity the previous step's D-x vx, D-y vy, D-z vz,
 * Dx+ vy, Dy+ vx, Dx+ vz, Dz+ vx, Dy+ vz, Dz+ vy) to host memory.
 * The split into parts only matters where the absorbing layer damps (Sec.
 * II-B): in the undamped cells (pstd3d_undamped_range) each field's whole
 * value sits in its first part and the other parts are zero. */
int pstd3d_get_state(pstd3d_ctx *c, int shot, float *fields_host);
/* Restore shot `shot`'s split fields from host memory and set the step index
 * of the context (the wavelet sample used by the next step).  In the
 * undamped cells the parts of each field are summed into its first part
 * (in a host copy of the state: PSTD_ENOMEM if that allocation fails). */
int pstd3d_set_state(pstd3d_ctx *c, int shot, const float *fields_host, long step);
/* Step index of the next step. */
long pstd3d_step(const pstd3d_ctx *c);
/* The undamped cells: those with lo[d] <= index <= hi[d] on every axis d
 * (x, y, z), where every absorbing-layer factor of the split update is
 * exactly 1 (hi[d] < lo[d]: none).  The update kernels read and write only
 * the first split part of each field there.  PSTD_EINVAL for NULL. */
int pstd3d_undamped_range(const pstd3d_ctx *c, int lo[3], int hi[3]);

/* Debug / test entry: the nine staggered spectral derivatives of one phase,
 * computed with the same kernels as a time step.  phase 0: in = 6 device
 * fields (sxx, syy, szz, sxy, sxz, syz) -> out = 9 device fields
 * (Dx+ sxx, Dy- sxy, Dz- sxz, Dx- sxy, Dy+ syy, Dz- syz, Dx- sxz, Dy- syz, Dz+ szz);
 * phase 1: in = 3 fields (vx, vy, vz) -> out = 9 fields
 * (Dx- vx, Dy- vy, Dz- vz, Dy+ vx, Dx+ vy, Dz+ vx, Dx+ vz, Dz+ vy, Dy+ vz).
 * D_d^{+-} f = IFFT[i k_d exp(+-i k_d h_d/2) kappa FFT f].  Uses shot 0's
 * scratch; the shot's state is kept. */
int pstd3d_derivs(pstd3d_ctx *c, int phase, const float *in_dev, float *out_dev, void *hip_stream);

/* Zero every shot's state and set the step index to 0 (the sources set by
 * pstd3d_set_sources are kept), enqueued on hip_stream. */
int pstd3d_reset(pstd3d_ctx *c, void *hip_stream);

/* Per-kernel timing with HIP events recorded around every launch of
 * pstd3d_run (off by default).  Kinds: */
#define PSTD_K_YFWD_S 0   /* y FFT of the 6 stress spectra */
#define PSTD_K_ZOP_V 1    /* z FFT, 9 derivative symbols, inverse z FFT (V phase) */
#define PSTD_K_YINV_V 2   /* inverse y FFT of the 9 stress derivatives */
#define PSTD_K_VEL 3      /* inverse x FFT + velocity update + receivers + x FFT of v */
#define PSTD_K_YFWD_V 4   /* y FFT of the 3 velocity spectra */
#define PSTD_K_ZOP_S 5    /* z operator of the S phase */
#define PSTD_K_YINV_S 6   /* inverse y FFT of the 9 velocity derivatives */
#define PSTD_K_STR 7      /* inverse x FFT + stress update + sources + receivers + x FFT */
#define PSTD_K_COUNT 8
/* enable != 0 turns timing on and clears the accumulators. */
int pstd3d_profile(pstd3d_ctx *c, int enable);
/* Accumulated milliseconds and launch count of one kernel kind since the
 * last pstd3d_profile(c, 1). */
int pstd3d_profile_read(const pstd3d_ctx *c, int kind, double *total_ms, long *launches);

/* Autotuner.  Six launch-shape knobs of a time step:
 *   PSTD_TUNE_Y, PSTD_TUNE_Z  the y and z transforms work on tiles of this
 *        many adjacent pencils (8, 16, 32 or 64, where the tile fits the LDS
 *        and register budget of its length; y tiles of 8 only where 16 does
 *        not fit);
 *   PSTD_TUNE_VEL, PSTD_TUNE_STR  threads per block of the velocity and the
 *        stress update kernels (x transforms fused with the split-PML
 *        updates): 128, 256 or 512, at most the cells of a block;
 *   PSTD_TUNE_ZT  threads per block of the z kernels: 256, or 512 where the
 *        tile gives each of 512 threads a butterfly of a radix-8 (or 16) first
 *        pass (half the registers per thread, so twice the waves in flight);
 *   PSTD_TUNE_ZF  input spectra per z block: 1, or 6 (every input of the
 *        phase in one block, which then reads its tile's kappa and symbols
 *        once for all of them).
 * The first pstd3d_set_sources of a context times every built value of every
 * knob on the context's own state (HIP events, one warm-up and three
 * launches each; the z knobs one after another, each with the ones before
 * at their choice) and keeps the fastest; the state is cleared afterwards.
 * pstd3d_set_tuning forces values (host int[PSTD_TUNE_COUNT]; a value must be
 * built, PSTD_EUNSUPPORTED otherwise, also for a z tile and z thread count
 * that are not built together); forced values take effect at once, and a 0
 * entry is tuned again at the next pstd3d_set_sources.  The traces agree
 * across values to FP32 rounding (the same butterflies and updates, possibly
 * contracted into fused multiply-adds differently, and radix-8 instead of
 * radix-16 passes in the 512-thread z kernels). */
#define PSTD_TUNE_Y 0
#define PSTD_TUNE_Z 1
#define PSTD_TUNE_VEL 2
#define PSTD_TUNE_STR 3
#define PSTD_TUNE_ZT 4
#define PSTD_TUNE_ZF 5
#define PSTD_TUNE_COUNT 6
int pstd3d_set_tuning(pstd3d_ctx *c, const int value[PSTD_TUNE_COUNT]);
/* The chosen value of `knob` (may be NULL), and its built values (host,
 * up to max entries) with the microseconds per launch measured by the last
 * tuning (0 where not measured).  Returns the number of built values or a
 * negative error code. */
int pstd3d_get_tuning(const pstd3d_ctx *c, int knob, int *chosen, int *values, float *us, int max);

/* Receivers of the context (the n_rec of its model), or PSTD_EINVAL for NULL. */
int pstd3d_n_rec(const pstd3d_ctx *c);

/* Bytes of device memory held by the context (not counting a workspace). */
long pstd3d_device_bytes(const pstd3d_ctx *c);

/* Caller-provided device memory for the shots' state (the split fields and
 * the spectra: the bulk of a context's memory, about 200 bytes per cell and
 * shot), for callers that manage their own device memory pool.
 * pstd3d_workspace_size: bytes n_shots shots need (with the current viscosity
 * setting), or a negative error code.  pstd3d_set_workspace: from the next
 * pstd3d_set_sources on, the shots' state lives in dev_ptr (device memory of
 * the context's device, 256-byte aligned, `bytes` long); that call fails with
 * PSTD_EINVAL if the shots need more.  NULL returns to memory the context
 * allocates itself.  The call clears the shots (call pstd3d_set_sources
 * again).  The memory stays the caller's: the context never frees it, and the
 * caller keeps it allocated and leaves it alone while the context uses it (up
 * to pstd3d_destroy, or a later pstd3d_set_workspace).  The source tables
 * (a few bytes per source) are still allocated by the context. */
long pstd3d_workspace_size(const pstd3d_ctx *c, int n_shots);
int pstd3d_set_workspace(pstd3d_ctx *c, void *dev_ptr, long bytes);
void pstd3d_destroy(pstd3d_ctx *c);
const char *pstd3d_last_error(void);

/* Superposition of single-event traces (Sec. IV; Case 2's shift-and-add with
 * real-valued shifts):
 *   out[c][r][m] = sum_e amp[e] * x_e(m dt_out - t_origin[e] - t0[c]),
 * x_e(t) the linear interpolation of tr[src_idx[e]][c][r][.] at t / dt_in,
 * zero outside [0, nt_in - 1].  Each output sample is accumulated in double
 * over its events grouped by source (sources ascending, event order within a
 * source) and rounded once to float.
 * tr: device float [n_src][4][n_rec][nt_in]; out: device float
 * [4][n_rec][nt_out]; t0: host double[4] (time of sample 0 per component);
 * src_idx, amp, t_origin: host arrays [n_ev].  The event lists (128 bytes per
 * event and record segment of up to 6144 samples for traces of up to 2044
 * samples, 88 for longer ones) go to a device buffer
 * allocated and freed by the call; runs on hip_stream and returns after the
 * stream has finished.  Errors: PSTD_EINVAL (sizes, nt_in above 2^30,
 * dt_out / dt_in outside [2^-20, 2^20], source index out of range,
 * non-finite value, more than 2^23
 * record segments in one call: 4 n_rec rounded up to a multiple of 8, times
 * ceil(nt_out / 6144)), PSTD_ENOMEM,
 * PSTD_EDEVICE; the message is returned by seis_combine_last_error(). */
int seis_combine(const float *tr, int n_src, int n_rec, int nt_in, double dt_in, const double t0[4],
                 int n_ev, const int32_t *src_idx, const double *amp, const double *t_origin,
                 int nt_out, double dt_out, float *out, void *hip_stream);
/* Message of the last seis_combine error on the calling thread. */
const char *seis_combine_last_error(void);

/* seis_combine for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results, but the event lists go to a
 * static device array of seis_combine_noalloc_max_bytes() bytes (4 MiB) that
 * the library holds on each device it runs on until the process ends; the
 * call makes no device allocation.  It needs 128 bytes per (event, record
 * segment of up to 6144 samples; 88 for traces longer than 2044 samples) plus
 * 16 per (source, segment) and a few hundred bytes: about 32 000
 * event-segments.  Larger event lists return
 * PSTD_EINVAL before any device work (use seis_combine).  Every call on one
 * device shares its array, so calls that overlap on one device (on other
 * streams or threads) race; each call returns after its stream has finished.
 * The other outputs and errors are those of seis_combine. */
int seis_combine_noalloc(const float *tr, int n_src, int n_rec, int nt_in, double dt_in, const double t0[4],
                         int n_ev, const int32_t *src_idx, const double *amp, const double *t_origin,
                         int nt_out, double dt_out, float *out, void *hip_stream);
long seis_combine_noalloc_max_bytes(void);

#ifdef __cplusplus
}
#endif
#endif
