/*
 * sno — spectral neural operator surrogate of the seismogram simulation, on
 * MI355X (gfx950).  Plain C ABI: host or device pointers and sizes only.
 *
 * The paper names a learned proxy of the forward simulation as future work
 * (Sec. VII).  The surrogate maps a point source (position and moment tensor,
 * 9 numbers) to four-component receiver traces on a line of receivers, with a
 * Fourier neural operator along time.  The elastic system is linear in its
 * source (eq. 2; Sec. IV's superposition rests on it), so the traces are a
 * combination of six responses weighted by the moment-tensor components, and
 * the network sees only the position:
 *   lift      V0 = P A + pb,  A = [p; t/T; cos, sin(2 pi c_f t/T) per Fourier
 *             feature frequency c_f]   (p: 3 normalised position features)
 *   layer l   Z = W_l V + b_l + IDFT_K( R_l[k] DFT_K(V)[k] ),  V = gelu(Z)
 *             (no activation after the last layer; K retained modes; complex
 *              C x C weights per mode)
 *   project   Y6 = Q2 gelu(Q1 V + q1b) + q2b           (6 O rows, O = 4 n_rec)
 *   output    Y[o] = sum_j m_j Y6[j O + o],  m_j = M_j / feat_scale[3 + j]
 * Every contraction runs on BF16 MFMA with FP32 accumulation; master weights,
 * gradients and Adam moments are FP32.  The projection's six responses are
 * weighted by the moment features before the product (one product per sample
 * instead of six), so the output is linear in the moment tensor to BF16
 * rounding.  Training minimises the mean squared
 * error of traces normalised per component by their training-set RMS.  An
 * error head predicts each sample's relative L2 error from the pooled last
 * hidden layer and the moment features; predictions whose estimate exceeds a tolerance are recomputed
 * by the pseudo-spectral solver (pstd3d), which stays the reference for accuracy.
 *
 * Layout: features X [n][9] (x, y, z cell indices, moment tensor xx yy zz xy xz
 * yz in N*m), traces Y [n][4][n_rec][T] (components p, vx, vy, vz).  Errors:
 * the PSTD_* codes of pstd3d.h.
 */
#ifndef SNO_H
#define SNO_H

#include <stdint.h>

#include "pstd3d.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sno sno;

typedef struct {
    int n_rec;          /* receivers on the line (O = 4 n_rec outputs) */
    int T;              /* time samples (power of two up to 4096) */
    int C;              /* width (multiple of 16) */
    int K;              /* retained Fourier modes (<= T/2) */
    int L;              /* Fourier layers */
    int H;              /* projection hidden width (multiple of 16) */
    double feat_off[9]; /* feature f = (x - off) / scale; off must be 0 for the 6
                           moment components (the output is linear in them) */
    double feat_scale[9];
    int n_four;         /* Fourier time features (0 .. SNO_MAX_FOUR) */
    double four_cycles[64]; /* their frequencies, cycles per window of T samples */
    int pos_mod;        /* 1: also each position feature times each cos and sin
                           feature (6 n_four more lift channels), so that a source
                           shift can move the phase of the time features; 0: off */
    /* Travel-time-aligned output (frames = 2): the projection gives two sets
     * of 6 O rows, a P frame and an S frame; row o of frame f is delayed by
     * (tau_f(source, receiver r(o)) - t_ref[f]) / dt samples before the frames
     * are summed, with tau_f the first-arrival time of the two-point ray
     * between the two cell centres through a medium whose slowness depends on
     * depth only (Snell's law across the cell layers: half a cell at each end,
     * whole cells between; a path within one layer, a vertical path or one
     * crossing a zero slowness takes the straight segment) and the fractional
     * delay evaluated by 4-point Lagrange (cubic) interpolation, zero outside
     * the window.  The direct arrivals then sit at fixed frame times for every
     * source.  frames = 1: no delay (the fields below are ignored). */
    int frames;
    const int32_t *rec_ijk;  /* host [n_rec][3] receiver cells (copied by sno_create) */
    int nz_slow;             /* depth cells of the profiles (source and receiver depths below it) */
    const double *slow_p;    /* host [nz_slow] P slowness per depth cell, s/m (copied) */
    const double *slow_s;    /* host [nz_slow] S slowness per depth cell, s/m (copied) */
    double h[3];             /* cell size (m) along x, y, z */
    double dt;               /* sample interval of the traces (s) */
    double t_ref[2];         /* reference time of the P and S frames (s) */
} sno_cfg;
#define SNO_MAX_FOUR 64  /* size of four_cycles */

typedef struct {
    int epochs;
    int batch;
    double lr;          /* peak learning rate, cosine decay to 0 */
    uint64_t seed;      /* shuffling (std::mt19937_64) */
    int n_calib;        /* last n_calib samples fit the error head, not the weights */
    /* optional (may be NULL): called on the calling thread after every epoch
     * with the epoch index and its mean training loss */
    void (*on_epoch)(int epoch, float loss, void *user);
    void *user;
    /* 0: the loss is the mean squared error of the per-component normalised
     * outputs; 1: each (sample, component) term is divided by that target's
     * mean square, so the loss is the mean squared relative L2 error over
     * samples and components (the measure the error head predicts) and a
     * weak seismogram counts as much as a strong one */
    int rel_loss;
} sno_train_cfg;

/* Create a model; params (host float, sno_n_params values, order P [C][NA]
 * with NA = 4 + 2 n_four (+ 6 n_four with pos_mod), pb [C], {W_l [C][C], b_l [C], Rr_l, Ri_l [K][C][C]}_l, Q1 [H][C],
 * q1b [H], Q2 [frames 6 O][H], q2b [frames 6 O]) are the initial weights; the
 * rows of Q2 are ordered (frame, moment component, output). */
int sno_create(const sno_cfg *cfg, const float *params, sno **out);
long sno_n_params(const sno_cfg *cfg);
void sno_destroy(sno *s);

/* Train on n device samples (X [n][9] float, Y [n][4][n_rec][T] float), then
 * fit the error head on the last n_calib samples.  loss_curve (host, may be
 * NULL) receives the mean training loss of each epoch. */
int sno_train(sno *s, const float *X, const float *Y, int n, const sno_train_cfg *cfg, float *loss_curve,
              void *hip_stream);

/* Predict n samples: Y [n][4][n_rec][T] device, est_err [n] device (the error
 * head's estimate of the relative L2 error; NaN-free). */
int sno_predict(sno *s, const float *X, int n, float *Y, float *est_err, void *hip_stream);

/* Predict, then recompute with the solver every sample whose estimated error
 * exceeds tol.  The solver context must have the surrogate's receivers, in
 * the same order (PSTD_EINVAL before any device work if its receiver count,
 * pstd3d_n_rec, differs from cfg.n_rec); sample i is a single point source at src_ijk[3i..] with
 * moment tensor m6[6i..] (host) and wavelet (host, nt_w samples, shared);
 * the solver runs decim * T steps and every decim-th sample is kept.  used
 * (host, n, may be NULL) returns 1 where the solver answered.  Solver calls go
 * in batches of at most max_batch shots. */
int sno_predict_or_solve(sno *s, pstd3d_ctx *solver, const float *X, const int32_t *src_ijk, const double *m6,
                         const double *wavelet, int nt_w, int decim, int n, double tol, int max_batch, float *Y,
                         float *est_err, int *used, void *hip_stream);

/* Test entries: forward of n samples with the current weights (Y device), and
 * the gradient of the mean squared error against targets Yt (device, already
 * normalised) into grad (device, sno_n_params floats). */
int sno_forward(sno *s, const float *X, int n, float *Y, void *hip_stream);
int sno_gradient(sno *s, const float *X, const float *Yt, int n, float *grad, float *loss, void *hip_stream);
/* The same with per-(sample, component) weights w (device float [n][4], NULL:
 * all 1): the loss is the mean over all outputs of w (Y - Yt)^2. */
int sno_gradient_weighted(sno *s, const float *X, const float *Yt, const float *w, int n, float *grad, float *loss,
                          void *hip_stream);
/* Copy the current FP32 weights to host memory. */
int sno_get_params(const sno *s, float *params);
/* Test entries of the optimiser: one Adam step of the weights with the device
 * gradient grad (sno_n_params floats) at learning rate lr, beta1 = 0.9,
 * beta2 = 0.999, eps = 1e-8 and the bias corrections 1 - beta^step of step
 * `step` (>= 1) -- the update sno_train makes after each batch; the moments
 * persist between calls (zero after sno_create, reset by sno_train).  And a
 * copy of the two moments (host, sno_n_params floats each). */
int sno_adam_step(sno *s, const float *grad, long step, double lr, void *hip_stream);
int sno_get_moments(const sno *s, float *m, float *v);
/* Output normalisation: per-component scale (4 floats, host). */
int sno_get_scale(const sno *s, float *scale4);

/* Message of the last surrogate error on the calling thread. */
const char *sno_last_error(void);

/* Keep every decim-th sample: in [n][4][n_rec][nt] -> out [n][4][n_rec][nt/decim]
 * (device). */
int sno_decimate(const float *in, int n, int n_rec, int nt, int decim, float *out, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
