/*
 * FP64 oracle of the trace superposition.  TEST INFRASTRUCTURE ONLY.
 *
 * Sec. IV: the wave equation is linear, so the record of many events is the
 * sum of single-event traces scaled by the event strength and shifted by the
 * event origin time, zero outside each shifted trace (the paper doubles the
 * record length and zero-pads; Case 2).  Reading: the shift is by a real
 * number of seconds, so the shifted trace is evaluated by linear
 * interpolation between samples, which is exactly the paper's integer shift
 * when the shift is a whole number of samples and the output sampling equals
 * the input sampling.
 *
 *   out[c][r][m] = sum_e amp[e] * x_e(m dt_out - t_origin[e] - t0[c])
 *   x_e(t) = linear interpolation of tr[src_idx[e]][c][r][.] at u = t / dt_in,
 *            with samples outside [0, nt_in - 1] taken as zero.
 *
 * Events are accumulated in their given order, in double precision.
 */
#include <math.h>

#include "oracle.h"

int ocombine(const float *tr, int n_src, int n_rec, int nt_in, double dt_in, const double *t0,
             int n_ev, const int *src_idx, const double *amp, const double *t_origin, int nt_out,
             double dt_out, double *out)
{
    if (n_src < 0 || n_rec < 0 || nt_in < 0 || nt_out < 0 || n_ev < 0 || !(dt_in > 0) ||
        !(dt_out > 0))
        return ORC_EINVAL;
    for (int e = 0; e < n_ev; ++e)
        if (src_idx[e] < 0 || src_idx[e] >= n_src) return ORC_EINVAL;
#pragma omp parallel for collapse(2) schedule(static)
    for (int c = 0; c < 4; ++c)
        for (int r = 0; r < n_rec; ++r) {
            double *o = out + ((long)c * n_rec + r) * nt_out;
            for (int m = 0; m < nt_out; ++m) o[m] = 0.0;
            for (int e = 0; e < n_ev; ++e) {
                const float *x = tr + (((long)src_idx[e] * 4 + c) * n_rec + r) * nt_in;
                for (int m = 0; m < nt_out; ++m) {
                    double u = (m * dt_out - t_origin[e] - t0[c]) / dt_in;
                    double fl = floor(u);
                    long i0 = (long)fl;
                    double f = u - fl;
                    double x0 = (i0 >= 0 && i0 < nt_in) ? x[i0] : 0.0;
                    double x1 = (i0 + 1 >= 0 && i0 + 1 < nt_in) ? x[i0 + 1] : 0.0;
                    o[m] += amp[e] * ((1.0 - f) * x0 + f * x1);
                }
            }
        }
    return ORC_OK;
}
