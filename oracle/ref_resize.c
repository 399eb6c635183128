/*
 * FP64 reference resampler in plain C (OpenMP over output rows).
 *
 * TEST INFRASTRUCTURE ONLY: this is the oracle the HIP library is checked
 * against and the CPU baseline the benchmark times. Only the tests, the smoke
 * check and the benchmark's CPU leg load it. It shares no code, header or
 * constant with the HIP path.
 *
 * It evaluates the same definition as oracle/ref_resize.py, one output pixel
 * at a time (paper section II.B, eqs. 1-5, generalised to 4x4 taps):
 *   s(x)  = ((2x+1) N_in - N_out) / (2 N_out)      half-pixel reading of eq. 1
 *   x0    = floor(s), t = s - x0                   eqs. 2-4, int() read as floor
 *   taps  = x0, x0+1 with (1-t, t)                 bilinear
 *         = x0-1 .. x0+2 with K(t - j)             Keys cubic, parameter a
 *   index = clamp(tap, 0, N_in - 1)                replicate edge
 *   v     = sum_j sum_i wy_j wx_i src[iy_j][ix_i]  eq. 5 generalised
 * all in double precision. Inputs are float32 arrays, which hold uint8,
 * float16 and float32 pixels exactly.
 *
 * Parity status: pinned by tests/test_oracle.py (brute force in exact
 * rationals on small images, and agreement with the numpy oracle).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_BILINEAR 0
#define ORACLE_BICUBIC 1

/* Keys (1981) cubic convolution kernel with parameter a. */
static double keys_kernel(double d, double a)
{
    double ad = fabs(d);
    if (ad <= 1.0)
        return (a + 2.0) * ad * ad * ad - (a + 3.0) * ad * ad + 1.0;
    if (ad < 2.0)
        return a * ad * ad * ad - 5.0 * a * ad * ad + 8.0 * a * ad - 4.0 * a;
    return 0.0;
}

static int64_t clamp_index(int64_t i, int64_t n)
{
    if (i < 0)
        return 0;
    if (i > n - 1)
        return n - 1;
    return i;
}

/* Taps of output index x along an axis of n_in -> n_out samples.
 * Writes k clamped indices and weights, returns k (2 or 4). */
static int axis_taps(int64_t x, int64_t n_in, int64_t n_out, int filt, double a,
                     int64_t *idx, double *w)
{
    double s = (double)((2 * x + 1) * n_in - n_out) / (double)(2 * n_out);
    double base = floor(s);
    double t = s - base;
    int64_t x0 = (int64_t)base;
    if (filt == ORACLE_BILINEAR) {
        idx[0] = clamp_index(x0, n_in);
        idx[1] = clamp_index(x0 + 1, n_in);
        w[0] = 1.0 - t;
        w[1] = t;
        return 2;
    }
    for (int j = -1; j <= 2; ++j) {
        idx[j + 1] = clamp_index(x0 + j, n_in);
        w[j + 1] = keys_kernel(t - (double)j, a);
    }
    return 4;
}

/*
 * Resize selected output rows.
 *   src  : planes x in_h x in_w x ch float32 (row-major, channels interleaved)
 *   dst  : planes x nrows x out_w x ch float64
 *   rows : nrows output row indices in [0, out_h)
 * Returns 0, or -1 on an invalid argument.
 */
int oracle_resize_rows(const float *src, int64_t planes, int64_t in_h, int64_t in_w, int64_t ch,
                       double *dst, int64_t out_h, int64_t out_w, int filt, double a,
                       const int64_t *rows, int64_t nrows, int nthreads)
{
    if (!src || !dst || !rows || planes < 1 || in_h < 1 || in_w < 1 || ch < 1 || out_h < 1 ||
        out_w < 1 || nrows < 0 || (filt != ORACLE_BILINEAR && filt != ORACLE_BICUBIC))
        return -1;
    for (int64_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= out_h)
            return -1;
    /* the thread count applies to this call only (num_threads clause) */
#ifdef _OPENMP
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    const int nt = 1;
    (void)nthreads;
#endif
    (void)nt;
    int64_t total = planes * nrows;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t pr = 0; pr < total; ++pr) {
        int64_t p = pr / nrows;
        int64_t r = pr % nrows;
        int64_t iy[4], ix[4];
        double wy[4], wx[4];
        int ky = axis_taps(rows[r], in_h, out_h, filt, a, iy, wy);
        const float *plane = src + p * in_h * in_w * ch;
        double *out_row = dst + (p * nrows + r) * out_w * ch;
        for (int64_t x = 0; x < out_w; ++x) {
            int kx = axis_taps(x, in_w, out_w, filt, a, ix, wx);
            for (int64_t c = 0; c < ch; ++c) {
                double v = 0.0;
                for (int j = 0; j < ky; ++j)
                    for (int i = 0; i < kx; ++i)
                        v += wy[j] * wx[i] * (double)plane[(iy[j] * in_w + ix[i]) * ch + c];
                out_row[x * ch + c] = v;
            }
        }
    }
    return 0;
}

/*
 * Adjoint of the resize with respect to its input.
 *   grad_out : planes x out_h x out_w x ch float32
 *   grad_src : planes x in_h x in_w x ch float64 (overwritten)
 * Every output pixel scatters wy_j wx_i g onto its clamped taps. Planes are
 * independent, so the planes are split over threads.
 */
int oracle_adjoint(const float *grad_out, int64_t planes, int64_t out_h, int64_t out_w, int64_t ch,
                   double *grad_src, int64_t in_h, int64_t in_w, int filt, double a, int nthreads)
{
    if (!grad_out || !grad_src || planes < 1 || in_h < 1 || in_w < 1 || ch < 1 || out_h < 1 ||
        out_w < 1 || (filt != ORACLE_BILINEAR && filt != ORACLE_BICUBIC))
        return -1;
    /* the thread count applies to this call only (num_threads clause) */
#ifdef _OPENMP
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    const int nt = 1;
    (void)nthreads;
#endif
    (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t p = 0; p < planes; ++p) {
        double *gs = grad_src + p * in_h * in_w * ch;
        const float *g = grad_out + p * out_h * out_w * ch;
        for (int64_t k = 0; k < in_h * in_w * ch; ++k)
            gs[k] = 0.0;
        int64_t iy[4], ix[4];
        double wy[4], wx[4];
        for (int64_t y = 0; y < out_h; ++y) {
            int ky = axis_taps(y, in_h, out_h, filt, a, iy, wy);
            for (int64_t x = 0; x < out_w; ++x) {
                int kx = axis_taps(x, in_w, out_w, filt, a, ix, wx);
                for (int64_t c = 0; c < ch; ++c) {
                    double gv = (double)g[(y * out_w + x) * ch + c];
                    for (int j = 0; j < ky; ++j)
                        for (int i = 0; i < kx; ++i)
                            gs[(iy[j] * in_w + ix[i]) * ch + c] += wy[j] * wx[i] * gv;
                }
            }
        }
    }
    return 0;
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
