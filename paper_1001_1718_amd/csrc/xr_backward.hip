// Adjoint of the resize with respect to its input for gfx950: gradients
// stored as float32 or float16, summed in float32.
//
// grad_src = A_y^T grad_dst A_x: every output pixel (y, x) scatters
// wy_j * wx_i * g[y][x] onto its clamped taps (the transpose of eq. 5).
//
// Owner computes: a workgroup owns a tile of grad_src (input pixels) and
// gathers every output pixel whose taps touch that tile, so each gradient
// pixel is written exactly once with a plain store: no global atomics, no
// clearing pass, and pixels no output touches come out as zero.
//
//  phase 0  for each tile column c the outputs x whose taps reach it with
//           their summed weight w(x, c), and the same for each tile row;
//  phase 1  horizontal adjoint, gather: u[y][c] = sum over x ascending of
//           w(x, c) * g[y][x];
//  phase 2  vertical adjoint, gather: grad[r][c] = sum over the output rows y
//           whose taps include r of wy_j(y) * u[y][c], summed in ascending y.
//
// Every sum has a fixed order, so the result is deterministic (bit for bit
// the same on every run and for every tiling of the launch). The exact-x2
// walk below (float32 and float16) is deterministic as well.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "xr_buffer.hpp"
#include "xr_device.hpp"
#include "xr_internal.h"

namespace xr {
using namespace dev;

namespace {

constexpr int kBwdThreads = 256;


// First output index whose clamped taps reach source index >= c, for the
// axis n_in -> n_out (the map is monotone; see eqs. 1-4).
template <int FILTER>
__device__ __forceinline__ int32_t first_output(int32_t c, int32_t n_in, int32_t n_out)
{
    using TP = Taps<FILTER>;
    if (c <= 0)
        return 0;
    // lo(x) + K - 1 >= c  <=>  floor(s(x)) >= m  <=>  s(x) >= m
    const int64_t m = static_cast<int64_t>(c) - TP::K + 1 - TP::LO;
    const int64_t num = 2 * static_cast<int64_t>(n_out) * m + n_out - n_in;
    const int64_t den = 2 * static_cast<int64_t>(n_in);
    const int64_t x = num >= 0 ? (num + den - 1) / den : -((-num) / den);  // ceil
    return static_cast<int32_t>(x < 0 ? 0 : (x > n_out - 1 ? n_out - 1 : x));
}

// Last output index whose clamped taps reach source index <= c.
template <int FILTER>
__device__ __forceinline__ int32_t last_output(int32_t c, int32_t n_in, int32_t n_out)
{
    using TP = Taps<FILTER>;
    if (c >= n_in - 1)
        return n_out - 1;
    // lo(x) <= c  <=>  floor(s(x)) <= c - LO  <=>  s(x) < c - LO + 1
    const int64_t m = static_cast<int64_t>(c) - TP::LO + 1;
    const int64_t num = 2 * static_cast<int64_t>(n_out) * m + n_out - n_in;
    const int64_t den = 2 * static_cast<int64_t>(n_in);
    const int64_t x = (num >= 0 ? (num + den - 1) / den : -((-num) / den)) - 1;  // ceil - 1
    return static_cast<int32_t>(x < 0 ? 0 : (x > n_out - 1 ? n_out - 1 : x));
}

// a.src = grad_dst (out_w x out_h), a.dst = grad_src (in_w x in_h), both
// stored as T (float or _Float16), summed in float32.
// Tile: tw columns x th rows of grad_src (tw a power of two). LDS holds
// max_rows x tw x C floats of u; per tile column the first output column, the
// count and nmax weights of the outputs that reach it; per tile row the first
// region row, the count and nmax_y weights of the output rows that reach it.
template <int FILTER, typename T, int C>
__global__ void __launch_bounds__(kBwdThreads) k_bwd_owner(ResizeArgs a, int32_t tw, int32_t th,
                                                           int32_t max_rows, int32_t nmax, int32_t nmax_y)
{
    using TP = Taps<FILTER>;
    constexpr int K = TP::K;
    constexpr int RU = 8;  // region rows per thread and step of the horizontal pass
    extern __shared__ float lds[];
    const int32_t row_floats = tw * C;
    float *u = lds;                                                             // [max_rows][tw*C]
    int32_t *colx = reinterpret_cast<int32_t *>(u + max_rows * row_floats);    // [tw]
    int32_t *coln = colx + tw;                                                  // [tw]
    float *colw = reinterpret_cast<float *>(coln + tw);                         // [tw][nmax]
    int32_t *rowk = reinterpret_cast<int32_t *>(colw + tw * nmax);              // [th]
    int32_t *rown = rowk + th;                                                  // [th]
    float *roww = reinterpret_cast<float *>(rown + th);                         // [th][nmax_y]

    const int32_t c_a = blockIdx.x * tw;
    const int32_t c_b = min(c_a + tw, a.in_w);
    const int32_t r_a = blockIdx.y * th;
    const int32_t r_b = min(r_a + th, a.in_h);
    const int32_t plane = blockIdx.z;
    const int32_t ya = first_output<FILTER>(r_a, a.in_h, a.out_h);
    const int32_t yb = min(last_output<FILTER>(r_b - 1, a.in_h, a.out_h), ya + max_rows - 1);
    const int32_t nrows = yb - ya + 1;
    const int32_t ntc = c_b - c_a;
    const int32_t ntr = r_b - r_a;
    const int32_t tid = threadIdx.x;

    // phase 0: for each tile column c (tile row r) the outputs whose clamped
    // taps reach it, x in [first_output(c), last_output(c)], and the summed
    // weight of those taps (taps ascending)
    auto axis_table = [](int32_t c, int32_t n_in, int32_t n_out, int32_t nm, int32_t &first, int32_t &count,
                         float *w) {
        first = first_output<FILTER>(c, n_in, n_out);
        count = min(max(last_output<FILTER>(c, n_in, n_out) - first + 1, 0), nm);
        for (int32_t m = 0; m < count; ++m) {
            int32_t x0;
            float t, omt;
            axis_tap(first + m, n_in, n_out, 1, x0, t, omt);
            float wt[K];
            weights<FILTER>(t, omt, wt);
            float sum = 0.0f;
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (clampi(x0 + TP::LO + i, 0, n_in - 1) == c)
                    sum += wt[i];
            w[m] = sum;
        }
    };
    for (int32_t t = tid; t < ntc + ntr; t += kBwdThreads) {
        if (t < ntc) {
            axis_table(c_a + t, a.in_w, a.out_w, nmax, colx[t], coln[t], colw + t * nmax);
        } else {
            const int32_t i = t - ntc;
            int32_t yf, n;
            axis_table(r_a + i, a.in_h, a.out_h, nmax_y, yf, n, roww + i * nmax_y);
            // first_output and last_output are monotone, so the rows lie in
            // the region ya .. yb (yf >= ya; the min only guards the LDS)
            rowk[i] = yf - ya;
            rown[i] = max(min(n, nrows - (yf - ya)), 0);
        }
    }
    __syncthreads();

    // phase 1: horizontal adjoint as a gather: u[k][c] = sum over x ascending
    // of w(x, c) g[ya + k][x]. A thread owns one tile column and RU region
    // rows per step, so RU loads are in flight per weight.
    const unsigned char *gsrc = a.src + static_cast<int64_t>(plane) * a.src_plane_pitch;
    const int32_t phases = kBwdThreads / tw;
    const int32_t cl = tid & (tw - 1), kq = tid / tw;
    if (cl < ntc) {
        const int32_t xf = colx[cl], n = coln[cl];
        const float *w = colw + cl * nmax;
        for (int32_t k0 = kq * RU; k0 < nrows; k0 += phases * RU) {
            const unsigned char *grow[RU];
#pragma unroll
            for (int q = 0; q < RU; ++q)
                grow[q] = gsrc + static_cast<int64_t>(ya + min(k0 + q, nrows - 1)) * a.src_pitch;
            float acc[RU][C];
            if (n > 0) {
                const float w0 = w[0];
#pragma unroll
                for (int q = 0; q < RU; ++q) {
                    float g[C];
                    Pix<T, C>::load(grow[q], xf, g);
                    fma_first(acc[q], w0, g);
                }
                for (int32_t m = 1; m < n; ++m) {
                    const float wm = w[m];
#pragma unroll
                    for (int q = 0; q < RU; ++q) {
                        float g[C];
                        Pix<T, C>::load(grow[q], xf + m, g);
                        fma_next(acc[q], wm, g);
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < RU; ++q)
#pragma unroll
                    for (int ch = 0; ch < C; ++ch)
                        acc[q][ch] = 0.0f;
            }
#pragma unroll
            for (int q = 0; q < RU; ++q)
                if (k0 + q < nrows) {
                    float *urow = u + (k0 + q) * row_floats + cl * C;
#pragma unroll
                    for (int ch = 0; ch < C; ++ch)
                        urow[ch] = acc[q][ch];
                }
        }
    }
    __syncthreads();

    // phase 2: vertical adjoint, one (column, channel) per thread:
    // grad[r][c] = sum over region rows k ascending of w(y, r) u[k][c]
    unsigned char *gdst = a.dst + static_cast<int64_t>(plane) * a.dst_plane_pitch;
    const int32_t ncols = ntc * C;
    for (int32_t f = tid; f < ncols; f += kBwdThreads) {
        for (int32_t i = 0; i < ntr; ++i) {
            const int32_t k0 = rowk[i], n = rown[i];
            const float *wr = roww + i * nmax_y;
            float acc = 0.0f;
            for (int32_t j = 0; j < n; ++j)
                acc = __builtin_fmaf(wr[j], u[(k0 + j) * row_floats + f], acc);
            const float v[1] = {acc};
            Pix<T, 1>::store(gdst + static_cast<int64_t>(r_a + i) * a.dst_pitch, c_a * C + f, v);
        }
    }
}

// ---------------------------------------------------------------------------
// Exact x2 upscale on both axes: transposed strip walk in registers
// ---------------------------------------------------------------------------
//
// For out = 2 in, output x taps source lo(x) + i with lo(2m) = m - 1 + LO
// (t = 3/4) and lo(2m+1) = m + LO (t = 1/4). Ignoring the clamp, source
// column c therefore receives the 2K outputs x = 2c - K + 1 + d, d = 0..2K-1,
// with weight wo[K-1-q] for d = 2q and we[K-1-q] for d = 2q+1; rows alike.
// k_bwd_x2 sums exactly those unclamped terms (outputs outside the image
// count as zero), and the threads that own the image's first or last row or
// column add the terms whose taps were clamped onto them, so every gradient
// is one sum rounded once.
//
// The walk: a thread owns P source columns c0 .. c0 + P - 1 and a strip of ns
// source rows (ns a multiple of 4). Per source row it needs the horizontal
// adjoints of the 2K output rows 2r - K + 1 .. 2r + K, of which two are new:
// output rows come in pairs, pair q being rows y_first + 2q and + 1
// (y_first = 2 r_a - K + 1), held as horizontal adjoints in a ring of 2K rows.
// A row's window is the W = 2P + 2K - 2 output pixels from column
// 2 c0 - K + 1 on; these sums leave out the taps that were clamped onto the
// image's first or last row or column, which the threads owning those pixels
// add on their own (see `clamped`). Every load and store is issued on every step, through
// buffer resources: output rows outside the image read as zero (outside the
// load resource), gradient rows past the strip or the image are dropped
// (outside the store resource); the first thread of a row loads from column
// 0 and moves its window right in registers, threads at either edge zero the
// pixels outside the image. Loads run PD pairs ahead. The float32 order per
// value is the one the previous register walk used (taps ascending), so the
// result does not depend on the launch.
template <int FILTER, typename T, int C, int P, int PD>
struct BwdX2Walk {
    using TP = Taps<FILTER>;
    static constexpr int K = TP::K;
    static constexpr int W = 2 * P + 2 * K - 2;
    static constexpr int PB = static_cast<int>(sizeof(T)) * C;
    static constexpr int MIS = ((K - 1) * PB) % 4;  // the window starts MIS bytes into its first dword
    static constexpr int LB = (MIS + W * PB + 3) / 4 * 4;
    static constexpr int Q = PD + 1;
    static_assert((2 * P * PB) % 4 == 0, "a thread's window must advance by whole dwords");
    static_assert(4 % Q == 0 && 4 % K == 0, "slots repeat every 4 steps");
    struct Pair {
        RawBuf<LB, 4> r[2];
    };

    __amdgpu_buffer_rsrc_t grsrc;  // upstream rows from y_res on
    int32_t y_res, y_first;
    int64_t g_pitch, d_pitch;
    uint32_t lane_src;
    int32_t xs, out_w;             // first window column, upstream width
    bool left, right;              // window starts before column 0 / ends past out_w - 1
    bool own_first;                // this thread owns column 0
    int32_t p_right;               // owned column index of column in_w - 1, or -1
    int32_t r_a, in_h;
    // clamped taps (see `clamped`): summed weight of the taps of output index
    // m (m = 0 .. K - 1 from the first, resp. last, output on) that land
    // before column / row 0, resp. past the last one
    float wlo[K], whi[K];
    RunStore<T, C, P> st;
    int32_t d_row_off;             // strip step of the store resource's first row
    float wt[2 * K];
    float ring[2 * K][P][C];
    Pair rawq[Q];

    __device__ __forceinline__ Pair load_pair(int32_t q) const
    {
        Pair pr;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int32_t y = y_first + 2 * q + h;
            const uint32_t roff = static_cast<uint32_t>(static_cast<int64_t>(y - y_res) * g_pitch);
            buf_load<LB>(pr.r[h].b, grsrc, roff + lane_src);
        }
        return pr;
    }

    // the window's pixels as floats; at an image edge, pixels outside are zero
    __device__ __forceinline__ void window(const RawBuf<LB, 4> &raw, float (&v)[W][C]) const
    {
        RawBuf<LB, 4> in = raw;
        if (left) {
            // loaded from column 0: pixel s of the window is loaded pixel
            // s + xs, i.e. the bytes move right by -xs pixels (1 .. K - 1)
#pragma unroll
            for (int n = 1; n < K; ++n) {
                const int SH = n * PB + MIS;  // bytes
                RawBuf<LB, 4> sh;
#pragma unroll
                for (int b = 0; b < LB; ++b)
                    sh.b[b] = b >= SH ? raw.b[b - SH] : 0;
                if (-xs == n)
                    in = sh;
            }
        }
#pragma unroll
        for (int s = 0; s < W; ++s) {
            float p[C];
            if constexpr (std::is_same_v<T, float>) {
#pragma unroll
                for (int ch = 0; ch < C; ++ch)
                    __builtin_memcpy(&p[ch], in.b + MIS + (s * C + ch) * 4, 4);
            } else {
#pragma unroll
                for (int ch = 0; ch < C; ++ch) {
                    _Float16 hv;
                    __builtin_memcpy(&hv, in.b + MIS + (s * C + ch) * 2, 2);
                    p[ch] = static_cast<float>(hv);
                }
            }
#pragma unroll
            for (int ch = 0; ch < C; ++ch)
                v[s][ch] = p[ch];
        }
        if (left || right) {
#pragma unroll
            for (int s = 0; s < W; ++s) {
                const int32_t x = xs + s;
                const bool ok = x >= 0 && x < out_w;
#pragma unroll
                for (int ch = 0; ch < C; ++ch)
                    v[s][ch] = ok ? v[s][ch] : 0.0f;
            }
        }
    }

    __device__ __forceinline__ void hadj(const RawBuf<LB, 4> &raw, float (&u)[P][C]) const
    {
        float v[W][C];
        window(raw, v);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            fma_first(u[p], wt[0], v[2 * p]);
#pragma unroll
            for (int d = 1; d < 2 * K; ++d)
                fma_next(u[p], wt[d], v[2 * p + d]);
        }
        if (own_first) {
            // column 0 (this thread's first, c0 = 0, window from column
            // 1 - K): taps clamped from the left; output column m is window
            // pixel m + K - 1
#pragma unroll
            for (int m = 0; m < K; ++m)
                fma_next(u[0], wlo[m], v[m + K - 1]);
        }
        if (p_right >= 0) {
            // column in_w - 1 = c0 + p_right: taps clamped from the right.
            // With c0 = in_w - 1 - p_right the window starts at column
            // out_w - 1 - K - 2 p_right, so output column out_w - K + m is
            // window pixel m + 1 + 2 p_right.
#pragma unroll
            for (int pr = 0; pr < P; ++pr)
                if (p_right == pr) {
#pragma unroll
                    for (int m = 0; m < K; ++m)
                        fma_next(u[pr], whi[m], v[m + 1 + 2 * pr]);
                }
        }
    }

    // source row r_a + j: pair K - 1 + j completes its window; ring slot of
    // pair q's first row is 2q mod 2K
    template <int I>  // j mod 4
    __device__ __forceinline__ void step(int32_t j, int32_t last_pair)
    {
        constexpr int QI = I + K - 1;  // pair index mod 4
        rawq[(QI + PD) % Q] = load_pair(min(j + K - 1 + PD, last_pair));
        __builtin_amdgcn_sched_barrier(0);
        hadj(rawq[QI % Q].r[0], ring[(2 * QI) % (2 * K)]);
        hadj(rawq[QI % Q].r[1], ring[(2 * QI + 1) % (2 * K)]);
        float g[P][C];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            fma_first(g[p], wt[0], ring[(2 * I) % (2 * K)][p]);
#pragma unroll
            for (int d = 1; d < 2 * K; ++d)
                fma_next(g[p], wt[d], ring[(2 * I + d) % (2 * K)][p]);
        }
        const int32_t r = r_a + j;
        if (r == 0) {
            // taps of output rows 0 .. K - 1 clamped onto row 0; output row m
            // sits at window row m + K - 1 (2j + K - 1 + m, j = 0 here)
#pragma unroll
            for (int m = 0; m < K; ++m)
#pragma unroll
                for (int p = 0; p < P; ++p)
                    fma_next(g[p], wlo[m], ring[(2 * I + K - 1 + m) % (2 * K)][p]);
        }
        if (r == in_h - 1) {
            // taps of output rows out_h - K + m clamped onto the last row;
            // this step's window starts at output row 2r - K + 1, so output
            // row 2 in_h - K + m is its window row m + 1
#pragma unroll
            for (int m = 0; m < K; ++m)
#pragma unroll
                for (int p = 0; p < P; ++p)
                    fma_next(g[p], whi[m], ring[(2 * I + 1 + m) % (2 * K)][p]);
        }
        RawBuf<P * PB, cmin(16, P * PB)> out;
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int ch = 0; ch < C; ++ch) {
                const T vv = static_cast<T>(g[p][ch]);
                __builtin_memcpy(out.b + (p * C + ch) * sizeof(T), &vv, sizeof(T));
            }
        st.store(static_cast<uint32_t>(static_cast<int64_t>(j - d_row_off) * d_pitch), out);
        __builtin_amdgcn_sched_barrier(0);
    }

    // Taps clamped onto the first or last source index of an axis (the same
    // on both axes at x2): output m (m = 0 .. K - 1) has x0 = floor((2m - 1)/4)
    // with t = 3/4 (even m) or 1/4 (odd m); its taps x0 + LO + i below 0 land
    // on index 0. Mirrored, output n - K + m has taps past n_in - 1 where
    // output K - 1 - m has them below 0, with the weights reversed.
    __device__ __forceinline__ void clamped()
    {
        float we[K], wo[K];
        weights<FILTER>(0.75f, 0.25f, we);
        weights<FILTER>(0.25f, 0.75f, wo);
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const int x0 = (m % 2 == 0) ? m / 2 - 1 : (m - 1) / 2;
            const float *w = (m % 2 == 0) ? we : wo;
            float lo = 0.0f;
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (x0 + TP::LO + i < 0)
                    lo += w[i];
            wlo[m] = lo;
        }
        // output n - K + m mirrors output K - 1 - m (the map and the kernel are
        // symmetric about the axis centre), so its taps past the end carry the
        // same weights; their sum is exact in float32 (dyadic weights)
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const int mm = K - 1 - m;
            const int x0 = (mm % 2 == 0) ? mm / 2 - 1 : (mm - 1) / 2;
            const float *w = (mm % 2 == 0) ? we : wo;
            float hi = 0.0f;
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (x0 + TP::LO + i < 0)
                    hi += w[i];
            whi[m] = hi;
        }
    }

    __device__ __forceinline__ void run(int32_t ns)
    {
        float we[K], wo[K];
        weights<FILTER>(0.75f, 0.25f, we);
        weights<FILTER>(0.25f, 0.75f, wo);
#pragma unroll
        for (int q = 0; q < K; ++q) {
            wt[2 * q] = wo[K - 1 - q];
            wt[2 * q + 1] = we[K - 1 - q];
        }
        clamped();
        const int32_t last_pair = ns + K - 2;
#pragma unroll
        for (int i = 0; i < PD; ++i)
            rawq[i % Q] = load_pair(min(i, last_pair));
#pragma unroll
        for (int q = 0; q + 1 < K; ++q) {
            rawq[(q + PD) % Q] = load_pair(min(q + PD, last_pair));
            hadj(rawq[q % Q].r[0], ring[(2 * q) % (2 * K)]);
            hadj(rawq[q % Q].r[1], ring[(2 * q + 1) % (2 * K)]);
        }
        step<0>(0, last_pair);
        step<1>(1, last_pair);
        step<2>(2, last_pair);
        step<3>(3, last_pair);
        for (int32_t j = 4; j < ns; j += 4) {
            step<0>(j, last_pair);
            step<1>(j + 1, last_pair);
            step<2>(j + 2, last_pair);
            step<3>(j + 3, last_pair);
        }
    }
};

// Pairs of upstream rows loaded ahead of use: one for windows of up to 64
// bytes per row, none for wider ones (RGBA float32 bicubic: 128 bytes a row;
// a queue of them would take most of the register file)
template <typename T, int C, int P, int K>
constexpr int bwd_x2_prefetch()
{
    return (2 * P + 2 * K - 2) * static_cast<int>(sizeof(T)) * C <= 64 ? 1 : 0;
}

// a.src = grad_dst (out_w x out_h), a.dst = grad_src (in_w x in_h); strip s of
// ns source rows covers rows [s ns, (s + 1) ns); threadIdx.y picks one of
// blockDim.y consecutive strips.
template <int FILTER, typename T, int C, int P>
__global__ void __launch_bounds__(256) k_bwd_x2(ResizeArgs a, int32_t ns)
{
    using Wk = BwdX2Walk<FILTER, T, C, P, bwd_x2_prefetch<T, C, P, Taps<FILTER>::K>()>;
    constexpr int K = Wk::K, W = Wk::W, PB = Wk::PB;
    const int32_t c0 = (static_cast<int32_t>(blockIdx.x * blockDim.x) + static_cast<int32_t>(threadIdx.x)) * P;
    if (!RunStore<T, C, P>::kExchange && c0 >= a.in_w)
        return;
    const int32_t r_a = __builtin_amdgcn_readfirstlane(
        static_cast<int32_t>(blockIdx.y * blockDim.y + threadIdx.y) * ns);
    if (r_a >= a.in_h)
        return;
    const int32_t r_b = min(r_a + ns, a.in_h);
    Wk w;
    w.y_first = 2 * r_a - K + 1;
    // upstream rows the strip reads, inside the image
    w.y_res = max(0, w.y_first);
    const int32_t y_end = min(a.out_h, 2 * (r_a + ns) + K);
    w.g_pitch = a.src_pitch;
    const unsigned char *g = a.src + static_cast<int64_t>(blockIdx.z) * a.src_plane_pitch +
                             static_cast<int64_t>(w.y_res) * a.src_pitch;
    w.grsrc = buf_rsrc(g, static_cast<uint32_t>(static_cast<int64_t>(y_end - w.y_res) * a.src_pitch));
    w.xs = 2 * c0 - K + 1;
    w.out_w = a.out_w;
    w.left = w.xs < 0;
    w.right = w.xs + W > a.out_w;
    w.lane_src = w.left ? 0u : static_cast<uint32_t>(w.xs * PB - Wk::MIS);
    w.own_first = c0 == 0;
    w.p_right = (a.in_w - 1 >= c0 && a.in_w - 1 < c0 + P) ? a.in_w - 1 - c0 : -1;
    w.r_a = r_a;
    w.in_h = a.in_h;
    unsigned char *d = a.dst + static_cast<int64_t>(blockIdx.z) * a.dst_plane_pitch +
                       static_cast<int64_t>(r_a) * a.dst_pitch;
    extern __shared__ __attribute__((aligned(16))) unsigned char xlds[];
    w.st.init(buf_rsrc(d, static_cast<uint32_t>(static_cast<int64_t>(r_b - r_a) * a.dst_pitch)), c0, a.in_w,
              static_cast<int32_t>(threadIdx.y * blockDim.x + threadIdx.x), xlds);
    w.d_pitch = a.dst_pitch;
    w.d_row_off = 0;
    w.run(ns);
}

template <int FILTER, typename T, int C>
hipError_t launch_bwd_up2(const ResizeArgs &a, hipStream_t stream)
{
    constexpr int P = (C == 1) ? 4 : 1;
    // strips of 8 source rows (measured on the 32x3x1024^2 bilinear FP32
    // adjoint: 8 rows 345 us, 16 rows 360 us, 32 rows 381 us), shortened so
    // that a strip's rows stay well inside a buffer resource's 2 GiB
    int32_t ns = 8;
    while (ns > 4 && (2 * ns + 8) * std::max(a.src_pitch, a.dst_pitch) >= (int64_t(1) << 30))
        ns -= 4;
    const int32_t cols_per_block = 256 * P;
    const size_t lds = RunStore<T, C, P>::kExchange ? 256 * RunStore<T, C, P>::OB : 0;
    hipLaunchKernelGGL((k_bwd_x2<FILTER, T, C, P>),
                       dim3((a.in_w + cols_per_block - 1) / cols_per_block, (a.in_h + ns - 1) / ns, a.planes),
                       dim3(256), lds, stream, a, ns);
    return hipGetLastError();
}

// Tile of the owner-computes kernel: tw source columns (tw * C = 256 values
// across the threads) and th source rows, shrunk until the region of output
// rows and the column tables fit the LDS budget.
struct BwdPlan {
    int32_t tw, th, max_rows, nmax, nmax_y;
    size_t lds;
};

template <int FILTER, int C>
BwdPlan plan_backward(const ResizeArgs &a)
{
    constexpr int K = Taps<FILTER>::K;
    constexpr size_t kBudget = 64 * 1024;
    BwdPlan p{};
    // outputs reaching one source column: at most ceil(K out / in) + 1 inside,
    // (1 - LO + 1/2) out / in + 1 at a clamped border; rows alike
    p.nmax = static_cast<int32_t>((static_cast<int64_t>(K) * a.out_w + a.in_w - 1) / a.in_w + 2);
    p.nmax_y = static_cast<int32_t>((static_cast<int64_t>(K) * a.out_h + a.in_h - 1) / a.in_h + 2);
    // first tile height: tall for shrinking and identity (few output rows per
    // source row), short for upscales (measured: x0.75 bilinear 0.26 -> 0.19 ms
    // at 32 rows, x1.5 bicubic 0.75 -> 0.71 ms at 8)
    const int32_t th0 = a.out_h <= a.in_h ? 32 : 8;
    p.tw = kBwdThreads / C;
    p.th = th0;
    for (;;) {
        // output rows touching th source rows: at most (th + K - 1) * out/in + 2
        const int64_t rows = (static_cast<int64_t>(p.th + K - 1) * a.out_h + a.in_h - 1) / a.in_h + 2;
        p.max_rows = static_cast<int32_t>(rows);
        p.lds = sizeof(float) * (static_cast<size_t>(rows) * p.tw * C +
                                 static_cast<size_t>(p.tw) * (2 + static_cast<size_t>(p.nmax)) +
                                 static_cast<size_t>(p.th) * (2 + static_cast<size_t>(p.nmax_y)));
        if (rows < (int64_t{1} << 24) && p.lds <= kBudget)
            return p;
        if (p.th > 1) {
            p.th /= 2;
        } else if (p.tw > 16) {
            p.tw /= 2;
            p.th = th0;
        } else {
            p.lds = 0;
            return p;
        }
    }
}

template <int FILTER, typename T, int C>
hipError_t launch_bwd_typed(const ResizeArgs &a, hipStream_t stream)
{
    if (a.out_w == 2 * a.in_w && a.out_h == 2 * a.in_h)
        return launch_bwd_up2<FILTER, T, C>(a, stream);
    const BwdPlan p = plan_backward<FILTER, C>(a);
    if (p.lds == 0)
        return hipErrorInvalidConfiguration;
    const dim3 grid((a.in_w + p.tw - 1) / p.tw, (a.in_h + p.th - 1) / p.th, a.planes);
    hipLaunchKernelGGL((k_bwd_owner<FILTER, T, C>), grid, dim3(kBwdThreads), p.lds, stream, a, p.tw, p.th,
                       p.max_rows, p.nmax, p.nmax_y);
    return hipGetLastError();
}

template <int FILTER, typename T>
hipError_t launch_bwd_channels(const ResizeArgs &a, int32_t channels, hipStream_t stream)
{
    return channels == 4 ? launch_bwd_typed<FILTER, T, 4>(a, stream) : launch_bwd_typed<FILTER, T, 1>(a, stream);
}

}  // namespace

bool backward_supported(const ResizeArgs &a, int32_t filter, int32_t channels)
{
    if (filter == XR_BICUBIC)
        return channels == 4 ? plan_backward<kBicubic, 4>(a).lds != 0
                             : plan_backward<kBicubic, 1>(a).lds != 0;
    return channels == 4 ? plan_backward<kBilinear, 4>(a).lds != 0
                         : plan_backward<kBilinear, 1>(a).lds != 0;
}

hipError_t launch_backward(const ResizeArgs &a, int32_t filter, int32_t dtype, int32_t channels,
                           hipStream_t stream)
{
    if (dtype == XR_F16)
        return filter == XR_BICUBIC ? launch_bwd_channels<kBicubic, _Float16>(a, channels, stream)
                                    : launch_bwd_channels<kBilinear, _Float16>(a, channels, stream);
    return filter == XR_BICUBIC ? launch_bwd_channels<kBicubic, float>(a, channels, stream)
                                : launch_bwd_channels<kBilinear, float>(a, channels, stream);
}

}  // namespace xr
