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
// path below (float32 and float16) is deterministic as well.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "xr_device.hpp"
#include "xr_internal.h"

namespace xr {
using namespace dev;

namespace {

constexpr int kBwdThreads = 256;

// N values of T moved as one aligned vector access (ALIGN bytes)
template <typename T, int N, int ALIGN>
struct alignas(ALIGN) RawVals {
    T v[N];
};

// Alignment of the x2 walk's row runs: they start at (2 c0 + SX0) C sizeof(T)
// bytes, a multiple of 16 for float32 and of 8 for float16.
template <typename T>
constexpr int kRunAlign = sizeof(T) == 4 ? 16 : 8;

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
// k_bwd_up2 sums exactly those unclamped terms (outputs outside the image
// count as zero); k_bwd_up2_border then adds, for the source pixels on the
// image border, the terms whose taps were clamped onto them.

template <int FILTER, int C, int P>
struct BwdUp2 {
    using TP = Taps<FILTER>;
    static constexpr int K = TP::K;
    static constexpr int W = 2 * P + 2 * K - 2;       // output pixels read per row
    static constexpr int SX0 = (C == 1) ? -4 : 1 - K;  // first loaded pixel relative to 2*c0
    static constexpr int SX = (C == 1) ? 16 : W;       // pixels loaded per row
    static constexpr int OFF = (1 - K) - SX0;          // window start within the loaded pixels
    static constexpr int Q = 2;                        // output rows per step
};

template <int FILTER, typename T, int C, int P>
__global__ void __launch_bounds__(256) k_bwd_up2(ResizeArgs a, int32_t strip_h)
{
    using B = BwdUp2<FILTER, C, P>;
    constexpr int K = B::K;
    constexpr int SX = B::SX;
    static_assert(C == 4 || P == 4, "one-channel rows are read 16 pixels at a time");
    float we[K], wo[K];
    weights<FILTER>(0.75f, 0.25f, we);
    weights<FILTER>(0.25f, 0.75f, wo);
    float wt[2 * K];  // transposed weights over the window of one source index
#pragma unroll
    for (int q = 0; q < K; ++q) {
        wt[2 * q] = wo[K - 1 - q];
        wt[2 * q + 1] = we[K - 1 - q];
    }

    const int32_t c0 = (blockIdx.x * blockDim.x + threadIdx.x) * P;
    const int32_t r_a = __builtin_amdgcn_readfirstlane(blockIdx.y * strip_h);
    if (c0 >= a.in_w || r_a >= a.in_h)
        return;
    const int32_t r_b = min(r_a + strip_h, a.in_h);
    const int32_t plane = blockIdx.z;
    const unsigned char *gsrc = a.src + static_cast<int64_t>(plane) * a.src_plane_pitch;
    const int32_t xs = 2 * c0 + B::SX0;  // first loaded output column
    const bool wide = a.aligned16 && xs >= 0 && xs + SX <= a.out_w && c0 + P <= a.in_w;

    // one output row's pixels [xs, xs + SX), zero outside the image
    auto load_row = [&](int32_t y, float (&v)[SX][C]) {
        const bool row_ok = y >= 0 && y < a.out_h;
        const int32_t yy = clampi(y, 0, a.out_h - 1);
        const unsigned char *row = gsrc + static_cast<int64_t>(yy) * a.src_pitch;
        if (wide) {
            const auto raw = *reinterpret_cast<const RawVals<T, SX * C, kRunAlign<T>> *>(
                __builtin_assume_aligned(row + static_cast<int64_t>(xs) * C * sizeof(T), kRunAlign<T>));
#pragma unroll
            for (int s = 0; s < SX; ++s)
#pragma unroll
                for (int ch = 0; ch < C; ++ch)
                    v[s][ch] = row_ok ? static_cast<float>(raw.v[s * C + ch]) : 0.0f;
        } else {
#pragma unroll
            for (int s = 0; s < SX; ++s) {
                const int32_t x = xs + s;
                const bool ok = row_ok && x >= 0 && x < a.out_w;
                float p[C];
                Pix<T, C>::load(row, clampi(x, 0, a.out_w - 1), p);
#pragma unroll
                for (int ch = 0; ch < C; ++ch)
                    v[s][ch] = ok ? p[ch] : 0.0f;
            }
        }
    };
    // horizontal adjoint of one output row for the P owned source columns
    auto hadj = [&](const float (&v)[SX][C], float (&u)[P][C]) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            fma_first(u[p], wt[0], v[B::OFF + 2 * p]);
#pragma unroll
            for (int d = 1; d < 2 * K; ++d)
                fma_next(u[p], wt[d], v[B::OFF + 2 * p + d]);
        }
    };

    // ring of the horizontal adjoints of output rows y, slot (y - y_first) mod 2K
    float ring[2 * K][P][C];
    const int32_t y_first = 2 * r_a - K + 1;
    float va[SX][C], vb[SX][C];
#pragma unroll
    for (int k = 0; k + 2 < 2 * K; k += 2) {  // rows y_first .. y_first + 2K - 3
        load_row(y_first + k, va);
        load_row(y_first + k + 1, vb);
        hadj(va, ring[k]);
        hadj(vb, ring[k + 1]);
    }
    unsigned char *gdst = a.dst + static_cast<int64_t>(plane) * a.dst_plane_pitch;
    const int32_t ncols = min(P, a.in_w - c0);
    auto step = [&](auto slot_tag, int32_t r) {
        constexpr int S = decltype(slot_tag)::value;  // slot of the first new row
        // rows 2r + K - 1 and 2r + K complete the window of source row r
        load_row(2 * r + K - 1, va);
        load_row(2 * r + K, vb);
        hadj(va, ring[S % (2 * K)]);
        hadj(vb, ring[(S + 1) % (2 * K)]);
        float g[P][C];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            fma_first(g[p], wt[0], ring[(S + 2) % (2 * K)][p]);
#pragma unroll
            for (int d = 1; d < 2 * K; ++d)
                fma_next(g[p], wt[d], ring[(S + 2 + d) % (2 * K)][p]);
        }
        unsigned char *drow = gdst + static_cast<int64_t>(r) * a.dst_pitch;
        if (wide) {
            RawVals<T, P * C, kRunAlign<T>> out;
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int ch = 0; ch < C; ++ch)
                    out.v[p * C + ch] = static_cast<T>(g[p][ch]);
            *reinterpret_cast<RawVals<T, P * C, kRunAlign<T>> *>(
                __builtin_assume_aligned(drow + static_cast<int64_t>(c0) * C * sizeof(T), kRunAlign<T>)) = out;
        } else {
#pragma unroll
            for (int p = 0; p < P; ++p)
                if (p < ncols)
                    Pix<T, C>::store(drow, c0 + p, g[p]);
        }
    };
    // the window of row r starts at slot (2(r - r_a)) mod 2K; unroll K rows so
    // that every slot index is a constant
    for (int32_t r = r_a; r < r_b; r += K) {
        step(std::integral_constant<int, 2 * K - 2>{}, r);
        if (r + 1 < r_b)
            step(std::integral_constant<int, 2 * K>{}, r + 1);
        if constexpr (K == 4) {
            if (r + 2 < r_b)
                step(std::integral_constant<int, 2 * K + 2>{}, r + 2);
            if (r + 3 < r_b)
                step(std::integral_constant<int, 2 * K + 4>{}, r + 3);
        }
    }
}

// Border source pixels: add the terms whose row or column tap was clamped onto
// them (the interior walk above left those out). One thread per border pixel
// and plane; index k walks row 0, row in_h-1, then columns 0 and in_w-1 of
// the rows in between. With float16 storage the walk's value is already
// rounded, so the border pixels are summed here in full (every term) and
// overwritten: each gradient is rounded once.
template <int FILTER, typename T, int C>
__global__ void __launch_bounds__(256) k_bwd_up2_border(ResizeArgs a)
{
    constexpr bool kFull = !std::is_same_v<T, float>;
    using TP = Taps<FILTER>;
    constexpr int K = TP::K;
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t n_rows_part = (a.in_h > 1) ? 2 * a.in_w : a.in_w;
    const int32_t inner = a.in_h > 2 ? a.in_h - 2 : 0;
    const int32_t n_cols_part = (a.in_w > 1) ? 2 * inner : inner;
    if (k >= n_rows_part + n_cols_part)
        return;
    int32_t r, c;
    if (k < n_rows_part) {
        r = (k < a.in_w) ? 0 : a.in_h - 1;
        c = k % a.in_w;
    } else {
        const int32_t j = k - n_rows_part;
        r = 1 + j % inner;
        c = (j < inner) ? 0 : a.in_w - 1;
    }
    const int32_t y_lo = first_output<FILTER>(r, a.in_h, a.out_h);
    const int32_t y_hi = last_output<FILTER>(r, a.in_h, a.out_h);
    const int32_t x_lo = first_output<FILTER>(c, a.in_w, a.out_w);
    const int32_t x_hi = last_output<FILTER>(c, a.in_w, a.out_w);
    const unsigned char *gsrc = a.src + static_cast<int64_t>(blockIdx.y) * a.src_plane_pitch;
    float extra[C];
#pragma unroll
    for (int ch = 0; ch < C; ++ch)
        extra[ch] = 0.0f;
    for (int32_t y = y_lo; y <= y_hi; ++y) {
        int32_t y0;
        float ty, uy;
        axis_tap(y, a.in_h, a.out_h, 1, y0, ty, uy);
        float wy[K];
        weights<FILTER>(ty, uy, wy);
        const unsigned char *grow = gsrc + static_cast<int64_t>(y) * a.src_pitch;
        for (int32_t x = x_lo; x <= x_hi; ++x) {
            int32_t x0;
            float tx, ux;
            axis_tap(x, a.in_w, a.out_w, 1, x0, tx, ux);
            float wx[K];
            weights<FILTER>(tx, ux, wx);
            float w = 0.0f;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int32_t ry = y0 + TP::LO + j;
                if (clampi(ry, 0, a.in_h - 1) != r)
                    continue;
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const int32_t cx = x0 + TP::LO + i;
                    if (clampi(cx, 0, a.in_w - 1) == c && (kFull || ry != r || cx != c))
                        w += wy[j] * wx[i];
                }
            }
            if (w != 0.0f) {
                float g[C];
                Pix<T, C>::load(grow, x, g);
#pragma unroll
                for (int ch = 0; ch < C; ++ch)
                    extra[ch] = __builtin_fmaf(w, g[ch], extra[ch]);
            }
        }
    }
    unsigned char *orow = a.dst + static_cast<int64_t>(blockIdx.y) * a.dst_plane_pitch +
                          static_cast<int64_t>(r) * a.dst_pitch;
    if constexpr (kFull) {
        Pix<T, C>::store(orow, c, extra);
    } else {
        float *out = reinterpret_cast<float *>(orow) + c * C;
#pragma unroll
        for (int ch = 0; ch < C; ++ch)
            out[ch] += extra[ch];
    }
}

template <int FILTER, typename T, int C>
hipError_t launch_bwd_up2(const ResizeArgs &a, hipStream_t stream)
{
    constexpr int P = (C == 1) ? 4 : 1;
    constexpr int32_t kStrip = 16;
    const int32_t cols_per_block = 256 * P;
    hipLaunchKernelGGL((k_bwd_up2<FILTER, T, C, P>),
                       dim3((a.in_w + cols_per_block - 1) / cols_per_block, (a.in_h + kStrip - 1) / kStrip,
                            a.planes),
                       dim3(256), 0, stream, a, kStrip);
    const int32_t inner = a.in_h > 2 ? a.in_h - 2 : 0;
    const int32_t border = ((a.in_h > 1) ? 2 * a.in_w : a.in_w) + ((a.in_w > 1) ? 2 * inner : inner);
    hipLaunchKernelGGL((k_bwd_up2_border<FILTER, T, C>), dim3((border + 255) / 256, a.planes), dim3(256), 0,
                       stream, a);
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
