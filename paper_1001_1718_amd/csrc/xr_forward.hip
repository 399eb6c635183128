// Forward resize kernels for gfx950.
//
//  k_gather     one thread per output pixel; a workgroup of block_w x block_h
//               threads covers a block_w x block_h tile (paper section III.A,
//               eq. 6). Every tap is read from memory. Kept as the paper's
//               own tiling, for the tile-shape study and as a reference
//               launch shape.
//  k_strip      each thread owns ppt_x adjacent output columns and walks a
//               strip of ppt_y output rows. The horizontally filtered source
//               rows (the inner sums of eq. 5) are kept in a ring of K
//               registers and reused by every output row that needs them, so
//               a source row is filtered once per strip instead of K times.
//  k_x2         the walk specialised for an exact x2 upscale on both axes:
//               output columns/rows alternate between t = 3/4 and t = 1/4, a
//               thread's ppt_x columns read one contiguous run of ppt_x/2 + K
//               source pixels, every source row completes a pair of output
//               rows, and every memory access goes through a buffer resource
//               so no branch separates the walk's loads and stores.
//  k_x05        the walk for an exact x0.5 on both axes: t = 1/2
//               everywhere, a contiguous run of 2 ppt_x - 2 + K source
//               pixels per row, two source rows per output row, with the
//               buffer-resource loads and stores of k_x2.
//  k_strip_lds  any scale, each source row staged once per workgroup in LDS.
//  k_batch_walk persistent launches over the tiles of many jobs, one per job
//               kind (filter x channels); one window load per column and
//               row weights from a per-wavefront LDS table.
//  k_gather_aa, k_tile_aa  the antialiased filters (support stretched when
//               shrinking): one pixel per thread from memory, or the block's
//               source window staged in LDS and filtered separably.
//
// The bilinear and bicubic kernels evaluate each output with the same float32
// operation sequence (xr_device.hpp), so their results are bit-identical; so
// are the two antialiased kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "xr_buffer.hpp"
#include "xr_device.hpp"
#include "xr_internal.h"

namespace xr {
using namespace dev;

// ---------------------------------------------------------------------------
// helpers: contiguous runs of pixels
// ---------------------------------------------------------------------------

// Storage type code of a pixel type.
template <typename T>
struct DType;
template <>
struct DType<uint8_t> {
    static constexpr int32_t kCode = XR_U8;
};
template <>
struct DType<_Float16> {
    static constexpr int32_t kCode = XR_F16;
};
template <>
struct DType<float> {
    static constexpr int32_t kCode = XR_F32;
};

template <typename T, int C>
struct PixRaw {
    static constexpr int kBytes = Pix<T, C>::kBytes;
};

// Decode pixel `i` of a byte buffer into floats.
template <typename T, int C>
__device__ __forceinline__ void decode(const unsigned char *buf, int i, float (&v)[C])
{
    Pix<T, C>::load(buf, i, v);
}


template <int BYTES, int ALIGN>
__device__ __forceinline__ RawBuf<BYTES, ALIGN> load_raw(const unsigned char *p)
{
    return *reinterpret_cast<const RawBuf<BYTES, ALIGN> *>(__builtin_assume_aligned(p, ALIGN));
}

template <int BYTES, int ALIGN>
__device__ __forceinline__ void store_raw(unsigned char *p, const RawBuf<BYTES, ALIGN> &v)
{
    *reinterpret_cast<RawBuf<BYTES, ALIGN> *>(__builtin_assume_aligned(p, ALIGN)) = v;
}

// Store of an output run that is written once and not read back by this
// launch: non-temporal vector stores (they do not keep the lines in the
// caches, which leaves room there for the source rows that neighbouring
// strips re-read; measured faster for the x2 walk).
template <int BYTES, int ALIGN>
__device__ __forceinline__ void store_stream(unsigned char *p, const RawBuf<BYTES, ALIGN> &v)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    if constexpr (ALIGN >= 16 && BYTES % 16 == 0) {
#pragma unroll
        for (int i = 0; i < BYTES / 16; ++i)
            __builtin_nontemporal_store(*reinterpret_cast<const u32x4 *>(v.b + 16 * i),
                                        reinterpret_cast<u32x4 *>(__builtin_assume_aligned(p, 16)) + i);
    } else if constexpr (ALIGN >= 8 && BYTES % 8 == 0) {
#pragma unroll
        for (int i = 0; i < BYTES / 8; ++i)
            __builtin_nontemporal_store(*reinterpret_cast<const u32x2 *>(v.b + 8 * i),
                                        reinterpret_cast<u32x2 *>(__builtin_assume_aligned(p, 8)) + i);
    } else if constexpr (ALIGN >= 4 && BYTES % 4 == 0) {
#pragma unroll
        for (int i = 0; i < BYTES / 4; ++i)
            __builtin_nontemporal_store(*reinterpret_cast<const uint32_t *>(v.b + 4 * i),
                                        reinterpret_cast<uint32_t *>(__builtin_assume_aligned(p, 4)) + i);
    } else {
        store_raw<BYTES, ALIGN>(p, v);
    }
}


// Encode N pixels into a byte buffer (uint8 pixels four to a dword).
template <typename T, int C, int N, int BYTES, int ALIGN>
__device__ __forceinline__ void encode_run(const float (&v)[N][C], RawBuf<BYTES, ALIGN> &out)
{
    if constexpr (std::is_same<T, uint8_t>::value && C == 1 && N % 4 == 0) {
#pragma unroll
        for (int g = 0; g < N / 4; ++g) {
            uint32_t r = u8_insert(v[4 * g][0], 0, 0u);
            r = u8_insert(v[4 * g + 1][0], 1, r);
            r = u8_insert(v[4 * g + 2][0], 2, r);
            r = u8_insert(v[4 * g + 3][0], 3, r);
            *reinterpret_cast<uint32_t *>(out.b + 4 * g) = r;
        }
    } else {
#pragma unroll
        for (int c = 0; c < N; ++c)
            Pix<T, C>::store(out.b, c, v[c]);
    }
}


// ---------------------------------------------------------------------------
// k_gather
// ---------------------------------------------------------------------------

template <int FILTER, typename T, int C>
__global__ void __launch_bounds__(1024) k_gather(ResizeArgs a)
{
    using TP = Taps<FILTER>;
    constexpr int K = TP::K;
    const int32_t px = blockIdx.x * blockDim.x + threadIdx.x;  // eq. 6
    const int32_t py = blockIdx.y * blockDim.y + threadIdx.y;
    if (px >= a.out_w || py >= a.dst_rows)
        return;
    const int32_t plane = blockIdx.z;
    int32_t x0, y0;
    float tx, ty, ux, uy;
    source_tap<FILTER>(px, a.in_w, a.out_w, a.map_off, x0, tx, ux);
    source_tap<FILTER>(a.dst_row0 + py, a.in_h, a.out_h, a.map_off, y0, ty, uy);
    float wx[K], wy[K];
    weights<FILTER>(tx, ux, wx);
    weights<FILTER>(ty, uy, wy);
    int32_t ix[K];
#pragma unroll
    for (int i = 0; i < K; ++i)
        ix[i] = clampi(x0 + TP::LO + i, 0, a.in_w - 1);
    const unsigned char *src = a.src + static_cast<int64_t>(plane) * a.src_plane_pitch;
    float acc[C];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int32_t r = clampi(y0 + TP::LO + j, 0, a.in_h - 1) - a.src_row0;
        const unsigned char *row = src + static_cast<int64_t>(r) * a.src_pitch;
        float h[C], p[C];
        Pix<T, C>::load(row, ix[0], p);
        fma_first(h, wx[0], p);
#pragma unroll
        for (int i = 1; i < K; ++i) {
            Pix<T, C>::load(row, ix[i], p);
            fma_next(h, wx[i], p);
        }
        if (j == 0)
            fma_first(acc, wy[0], h);
        else
            fma_next(acc, wy[j], h);
    }
    unsigned char *dst = a.dst + static_cast<int64_t>(plane) * a.dst_plane_pitch +
                         static_cast<int64_t>(py) * a.dst_pitch;
    Pix<T, C>::store(dst, px, acc);
}

// ---------------------------------------------------------------------------
// k_gather_aa (antialiased: filter stretched by the shrink factor)
// ---------------------------------------------------------------------------

// Taps of output index x for an antialiased filter of radius R (1 bilinear,
// 2 Keys): sigma = max(1, n_in / n_out), every source i with
// s - R sigma < i <= s + R sigma inside [0, n_in - 1], from exact integers
// (s = num / (2 n_out), num = (2x + 1) n_in - n_out). Not in the paper: the
// usual remedy for aliasing when shrinking.
__device__ __forceinline__ void aa_range(int32_t x, int32_t n_in, int32_t n_out, int32_t r,
                                         int32_t &lo, int32_t &hi)
{
    const int64_t num = (2 * static_cast<int64_t>(x) + 1) * n_in - n_out;
    const int64_t den = 2 * static_cast<int64_t>(n_out);
    const int64_t reach = 2 * static_cast<int64_t>(r) * (n_in > n_out ? n_in : n_out);
    // floor division of possibly negative numerators
    auto fdiv = [](int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
    lo = static_cast<int32_t>(max<int64_t>(fdiv(num - reach, den) + 1, 0));
    hi = static_cast<int32_t>(min<int64_t>(fdiv(num + reach, den), n_in - 1));
}

// K(d) in factored forms whose factors do not cancel: 1 - u; Keys a = -1/2
// as (1 - u)(1 + u (1 - 3u/2)) for u <= 1 and -(u - 1)(u - 2)^2 / 2 for
// 1 < u < 2 (u - 1 and u - 2 are exact there).
template <int R>
__device__ __forceinline__ float aa_kernel(float d)
{
    const float u = fabsf(d);
    if constexpr (R == 1) {
        return u < 1.0f ? 1.0f - u : 0.0f;
    } else {
        if (u <= 1.0f)
            return (1.0f - u) * (1.0f + u * (1.0f - 1.5f * u));
        if (u < 2.0f) {
            const float v = u - 2.0f;
            return (-0.5f * (u - 1.0f)) * (v * v);
        }
        return 0.0f;
    }
}

// Taps and normalised weights of one output index into an LDS table: the
// kernel values K((i - s) / sigma) for i = lo .. hi, then each divided by
// their sum (summed in ascending i).
template <int R>
__device__ __forceinline__ void aa_table(int32_t x, int32_t n_in, int32_t n_out, int32_t kmax,
                                         int32_t *lo_out, int32_t *n_out_taps, float *w)
{
    int32_t lo, hi;
    aa_range(x, n_in, n_out, R, lo, hi);
    const int32_t n = min(hi - lo + 1, kmax);
    // (i - s) / sigma = (2 i n_out - num) / (2 max(n_in, n_out)) from exact
    // integers: one rounding, no cancellation
    const int64_t num = (2 * static_cast<int64_t>(x) + 1) * n_in - n_out;
    const float den = static_cast<float>(2 * static_cast<int64_t>(n_in > n_out ? n_in : n_out));
    float sum = 0.0f;
    for (int32_t k = 0; k < n; ++k) {
        const int64_t dn = 2 * static_cast<int64_t>(lo + k) * n_out - num;
        const float v = aa_kernel<R>(static_cast<float>(dn) / den);
        w[k] = v;
        sum += v;
    }
    const float inv = 1.0f / sum;
    for (int32_t k = 0; k < n; ++k)
        w[k] *= inv;
    *lo_out = lo;
    *n_out_taps = n;
}

// One output pixel per thread in a block_w x block_h tile (the paper's
// tiling, eq. 6). The workgroup first fills LDS tables of taps and weights
// for its block_w columns and block_h rows (kx / ky weights each), then every
// thread sums its window: per source row the taps ascending (multiply, then
// FMAs), then the rows ascending.
template <int R, typename T, int C>
__global__ void __launch_bounds__(1024) k_gather_aa(ResizeArgs a, int32_t kx, int32_t ky)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int32_t bw = static_cast<int32_t>(blockDim.x), bh = static_cast<int32_t>(blockDim.y);
    int32_t *xlo = reinterpret_cast<int32_t *>(lds);
    int32_t *xn = xlo + bw;
    int32_t *ylo = xn + bw;
    int32_t *yn = ylo + bh;
    float *xw = reinterpret_cast<float *>(yn + bh);
    float *yw = xw + bw * kx;
    const int32_t tid = threadIdx.y * bw + threadIdx.x;
    for (int32_t t = tid; t < bw + bh; t += bw * bh) {
        if (t < bw) {
            const int32_t x = min(static_cast<int32_t>(blockIdx.x) * bw + t, a.out_w - 1);
            aa_table<R>(x, a.in_w, a.out_w, kx, xlo + t, xn + t, xw + t * kx);
        } else {
            const int32_t u = t - bw;
            const int32_t y = a.dst_row0 + min(static_cast<int32_t>(blockIdx.y) * bh + u, a.dst_rows - 1);
            aa_table<R>(y, a.in_h, a.out_h, ky, ylo + u, yn + u, yw + u * ky);
        }
    }
    __syncthreads();
    const int32_t px = blockIdx.x * bw + threadIdx.x;
    const int32_t py = blockIdx.y * bh + threadIdx.y;
    if (px >= a.out_w || py >= a.dst_rows)
        return;
    const unsigned char *src = a.src + static_cast<int64_t>(blockIdx.z) * a.src_plane_pitch;
    const int32_t x0 = xlo[threadIdx.x], nx = xn[threadIdx.x];
    const int32_t y0 = ylo[threadIdx.y], ny = yn[threadIdx.y];
    const float *wxr = xw + threadIdx.x * kx;
    const float *wyr = yw + threadIdx.y * ky;
    float acc[C];
    for (int32_t j = 0; j < ny; ++j) {
        const unsigned char *row = src + static_cast<int64_t>(y0 + j - a.src_row0) * a.src_pitch;
        float h[C], p[C];
        Pix<T, C>::load(row, x0, p);
        fma_first(h, wxr[0], p);
        for (int32_t i = 1; i < nx; ++i) {
            Pix<T, C>::load(row, x0 + i, p);
            fma_next(h, wxr[i], p);
        }
        if (j == 0)
            fma_first(acc, wyr[0], h);
        else
            fma_next(acc, wyr[j], h);
    }
    unsigned char *dst = a.dst + static_cast<int64_t>(blockIdx.z) * a.dst_plane_pitch +
                         static_cast<int64_t>(py) * a.dst_pitch;
    Pix<T, C>::store(dst, px, acc);
}

// ---------------------------------------------------------------------------
// k_strip (any scale)
// ---------------------------------------------------------------------------

// Copy one pixel of PB bytes between PB-aligned addresses.
template <int PB>
__device__ __forceinline__ void copy_pixel(unsigned char *dst, const unsigned char *src)
{
    if constexpr (PB == 1) {
        *dst = *src;
    } else if constexpr (PB == 2) {
        *reinterpret_cast<uint16_t *>(dst) = *reinterpret_cast<const uint16_t *>(src);
    } else if constexpr (PB == 4) {
        *reinterpret_cast<uint32_t *>(dst) = *reinterpret_cast<const uint32_t *>(src);
    } else if constexpr (PB == 8) {
        *reinterpret_cast<uint2 *>(dst) = *reinterpret_cast<const uint2 *>(src);
    } else {
        *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(src);
    }
}

// The antialiased filter on block_w x block_h tiles of output pixels with
// the source window staged in LDS (separable). A workgroup takes `tpb`
// vertically adjacent tiles of one tile column: the column tables (taps and
// kx weights per output column, the same as k_gather_aa's) are built once,
// the row tables once per tile. Per tile the source window (rows ylo(first)
// .. yhi(last), columns xlo(first) .. xhi(last)) is copied to LDS with
// coalesced loads, the horizontal pass filters every window row for every
// tile column into an LDS row buffer, and each thread then sums its rows. Per
// pixel the float32 sequence is exactly k_gather_aa's (taps ascending per
// row, rows ascending), so the two kernels agree bit for bit. The window is
// at most win_w x win_h pixels (bounded on the host from the scale).
constexpr int kAaRegTaps = 12;  // register-held horizontal weights (bicubic to 1/2.75)
constexpr int32_t kAaTilesPerBlock = 4;  // most tiles a workgroup walks down its column
constexpr int64_t kAaMinBlocks = 1024;    // workgroups the multi-tile grid keeps

template <int R, typename T, int C>
__global__ void __launch_bounds__(1024) k_tile_aa(ResizeArgs a, int32_t kx, int32_t ky, int32_t win_w,
                                                  int32_t win_h, int32_t tpb)
{
    constexpr int PB = Pix<T, C>::kBytes;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int32_t bw = static_cast<int32_t>(blockDim.x), bh = static_cast<int32_t>(blockDim.y);
    const int32_t nthreads = bw * bh;
    int32_t *xlo = reinterpret_cast<int32_t *>(lds);
    int32_t *xn = xlo + bw;
    int32_t *ylo = xn + bw;
    int32_t *yn = ylo + bh;
    float *xw = reinterpret_cast<float *>(yn + bh);
    float *yw = xw + bw * kx;
    const int64_t table_bytes = 4 * (2 * static_cast<int64_t>(bw) + 2 * bh +
                                     static_cast<int64_t>(bw) * kx + static_cast<int64_t>(bh) * ky);
    unsigned char *win = lds + (table_bytes + 15) / 16 * 16;
    float *hbuf = reinterpret_cast<float *>(win + (static_cast<int64_t>(win_w) * win_h * PB + 15) / 16 * 16);
    const int32_t tid = threadIdx.y * bw + threadIdx.x;
    const unsigned char *src = a.src + static_cast<int64_t>(blockIdx.z) * a.src_plane_pitch;
    const int32_t n_tiles_y = (a.dst_rows + bh - 1) / bh;
    const int32_t tile_end = min(static_cast<int32_t>(blockIdx.y + 1) * tpb, n_tiles_y);
    // Every bound below is uniform over the workgroup, and no thread leaves
    // the loop early, so every thread reaches every barrier.
    for (int32_t by = static_cast<int32_t>(blockIdx.y) * tpb; by < tile_end; ++by) {
        const bool first = by == static_cast<int32_t>(blockIdx.y) * tpb;
        for (int32_t t = tid + (first ? 0 : bw); t < bw + bh; t += nthreads) {
            if (t < bw) {
                const int32_t x = min(static_cast<int32_t>(blockIdx.x) * bw + t, a.out_w - 1);
                aa_table<R>(x, a.in_w, a.out_w, kx, xlo + t, xn + t, xw + t * kx);
            } else {
                const int32_t u = t - bw;
                const int32_t y = a.dst_row0 + min(by * bh + u, a.dst_rows - 1);
                aa_table<R>(y, a.in_h, a.out_h, ky, ylo + u, yn + u, yw + u * ky);
            }
        }
        __syncthreads();
        // the tile's source window (tap ranges are monotone in x and y)
        const int32_t wx0 = xlo[0];
        const int32_t ww = min(xlo[bw - 1] + xn[bw - 1] - wx0, win_w);
        const int32_t wy0 = ylo[0];
        const int32_t wh = min(ylo[bh - 1] + yn[bh - 1] - wy0, win_h);
        // NB loads in flight per thread before any LDS store. Element i of the
        // window is (i / ww, i % ww); a thread's elements step by nthreads,
        // i.e. by dr rows and dc columns with a carry, so no division per
        // element.
        constexpr int NB = 8;
        const int32_t total = ww * wh;
        const int32_t dr = nthreads / ww, dc = nthreads - dr * ww;
        int32_t r = tid / ww, c = tid - (tid / ww) * ww;
        const unsigned char *wsrc = src + static_cast<int64_t>(wy0 - a.src_row0) * a.src_pitch +
                                    static_cast<int64_t>(wx0) * PB;
        for (int32_t base = tid; base < total; base += nthreads * NB) {
            RawBuf<PB, PB> v[NB];
            int32_t off[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                // past the end: reload the window's last element (a valid address)
                const bool in = base + k * nthreads < total;
                const int32_t rr = in ? r : wh - 1, cc = in ? c : ww - 1;
                off[k] = (rr * win_w + cc) * PB;
                v[k] = load_raw<PB, PB>(wsrc + static_cast<int64_t>(rr) * a.src_pitch + cc * PB);
                c += dc;
                r += dr + (c >= ww ? 1 : 0);
                c -= c >= ww ? ww : 0;
            }
#pragma unroll
            for (int k = 0; k < NB; ++k)
                if (base + k * nthreads < total)
                    store_raw<PB, PB>(win + off[k], v[k]);
        }
        __syncthreads();
        // horizontal pass: window row r, tile column hc (threads of one
        // column take rows ty, ty + bh, ...). A column's weights are the same
        // on every row, so up to kAaRegTaps of them are held in registers.
        const int32_t hc = threadIdx.x;
        const int32_t hx0 = xlo[hc] - wx0, hnx = xn[hc];
        const float *hwx = xw + hc * kx;
        if (kx <= kAaRegTaps) {
            float wr[kAaRegTaps];
#pragma unroll
            for (int k = 0; k < kAaRegTaps; ++k)
                wr[k] = k < hnx ? hwx[k] : 0.0f;
            for (int32_t rr = threadIdx.y; rr < wh; rr += bh) {
                const unsigned char *wrow = win + static_cast<int64_t>(rr) * win_w * PB;
                float h[C], p[C];
                Pix<T, C>::load(wrow, hx0, p);
                fma_first(h, wr[0], p);
#pragma unroll
                for (int k = 1; k < kAaRegTaps; ++k) {
                    if (k < hnx) {
                        Pix<T, C>::load(wrow, hx0 + k, p);
                        fma_next(h, wr[k], p);
                    }
                }
                float *hp = hbuf + (static_cast<int64_t>(rr) * bw + hc) * C;
#pragma unroll
                for (int ch = 0; ch < C; ++ch)
                    hp[ch] = h[ch];
            }
        } else {
            for (int32_t rr = threadIdx.y; rr < wh; rr += bh) {
                const unsigned char *wrow = win + static_cast<int64_t>(rr) * win_w * PB;
                float h[C], p[C];
                Pix<T, C>::load(wrow, hx0, p);
                fma_first(h, hwx[0], p);
                for (int32_t k = 1; k < hnx; ++k) {
                    Pix<T, C>::load(wrow, hx0 + k, p);
                    fma_next(h, hwx[k], p);
                }
                float *hp = hbuf + (static_cast<int64_t>(rr) * bw + hc) * C;
#pragma unroll
                for (int ch = 0; ch < C; ++ch)
                    hp[ch] = h[ch];
            }
        }
        __syncthreads();
        const int32_t px = blockIdx.x * bw + threadIdx.x;
        const int32_t py = by * bh + threadIdx.y;
        if (px < a.out_w && py < a.dst_rows) {
            const int32_t r0 = ylo[threadIdx.y] - wy0, ny = yn[threadIdx.y];
            const float *wyr = yw + threadIdx.y * ky;
            float acc[C], h[C];
            for (int32_t j = 0; j < ny; ++j) {
                const float *hp = hbuf + (static_cast<int64_t>(r0 + j) * bw + threadIdx.x) * C;
#pragma unroll
                for (int ch = 0; ch < C; ++ch)
                    h[ch] = hp[ch];
                if (j == 0)
                    fma_first(acc, wyr[0], h);
                else
                    fma_next(acc, wyr[j], h);
            }
            unsigned char *dst = a.dst + static_cast<int64_t>(blockIdx.z) * a.dst_plane_pitch +
                                 static_cast<int64_t>(py) * a.dst_pitch;
            Pix<T, C>::store(dst, px, acc);
        }
        // the next tile rewrites the row tables, the window and the row buffer
        __syncthreads();
    }
}

// Any scale: a thread owns PPX adjacent output columns (each with its own
// taps) and walks the source rows its strip of output rows reads, in order.
// Each source row is filtered once into ring slot (row - first row) mod K;
// an output row is emitted as soon as its last tap row has been filtered,
// reading its K rows from slots that are constants of the 4-row unrolled
// walk. The PPX*K tap pixels of the row PD rows ahead are requested before
// the current row is filtered.
template <int FILTER, typename T, int C, int PPX>
struct StripBody {
    using TP = Taps<FILTER>;
    static constexpr int K = TP::K;
    static constexpr int PB = Pix<T, C>::kBytes;
    static constexpr int ROWB = PPX * K * PB;       // tap bytes per source row
    static constexpr int PD = ROWB <= 32 ? 3 : 1;   // prefetch distance in rows
    static constexpr int Q = PD + 1;                // divides 4
    using Raw = RawBuf<ROWB, PB>;

    int32_t ixb[PPX][K];  // byte offsets of the clamped tap columns
    float wx[PPX][K];
    float ring[K][PPX][C];
    Raw rawq[Q];

    __device__ __forceinline__ Raw load_row(const ResizeArgs &a, const unsigned char *src,
                                            int32_t r) const
    {
        // clamped into the stored band (which holds every needed row)
        const int32_t rr = clampi(r, a.src_row0, a.src_row0 + a.src_rows - 1) - a.src_row0;
        const unsigned char *row = src + static_cast<int64_t>(rr) * a.src_pitch;
        Raw raw;
#pragma unroll
        for (int c = 0; c < PPX; ++c)
#pragma unroll
            for (int i = 0; i < K; ++i)
                copy_pixel<PB>(raw.b + (c * K + i) * PB, row + ixb[c][i]);
        return raw;
    }

    __device__ __forceinline__ void hfilter(const Raw &raw, float (&out)[PPX][C]) const
    {
#pragma unroll
        for (int c = 0; c < PPX; ++c) {
            float p[C];
            decode<T, C>(raw.b, c * K, p);
            fma_first(out[c], wx[c][0], p);
#pragma unroll
            for (int i = 1; i < K; ++i) {
                decode<T, C>(raw.b, c * K + i, p);
                fma_next(out[c], wx[c][i], p);
            }
        }
    }

    // Process output rows [r_begin, r_end) (band coordinates) of one plane for
    // the PPX columns starting at col0.
    __device__ __forceinline__ void run(const ResizeArgs &a, int32_t plane, int32_t col0,
                                        int32_t r_begin, int32_t r_end)
    {
#pragma unroll
        for (int c = 0; c < PPX; ++c) {
            const int32_t x = min(col0 + c, a.out_w - 1);
            int32_t x0;
            float t, u;
            source_tap<FILTER>(x, a.in_w, a.out_w, a.map_off, x0, t, u);
            weights<FILTER>(t, u, wx[c]);
#pragma unroll
            for (int i = 0; i < K; ++i)
                ixb[c][i] = clampi(x0 + TP::LO + i, 0, a.in_w - 1) * PB;
        }
        const unsigned char *src = a.src + static_cast<int64_t>(plane) * a.src_plane_pitch;
        unsigned char *dst = a.dst + static_cast<int64_t>(plane) * a.dst_plane_pitch;
        const int32_t ncols = min(PPX, a.out_w - col0);
        // the whole run of PPX pixels is inside the row and aligned for one
        // vector store (PPX * PB bytes at a multiple of that size)
        const bool full_run = ncols == PPX && a.aligned16;

        int32_t y = a.dst_row0 + r_begin;  // next output row to emit (logical)
        const int32_t y_end = a.dst_row0 + r_end;
        int32_t y0, y0_last;
        float ty, uy, tl, ul;
        // one division per strip: the rows' taps use its reciprocal
        const float rcp_h = __fdiv_rn(1.0f, static_cast<float>(2 * a.out_h));
        source_tap_rcp<FILTER>(y, a.in_h, a.out_h, a.map_off, rcp_h, y0, ty, uy);
        source_tap_rcp<FILTER>(y_end - 1, a.in_h, a.out_h, a.map_off, rcp_h, y0_last, tl, ul);
        float wy[K];
        weights<FILTER>(ty, uy, wy);
        int32_t last = y0 + TP::LO + K - 1;  // last tap row of output y
        const int32_t rho0 = y0 + TP::LO;
        const int32_t rho1 = y0_last + TP::LO + K - 1;

        // emit every output row whose last tap row is rho (ring slot I of rho)
        auto emit_all = [&](auto slot_tag, int32_t rho) {
            constexpr int I = decltype(slot_tag)::value;
            while (y < y_end && last == rho) {
                unsigned char *drow = dst + static_cast<int64_t>(y - a.dst_row0) * a.dst_pitch;
                float v[PPX][C];
#pragma unroll
                for (int c = 0; c < PPX; ++c) {
                    fma_first(v[c], wy[0], ring[(I + 1) % K][c]);
#pragma unroll
                    for (int j = 1; j < K; ++j)
                        fma_next(v[c], wy[j], ring[(I + 1 + j) % K][c]);
                }
                if (full_run) {
                    RawBuf<PPX * PB, cmin(16, PPX * PB)> out;
                    encode_run<T, C, PPX>(v, out);
                    store_stream<PPX * PB, cmin(16, PPX * PB)>(drow + static_cast<int64_t>(col0) * PB, out);
                } else {
#pragma unroll
                    for (int c = 0; c < PPX; ++c)
                        if (c < ncols)
                            Pix<T, C>::store(drow, col0 + c, v[c]);
                }
                ++y;
                if (y < y_end) {
                    source_tap_rcp<FILTER>(y, a.in_h, a.out_h, a.map_off, rcp_h, y0, ty, uy);
                    weights<FILTER>(ty, uy, wy);
                    last = y0 + TP::LO + K - 1;
                }
            }
        };
        // Requests past the last needed row re-read that row (a cache hit)
        // instead of fetching rows this strip never uses.
        auto step = [&](auto slot_tag, int32_t rho) {
            constexpr int I = decltype(slot_tag)::value;
            rawq[(I + PD) % Q] = load_row(a, src, min(rho + PD, rho1));
            if (rho <= rho1) {
                hfilter(rawq[I % Q], ring[I % K]);
                emit_all(slot_tag, rho);
            }
        };
#pragma unroll
        for (int i = 0; i < PD; ++i)
            rawq[i % Q] = load_row(a, src, min(rho0 + i, rho1));
        for (int32_t rho = rho0; rho <= rho1; rho += 4) {
            step(std::integral_constant<int, 0>{}, rho);
            step(std::integral_constant<int, 1>{}, rho + 1);
            step(std::integral_constant<int, 2>{}, rho + 2);
            step(std::integral_constant<int, 3>{}, rho + 3);
        }
    }
};

// Logical tile (bx, by) of this workgroup within its plane. order 0 keeps the
// launch order. order 1 relies on the hardware dealing consecutive workgroups
// to the 8 XCDs in turn and gives XCD k the k-th contiguous band of tiles
// (a bijection for any tile count), so neighbouring tiles share an L2.
__device__ __forceinline__ void tile_coords(int32_t order, int32_t &bx, int32_t &by)
{
    if (order == 0) {
        bx = blockIdx.x;
        by = blockIdx.y;
        return;
    }
    const uint32_t gx = gridDim.x;
    const uint32_t n = gx * gridDim.y;
    const uint32_t h = blockIdx.y * gx + blockIdx.x;
    const uint32_t q = n / 8, r = n % 8;
    const uint32_t xcd = h % 8, slot = h / 8;
    const uint32_t logical = xcd * q + min(xcd, r) + slot;
    bx = static_cast<int32_t>(logical % gx);
    by = static_cast<int32_t>(logical / gx);
}

// Row strip of a thread: threadIdx.y selects one of blockDim.y strips stacked
// vertically in the tile. blockDim.x is a multiple of the wavefront size, so
// the strip is uniform across a wavefront.
__device__ __forceinline__ int32_t strip_begin(int32_t by, int32_t strip_h)
{
    return __builtin_amdgcn_readfirstlane((by * static_cast<int32_t>(blockDim.y) + threadIdx.y) * strip_h);
}

template <int FILTER, typename T, int C, int PPX>
__global__ void __launch_bounds__(512) k_strip(ResizeArgs a, int32_t strip_h, int32_t order)
{
    int32_t bx, by;
    tile_coords(order, bx, by);
    const int32_t col0 = (bx * static_cast<int32_t>(blockDim.x) + threadIdx.x) * PPX;
    const int32_t r_begin = strip_begin(by, strip_h);
    if (col0 >= a.out_w || r_begin >= a.dst_rows)
        return;
    const int32_t r_end = min(r_begin + strip_h, a.dst_rows);
    StripBody<FILTER, T, C, PPX> body;
    body.run(a, blockIdx.z, col0, r_begin, r_end);
}

// ---------------------------------------------------------------------------
// k_strip_lds (any scale, each source row staged once per workgroup in LDS)
// ---------------------------------------------------------------------------

// Staging plan of the LDS strip walk. A lane moves CB-byte chunks: whole
// pixels of 4 bytes or more, else aligned 4-byte words (which needs a 4-byte
// aligned source with rows of a whole number of words). One workgroup of bw
// threads covers cols = min(bw * PPX, out_w) output columns and reads a
// segment of at most seg_max = floor((cols - 1) * in_w / out_w) + K + 1
// source pixels,
// since x0(c2) - x0(c1) <= floor((c2 - c1) * in_w / out_w) + 1 (eqs. 1-4);
// with the word alignment slack that is at most `chunks` chunks, `need`
// chunks per lane, in an LDS row buffer of `buf_bytes`.
template <int FILTER, typename T, int C, int PPX>
struct LdsPlan {
    static constexpr int K = Taps<FILTER>::K;
    static constexpr int PB = Pix<T, C>::kBytes;
    static constexpr int CB = PB < 4 ? 4 : PB;
    static constexpr int MAX_CH = 64 / CB;  // registers for one row's chunks
    int64_t chunks, need, buf_bytes;
    bool ok;
    LdsPlan(int32_t in_w, int32_t out_w, int32_t bw, bool aligned4)
    {
        const int64_t cols = std::min<int64_t>(static_cast<int64_t>(bw) * PPX, out_w);
        const int64_t seg = (cols - 1) * in_w / out_w + K + 1;
        chunks = (seg * PB + (CB - PB) + CB - 1) / CB;
        need = (chunks + bw - 1) / bw;
        buf_bytes = (chunks * CB + 15) / 16 * 16;
        ok = need <= MAX_CH && 3 * buf_bytes <= static_cast<int64_t>(kLdsBudget) &&
             (PB >= 4 || aligned4);
    }
};

// The workgroup is one row strip (block_h = 1): all its threads read the same
// source rows. Per source row, every lane loads CH chunks of the row segment
// (coalesced, clamped into the segment, so the loads are unconditional) and
// writes them to one of three LDS row buffers; after one barrier per row each
// thread gathers its PPX * K taps from LDS, filters them into its ring, and
// emits output rows exactly like k_strip (same weights, same order). Row
// rho + 1 is written to LDS while row rho is filtered; row rho + 2 is in
// flight from memory meanwhile. Every thread of the workgroup runs the same
// loop and barrier sequence (the strip and trip count are uniform; threads
// past the right edge only skip their stores).
template <int FILTER, typename T, int C, int PPX, int CH>
__global__ void __launch_bounds__(512) k_strip_lds(ResizeArgs a, int32_t strip_h, int32_t order,
                                                   int32_t buf_bytes)
{
    using TP = Taps<FILTER>;
    constexpr int K = TP::K;
    constexpr int PB = Pix<T, C>::kBytes;
    constexpr int CB = PB < 4 ? 4 : PB;
    using Chunk = RawBuf<CB, CB>;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];

    int32_t bx, by;
    tile_coords(order, bx, by);
    const int32_t bw = static_cast<int32_t>(blockDim.x);
    const int32_t tid = static_cast<int32_t>(threadIdx.x);
    const int32_t c_first = bx * bw * PPX;
    const int32_t r_begin = by * strip_h;
    if (c_first >= a.out_w || r_begin >= a.dst_rows)  // uniform over the workgroup
        return;
    const int32_t r_end = min(r_begin + strip_h, a.dst_rows);
    const int32_t col0 = c_first + tid * PPX;
    const int32_t c_last = min(c_first + bw * PPX - 1, a.out_w - 1);

    // the workgroup's segment of source columns [seg0, seg1], staged from the
    // chunk-aligned byte seg_b0 on
    int32_t xa, xb;
    float tq, uq;
    source_tap<FILTER>(c_first, a.in_w, a.out_w, a.map_off, xa, tq, uq);
    source_tap<FILTER>(c_last, a.in_w, a.out_w, a.map_off, xb, tq, uq);
    const int32_t seg0 = clampi(xa + TP::LO, 0, a.in_w - 1);
    const int32_t seg1 = clampi(xb + TP::LO + K - 1, 0, a.in_w - 1);
    const int32_t seg_b0 = (seg0 * PB) & ~(CB - 1);
    const int32_t nch = ((seg1 + 1) * PB - seg_b0 + CB - 1) / CB;

    // this thread's taps, as byte offsets into the staged segment
    int32_t toff[PPX][K];
    float wx[PPX][K];
#pragma unroll
    for (int c = 0; c < PPX; ++c) {
        const int32_t x = min(col0 + c, a.out_w - 1);
        int32_t x0;
        float t, u;
        source_tap<FILTER>(x, a.in_w, a.out_w, a.map_off, x0, t, u);
        weights<FILTER>(t, u, wx[c]);
#pragma unroll
        for (int i = 0; i < K; ++i)
            toff[c][i] = clampi(x0 + TP::LO + i, 0, a.in_w - 1) * PB - seg_b0;
    }
    const unsigned char *src = a.src + static_cast<int64_t>(blockIdx.z) * a.src_plane_pitch;
    unsigned char *dst = a.dst + static_cast<int64_t>(blockIdx.z) * a.dst_plane_pitch;
    const int32_t ncols = min(PPX, a.out_w - col0);
    const bool full_run = ncols == PPX && a.aligned16;

    int32_t y = a.dst_row0 + r_begin;  // next output row to emit (logical)
    const int32_t y_end = a.dst_row0 + r_end;
    int32_t y0, y0_last;
    float ty, uy, tl, ul;
    // one division per strip: the rows' taps use its reciprocal
    const float rcp_h = __fdiv_rn(1.0f, static_cast<float>(2 * a.out_h));
    source_tap_rcp<FILTER>(y, a.in_h, a.out_h, a.map_off, rcp_h, y0, ty, uy);
    source_tap_rcp<FILTER>(y_end - 1, a.in_h, a.out_h, a.map_off, rcp_h, y0_last, tl, ul);
    float wy[K];
    weights<FILTER>(ty, uy, wy);
    int32_t last = y0 + TP::LO + K - 1;  // last tap row of output y
    const int32_t rho0 = y0 + TP::LO;
    const int32_t rho1 = y0_last + TP::LO + K - 1;

    Chunk q[CH];
    // the CH chunks of source row rho (clamped into the band, and to rho1:
    // requests past the last needed row re-read it) that this lane stages
    auto fetch = [&](int32_t rho) {
        const int32_t rr = clampi(min(rho, rho1), a.src_row0, a.src_row0 + a.src_rows - 1) - a.src_row0;
        const unsigned char *row = src + static_cast<int64_t>(rr) * a.src_pitch + seg_b0;
#pragma unroll
        for (int k = 0; k < CH; ++k)
            q[k] = load_raw<CB, CB>(row + min(tid + k * bw, nch - 1) * CB);
    };
    auto stage = [&](int32_t buf) {
        unsigned char *b = lds + buf * buf_bytes;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int32_t i = tid + k * bw;
            if (i < nch)
                store_raw<CB, CB>(b + i * CB, q[k]);
        }
    };
    float ring[K][PPX][C];
    auto filter_row = [&](int32_t buf, float (&out)[PPX][C]) {
        const unsigned char *b = lds + buf * buf_bytes;
#pragma unroll
        for (int c = 0; c < PPX; ++c) {
            float p[C];
            Pix<T, C>::load(b + toff[c][0], 0, p);
            fma_first(out[c], wx[c][0], p);
#pragma unroll
            for (int i = 1; i < K; ++i) {
                Pix<T, C>::load(b + toff[c][i], 0, p);
                fma_next(out[c], wx[c][i], p);
            }
        }
    };
    auto emit_all = [&](auto slot_tag, int32_t rho) {
        constexpr int I = decltype(slot_tag)::value;
        while (y < y_end && last == rho) {
            unsigned char *drow = dst + static_cast<int64_t>(y - a.dst_row0) * a.dst_pitch;
            float v[PPX][C];
#pragma unroll
            for (int c = 0; c < PPX; ++c) {
                fma_first(v[c], wy[0], ring[(I + 1) % K][c]);
#pragma unroll
                for (int j = 1; j < K; ++j)
                    fma_next(v[c], wy[j], ring[(I + 1 + j) % K][c]);
            }
            if (full_run) {
                RawBuf<PPX * PB, cmin(16, PPX * PB)> out;
                encode_run<T, C, PPX>(v, out);
                store_stream<PPX * PB, cmin(16, PPX * PB)>(drow + static_cast<int64_t>(col0) * PB, out);
            } else {
#pragma unroll
                for (int c = 0; c < PPX; ++c)
                    if (c < ncols)
                        Pix<T, C>::store(drow, col0 + c, v[c]);
            }
            ++y;
            if (y < y_end) {
                source_tap_rcp<FILTER>(y, a.in_h, a.out_h, a.map_off, rcp_h, y0, ty, uy);
                weights<FILTER>(ty, uy, wy);
                last = y0 + TP::LO + K - 1;
            }
        }
    };
    // Row rho sits in LDS buffer (rho - rho0) mod 3 and ring slot
    // (rho - rho0) mod K. Buffer (b + 1) mod 3 was last read two rows ago,
    // before the previous barrier, so it can be refilled now.
    auto step = [&](auto slot_tag, int32_t rho) {
        constexpr int I = decltype(slot_tag)::value;
        if (rho <= rho1) {  // uniform over the workgroup
            const int32_t b = (rho - rho0) % 3;
            stage(b == 2 ? 0 : b + 1);  // row rho + 1
            fetch(rho + 2);
            __syncthreads();
            filter_row(b, ring[I % K]);
            emit_all(slot_tag, rho);
        }
    };
    fetch(rho0);
    stage(0);
    fetch(rho0 + 1);
    __syncthreads();
    for (int32_t rho = rho0; rho <= rho1; rho += 4) {
        step(std::integral_constant<int, 0>{}, rho);
        step(std::integral_constant<int, 1>{}, rho + 1);
        step(std::integral_constant<int, 2>{}, rho + 2);
        step(std::integral_constant<int, 3>{}, rho + 3);
    }
}

// ---------------------------------------------------------------------------
// edge runs of the exact-ratio walks
// ---------------------------------------------------------------------------
//
// A thread at the image's left or right edge loads its run of N pixels
// (pixels of a multiple of 4 bytes) from column ld0, clamped so the load stays
// inside the row (0 for images narrower than the run). Pixel s of the run
// must be column clamp(run0 + s, 0, in_w - 1): first every loaded pixel past
// the last column repeats its left neighbour, then the window moves right by
// ld0 - run0 pixels (at most MAXL) repeating its first pixel, or left by
// run0 - ld0 (at most MAXR) repeating its last. Lane values only select,
// never index, so the rebuild stays in registers.
template <int N, int PB, int MAXL, int MAXR, int LBYTES>
__device__ __forceinline__ RawBuf<LBYTES, 4> clamp_window(const RawBuf<LBYTES, 4> &in, int32_t run0,
                                                         int32_t ld0, int32_t in_w)
{
    static_assert(PB % 4 == 0 && N * PB <= LBYTES, "whole-dword pixels");
    constexpr int DW = PB / 4;
    uint32_t w[N][DW];
    __builtin_memcpy(w, in.b, N * PB);
    const int32_t last = in_w - 1 - ld0;
#pragma unroll
    for (int t = 1; t < N; ++t)
#pragma unroll
        for (int d = 0; d < DW; ++d)
            w[t][d] = t > last ? w[t - 1][d] : w[t][d];
    const int32_t sh = run0 - ld0;
#pragma unroll
    for (int step = 0; step < MAXL; ++step) {
        const bool go = step < -sh;
#pragma unroll
        for (int t = N - 1; t > 0; --t)
#pragma unroll
            for (int d = 0; d < DW; ++d)
                w[t][d] = go ? w[t - 1][d] : w[t][d];
    }
#pragma unroll
    for (int step = 0; step < MAXR; ++step) {
        const bool go = step < sh;
#pragma unroll
        for (int t = 0; t + 1 < N; ++t)
#pragma unroll
            for (int d = 0; d < DW; ++d)
                w[t][d] = go ? w[t + 1][d] : w[t][d];
    }
    RawBuf<LBYTES, 4> out = in;
    __builtin_memcpy(out.b, w, N * PB);
    return out;
}

// ---------------------------------------------------------------------------
// k_x2 (exact x2 upscale on both axes)
// ---------------------------------------------------------------------------
//
// Output rows pair up as (2m+1, 2m+2): both tap the K source rows
// m+LO .. m+LO+K-1, with t = 1/4 and t = 3/4 (s(y) = (2y - 1)/4). A strip of
// np pairs (np a multiple of 4) filters np + K - 1 source rows, the first
// K - 1 before its first pair, and emits both rows of every pair. A thread
// owns PPX output columns (PPX/2 source columns plus the K/2 taps on either
// side: a run of SPAN source pixels per row).
//
// Every load and store is issued on every step, so the compiler's counts of
// memory operations in flight are exact and each wait covers only the row it
// needs (loads run PD rows ahead):
// * source rows are clamped to the image and the stored band;
// * output rows outside the caller's band fall outside the store resource
//   and are dropped;
// * a thread whose run crosses the left or right image edge loads the run
//   clamped into the row and rebuilds the edge-replicated pixels in
//   registers (pixels of 4 bytes or more), or loads each pixel from its
//   clamped column (1- and 2-byte pixels);
// * a thread whose output run crosses the right image edge has its run store
//   dropped (offset moved past the resource) and stores its pixels one by
//   one.
// The output stores stream past the L2 (kStoreStream). The float32 operation
// order per pixel is the one every kernel uses.
template <int FILTER, typename T, int C, int PPX, int PD>
struct X2Walk {
    using TP = Taps<FILTER>;
    static constexpr int K = TP::K;
    static constexpr int LO = TP::LO;
    static constexpr int M = PPX / 2;
    static constexpr int SPAN = M + K;
    static constexpr int PB = Pix<T, C>::kBytes;
    // a run starts at source column M t - K/2; loads start MIS bytes lower so
    // that they begin on a dword (the same MIS for every interior thread)
    static_assert((M * PB) % 4 == 0, "a thread's run must advance by whole dwords");
    static constexpr int MIS = (4 - ((K / 2) * PB) % 4) % 4;
    static constexpr int LB = (MIS + SPAN * PB + 3) / 4 * 4;  // bytes loaded per row
    static constexpr int OB = PPX * PB;                         // bytes stored per row
    static constexpr int Q = PD + 1;
    static_assert(4 % K == 0 && 4 % Q == 0, "slots repeat every 4 rows");
    using Raw = RawBuf<LB, 4>;

    __amdgpu_buffer_rsrc_t srsrc;
    int32_t row_first;   // logical source row of window row 0 of the strip
    int32_t row_lo, row_hi;  // clamp range (row_lo: the source resource's first row)
    int64_t src_pitch, dst_pitch;
    uint32_t lane_src;   // byte offset of this thread's load within a row (dword aligned)
    int32_t run0, ld0, in_w;  // run: columns run0 .. run0 + SPAN - 1 clamped; edge load at ld0
    bool edge;
    RunStore<T, C, PPX> st;
    int32_t dst_row_off; // strip row of the store resource's first row
    float we[K], wo[K];
    float ring[K][PPX][C];
    Raw rawq[Q];

    __device__ __forceinline__ Raw load_row(int32_t j) const
    {
        const int32_t r = clampi(row_first + j, row_lo, row_hi) - row_lo;
        const uint32_t roff = static_cast<uint32_t>(static_cast<int64_t>(r) * src_pitch);
        Raw raw;
        if constexpr (PB % 4 == 0) {
            buf_load<LB>(raw.b, srsrc, roff + lane_src);
        } else {
            if (!edge) {
                buf_load<LB>(raw.b, srsrc, roff + lane_src);
            } else {
#pragma unroll
                for (int s = 0; s < SPAN; ++s)
                    buf_load_px<PB>(raw.b + MIS + s * PB, srsrc,
                                    roff + static_cast<uint32_t>(clampi(run0 + s, 0, in_w - 1) * PB));
            }
        }
        return raw;
    }

    __device__ __forceinline__ void hfilter(const Raw &loaded, float (&out)[PPX][C]) const
    {
        Raw raw = loaded;
        if constexpr (PB % 4 == 0) {
            if (edge)  // image edge: rebuild the replicated pixels in registers
                raw = clamp_window<SPAN, PB, K / 2, M + K / 2>(loaded, run0, ld0, in_w);
        }
        float p[SPAN][C];
#pragma unroll
        for (int s = 0; s < SPAN; ++s)
            decode<T, C>(raw.b + MIS, s, p[s]);
#pragma unroll
        for (int q = 0; q < M; ++q) {
            fma_first(out[2 * q], we[0], p[q]);
#pragma unroll
            for (int i = 1; i < K; ++i)
                fma_next(out[2 * q], we[i], p[q + i]);
            fma_first(out[2 * q + 1], wo[0], p[q + 1]);
#pragma unroll
            for (int i = 1; i < K; ++i)
                fma_next(out[2 * q + 1], wo[i], p[q + 1 + i]);
        }
    }

    // strip row `row` (0-based; it may lie outside the band) from the window
    // whose oldest row sits in ring slot OLD
    template <int OLD>
    __device__ __forceinline__ void emit_row(int32_t row, const float (&w)[K]) const
    {
        float v[PPX][C];
#pragma unroll
        for (int c = 0; c < PPX; ++c) {
            fma_first(v[c], w[0], ring[OLD % K][c]);
#pragma unroll
            for (int j = 1; j < K; ++j)
                fma_next(v[c], w[j], ring[(OLD + j) % K][c]);
        }
        RawBuf<OB, cmin(16, OB)> out;
        encode_run<T, C, PPX>(v, out);
        st.store(static_cast<uint32_t>(static_cast<int64_t>(row - dst_row_off) * dst_pitch), out);
    }

    // pair k of the strip: source row k + K - 1 completes its window
    template <int I>
    __device__ __forceinline__ void step(int32_t k, int32_t np)
    {
        constexpr int J = I + K - 1;  // window row index mod 4
        rawq[(J + PD) % Q] = load_row(min(k + K - 1 + PD, np + K - 2));
        __builtin_amdgcn_sched_barrier(0);
        hfilter(rawq[J % Q], ring[J % K]);
        emit_row<I>(2 * k, wo);      // row 2m+1, t = 1/4
        emit_row<I>(2 * k + 1, we);  // row 2m+2, t = 3/4
        __builtin_amdgcn_sched_barrier(0);
    }

    __device__ __forceinline__ void run(int32_t np)
    {
        weights<FILTER>(0.75f, 0.25f, we);
        weights<FILTER>(0.25f, 0.75f, wo);
#pragma unroll
        for (int i = 0; i < PD; ++i)
            rawq[i % Q] = load_row(min(i, np + K - 2));
#pragma unroll
        for (int j = 0; j + 1 < K; ++j) {
            rawq[(j + PD) % Q] = load_row(min(j + PD, np + K - 2));
            hfilter(rawq[j % Q], ring[j % K]);
        }
        // the first four pairs ahead of the loop: the loop's waits then see
        // the same rows of loads and stores in flight on every iteration
        step<0>(0, np);
        step<1>(1, np);
        step<2>(2, np);
        step<3>(3, np);
        for (int32_t k = 4; k < np; k += 4) {
            step<0>(k, np);
            step<1>(k + 1, np);
            step<2>(k + 2, np);
            step<3>(k + 3, np);
        }
    }
};

// Rows ahead of use that the x2 walk loads (one row keeps a 4-byte RGBA walk
// at 98 VGPRs, five wavefronts per SIMD; three rows measured the same)
constexpr int kX2Prefetch = 1;

// Strip s of np pairs covers logical output rows [2 s np - 1, 2 (s+1) np - 1);
// threadIdx.y picks one of blockDim.y consecutive strips from s_first on.
template <int FILTER, typename T, int C, int PPX>
__global__ void __launch_bounds__(512) k_x2(ResizeArgs a, int32_t np, int32_t s_first, int32_t order)
{
    int32_t bx, by;
    tile_coords(order, bx, by);
    using W = X2Walk<FILTER, T, C, PPX, kX2Prefetch>;
    constexpr int K = W::K, LO = W::LO, SPAN = W::SPAN, PB = W::PB;
    const int32_t col0 = (bx * static_cast<int32_t>(blockDim.x) + static_cast<int32_t>(threadIdx.x)) * PPX;
    if (!RunStore<T, C, PPX>::kExchange && col0 >= a.out_w)  // (an exchange needs every lane)
        return;
    const int32_t s = s_first + __builtin_amdgcn_readfirstlane(by * static_cast<int32_t>(blockDim.y) +
                                                               static_cast<int32_t>(threadIdx.y));
    const int32_t ys = 2 * s * np - 1;
    const int32_t y_lo = max(ys, max(a.dst_row0, 0));
    const int32_t y_hi = min(ys + 2 * np, min(a.dst_row0 + a.dst_rows, a.out_h));
    if (y_lo >= y_hi)
        return;
    W w;
    // source: the stored band's rows from the strip's first clamped row on
    const int32_t band_lo = max(0, a.src_row0);
    const int32_t band_hi = min(a.in_h - 1, a.src_row0 + a.src_rows - 1);
    w.row_first = s * np - 1 + LO;
    w.row_lo = clampi(w.row_first, band_lo, band_hi);
    w.row_hi = clampi(w.row_first + np + K - 2, band_lo, band_hi);  // the strip's last source row
    w.src_pitch = a.src_pitch;
    const unsigned char *src = a.src + static_cast<int64_t>(blockIdx.z) * a.src_plane_pitch +
                               static_cast<int64_t>(w.row_lo - a.src_row0) * a.src_pitch;
    w.srsrc = buf_rsrc(src, static_cast<uint32_t>(static_cast<int64_t>(w.row_hi - w.row_lo) * a.src_pitch +
                                                  static_cast<int64_t>(a.in_w) * PB));
    w.run0 = col0 / 2 - K / 2;
    w.in_w = a.in_w;
    w.edge = w.run0 < 0 || w.run0 + SPAN > a.in_w;
    w.ld0 = max(0, min(w.run0, a.in_w - SPAN));
    w.lane_src = static_cast<uint32_t>((w.edge && PB % 4 == 0) ? w.ld0 * PB : w.run0 * PB - W::MIS);
    // destination: rows [y_lo, y_hi) of the band
    unsigned char *dst = a.dst + static_cast<int64_t>(blockIdx.z) * a.dst_plane_pitch +
                         static_cast<int64_t>(y_lo - a.dst_row0) * a.dst_pitch;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    w.st.init(buf_rsrc(dst, static_cast<uint32_t>(static_cast<int64_t>(y_hi - y_lo) * a.dst_pitch)), col0,
              a.out_w, static_cast<int32_t>(threadIdx.y * blockDim.x + threadIdx.x), lds);
    w.dst_pitch = a.dst_pitch;
    w.dst_row_off = y_lo - ys;
    w.run(np);
}

// ---------------------------------------------------------------------------
// k_x05 (exact x0.5 on both axes)
// ---------------------------------------------------------------------------
//
// For out = in / 2 every output column and row has s = 2x + 1/2: x0 = 2x and
// t = 1/2, so output x taps source 2x + LO + i with the weights of t = 1/2
// (bicubic (-1, 9, 9, -1) / 16, bilinear (1/2, 1/2)). A thread's PPX columns
// read one run of NEED = 2 PPX - 2 + K source pixels per row; output row y
// reads the K source rows from 2y + LO on, so a strip of nr output rows (nr
// even) filters 2 nr + K - 2 source rows, K - 2 before its first output row,
// into a ring of K, two per output row. Loads and stores are issued on every
// step, through buffer resources, with the edge rules of k_x2: rows clamped on
// load, output rows outside the band dropped by the store resource, edge runs
// rebuilt in registers (or loaded pixel by pixel for 1- and 2-byte pixels),
// right-edge output runs stored pixel by pixel.
template <int FILTER, typename T, int C, int PPX, int PD>
struct D2Walk {
    using TP = Taps<FILTER>;
    static constexpr int K = TP::K;
    static constexpr int LO = TP::LO;
    static constexpr int PB = Pix<T, C>::kBytes;
    static constexpr int NEED = 2 * PPX - 2 + K;
    // a run starts at column 2 col0 + LO; loads start MIS bytes lower, on a dword
    static_assert((2 * PPX * PB) % 4 == 0, "a thread's run must advance by whole dwords");
    static constexpr int MIS = (4 - ((-LO) * PB) % 4) % 4;
    static constexpr int LB = (MIS + NEED * PB + 3) / 4 * 4;
    static constexpr int OB = PPX * PB;
    static constexpr int Q = PD + 1;
    static_assert(4 % K == 0 && 4 % Q == 0, "slots repeat every 4 rows");
    using Raw = RawBuf<LB, 4>;

    __amdgpu_buffer_rsrc_t srsrc;
    int32_t row_first, row_lo, row_hi;
    int64_t src_pitch, dst_pitch;
    uint32_t lane_src;
    int32_t run0, ld0, in_w, dst_row_off;
    bool edge;
    RunStore<T, C, PPX> st;
    float w[K];
    float ring[K][PPX][C];
    Raw rawq[Q];

    __device__ __forceinline__ Raw load_row(int32_t j) const
    {
        const int32_t r = clampi(row_first + j, row_lo, row_hi) - row_lo;
        const uint32_t roff = static_cast<uint32_t>(static_cast<int64_t>(r) * src_pitch);
        Raw raw;
        if constexpr (PB % 4 == 0) {
            buf_load<LB>(raw.b, srsrc, roff + lane_src);
        } else {
            if (!edge) {
                buf_load<LB>(raw.b, srsrc, roff + lane_src);
            } else {
#pragma unroll
                for (int s = 0; s < NEED; ++s)
                    buf_load_px<PB>(raw.b + MIS + s * PB, srsrc,
                                    roff + static_cast<uint32_t>(clampi(run0 + s, 0, in_w - 1) * PB));
            }
        }
        return raw;
    }

    __device__ __forceinline__ void hfilter(const Raw &loaded, float (&out)[PPX][C]) const
    {
        Raw raw = loaded;
        if constexpr (PB % 4 == 0) {
            if (edge)
                raw = clamp_window<NEED, PB, -LO, NEED>(loaded, run0, ld0, in_w);
        }
        float p[NEED][C];
#pragma unroll
        for (int s = 0; s < NEED; ++s)
            decode<T, C>(raw.b + MIS, s, p[s]);
#pragma unroll
        for (int c = 0; c < PPX; ++c) {
            fma_first(out[c], w[0], p[2 * c]);
#pragma unroll
            for (int i = 1; i < K; ++i)
                fma_next(out[c], w[i], p[2 * c + i]);
        }
    }

    // strip row `row` from the window whose oldest row sits in ring slot OLD
    template <int OLD>
    __device__ __forceinline__ void emit_row(int32_t row) const
    {
        float v[PPX][C];
#pragma unroll
        for (int c = 0; c < PPX; ++c) {
            fma_first(v[c], w[0], ring[OLD % K][c]);
#pragma unroll
            for (int j = 1; j < K; ++j)
                fma_next(v[c], w[j], ring[(OLD + j) % K][c]);
        }
        RawBuf<OB, cmin(16, OB)> out;
        encode_run<T, C, PPX>(v, out);
        st.store(static_cast<uint32_t>(static_cast<int64_t>(row - dst_row_off) * dst_pitch), out);
    }

    // filter window row j (slot J mod K), requesting row j + PD first
    template <int J>
    __device__ __forceinline__ void filter(int32_t j, int32_t last)
    {
        rawq[(J + PD) % Q] = load_row(min(j + PD, last));
        __builtin_amdgcn_sched_barrier(0);
        hfilter(rawq[J % Q], ring[J % K]);
    }

    // output row k of the strip: window rows 2k + K - 2 and 2k + K - 1 complete it
    template <int I>  // k mod 2
    __device__ __forceinline__ void step(int32_t k, int32_t last)
    {
        constexpr int J0 = 2 * I + K - 2;  // window row index mod 4
        filter<J0>(2 * k + K - 2, last);
        filter<J0 + 1>(2 * k + K - 1, last);
        emit_row<2 * I>(k);
        __builtin_amdgcn_sched_barrier(0);
    }

    __device__ __forceinline__ void run(int32_t nr)
    {
        weights<FILTER>(0.5f, 0.5f, w);
        const int32_t last = 2 * nr + K - 3;  // the strip's last window row
#pragma unroll
        for (int i = 0; i < PD; ++i)
            rawq[i % Q] = load_row(min(i, last));
        if constexpr (K == 4) {
            filter<0>(0, last);
            filter<1>(1, last);
        }
        step<0>(0, last);
        step<1>(1, last);
        for (int32_t k = 2; k < nr; k += 2) {
            step<0>(k, last);
            step<1>(k + 1, last);
        }
    }
};

constexpr int kX05Prefetch = 1;

// Strip s covers logical output rows [s nr, (s + 1) nr); threadIdx.y picks
// one of blockDim.y consecutive strips from s_first on.
template <int FILTER, typename T, int C, int PPX>
__global__ void __launch_bounds__(512) k_x05(ResizeArgs a, int32_t nr, int32_t s_first, int32_t order)
{
    int32_t bx, by;
    tile_coords(order, bx, by);
    using W = D2Walk<FILTER, T, C, PPX, kX05Prefetch>;
    constexpr int K = W::K, LO = W::LO, NEED = W::NEED, PB = W::PB;
    const int32_t col0 = (bx * static_cast<int32_t>(blockDim.x) + static_cast<int32_t>(threadIdx.x)) * PPX;
    if (!RunStore<T, C, PPX>::kExchange && col0 >= a.out_w)  // (an exchange needs every lane)
        return;
    const int32_t s = s_first + __builtin_amdgcn_readfirstlane(by * static_cast<int32_t>(blockDim.y) +
                                                               static_cast<int32_t>(threadIdx.y));
    const int32_t ys = s * nr;
    const int32_t y_lo = max(ys, max(a.dst_row0, 0));
    const int32_t y_hi = min(ys + nr, min(a.dst_row0 + a.dst_rows, a.out_h));
    if (y_lo >= y_hi)
        return;
    W w;
    const int32_t band_lo = max(0, a.src_row0);
    const int32_t band_hi = min(a.in_h - 1, a.src_row0 + a.src_rows - 1);
    w.row_first = 2 * ys + LO;
    w.row_lo = clampi(w.row_first, band_lo, band_hi);
    w.row_hi = clampi(w.row_first + 2 * nr + K - 3, band_lo, band_hi);
    w.src_pitch = a.src_pitch;
    const unsigned char *src = a.src + static_cast<int64_t>(blockIdx.z) * a.src_plane_pitch +
                               static_cast<int64_t>(w.row_lo - a.src_row0) * a.src_pitch;
    w.srsrc = buf_rsrc(src, static_cast<uint32_t>(static_cast<int64_t>(w.row_hi - w.row_lo) * a.src_pitch +
                                                  static_cast<int64_t>(a.in_w) * PB));
    w.run0 = 2 * col0 + LO;
    w.in_w = a.in_w;
    w.edge = w.run0 < 0 || w.run0 + NEED > a.in_w;
    w.ld0 = max(0, min(w.run0, a.in_w - NEED));
    w.lane_src = static_cast<uint32_t>((w.edge && PB % 4 == 0) ? w.ld0 * PB : w.run0 * PB - W::MIS);
    unsigned char *dst = a.dst + static_cast<int64_t>(blockIdx.z) * a.dst_plane_pitch +
                         static_cast<int64_t>(y_lo - a.dst_row0) * a.dst_pitch;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    w.st.init(buf_rsrc(dst, static_cast<uint32_t>(static_cast<int64_t>(y_hi - y_lo) * a.dst_pitch)), col0,
              a.out_w, static_cast<int32_t>(threadIdx.y * blockDim.x + threadIdx.x), lds);
    w.dst_pitch = a.dst_pitch;
    w.dst_row_off = y_lo - ys;
    w.run(nr);
}

// ---------------------------------------------------------------------------
// k_batch_walk: persistent launches over the tiles of many jobs
// ---------------------------------------------------------------------------
//
// The jobs are grouped by kind (filter x channel count). Each kind has a
// launch of its own, compiled for it (its own columns per thread and register
// budget); the launches follow one another on the stream. Within a kind,
// workgroups take tiles from the kind's ticket counter; its jobs are ordered
// largest first, so long tiles start early and short ones fill the tail. A
// tile is (blockDim.x * PPX) columns by (blockDim.y * strip_h) rows of one
// plane of one job (strip_h per job). The last workgroup of a launch to finish
// resets its kind's counters, so the launches can be replayed (e.g. from a HIP
// graph) without host-side clearing. Jobs whose source is narrower than the
// filter's taps, or whose output is narrower than a run, form a fifth kind
// that runs the per-tap strip walk.
//
// The walk of one thread (SrcWalk) covers PPX adjacent output columns of a
// strip of output rows:
//  * columns: a column's K taps are K adjacent source pixels (eqs. 2-5).
//    Pixels of under 4 bytes are read with one window load of K pixels from
//    the first tap clamped into the row, the taps then picked out of it with
//    byte permutes (the identity away from the image edges); wider pixels
//    with one load per tap at its clamped offset. The last run of a row is
//    moved left to end at the image edge (its pixels are computed twice, to
//    the same bits), so every store writes a whole run;
//  * rows: each source row the strip reads is loaded a few rows ahead and
//    filtered once into ring slot (row mod K), and every output row is
//    emitted as soon as its last tap row is filtered, reading its K rows
//    from slots that are constants of the 4-row unrolled loop; the row taps
//    advance by a constant quotient and remainder (one division per strip),
//    and the rows' weights are computed once per strip, one row per lane,
//    into a table of the wavefront in LDS read back per output row as a
//    broadcast;
//  * memory: loads and stores go through buffer resources over the strip's
//    source rows and output rows.
// The float32 sequence per output value is the one every kernel uses, so
// the results are bit-identical to the single-image launches.

// K pixels (TB bytes) of a column's window; 2-byte windows (one-channel uint8
// bilinear) take one 16-bit load, zero-extended into the window's dword
template <int TB>
__device__ __forceinline__ void buf_load_win(unsigned char *dst, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    if constexpr (TB % 4 == 0) {
        buf_load<TB>(dst, r, off);
    } else {
        static_assert(TB == 2, "2-byte windows");
        const uint32_t v = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
        __builtin_memcpy(dst, &v, 4);
    }
}

// The column side of the batched walk: PPX adjacent output columns of one
// thread, their weights and how their taps are loaded from a source row.
template <int FILTER, typename T, int C, int PPX>
struct ColTaps {
    using TP = Taps<FILTER>;
    static constexpr int K = TP::K;
    static constexpr int PB = Pix<T, C>::kBytes;
    static constexpr int TB = K * PB;                 // tap bytes of a column
    static constexpr int WB = TB < 4 ? 4 : TB;        // their registers
    static constexpr int OB = PPX * PB;
    static constexpr bool kWindow = PB <= 2;
    static constexpr int NS = kWindow ? (TB + 3) / 4 : 1;
    static constexpr int NO = kWindow ? 1 : K;        // load offsets per column
    using Win = RawBuf<WB, 4>;
    using WRow = BatchWeights<K>;

    uint32_t off[PPX][NO];    // byte offsets within a row: the window, or each tap
    uint32_t psel[PPX][NS];   // window: permute selectors of the taps
    float wx[PPX][K];
    __amdgpu_buffer_rsrc_t srsrc;
    int32_t row_lo, row_hi;   // logical source rows the source resource starts and ends with
    uint32_t src_pitch;

    // the taps of source row r (clamped into the resource's rows)
    __device__ __forceinline__ void load_row(Win (&w)[PPX], int32_t r) const
    {
        const int32_t rr = clampi(r, row_lo, row_hi);
        const uint32_t ro = static_cast<uint32_t>(rr - row_lo) * src_pitch;
#pragma unroll
        for (int c = 0; c < PPX; ++c) {
            if constexpr (kWindow) {
                buf_load_win<TB>(w[c].b, srsrc, ro + off[c][0]);
            } else {
#pragma unroll
                for (int i = 0; i < K; ++i)
                    buf_load<PB>(w[c].b + i * PB, srsrc, ro + off[c][i]);
            }
        }
    }

    // window: tap i of column c is pixel clamp(f + i, 0, n_in - 1) - ld of it
    __device__ __forceinline__ void pick(Win (&w)[PPX]) const
    {
        if constexpr (kWindow) {
#pragma unroll
            for (int c = 0; c < PPX; ++c) {
                uint32_t d[2];
                __builtin_memcpy(d, w[c].b, 4);
                d[1] = 0;
                if constexpr (WB >= 8)
                    __builtin_memcpy(&d[1], w[c].b + 4, 4);
                uint32_t r[NS];
#pragma unroll
                for (int k = 0; k < NS; ++k)
                    r[k] = __builtin_amdgcn_perm(d[1], d[0], psel[c][k]);
                __builtin_memcpy(w[c].b, r, 4 * NS);
            }
        }
    }

    // the load offsets (and selectors) of column c, first tap f; the
    // window needs n_in >= K
    __device__ __forceinline__ void make_taps(int c, int32_t f, int32_t in_w)
    {
        if constexpr (kWindow) {
            const int32_t ld = max(0, min(f, in_w - K));
            off[c][0] = static_cast<uint32_t>(ld * PB);
            uint32_t sel[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k)
                sel[k] = 0x0c0c0c0cu;  // bytes past the taps: zero
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const uint32_t idx = static_cast<uint32_t>(clampi(f + i, 0, in_w - 1) - ld);
#pragma unroll
                for (int b = 0; b < PB; ++b) {
                    const int pos = i * PB + b;  // byte of the picked taps
                    const uint32_t from = idx * PB + b;
                    sel[pos / 4] = (sel[pos / 4] & ~(0xffu << (8 * (pos % 4)))) | (from << (8 * (pos % 4)));
                }
            }
#pragma unroll
            for (int k = 0; k < NS; ++k)
                psel[c][k] = sel[k];
        } else {
#pragma unroll
            for (int i = 0; i < K; ++i)
                off[c][i] = static_cast<uint32_t>(clampi(f + i, 0, in_w - 1) * PB);
        }
    }

    __device__ __forceinline__ void hfilter(const Win (&w)[PPX], float (&out)[PPX][C]) const
    {
#pragma unroll
        for (int c = 0; c < PPX; ++c) {
            float p[C];
            decode<T, C>(w[c].b, 0, p);
            fma_first(out[c], wx[c][0], p);
#pragma unroll
            for (int i = 1; i < K; ++i) {
                decode<T, C>(w[c].b, i, p);
                fma_next(out[c], wx[c][i], p);
            }
        }
    }

    // columns c0 .. c0 + PPX - 1 (inside the image)
    __device__ __forceinline__ void set_columns(const ResizeArgs &a, int32_t c0)
    {
#pragma unroll
        for (int c = 0; c < PPX; ++c) {
            int32_t x0;
            float t, u;
            source_tap<FILTER>(c0 + c, a.in_w, a.out_w, a.map_off, x0, t, u);
            weights<FILTER>(t, u, wx[c]);
            make_taps(c, x0 + TP::LO, a.in_w);
        }
    }

    // the source resource over logical rows [lo, hi] clamped into the band
    __device__ __forceinline__ void set_source(const ResizeArgs &a, int32_t plane, int32_t lo, int32_t hi)
    {
        const int32_t band_lo = a.src_row0, band_hi = a.src_row0 + a.src_rows - 1;
        row_lo = clampi(lo, band_lo, band_hi);
        row_hi = clampi(hi, band_lo, band_hi);
        src_pitch = static_cast<uint32_t>(a.src_pitch);
        const unsigned char *sbase = a.src + static_cast<int64_t>(plane) * a.src_plane_pitch +
                                     static_cast<int64_t>(row_lo - a.src_row0) * a.src_pitch;
        srsrc = buf_rsrc(sbase, static_cast<uint32_t>(static_cast<int64_t>(row_hi - row_lo + 1) * a.src_pitch));
    }
};

// The row side of the batched walk: the strip's row taps (one floor
// division for its first and last row, then steps of 2 n_in = sq den + sr)
// and its row weights, computed one row per lane into the wavefront's LDS
// table.
template <int FILTER>
struct RowTaps {
    using TP = Taps<FILTER>;
    static constexpr int K = TP::K;
    using WRow = BatchWeights<K>;
    int32_t den, sq, sr;
    int32_t y_first, rows;

    __device__ __forceinline__ void floor_div(const ResizeArgs &a, int32_t yy, int32_t &qq, int32_t &rr) const
    {
        const int32_t num = (2 * yy + a.map_off) * a.in_h - a.map_off * a.out_h;
        qq = num / den;
        rr = num - qq * den;
        if (rr < 0) {
            qq -= 1;
            rr += den;
        }
    }

    __device__ __forceinline__ void advance(int32_t &q, int32_t &r) const
    {
        r += sr;
        q += sq;
        if (r >= den) {
            r -= den;
            ++q;
        }
    }

    __device__ __forceinline__ void init(const ResizeArgs &a, int32_t r_begin, int32_t r_end, WRow *table,
                                         int32_t tid)
    {
        y_first = a.dst_row0 + r_begin;
        rows = r_end - r_begin;
        den = 2 * a.out_h;
        sq = (2 * a.in_h) / den;
        sr = 2 * a.in_h - sq * den;
        const int32_t lane = tid & 63;
        const float rcp_h = __fdiv_rn(1.0f, static_cast<float>(den));
        for (int32_t base = 0; base < rows; base += 64) {
            const int32_t yy = y_first + min(base + lane, rows - 1);
            int32_t y0;
            float t, u;
            source_tap_rcp<FILTER>(yy, a.in_h, a.out_h, a.map_off, rcp_h, y0, t, u);
            WRow e;
            weights<FILTER>(t, u, e.w);
            if (base + lane < kBatchMaxStrip)
                table[base + lane] = e;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
};

// Cache policy of the batched walk's output stores: non-temporal only. The
// batch's rows start at arbitrary byte offsets, so a wavefront's run covers
// partial lines at both ends; measured on the uneven 256-image batch, plain
// non-temporal stores beat the streaming past-the-L2 policy of the exact
// walks by 8% (and write-back stores by 12%).
constexpr int kBatchStore = 2;

// Source-row driven walk (any scale): each source row the strip reads is
// loaded PD rows ahead, filtered once into ring slot (row mod K), and every
// output row is emitted as soon as its last tap row is filtered, reading its
// K rows from slots that are constants of the 4-row unrolled loop.
template <int FILTER, typename T, int C, int PPX>
struct SrcWalk : ColTaps<FILTER, T, C, PPX> {
    using B = ColTaps<FILTER, T, C, PPX>;
    using typename B::Win;
    using typename B::WRow;
    using TP = Taps<FILTER>;
    static constexpr int K = B::K, PB = B::PB, OB = B::OB, WB = B::WB;
    static constexpr int PD = PPX * WB <= 32 ? 3 : 1;  // rows loaded ahead
    static constexpr int Q = PD + 1;                  // divides 4

    float ring[K][PPX][C];
    Win rawq[Q][PPX];
    float wy[K];
    RowTaps<FILTER> rt;
    const WRow *wt;
    __amdgpu_buffer_rsrc_t drsrc;
    uint32_t dst_off, dst_pitch, lane_off;
    int32_t y, y_end, q, rem, last;

    __device__ __forceinline__ void read_weights()
    {
        const WRow e = wt[min(y - rt.y_first, rt.rows - 1)];
#pragma unroll
        for (int j = 0; j < K; ++j)
            wy[j] = e.w[j];
    }

    template <int I>
    __device__ __forceinline__ void emit()
    {
        float v[PPX][C];
#pragma unroll
        for (int c = 0; c < PPX; ++c) {
            fma_first(v[c], wy[0], ring[(I + 1) % K][c]);
#pragma unroll
            for (int j = 1; j < K; ++j)
                fma_next(v[c], wy[j], ring[(I + 1 + j) % K][c]);
        }
        RawBuf<OB, cmin(16, cgcd(OB, 16))> out;
        encode_run<T, C, PPX>(v, out);
        buf_store<OB, kBatchStore>(out.b, drsrc, dst_off + lane_off);
        ++y;
        dst_off += dst_pitch;
        rt.advance(q, rem);
        last = q + TP::LO + K - 1;
        read_weights();
    }

    template <int I>
    __device__ __forceinline__ void step(int32_t rho, int32_t rho1)
    {
        this->load_row(rawq[(I + PD) % Q], min(rho + PD, rho1));
        if (rho <= rho1) {
            this->pick(rawq[I % Q]);
            this->hfilter(rawq[I % Q], ring[I % K]);
            while (y < y_end && last == rho)
                emit<I>();
        }
    }

    __device__ __forceinline__ void run(const ResizeArgs &a, int32_t plane, int32_t col0, int32_t r_begin,
                                        int32_t r_end, WRow *table, int32_t tid)
    {
        const int32_t c0 = min(col0, a.out_w - PPX);
        lane_off = col0 < a.out_w ? static_cast<uint32_t>(c0 * PB) : 0x80000000u;
        this->set_columns(a, c0);
        rt.init(a, r_begin, r_end, table, tid);
        wt = table;
        y = rt.y_first;
        y_end = y + rt.rows;
        int32_t q_last, r_last;
        rt.floor_div(a, y, q, rem);
        rt.floor_div(a, y_end - 1, q_last, r_last);
        last = q + TP::LO + K - 1;
        read_weights();
        const int32_t rho0 = q + TP::LO;
        const int32_t rho1 = q_last + TP::LO + K - 1;
        this->set_source(a, plane, rho0, rho1);
        unsigned char *dbase = a.dst + static_cast<int64_t>(plane) * a.dst_plane_pitch +
                               static_cast<int64_t>(r_begin) * a.dst_pitch;
        drsrc = buf_rsrc(dbase, static_cast<uint32_t>(static_cast<int64_t>(rt.rows) * a.dst_pitch));
        dst_pitch = static_cast<uint32_t>(a.dst_pitch);
        dst_off = 0;
#pragma unroll
        for (int i = 0; i < PD; ++i)
            this->load_row(rawq[i % Q], min(rho0 + i, rho1));
        for (int32_t rho = rho0; rho <= rho1; rho += 4) {
            step<0>(rho, rho1);
            step<1>(rho + 1, rho1);
            step<2>(rho + 2, rho1);
            step<3>(rho + 3, rho1);
        }
    }
};

template <int FILTER, typename T, int C>
__global__ void __launch_bounds__(256) k_batch_walk(unsigned char *ws, int32_t kind)
{
    constexpr int PPX = batch_ppx(FILTER == kBicubic ? XR_BICUBIC : XR_BILINEAR, DType<T>::kCode, C);
    using W = SrcWalk<FILTER, T, C, PPX>;
    __shared__ typename W::WRow table[4][kBatchMaxStrip];
    __shared__ uint32_t s_tile;
    BatchHeader *hdr = reinterpret_cast<BatchHeader *>(ws);
    const BatchJob *jobs = reinterpret_cast<const BatchJob *>(ws + kBatchHeaderBytes);
    const int64_t total = hdr->tiles[kind];
    const int32_t j_lo = hdr->job_lo[kind], j_hi = hdr->job_hi[kind];
    const int32_t tid = static_cast<int32_t>(threadIdx.y * blockDim.x + threadIdx.x);
    for (;;) {
        if (tid == 0)
            s_tile = atomicAdd(&hdr->ticket[kind], 1u);
        __syncthreads();
        const int64_t tile = static_cast<int64_t>(__builtin_amdgcn_readfirstlane(s_tile));
        __syncthreads();
        if (tile >= total)
            break;
        int32_t lo = j_lo, hi = j_hi - 1;  // last job of the kind whose tile_begin <= tile
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_begin <= tile)
                lo = mid;
            else
                hi = mid - 1;
        }
        const BatchJob &job = jobs[lo];
        const ResizeArgs a = job.a;
        const int64_t local = tile - job.tile_begin;
        const int64_t per_plane = static_cast<int64_t>(job.tiles_x) * job.tiles_y;
        const int32_t plane = static_cast<int32_t>(local / per_plane);
        const int32_t rem = static_cast<int32_t>(local - plane * per_plane);
        const int32_t ty = rem / job.tiles_x;
        const int32_t tx = rem - ty * job.tiles_x;
        const int32_t col0 = (tx * static_cast<int32_t>(blockDim.x) + static_cast<int32_t>(threadIdx.x)) * PPX;
        const int32_t strip_h = job.strip_h;
        const int32_t r_begin =
            __builtin_amdgcn_readfirstlane((ty * static_cast<int32_t>(blockDim.y) + threadIdx.y) * strip_h);
        const int32_t wave_col0 = __builtin_amdgcn_readfirstlane(col0);
        if (wave_col0 < a.out_w && r_begin < a.dst_rows) {
            W w;
            w.run(a, plane, col0, r_begin, min(r_begin + strip_h, a.dst_rows), table[tid >> 6], tid);
        }
    }
    if (tid == 0) {
        __threadfence();
        if (atomicAdd(&hdr->done[kind], 1u) == gridDim.x - 1) {
            atomicExch(&hdr->ticket[kind], 0u);
            atomicExch(&hdr->done[kind], 0u);
        }
    }
}

// Jobs whose source is narrower than the filter's taps or whose output is
// narrower than the walk's run (any filter and channel count): the per-tap
// strip walk, one column per thread.
template <typename T>
__global__ void __launch_bounds__(256) k_batch_narrow(unsigned char *ws)
{
    constexpr int32_t kind = kBatchNarrow;
    __shared__ uint32_t s_tile;
    BatchHeader *hdr = reinterpret_cast<BatchHeader *>(ws);
    const BatchJob *jobs = reinterpret_cast<const BatchJob *>(ws + kBatchHeaderBytes);
    const int64_t total = hdr->tiles[kind];
    const int32_t j_lo = hdr->job_lo[kind], j_hi = hdr->job_hi[kind];
    const int32_t tid = static_cast<int32_t>(threadIdx.y * blockDim.x + threadIdx.x);
    for (;;) {
        if (tid == 0)
            s_tile = atomicAdd(&hdr->ticket[kind], 1u);
        __syncthreads();
        const int64_t tile = static_cast<int64_t>(__builtin_amdgcn_readfirstlane(s_tile));
        __syncthreads();
        if (tile >= total)
            break;
        int32_t lo = j_lo, hi = j_hi - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_begin <= tile)
                lo = mid;
            else
                hi = mid - 1;
        }
        const BatchJob &job = jobs[lo];
        const ResizeArgs a = job.a;
        const int64_t local = tile - job.tile_begin;
        const int64_t per_plane = static_cast<int64_t>(job.tiles_x) * job.tiles_y;
        const int32_t plane = static_cast<int32_t>(local / per_plane);
        const int32_t rem = static_cast<int32_t>(local - plane * per_plane);
        const int32_t ty = rem / job.tiles_x;
        const int32_t tx = rem - ty * job.tiles_x;
        const int32_t col0 = tx * static_cast<int32_t>(blockDim.x) + static_cast<int32_t>(threadIdx.x);
        const int32_t r_begin =
            __builtin_amdgcn_readfirstlane((ty * static_cast<int32_t>(blockDim.y) + threadIdx.y) * job.strip_h);
        if (col0 < a.out_w && r_begin < a.dst_rows) {
            const int32_t r_end = min(r_begin + job.strip_h, a.dst_rows);
            switch (job.kind_fc) {
            case 0: {
                StripBody<kBilinear, T, 1, 1> b;
                b.run(a, plane, col0, r_begin, r_end);
                break;
            }
            case 1: {
                StripBody<kBilinear, T, 4, 1> b;
                b.run(a, plane, col0, r_begin, r_end);
                break;
            }
            case 2: {
                StripBody<kBicubic, T, 1, 1> b;
                b.run(a, plane, col0, r_begin, r_end);
                break;
            }
            default: {
                StripBody<kBicubic, T, 4, 1> b;
                b.run(a, plane, col0, r_begin, r_end);
                break;
            }
            }
        }
    }
    if (tid == 0) {
        __threadfence();
        if (atomicAdd(&hdr->done[kind], 1u) == gridDim.x - 1) {
            atomicExch(&hdr->ticket[kind], 0u);
            atomicExch(&hdr->done[kind], 0u);
        }
    }
}

namespace {
// kind = 2 * bicubic + four channels; kBatchNarrow last
template <typename T, int FILTER, int C>
void launch_kind(unsigned char *p, dim3 block, const int32_t *grid, hipStream_t stream)
{
    constexpr int kind = (FILTER == kBicubic ? 2 : 0) + (C == 4 ? 1 : 0);
    if (grid[kind] > 0)
        hipLaunchKernelGGL((k_batch_walk<FILTER, T, C>), dim3(grid[kind]), block, 0, stream, p, kind);
}

template <typename T, int FILTER, int C>
int32_t kind_occupancy(int32_t threads)
{
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_walk<FILTER, T, C>, threads, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

template <typename T>
hipError_t launch_batch_kinds(unsigned char *p, int32_t block_w, int32_t block_h, const int32_t *grid,
                              hipStream_t stream)
{
    const dim3 block(block_w, block_h, 1);
    launch_kind<T, kBilinear, 1>(p, block, grid, stream);
    launch_kind<T, kBilinear, 4>(p, block, grid, stream);
    launch_kind<T, kBicubic, 1>(p, block, grid, stream);
    launch_kind<T, kBicubic, 4>(p, block, grid, stream);
    if (grid[kBatchNarrow] > 0)
        hipLaunchKernelGGL(k_batch_narrow<T>, dim3(grid[kBatchNarrow]), block, 0, stream, p);
    return hipGetLastError();
}

template <typename T>
int32_t batch_kind_occupancy(int32_t kind, int32_t threads)
{
    switch (kind) {
    case 0:
        return kind_occupancy<T, kBilinear, 1>(threads);
    case 1:
        return kind_occupancy<T, kBilinear, 4>(threads);
    case 2:
        return kind_occupancy<T, kBicubic, 1>(threads);
    case 3:
        return kind_occupancy<T, kBicubic, 4>(threads);
    default: {
        int n = 0;
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_narrow<T>, threads, 0);
        return (e == hipSuccess && n > 0) ? n : 1;
    }
    }
}
}  // namespace

hipError_t launch_batched(const void *ws, int32_t dtype, int32_t block_w, int32_t block_h, const int32_t *grid,
                          hipStream_t stream)
{
    unsigned char *p = const_cast<unsigned char *>(static_cast<const unsigned char *>(ws));
    switch (dtype) {
    case XR_U8:
        return launch_batch_kinds<uint8_t>(p, block_w, block_h, grid, stream);
    case XR_F16:
        return launch_batch_kinds<_Float16>(p, block_w, block_h, grid, stream);
    default:
        return launch_batch_kinds<float>(p, block_w, block_h, grid, stream);
    }
}

int32_t batched_blocks_per_cu(int32_t dtype, int32_t kind, int32_t threads)
{
    switch (dtype) {
    case XR_U8:
        return batch_kind_occupancy<uint8_t>(kind, threads);
    case XR_F16:
        return batch_kind_occupancy<_Float16>(kind, threads);
    default:
        return batch_kind_occupancy<float>(kind, threads);
    }
}
// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------

namespace {
template <int FILTER, typename T, int C>
bool lds_fits(int32_t in_w, int32_t out_w, int32_t block_w, bool aligned4)
{
    return LdsPlan<FILTER, T, C, kLdsPpx[C == 4 ? 1 : 0]>(in_w, out_w, block_w, aligned4).ok;
}
template <int FILTER>
bool lds_fits_filter(int32_t dtype, int32_t channels, int32_t in_w, int32_t out_w, int32_t block_w,
                     bool aligned4)
{
    switch (dtype) {
    case XR_U8:
        return channels == 4 ? lds_fits<FILTER, uint8_t, 4>(in_w, out_w, block_w, aligned4)
                             : lds_fits<FILTER, uint8_t, 1>(in_w, out_w, block_w, aligned4);
    case XR_F16:
        return channels == 4 ? lds_fits<FILTER, _Float16, 4>(in_w, out_w, block_w, aligned4)
                             : lds_fits<FILTER, _Float16, 1>(in_w, out_w, block_w, aligned4);
    case XR_F32:
        return channels == 4 ? lds_fits<FILTER, float, 4>(in_w, out_w, block_w, aligned4)
                             : lds_fits<FILTER, float, 1>(in_w, out_w, block_w, aligned4);
    default:
        return false;
    }
}
}  // namespace

bool strip_lds_fits(int32_t filter, int32_t dtype, int32_t channels, int32_t in_w, int32_t out_w,
                    int32_t block_w, bool aligned4)
{
    if (filter == XR_BICUBIC)
        return lds_fits_filter<kBicubic>(dtype, channels, in_w, out_w, block_w, aligned4);
    if (filter == XR_NEAREST)
        return lds_fits_filter<kNearest>(dtype, channels, in_w, out_w, block_w, aligned4);
    return lds_fits_filter<kBilinear>(dtype, channels, in_w, out_w, block_w, aligned4);
}

bool strip_ppx_supported(int32_t dtype, int32_t channels, int32_t ppx)
{
    (void)dtype;
    if (channels == 4)
        return ppx == 1 || ppx == 2 || ppx == 4 || ppx == 8;
    return ppx == 4 || ppx == 8 || ppx == 16;
}

namespace {

template <int FILTER, typename T, int C>
hipError_t launch_lds(const ResizeArgs &a, const xr_tile &tile, hipStream_t stream)
{
    constexpr int PPX = kLdsPpx[C == 4 ? 1 : 0];
    using Plan = LdsPlan<FILTER, T, C, PPX>;
    const Plan plan(a.in_w, a.out_w, tile.block_w, a.aligned4 != 0);
    if (!plan.ok)
        return hipErrorInvalidValue;
    const size_t lds = 3 * static_cast<size_t>(plan.buf_bytes);
    const int32_t buf_bytes = static_cast<int32_t>(plan.buf_bytes);
    const int32_t cols_per_block = tile.block_w * PPX;
    const dim3 block(tile.block_w, 1, 1);
    const dim3 grid((a.out_w + cols_per_block - 1) / cols_per_block,
                    (a.dst_rows + tile.ppt_y - 1) / tile.ppt_y, a.planes);
#define XR_LDS_CASE(N)                                                                        \
    if (plan.need <= N) {                                                                     \
        hipLaunchKernelGGL((k_strip_lds<FILTER, T, C, PPX, N>), grid, block, lds, stream, a,  \
                           tile.ppt_y, tile.order, buf_bytes);                                \
        return hipGetLastError();                                                             \
    }
    XR_LDS_CASE(1)
    XR_LDS_CASE(2)
    XR_LDS_CASE(4)
    if constexpr (Plan::MAX_CH >= 8) {
        XR_LDS_CASE(8)
    }
    if constexpr (Plan::MAX_CH >= 16) {
        XR_LDS_CASE(16)
    }
#undef XR_LDS_CASE
    return hipErrorInvalidValue;
}

// The x2 walk needs whole-dword runs: (PPX/2) pixels of a thread a multiple
// of 4 bytes (one-byte pixels: PPX 8 or 16).
// Runs of more than 64 output bytes per thread (float32 RGBA with 8 columns)
// take the general walk: their rings exceed the register file.
template <typename T, int C, int PPX>
constexpr bool x2_ppx_ok()
{
    return PPX % 2 == 0 && ((PPX / 2) * Pix<T, C>::kBytes) % 4 == 0 && PPX * Pix<T, C>::kBytes <= 64;
}

// Strips of 2 np output rows, np = ppt_y / 2 rounded up to a multiple of 4
// (at least 4), and shortened until a strip's source and output rows stay
// well inside a buffer resource's 2 GiB.
template <int FILTER, typename T, int C, int PPX>
hipError_t launch_x2(const ResizeArgs &a, const xr_tile &tile, hipStream_t stream)
{
    int64_t np = std::max<int64_t>(4, (static_cast<int64_t>(tile.ppt_y) + 7) / 8 * 4);
    const int64_t pitch = std::max(a.src_pitch, a.dst_pitch);
    while (np > 4 && (2 * np + 8) * pitch >= (int64_t(1) << 30))
        np -= 4;
    const int64_t s_first = (static_cast<int64_t>(a.dst_row0) + 1) / (2 * np);
    const int64_t s_last = (static_cast<int64_t>(a.dst_row0) + a.dst_rows) / (2 * np);
    const int64_t strips = s_last - s_first + 1;
    const int32_t cols_per_block = tile.block_w * PPX;
    const dim3 block(tile.block_w, tile.block_h, 1);
    const dim3 grid((a.out_w + cols_per_block - 1) / cols_per_block,
                    static_cast<uint32_t>((strips + tile.block_h - 1) / tile.block_h), a.planes);
    const size_t lds = run_store_lds<T, C, PPX>(tile.block_w * tile.block_h);
    hipLaunchKernelGGL((k_x2<FILTER, T, C, PPX>), grid, block, lds, stream, a, static_cast<int32_t>(np),
                       static_cast<int32_t>(s_first), tile.order);
    return hipGetLastError();
}

// Strips of nr output rows, nr = ppt_y rounded up to an even count, shortened
// until a strip's rows stay well inside a buffer resource's 2 GiB.
template <int FILTER, typename T, int C, int PPX>
hipError_t launch_x05(const ResizeArgs &a, const xr_tile &tile, hipStream_t stream)
{
    int64_t nr = std::max<int64_t>(2, (static_cast<int64_t>(tile.ppt_y) + 1) / 2 * 2);
    const int64_t pitch = std::max(a.src_pitch, a.dst_pitch);
    while (nr > 2 && (2 * nr + 8) * pitch >= (int64_t(1) << 30))
        nr -= 2;
    const int64_t s_first = static_cast<int64_t>(a.dst_row0) / nr;
    const int64_t s_last = (static_cast<int64_t>(a.dst_row0) + a.dst_rows - 1) / nr;
    const int64_t strips = s_last - s_first + 1;
    const int32_t cols_per_block = tile.block_w * PPX;
    const dim3 block(tile.block_w, tile.block_h, 1);
    const dim3 grid((a.out_w + cols_per_block - 1) / cols_per_block,
                    static_cast<uint32_t>((strips + tile.block_h - 1) / tile.block_h), a.planes);
    const size_t lds = run_store_lds<T, C, PPX>(tile.block_w * tile.block_h);
    hipLaunchKernelGGL((k_x05<FILTER, T, C, PPX>), grid, block, lds, stream, a, static_cast<int32_t>(nr),
                       static_cast<int32_t>(s_first), tile.order);
    return hipGetLastError();
}

template <int FILTER, typename T, int C>
hipError_t launch_typed(const ResizeArgs &a, const xr_tile &tile, int32_t mode, hipStream_t stream)
{
    if (tile.kernel == XR_KERNEL_STRIP_LDS)
        return launch_lds<FILTER, T, C>(a, tile, stream);
    if (tile.kernel == XR_KERNEL_GATHER) {
        const dim3 block(tile.block_w, tile.block_h, 1);
        const dim3 grid((a.out_w + tile.block_w - 1) / tile.block_w,
                        (a.dst_rows + tile.block_h - 1) / tile.block_h, a.planes);
        hipLaunchKernelGGL((k_gather<FILTER, T, C>), grid, block, 0, stream, a);
        return hipGetLastError();
    }
    const int32_t cols_per_block = tile.block_w * tile.ppt_x;
    const int32_t rows_per_block = tile.block_h * tile.ppt_y;
    const dim3 block(tile.block_w, tile.block_h, 1);
    const dim3 grid((a.out_w + cols_per_block - 1) / cols_per_block,
                    (a.dst_rows + rows_per_block - 1) / rows_per_block, a.planes);
#define XR_STRIP_CASE(P)                                                                        \
    case P:                                                                                     \
        if constexpr (FILTER != kNearest) {                                                     \
            if (mode == kUp2) {                                                                 \
                if constexpr (x2_ppx_ok<T, C, P>())                                             \
                    return launch_x2<FILTER, T, C, P>(a, tile, stream);                         \
            }                                                                                   \
            if (mode == kDown2) {                                                               \
                if constexpr ((2 * P * Pix<T, C>::kBytes) % 4 == 0 && P * Pix<T, C>::kBytes <= 64) \
                    return launch_x05<FILTER, T, C, P>(a, tile, stream);                        \
            }                                                                                   \
        }                                                                                       \
        hipLaunchKernelGGL((k_strip<FILTER, T, C, P>), grid, block, 0, stream, a, tile.ppt_y,   \
                           tile.order);                                                         \
        return hipGetLastError();
    if constexpr (C == 4) {
        switch (tile.ppt_x) {
            XR_STRIP_CASE(1)
            XR_STRIP_CASE(2)
            XR_STRIP_CASE(4)
            XR_STRIP_CASE(8)
        default:
            return hipErrorInvalidValue;
        }
    } else {
        switch (tile.ppt_x) {
            XR_STRIP_CASE(4)
            XR_STRIP_CASE(8)
            XR_STRIP_CASE(16)
        default:
            return hipErrorInvalidValue;
        }
    }
#undef XR_STRIP_CASE
}

template <int FILTER>
hipError_t launch_filter(const ResizeArgs &a, int32_t dtype, int32_t channels, const xr_tile &tile,
                         int32_t mode, hipStream_t stream)
{
    switch (dtype) {
    case XR_U8:
        return channels == 4 ? launch_typed<FILTER, uint8_t, 4>(a, tile, mode, stream)
                             : launch_typed<FILTER, uint8_t, 1>(a, tile, mode, stream);
    case XR_F16:
        return channels == 4 ? launch_typed<FILTER, _Float16, 4>(a, tile, mode, stream)
                             : launch_typed<FILTER, _Float16, 1>(a, tile, mode, stream);
    case XR_F32:
        return channels == 4 ? launch_typed<FILTER, float, 4>(a, tile, mode, stream)
                             : launch_typed<FILTER, float, 1>(a, tile, mode, stream);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace

namespace {
template <int R, typename T, int C>
hipError_t launch_aa_typed(const ResizeArgs &a, const xr_tile &tile, hipStream_t stream)
{
    const dim3 block(tile.block_w, tile.block_h, 1);
    const dim3 grid((a.out_w + tile.block_w - 1) / tile.block_w,
                    (a.dst_rows + tile.block_h - 1) / tile.block_h, a.planes);
    if (tile.kernel == XR_KERNEL_GATHER) {
        const AaPlan plan = aa_plan(a.in_w, a.in_h, a.out_w, a.out_h, R, tile.block_w, tile.block_h);
        hipLaunchKernelGGL((k_gather_aa<R, T, C>), grid, block, plan.lds_bytes, stream, a, plan.kx, plan.ky);
    } else {
        const AaPlan plan = aa_tile_plan(a.in_w, a.in_h, a.out_w, a.out_h, R, tile.block_w, tile.block_h,
                                         Pix<T, C>::kBytes, C);
        // tiles per workgroup down a tile column: the column tables are then
        // built once per tpb tiles, while the grid keeps kAaMinBlocks
        // workgroups
        const int64_t cols = static_cast<int64_t>(grid.x) * grid.z;
        int32_t tpb = 1;
        while (tpb < kAaTilesPerBlock && cols * ((grid.y + 2 * tpb - 1) / (2 * tpb)) >= kAaMinBlocks)
            tpb *= 2;
        const dim3 grid_t(grid.x, (grid.y + tpb - 1) / tpb, grid.z);
        hipLaunchKernelGGL((k_tile_aa<R, T, C>), grid_t, block, plan.lds_bytes, stream, a, plan.kx, plan.ky,
                           plan.win_w, plan.win_h, tpb);
    }
    return hipGetLastError();
}

template <int R>
hipError_t launch_aa(const ResizeArgs &a, int32_t dtype, int32_t channels, const xr_tile &tile,
                     hipStream_t stream)
{
    switch (dtype) {
    case XR_U8:
        return channels == 4 ? launch_aa_typed<R, uint8_t, 4>(a, tile, stream)
                             : launch_aa_typed<R, uint8_t, 1>(a, tile, stream);
    case XR_F16:
        return channels == 4 ? launch_aa_typed<R, _Float16, 4>(a, tile, stream)
                             : launch_aa_typed<R, _Float16, 1>(a, tile, stream);
    case XR_F32:
        return channels == 4 ? launch_aa_typed<R, float, 4>(a, tile, stream)
                             : launch_aa_typed<R, float, 1>(a, tile, stream);
    default:
        return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_forward(const ResizeArgs &a, int32_t filter, int32_t dtype, int32_t channels,
                          const xr_tile &tile, int32_t mode, hipStream_t stream)
{
    if (filter == XR_BILINEAR_AA)
        return launch_aa<1>(a, dtype, channels, tile, stream);
    if (filter == XR_BICUBIC_AA)
        return launch_aa<2>(a, dtype, channels, tile, stream);
    if (filter == XR_BICUBIC)
        return launch_filter<kBicubic>(a, dtype, channels, tile, mode, stream);
    if (filter == XR_NEAREST)
        return launch_filter<kNearest>(a, dtype, channels, tile, mode, stream);
    return launch_filter<kBilinear>(a, dtype, channels, tile, mode, stream);
}

}  // namespace xr
