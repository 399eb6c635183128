// Adjoint of the resize with respect to its input, float32, for gfx950.
//
// grad_src = A^T grad_dst: every output pixel (y, x) scatters
// wy_j * wx_i * g[y][x] onto its clamped taps (the transpose of eq. 5).
//
// One workgroup takes an output tile. Its contributions are accumulated in an
// LDS copy of the tile's source footprint (LDS float atomics), then the
// footprint is merged into global memory:
//   * pixels that no neighbouring tile touches are written with plain stores;
//   * pixels on the footprint ring that the left/right/upper/lower neighbour
//     also touches are merged with global float32 atomics. Before the main
//     kernel, a small fill kernel zeroes exactly those ring rows and columns.
// When an axis shrinks some source pixels may be touched by no output at all,
// so for any downscale the whole gradient is zeroed first and every footprint
// pixel is merged with atomics.
#include <hip/hip_runtime.h>

#include "xr_device.hpp"
#include "xr_internal.h"

namespace xr {
using namespace dev;

namespace {

constexpr int kBwdBlockW = 64;
constexpr int kBwdBlockH = 4;
constexpr int kBwdRows = 8;  // output rows per thread

template <int C>
struct BwdPpx {
    static constexpr int P = (C == 4) ? 1 : 4;  // output columns per thread
};

// first clamped source index a run of outputs [b, e) touches, and the last
template <int FILTER>
__device__ __forceinline__ int32_t first_tap(int32_t b, int32_t n_in, int32_t n_out)
{
    int32_t x0;
    float t, u;
    axis_tap(b, n_in, n_out, x0, t, u);
    return clampi(x0 + Taps<FILTER>::LO, 0, n_in - 1);
}

template <int FILTER>
__device__ __forceinline__ int32_t last_tap(int32_t e, int32_t n_in, int32_t n_out)
{
    int32_t x0;
    float t, u;
    axis_tap(e - 1, n_in, n_out, x0, t, u);
    return clampi(x0 + Taps<FILTER>::LO + Taps<FILTER>::K - 1, 0, n_in - 1);
}

// Zero the source rows shared by the tiles above and below each tile-row
// boundary. blockIdx.y = boundary index - 1, blockIdx.z = plane.
template <int FILTER, int C>
__global__ void __launch_bounds__(256) k_bwd_zero_rows(ResizeArgs a, int32_t tile_h)
{
    const int32_t yb = (blockIdx.y + 1) * tile_h;
    const int32_t r_first = first_tap<FILTER>(yb, a.in_h, a.out_h);
    const int32_t r_last = last_tap<FILTER>(yb, a.in_h, a.out_h);
    const int32_t col = blockIdx.x * blockDim.x + threadIdx.x;  // float index in the row
    if (col >= a.in_w * C)
        return;
    unsigned char *dst = a.dst + static_cast<int64_t>(blockIdx.z) * a.dst_plane_pitch;
    for (int32_t r = r_first; r <= r_last; ++r)
        reinterpret_cast<float *>(dst + static_cast<int64_t>(r) * a.dst_pitch)[col] = 0.0f;
}

// Zero the source columns shared by the tiles left and right of each tile-column
// boundary. blockIdx.x = boundary index - 1, threads run down the rows.
template <int FILTER, int C>
__global__ void __launch_bounds__(256) k_bwd_zero_cols(ResizeArgs a, int32_t tile_w)
{
    const int32_t xb = (blockIdx.x + 1) * tile_w;
    const int32_t c_first = first_tap<FILTER>(xb, a.in_w, a.out_w);
    const int32_t c_last = last_tap<FILTER>(xb, a.in_w, a.out_w);
    const int32_t r = blockIdx.y * blockDim.x + threadIdx.x;
    if (r >= a.in_h)
        return;
    float *row = reinterpret_cast<float *>(a.dst + static_cast<int64_t>(blockIdx.z) * a.dst_plane_pitch +
                                           static_cast<int64_t>(r) * a.dst_pitch);
    for (int32_t c = c_first; c <= c_last; ++c)
#pragma unroll
        for (int ch = 0; ch < C; ++ch)
            row[c * C + ch] = 0.0f;
}

// Zero a whole gradient image.
template <int C>
__global__ void __launch_bounds__(256) k_bwd_zero_all(ResizeArgs a)
{
    const int32_t col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= a.in_w * C)
        return;
    float *row = reinterpret_cast<float *>(a.dst + static_cast<int64_t>(blockIdx.z) * a.dst_plane_pitch +
                                           static_cast<int64_t>(blockIdx.y) * a.dst_pitch);
    row[col] = 0.0f;
}

// a.src = grad_dst (out_w x out_h), a.dst = grad_src (in_w x in_h).
template <int FILTER, int C>
__global__ void __launch_bounds__(256) k_bwd_scatter(ResizeArgs a, int32_t all_atomic)
{
    using TP = Taps<FILTER>;
    constexpr int K = TP::K;
    constexpr int P = BwdPpx<C>::P;
    constexpr int TW = kBwdBlockW * P;
    constexpr int TH = kBwdBlockH * kBwdRows;
    extern __shared__ float acc[];

    const int32_t xa = blockIdx.x * TW;
    const int32_t ya = blockIdx.y * TH;
    const int32_t xe = min(xa + TW, a.out_w);
    const int32_t ye = min(ya + TH, a.out_h);
    const int32_t plane = blockIdx.z;

    const int32_t fa = first_tap<FILTER>(xa, a.in_w, a.out_w);
    const int32_t fb = last_tap<FILTER>(xe, a.in_w, a.out_w);
    const int32_t ra = first_tap<FILTER>(ya, a.in_h, a.out_h);
    const int32_t rb = last_tap<FILTER>(ye, a.in_h, a.out_h);
    const int32_t fw = fb - fa + 1;
    const int32_t fh = rb - ra + 1;
    const int32_t tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int32_t nthreads = blockDim.x * blockDim.y;

    for (int32_t k = tid; k < fw * fh * C; k += nthreads)
        acc[k] = 0.0f;
    __syncthreads();

    // scatter this thread's outputs into the LDS footprint
    const int32_t xc = xa + threadIdx.x * P;
    if (xc < xe) {
        int32_t lx[P][K];
        float wx[P][K];
#pragma unroll
        for (int c = 0; c < P; ++c) {
            int32_t x0;
            float t, u;
            axis_tap(min(xc + c, xe - 1), a.in_w, a.out_w, x0, t, u);
            weights<FILTER>(t, u, wx[c]);
#pragma unroll
            for (int i = 0; i < K; ++i)
                lx[c][i] = clampi(x0 + TP::LO + i, 0, a.in_w - 1) - fa;
            if (xc + c >= xe) {
#pragma unroll
                for (int i = 0; i < K; ++i)
                    wx[c][i] = 0.0f;
            }
        }
        const unsigned char *gsrc = a.src + static_cast<int64_t>(plane) * a.src_plane_pitch;
        const int32_t y_begin = ya + __builtin_amdgcn_readfirstlane(threadIdx.y * kBwdRows);
        const int32_t y_end = min(y_begin + kBwdRows, ye);
        for (int32_t y = y_begin; y < y_end; ++y) {
            int32_t y0;
            float ty, uy;
            axis_tap(y, a.in_h, a.out_h, y0, ty, uy);
            float wy[K];
            weights<FILTER>(ty, uy, wy);
            const unsigned char *grow = gsrc + static_cast<int64_t>(y) * a.src_pitch;
            float g[P][C];
#pragma unroll
            for (int c = 0; c < P; ++c) {
                if (xc + c < xe)
                    Pix<float, C>::load(grow, xc + c, g[c]);
                else
#pragma unroll
                    for (int ch = 0; ch < C; ++ch)
                        g[c][ch] = 0.0f;
            }
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int32_t ly = clampi(y0 + TP::LO + j, 0, a.in_h - 1) - ra;
                float *arow = acc + static_cast<int32_t>(ly * fw) * C;
#pragma unroll
                for (int c = 0; c < P; ++c)
#pragma unroll
                    for (int i = 0; i < K; ++i) {
                        const float w = wy[j] * wx[c][i];
#pragma unroll
                        for (int ch = 0; ch < C; ++ch)
                            atomicAdd(arow + lx[c][i] * C + ch, w * g[c][ch]);
                    }
            }
        }
    }
    __syncthreads();

    // merge the footprint into global memory
    int32_t up_last = -1, down_first = a.in_h, left_last = -1, right_first = a.in_w;
    if (!all_atomic) {
        if (ya > 0)
            up_last = last_tap<FILTER>(ya, a.in_h, a.out_h);
        if (ye < a.out_h)
            down_first = first_tap<FILTER>(ye, a.in_h, a.out_h);
        if (xa > 0)
            left_last = last_tap<FILTER>(xa, a.in_w, a.out_w);
        if (xe < a.out_w)
            right_first = first_tap<FILTER>(xe, a.in_w, a.out_w);
    }
    unsigned char *gdst = a.dst + static_cast<int64_t>(plane) * a.dst_plane_pitch;
    for (int32_t k = tid; k < fw * fh; k += nthreads) {
        const int32_t r = ra + k / fw;
        const int32_t c = fa + k % fw;
        float *out = reinterpret_cast<float *>(gdst + static_cast<int64_t>(r) * a.dst_pitch) + c * C;
        const float *v = acc + k * C;
        const bool exclusive =
            !all_atomic && r > up_last && r < down_first && c > left_last && c < right_first;
        if (exclusive) {
#pragma unroll
            for (int ch = 0; ch < C; ++ch)
                out[ch] = v[ch];
        } else {
#pragma unroll
            for (int ch = 0; ch < C; ++ch)
                unsafeAtomicAdd(out + ch, v[ch]);
        }
    }
}

// Fallback for footprints too large for LDS (strong shrinking): every output
// pixel adds its contributions straight to the zeroed gradient with atomics.
template <int FILTER, int C>
__global__ void __launch_bounds__(256) k_bwd_direct(ResizeArgs a)
{
    using TP = Taps<FILTER>;
    constexpr int K = TP::K;
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= a.out_w || y >= a.out_h)
        return;
    int32_t x0, y0;
    float tx, ty, ux, uy;
    axis_tap(x, a.in_w, a.out_w, x0, tx, ux);
    axis_tap(y, a.in_h, a.out_h, y0, ty, uy);
    float wx[K], wy[K];
    weights<FILTER>(tx, ux, wx);
    weights<FILTER>(ty, uy, wy);
    float g[C];
    Pix<float, C>::load(a.src + static_cast<int64_t>(blockIdx.z) * a.src_plane_pitch +
                            static_cast<int64_t>(y) * a.src_pitch,
                        x, g);
    unsigned char *gdst = a.dst + static_cast<int64_t>(blockIdx.z) * a.dst_plane_pitch;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int32_t r = clampi(y0 + TP::LO + j, 0, a.in_h - 1);
        float *row = reinterpret_cast<float *>(gdst + static_cast<int64_t>(r) * a.dst_pitch);
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int32_t c = clampi(x0 + TP::LO + i, 0, a.in_w - 1);
            const float w = wy[j] * wx[i];
#pragma unroll
            for (int ch = 0; ch < C; ++ch)
                unsafeAtomicAdd(row + c * C + ch, w * g[ch]);
        }
    }
}

template <int FILTER, int C>
hipError_t launch_bwd_typed(const ResizeArgs &a, hipStream_t stream)
{
    constexpr int K = Taps<FILTER>::K;
    constexpr int TW = kBwdBlockW * BwdPpx<C>::P;
    constexpr int TH = kBwdBlockH * kBwdRows;
    const int32_t tiles_x = (a.out_w + TW - 1) / TW;
    const int32_t tiles_y = (a.out_h + TH - 1) / TH;
    const bool all_atomic = a.in_w > a.out_w || a.in_h > a.out_h;
    // largest footprint of a tile: (T-1) * in/out + 1 + K per axis
    const int64_t fw = (static_cast<int64_t>(TW - 1) * a.in_w) / a.out_w + K + 2;
    const int64_t fh = (static_cast<int64_t>(TH - 1) * a.in_h) / a.out_h + K + 2;
    const size_t lds = static_cast<size_t>(fw) * fh * C * sizeof(float);
    const int32_t row_threads = a.in_w * C;
    if (lds > 64 * 1024) {
        hipLaunchKernelGGL(k_bwd_zero_all<C>, dim3((row_threads + 255) / 256, a.in_h, a.planes),
                           dim3(256), 0, stream, a);
        hipLaunchKernelGGL((k_bwd_direct<FILTER, C>),
                           dim3((a.out_w + 63) / 64, (a.out_h + 3) / 4, a.planes), dim3(64, 4), 0,
                           stream, a);
        return hipGetLastError();
    }
    if (all_atomic) {
        hipLaunchKernelGGL(k_bwd_zero_all<C>, dim3((row_threads + 255) / 256, a.in_h, a.planes),
                           dim3(256), 0, stream, a);
    } else {
        if (tiles_y > 1)
            hipLaunchKernelGGL((k_bwd_zero_rows<FILTER, C>),
                               dim3((row_threads + 255) / 256, tiles_y - 1, a.planes), dim3(256), 0,
                               stream, a, TH);
        if (tiles_x > 1)
            hipLaunchKernelGGL((k_bwd_zero_cols<FILTER, C>),
                               dim3(tiles_x - 1, (a.in_h + 255) / 256, a.planes), dim3(256), 0,
                               stream, a, TW);
    }
    hipLaunchKernelGGL((k_bwd_scatter<FILTER, C>), dim3(tiles_x, tiles_y, a.planes),
                       dim3(kBwdBlockW, kBwdBlockH), lds, stream, a, all_atomic ? 1 : 0);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_backward(const ResizeArgs &a, int32_t filter, int32_t channels, hipStream_t stream)
{
    if (filter == XR_BICUBIC)
        return channels == 4 ? launch_bwd_typed<kBicubic, 4>(a, stream)
                             : launch_bwd_typed<kBicubic, 1>(a, stream);
    return channels == 4 ? launch_bwd_typed<kBilinear, 4>(a, stream)
                         : launch_bwd_typed<kBilinear, 1>(a, stream);
}

}  // namespace xr
