// Internal interface between the C-ABI layer (xr_api.cpp) and the kernels
// (xr_forward.hip, xr_backward.hip). Not installed; callers use include/xresize.h.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/xresize.h"

namespace xr {

// One resize job, resolved to byte addresses and validated on the host.
// `src` / `dst` point at the first stored row of plane 0.
struct ResizeArgs {
    const unsigned char *src;
    unsigned char *dst;
    int64_t src_pitch, src_plane_pitch;
    int64_t dst_pitch, dst_plane_pitch;
    int32_t in_w, in_h;      // full logical source size
    int32_t out_w, out_h;    // full logical destination size
    int32_t src_row0;        // logical row stored first in src
    int32_t src_rows;        // logical rows stored in src
    int32_t dst_row0;        // first logical output row to compute
    int32_t dst_rows;        // number of output rows to compute
    int32_t planes;
    int32_t aligned16;       // src, dst and pitches are 16-byte aligned
    int32_t aligned4;        // src and its pitches are 4-byte aligned and a
                             // source row is a whole number of 4-byte words
    int32_t map_off;         // 1: pixel-centre map; 0: the map eq. 1 prints
};

// Entry of the device job table of the batched launch.
struct BatchJob {
    ResizeArgs a;
    int32_t tiles_x;         // tiles per row of the output (per plane)
    int32_t tiles_y;         // tiles per column of the output (per plane)
    int64_t tile_begin;      // tiles of the jobs of the same kind before this one
    int32_t strip_h;         // output rows per thread strip of this job
    int32_t kind;            // launch of the job (kBatchKinds)
    int32_t kind_fc;         // 2 * (bicubic) + (four channels)
    int32_t pad_;
};

// Launches of the batched resize, one per job kind: kinds 0-3 are
// 2 * (bicubic) + (four channels); kind 4 holds the jobs with a source
// narrower than the filter's taps or an output narrower than the walk's run.
constexpr int32_t kBatchKinds = 5;
constexpr int32_t kBatchNarrow = 4;

// Header of the batched workspace; jobs follow at offset kBatchHeaderBytes,
// grouped by kind.
struct BatchHeader {
    int32_t n_jobs;
    int32_t dtype;
    int32_t block_w;         // threads per workgroup along x
    int32_t block_h;         // thread rows per workgroup
    int32_t ppt_y;           // rows per thread strip (before per-job scaling)
    int32_t pad_;
    int32_t job_lo[kBatchKinds];    // jobs [job_lo, job_hi) are of kind k
    int32_t job_hi[kBatchKinds];
    int64_t tiles[kBatchKinds];     // tiles of kind k
    int32_t grid[kBatchKinds];      // workgroups of kind k's launch (0: no launch)
    uint32_t ticket[kBatchKinds];   // next tile to hand out (self-resetting)
    uint32_t done[kBatchKinds];     // workgroups that have finished (self-resetting)
};
constexpr size_t kBatchHeaderBytes = 256;
static_assert(sizeof(BatchHeader) <= kBatchHeaderBytes, "batch header");

// Longest thread strip of the batched walk (rows of its per-wavefront weight
// table in LDS).
constexpr int32_t kBatchMaxStrip = 256;

// Row weights of one output row in that table.
template <int K>
struct alignas(K * 4) BatchWeights {
    float w[K];
};

// Output columns per thread of the batched walk, per filter, storage type and
// channel count: 16-byte runs for bilinear, 8 to 16 for bicubic (whose four
// tap rows per column would leave fewer waves with 16-byte uint8 runs); the
// narrow kind takes one column.
constexpr int32_t batch_ppx(int32_t filter, int32_t dtype, int32_t channels)
{
    return dtype == XR_U8 ? (channels == 1 ? (filter == XR_BILINEAR ? 16 : 8) : (filter == XR_BILINEAR ? 4 : 2))
         : dtype == XR_F16 ? (channels == 1 ? 8 : 2)
                           : (channels == 1 ? 4 : 1);
}

// Shape of an axis that a kernel can specialise on.
enum AxisMode : int32_t { kGeneral = 0, kUp2 = 1, kDown2 = 2 };

hipError_t launch_forward(const ResizeArgs &a, int32_t filter, int32_t dtype, int32_t channels,
                          const xr_tile &tile, int32_t mode, hipStream_t stream);
// The batched launches of a prepared workspace: one per kind with grid[kind] > 0.
hipError_t launch_batched(const void *ws, int32_t dtype, int32_t block_w, int32_t block_h, const int32_t *grid,
                          hipStream_t stream);
// Workgroups of the batched walk of `kind` that fit on one compute unit.
int32_t batched_blocks_per_cu(int32_t dtype, int32_t kind, int32_t threads);
hipError_t launch_backward(const ResizeArgs &a, int32_t filter, int32_t dtype, int32_t channels,
                           hipStream_t stream);
// False when the adjoint's smallest LDS tile cannot hold the output rows of
// one source row and the column tables (upscales beyond roughly 190x rows or
// a few hundred x columns).
bool backward_supported(const ResizeArgs &a, int32_t filter, int32_t channels);

// Weight tables of the antialiased kernel: at most kx (ky) taps per output
// column (row), floor(2 R sigma) + 1 with sigma = max(1, n_in / n_out), and
// the LDS bytes of one workgroup's tables.
struct AaPlan {
    int32_t kx, ky;
    int64_t lds_bytes;
    int32_t win_w = 0, win_h = 0;  // source window of the LDS-tiled kernel
};
inline AaPlan aa_plan(int32_t in_w, int32_t in_h, int32_t out_w, int32_t out_h, int32_t r,
                      int32_t block_w, int32_t block_h)
{
    const auto taps = [r](int64_t n_in, int64_t n_out) {
        return static_cast<int32_t>((n_in > n_out ? (2 * r * n_in) / n_out : 2 * r) + 1);
    };
    AaPlan p;
    p.kx = taps(in_w, out_w);
    p.ky = taps(in_h, out_h);
    p.lds_bytes = 4 * (2 * static_cast<int64_t>(block_w) + 2 * block_h +
                       static_cast<int64_t>(block_w) * p.kx + static_cast<int64_t>(block_h) * p.ky);
    return p;
}
// gfx950 gives a workgroup up to 160 KiB of LDS; 96 KiB admits the taller
// blocks of the LDS-tiled kernel (bilinear x0.25: 64x8 blocks, 11% faster than
// the 16x16 that fits 64 KiB)
constexpr int64_t kAaLdsBudget = 96 * 1024;
// The LDS-tiled antialiased kernel adds the tile's source window (pixels of
// pb bytes) and one float32 row buffer per window row: a block of bw output
// columns reads at most floor(((bw - 1) n_in + 2 R max(n_in, n_out)) / n_out) + 2
// source columns (its first and last columns' tap ranges, eq. 1).
inline AaPlan aa_tile_plan(int32_t in_w, int32_t in_h, int32_t out_w, int32_t out_h, int32_t r,
                           int32_t block_w, int32_t block_h, int32_t pb, int32_t channels)
{
    AaPlan p = aa_plan(in_w, in_h, out_w, out_h, r, block_w, block_h);
    const auto span = [r](int64_t n, int64_t n_in, int64_t n_out) {
        return static_cast<int32_t>(((n - 1) * n_in + 2 * r * (n_in > n_out ? n_in : n_out)) / n_out + 2);
    };
    p.win_w = std::min<int32_t>(span(block_w, in_w, out_w), in_w);
    p.win_h = std::min<int32_t>(span(block_h, in_h, out_h), in_h);
    const int64_t tables = (p.lds_bytes + 15) / 16 * 16;
    const int64_t window = (static_cast<int64_t>(p.win_w) * p.win_h * pb + 15) / 16 * 16;
    const int64_t rows = static_cast<int64_t>(p.win_h) * block_w * channels * 4;
    p.lds_bytes = tables + window + rows;
    return p;
}

// Pixels per thread along x that the strip kernel is instantiated for.
bool strip_ppx_supported(int32_t dtype, int32_t channels, int32_t ppx);
// Columns per thread of the LDS-staged strip kernel: {one channel, four}.
constexpr int32_t kLdsPpx[2] = {8, 4};
// Dynamic LDS of the LDS-staged strip kernel (three row buffers) is kept
// within this many bytes per workgroup.
constexpr size_t kLdsBudget = 64 * 1024;
// True when a workgroup of block_w threads of the LDS-staged strip kernel can
// stage its source row segment for an in_w -> out_w resize (`aligned4` as in
// ResizeArgs; pixels of fewer than 4 bytes are staged as 4-byte words).
bool strip_lds_fits(int32_t filter, int32_t dtype, int32_t channels, int32_t in_w, int32_t out_w,
                    int32_t block_w, bool aligned4);

}  // namespace xr
