/*
 * xresize.h - C ABI of libxresize.so, bilinear and Keys-bicubic image resize
 * for AMD Instinct MI355X (gfx950).
 *
 * What is computed (paper section II.B, eqs. 1-5, generalised to 4x4 taps).
 * Along each axis an output index x of an image resized from N_in to N_out
 * samples reads the source at the half-pixel coordinate
 *     s(x) = ((2x + 1) N_in - N_out) / (2 N_out)          (eq. 1)
 * (xr_resize also offers eq. 1 as printed, s(x) = x N_in / N_out, and
 * nearest neighbour)
 * with base tap x0 = floor(s) and offset t = s - x0        (eqs. 2-4)
 * evaluated from exact integers. Bilinear takes taps x0, x0+1 with weights
 * (1 - t, t); bicubic takes x0-1 .. x0+2 with the Keys (1981) cubic weights
 * for a = -1/2. Each tap index is clamped to [0, N_in - 1]. Per channel the
 * output is sum_j wy_j * (sum_i wx_i * src[y0+j][x0+i])     (eq. 5)
 * in float32: the inner sum over columns first, taps in ascending order, then
 * the sum over rows in ascending order. That order is the same in every
 * kernel of the library, so a pixel's value never depends on the tile shape,
 * the launch, the band split or the batch it was computed in.
 * uint8 outputs are rounded half-to-even and clamped to [0, 255]; float16
 * outputs are rounded to nearest even; float32 outputs are stored as is.
 *
 * Conventions for every entry point:
 *  - Image pointers are DEVICE pointers owned by the caller. The library never
 *    frees or retains them.
 *  - `stream` is a hipStream_t (NULL = the null stream). Work is enqueued and
 *    the call returns without synchronising.
 *  - The resize, batched and backward calls allocate nothing and may be
 *    captured into a HIP graph; xr_batch_prepare and xr_autotune may not.
 *  - Every argument is validated on the host before any HIP call. A non-zero
 *    return value is an XR_ERR_* code; xr_last_error() then gives a
 *    description (thread-local). No exception crosses the ABI.
 */
#ifndef XRESIZE_H
#define XRESIZE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define XR_OK 0
#define XR_ERR_NULL 1       /* a required pointer is NULL                          */
#define XR_ERR_SHAPE 2      /* a size <= 0, a side > XR_MAX_SIDE, planes < 1         */
#define XR_ERR_DTYPE 3      /* unsupported dtype, or src/dst dtypes differ           */
#define XR_ERR_CHANNELS 4   /* channels not 1 or 4, or src/dst channels differ       */
#define XR_ERR_PITCH 5      /* row/plane pitch too small or misaligned               */
#define XR_ERR_RANGE 6      /* band outside the image, or src band misses needed rows */
#define XR_ERR_ALIAS 7      /* src and dst memory ranges overlap                     */
#define XR_ERR_WORKSPACE 8  /* workspace NULL, too small or misaligned               */
#define XR_ERR_CAPTURE 9    /* a non-capturable call was made on a capturing stream  */
#define XR_ERR_HIP 10       /* a HIP runtime call failed; see xr_last_error()        */
#define XR_ERR_ARG 11       /* any other invalid argument (filter, tile, count)      */

/* ---- element types, filters, limits ------------------------------------ */
#define XR_U8 0
#define XR_F16 1
#define XR_F32 2

#define XR_BILINEAR 0
#define XR_BICUBIC 1
#define XR_NEAREST 2        /* xr_resize only */
#define XR_BILINEAR_AA 3    /* xr_resize only: antialiased (filter stretched when shrinking) */
#define XR_BICUBIC_AA 4     /* xr_resize only: antialiased Keys a = -1/2 */

/* coordinate maps of xr_resize (eq. 1) */
#define XR_MAP_HALF_PIXEL 0 /* s = ((2x + 1) N_in - N_out) / (2 N_out): pixel centres aligned */
#define XR_MAP_PAPER 1      /* s = x N_in / N_out: eq. 1 as printed, x_p = x_f / scale      */

#define XR_MAX_SIDE 32768   /* largest width/height of any image (keeps (2x+1)N in int32) */

/*
 * Image descriptor. Pixels are row-major with `channels` interleaved values
 * per pixel (HWC). Planar data (NCHW) is described with channels = 1 and
 * planes = N*C. `data` points at the first stored row of plane 0, which is
 * logical row `row0`; rows [row0, row0 + rows) of every plane are stored.
 * `width` and `height` are always the FULL logical sizes: the coordinate map
 * of eq. 1 uses them, so a band computes exactly the rows of the whole image.
 * For a whole image: row0 = 0, rows = height.
 */
typedef struct {
    void *data;          /* device pointer, caller-owned                     */
    int32_t width;       /* logical width in pixels                          */
    int32_t height;      /* logical height in pixels                         */
    int32_t channels;    /* 1 or 4                                           */
    int32_t dtype;       /* XR_U8, XR_F16, XR_F32                            */
    int64_t row_pitch;   /* bytes between rows, >= width*channels*elem_size, */
                         /* multiple of the element size                     */
    int32_t planes;      /* >= 1                                             */
    int64_t plane_pitch; /* bytes between planes, >= rows*row_pitch (planes>1) */
    int32_t row0;        /* first logical row held in `data`                 */
    int32_t rows;        /* number of logical rows held in `data`            */
} xr_image;

/*
 * Launch shape. A workgroup has block_w x block_h threads; each thread
 * computes ppt_x adjacent output columns and ppt_y output rows, so a tile
 * covers (block_w*ppt_x) x (block_h*ppt_y) output pixels (eq. 6 with
 * b_width = block_w*ppt_x, b_height = block_h*ppt_y).
 *  kernel = XR_KERNEL_AUTO    : use the tuned (or default) shape; other fields ignored
 *         = XR_KERNEL_GATHER  : one thread per pixel group, every tap read from
 *                               memory (the paper's block tiling); ppt_x = ppt_y = 1
 *         = XR_KERNEL_STRIP   : each thread walks ppt_y rows down a strip of
 *                               ppt_x columns and reuses the filtered rows
 *                               from registers; block_w a multiple of 64 and
 *                               block_w * block_h <= 512. An exact x2 upscale
 *                               or x0.5 downscale on both axes runs a variant
 *                               specialised for it.
 *         = XR_KERNEL_STRIP_ANY : the strip kernel without the x2 and x0.5
 *                               variants (the same results; for comparisons)
 *         = XR_KERNEL_STRIP_LDS : the strip walk with each source row staged
 *                               once per workgroup in LDS, taps read from LDS
 *                               (any scale; block_h = 1, block_w a multiple of
 *                               64 up to 512, ppt_x = 4 for 4 channels and 8
 *                               for one). XR_ERR_ARG when one workgroup's row
 *                               segment does not fit its LDS budget (strong
 *                               downscales with wide workgroups). With the
 *                               antialiased filters of xr_resize: the
 *                               LDS-tiled separable kernel (see there)
 *  order  = 0 : tiles are processed in launch order (row-major)
 *         = 1 : the launch is split into 8 contiguous bands of tiles, one per
 *               XCD (the hardware deals workgroups to the 8 XCDs in turn), so
 *               each XCD's L2 sees vertically adjacent tiles (strip kernels)
 */
#define XR_KERNEL_AUTO 0
#define XR_KERNEL_GATHER 1
#define XR_KERNEL_STRIP 2
#define XR_KERNEL_STRIP_ANY 3
#define XR_KERNEL_STRIP_LDS 4

typedef struct {
    int32_t kernel;
    int32_t block_w;
    int32_t block_h;
    int32_t ppt_x;
    int32_t ppt_y;
    int32_t order;
} xr_tile;

/*
 * Forward resize, bilinear (paper eqs. 1-5 with half-pixel centres and
 * clamp-to-edge taps). Computes dst rows [dst->row0, dst->row0 + dst->rows)
 * of every plane. src and dst must agree in dtype, channels and planes; the
 * src band must hold every source row those output rows read (rows
 * floor(s(first)) .. floor(s(last)) + 1, clamped), else XR_ERR_RANGE.
 * `tile` = NULL or kernel = XR_KERNEL_AUTO selects the tuned shape.
 */
int xr_resize_bilinear(const xr_image *src, const xr_image *dst, const xr_tile *tile, void *stream);

/*
 * Forward resize, Keys bicubic with a = -1/2, 4x4 taps per output pixel
 * (paper section II.B names bicubic interpolation; the kernel is Keys 1981).
 * Same contract as xr_resize_bilinear; the src band must hold source rows
 * floor(s(first)) - 1 .. floor(s(last)) + 2, clamped. No antialiasing when
 * shrinking: the 4 taps are used at every scale.
 */
int xr_resize_bicubic(const xr_image *src, const xr_image *dst, const xr_tile *tile, void *stream);

/*
 * Forward resize with a chosen filter and coordinate map.
 *  filter  = XR_BILINEAR, XR_BICUBIC, or XR_NEAREST: one tap, the source
 *            pixel whose area contains the mapped point, floor(s + 1/2) under
 *            XR_MAP_HALF_PIXEL (pixel i covers [i - 1/2, i + 1/2)) and
 *            floor(s) under XR_MAP_PAPER (pixel i covers [i, i + 1)); it
 *            copies source values exactly. Nearest neighbour is one of the
 *            interpolation methods section II of the paper names.
 *          XR_BILINEAR_AA / XR_BICUBIC_AA (not in the paper; PIL's
 *            convention): the filter stretched by sigma = max(1, N_in/N_out),
 *            taps |i - s| < R sigma (R = 1, 2) inside the image (dropped, not
 *            clamped, at the edges), weights K((i - s)/sigma) divided by their
 *            sum (float32). Pixel-centre map only. One output pixel per thread
 *            in a block of block_w x block_h threads (ppt 1 x 1, order 0):
 *            XR_KERNEL_GATHER reads every tap from global memory;
 *            XR_KERNEL_STRIP_LDS stages the block's source window in LDS and
 *            filters it separably (rows, then columns); when the grid holds
 *            enough workgroups, one takes up to 4 tiles down its column. Both
 *            give identical bits. Strip kinds (and XR_KERNEL_AUTO before tuning) take the
 *            first LDS block of 64x4, 64x2, 32x2, 16x2 that fits, else a 64x4
 *            gather. XR_ERR_ARG when the workgroup's LDS exceeds 96 KiB: the
 *            weight tables, 4 (2 bw + 2 bh + bw kx + bh ky) bytes with
 *            k = floor(2 R sigma) + 1, plus for LDS blocks the source window
 *            (W x H pixels, W = floor(((bw - 1) N_in + 2 R max(N_in, N_out)) / N_out) + 2
 *            clipped to the width, H likewise) and an H x bw x channels float32
 *            row buffer.
 *  mapping = XR_MAP_HALF_PIXEL (as xr_resize_bilinear / _bicubic) or
 *            XR_MAP_PAPER: s = x N_in / N_out, the map of eq. 1 as printed
 *            (x_p = x_f / scale with scale = N_out / N_in from the sizes);
 *            eqs. 2-5 then apply unchanged, taps clamped to the image.
 * xr_resize(src, dst, XR_BILINEAR, XR_MAP_HALF_PIXEL, tile, stream) is
 * xr_resize_bilinear(src, dst, tile, stream); likewise for bicubic. Same
 * contract otherwise (bands: see xr_needed_rows_map). XR_ERR_ARG for an
 * unknown filter or mapping.
 */
int xr_resize(const xr_image *src, const xr_image *dst, int32_t filter, int32_t mapping,
              const xr_tile *tile, void *stream);

/*
 * Batched resize of many images of uneven sizes and scales in ONE persistent
 * launch (the paper's per-image tiling question asked for a whole batch,
 * section III.B).
 *
 * xr_batch_workspace_bytes(n): bytes of device workspace for n jobs.
 * xr_batch_prepare: validates every job exactly like xr_resize_*, groups
 *   the jobs by kind (filter x channel count; jobs narrower than the
 *   filter's taps or than one thread's run form a fifth kind), splits every
 *   output into tiles of `tile` (NULL = the shape xr_batch_autotune chose for
 *   this dtype, else 256x1 threads with 14-row strips; block_w a multiple of
 *   64, block_w * block_h <= 256, ppt_y <= 256; the output columns per
 *   thread are fixed per kind, tile.ppt_x is ignored), orders each kind's
 *   jobs largest-first, and uploads the job table and tile prefix sums to
 *   `dev_ws` (device memory, 256-byte aligned, >= xr_batch_workspace_bytes(n))
 *   with an asynchronous copy on `stream`. The host copy of `jobs` may be
 *   reused once the call returns. NOT capturable (XR_ERR_CAPTURE).
 *   All jobs must share one dtype.
 * xr_resize_batched: one persistent launch per job kind present, back to
 *   back on `stream`, that together process every tile of every prepared
 *   job. Capturable and replayable; it allocates nothing. The workspace must
 *   not be used by two launches at the same time.
 * Each output pixel is bit-identical to the one xr_resize_bilinear /
 * xr_resize_bicubic writes for the same job.
 */
typedef struct {
    xr_image src;
    xr_image dst;
    int32_t filter;    /* XR_BILINEAR or XR_BICUBIC (pixel-centre map) */
} xr_job;

size_t xr_batch_workspace_bytes(int32_t n_jobs);
int xr_batch_prepare(const xr_job *jobs, int32_t n_jobs, const xr_tile *tile, void *dev_ws,
                     size_t ws_bytes, void *stream);
int xr_resize_batched(const void *dev_ws, int32_t n_jobs, void *stream);

/*
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): xr_batch_prepare + xr_resize_batched in
 * one call whose workspace is a static array of the library in device memory
 * instead of a caller's buffer. It validates exactly like xr_batch_prepare
 * (same error codes), uploads the job table with a copy on `stream` that it
 * waits for, and launches like xr_resize_batched; outputs are bit-identical
 * to that pair's. At most 1024 jobs per call (XR_ERR_WORKSPACE beyond).
 * Allocates nothing: no hipMalloc, hipFree or allocating library call. Each
 * GPU holds one such workspace (128.25 KiB) until the process ends, shared
 * by every call on that GPU: calls whose launches can overlap on one GPU (on
 * different streams) race, and must be ordered by the caller (one stream, or
 * a synchronisation between them). NOT capturable (XR_ERR_CAPTURE).
 */
int xr_resize_batched_static(const xr_job *jobs, int32_t n_jobs, const xr_tile *tile, void *stream);

/*
 * Autotuner of the batched launch (the paper's tile-shape question, sections
 * III.A and IV, asked for a whole batch): prepares `dev_ws` with each
 * candidate shape in turn (NULL = built-in list: 64x4, 128x2 and 256x1
 * threads, strips of 4 to 190 rows; ppt_x is ignored), times `groups` groups
 * of `reps` launches with HIP events on `stream`, and keeps the shape with
 * the smallest median time per launch. On return `dev_ws` is prepared with
 * that shape, *best / *best_ms (either may be NULL) hold it, and later
 * xr_batch_prepare calls with tile = NULL and the same dtype use it.
 * Every timed launch writes every dst (the results do not depend on the
 * shape). Synchronises `stream`; NOT capturable (XR_ERR_CAPTURE). Errors as
 * xr_batch_prepare, plus XR_ERR_ARG for reps, groups or candidates < 1.
 */
int xr_batch_autotune(const xr_job *jobs, int32_t n_jobs, const xr_tile *candidates,
                      int32_t n_candidates, int32_t reps, int32_t groups, void *dev_ws,
                      size_t ws_bytes, xr_tile *best, float *best_ms, void *stream);

/*
 * Adjoint of the resize with respect to its input: grad_src = A^T grad_dst,
 * where A is the linear map of the forward call with the same filter and
 * sizes; every output pixel scatters wy_j * wx_i * g onto its clamped taps
 * (the transpose of eq. 5). Gradients stored as float32 or float16 (both
 * images of one type; XR_ERR_DTYPE otherwise), summed in float32 and rounded
 * once to the storage type. Whole images only (row0 = 0, rows = height on
 * both), planes map one to one, channels 1 or 4.
 * grad_src is OVERWRITTEN: each workgroup owns a tile of grad_src, gathers the
 * contributions of every output pixel that touches the tile (rows of the
 * horizontal adjoint in LDS, then columns) and stores the tile once: no
 * atomics, no clearing pass. Every sum runs in a fixed order, so the result
 * is deterministic. Exact x2 takes a register walk plus a border pass
 * instead (also deterministic; with float16 storage the border pixels are
 * summed in full there, so every gradient is rounded once). XR_ERR_SHAPE if the upscale is too
 * strong for one tile (rows beyond about 190x, columns beyond a few hundred x).
 */
int xr_resize_backward(const xr_image *grad_dst, const xr_image *grad_src, int32_t filter,
                       void *stream);

/*
 * Launch-shape tuning (the paper's tiling question, section IV, measured on
 * this GPU). Times every candidate with HIP events (one warm-up launch, then
 * `groups` groups of `reps` launches; the candidate's time is the median
 * group's mean), cycling through the `n_pairs` image pairs srcs[k] -> dsts[k]
 * so that a working set larger than the caches can be tuned honestly. All
 * pairs must have the same filter key, sizes, dtype and channels. Writes the
 * fastest shape to *best and its time per launch in ms to *best_ms (either
 * may be NULL) and remembers it for later XR_KERNEL_AUTO calls with the same
 * key (filter, dtype, channels, the scale class of each axis: x2, identity,
 * other up, x0.5, other down; and the size class of the output's
 * width x height x planes pixels: up to 2^16, 2^20, 2^24, 2^26, beyond).
 * Overwrites the dsts.
 * candidates = NULL uses the built-in candidate list. Synchronises the
 * stream; NOT capturable.
 * xr_tune_candidates: copies up to `cap` built-in candidates for the given
 * key into `out` and returns how many exist.
 */
int xr_autotune(const xr_image *srcs, const xr_image *dsts, int32_t n_pairs, int32_t filter,
                const xr_tile *candidates, int32_t n_candidates, int32_t reps, int32_t groups,
                xr_tile *best, float *best_ms, void *stream);
int32_t xr_tune_candidates(int32_t filter, int32_t dtype, int32_t channels, int32_t in_w,
                           int32_t in_h, int32_t out_w, int32_t out_h, xr_tile *out, int32_t cap);

/*
 * The shape XR_KERNEL_AUTO resolves to for a key (images of one plane): the
 * tuned one if xr_autotune (or xr_set_tile) stored one, else the built-in
 * default. xr_set_tile with kernel XR_KERNEL_AUTO forgets the key's shape.
 */
int xr_get_tile(int32_t filter, int32_t dtype, int32_t channels, int32_t in_w, int32_t in_h,
                int32_t out_w, int32_t out_h, xr_tile *out);
int xr_set_tile(int32_t filter, int32_t dtype, int32_t channels, int32_t in_w, int32_t in_h,
                int32_t out_w, int32_t out_h, const xr_tile *tile);

/*
 * Persisted launch shapes (the tuned table of xr_autotune / xr_set_tile).
 * xr_tune_save writes the table to the text file `path`, headed by the
 * current device's architecture name, its compute-unit count and the
 * library's build identity (a hash of its kernel sources).
 * xr_tune_load merges the shapes of such a file into the table and sets
 * *n_loaded to their number; a file of another architecture, CU count or
 * build loads nothing (*n_loaded = 0, XR_OK), so a stale cache is ignored.
 * Both query the current device (HIP calls); XR_ERR_ARG when the file cannot
 * be written or read.
 */
int xr_tune_save(const char *path);
int xr_tune_load(const char *path, int32_t *n_loaded);

/*
 * Host-side geometry (no HIP call; usable without a GPU).
 * xr_source_taps: for output index x of an axis n_in -> n_out, the base tap
 *   x0 = floor(s(x)) and the numerator / denominator of t = num/den (eqs. 1-4).
 * xr_needed_rows: inclusive range of clamped source rows that output rows
 *   [row0, row0 + rows) read (pixel-centre map; XR_BILINEAR or XR_BICUBIC).
 * xr_needed_rows_map: the same for any filter of xr_resize and either map.
 * xr_thread_of_pixel: eq. 6 inverted for a tile shape: the workgroup
 *   (block_x, block_y) and the thread (thread_x, thread_y) that compute output
 *   pixel (px, py), plus the pixel's index within that thread's ppt_x x ppt_y
 *   group (sub_x, sub_y).
 */
int xr_source_taps(int32_t n_in, int32_t n_out, int32_t x, int32_t *x0, int64_t *t_num,
                   int64_t *t_den);
int xr_needed_rows(int32_t in_h, int32_t out_h, int32_t row0, int32_t rows, int32_t filter,
                   int32_t *first, int32_t *last);
int xr_needed_rows_map(int32_t in_h, int32_t out_h, int32_t row0, int32_t rows, int32_t filter,
                       int32_t mapping, int32_t *first, int32_t *last);
int xr_thread_of_pixel(const xr_tile *tile, int32_t px, int32_t py, int32_t *block_x,
                       int32_t *block_y, int32_t *thread_x, int32_t *thread_y, int32_t *sub_x,
                       int32_t *sub_y);

/* Strings. xr_strerror never returns NULL; xr_last_error is thread-local and
 * describes the most recent failing call on the calling thread. */
const char *xr_strerror(int code);
const char *xr_last_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int xr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* XRESIZE_H */
