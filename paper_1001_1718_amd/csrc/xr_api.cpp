// C-ABI layer of libxresize.so: argument validation (always before any HIP
// call), launch-shape selection, the batched job table, tuning, and error
// reporting. The kernels live in xr_forward.hip and xr_backward.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/xresize.h"
#include "xr_internal.h"

// Identity of the kernel build (a hash of the kernel sources, set by the build).
#ifndef XR_BUILD_ID
#define XR_BUILD_ID "unversioned"
#endif

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int fail_hip(hipError_t e, const char *what)
{
    return fail(XR_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), static_cast<int>(e));
}

int elem_size(int32_t dtype)
{
    switch (dtype) {
    case XR_U8:
        return 1;
    case XR_F16:
        return 2;
    case XR_F32:
        return 4;
    default:
        return 0;
    }
}

// ---- exact host geometry (eqs. 1-4) ------------------------------------

int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0)))
        --q;
    return q;
}

bool valid_filter(int32_t filter)
{
    return filter == XR_BILINEAR || filter == XR_BICUBIC || filter == XR_NEAREST ||
           filter == XR_BILINEAR_AA || filter == XR_BICUBIC_AA;
}
bool is_aa(int32_t filter) { return filter == XR_BILINEAR_AA || filter == XR_BICUBIC_AA; }
int32_t aa_radius(int32_t filter) { return filter == XR_BICUBIC_AA ? 2 : 1; }

// Antialiased taps of output index x (radius r): every i with
// s - r sigma < i <= s + r sigma inside [0, n_in - 1], sigma = max(1, n_in/n_out).
void aa_taps(int64_t x, int64_t n_in, int64_t n_out, int32_t r, int64_t *lo, int64_t *hi);
bool valid_mapping(int32_t mapping) { return mapping == XR_MAP_HALF_PIXEL || mapping == XR_MAP_PAPER; }

// Base tap of output index x (eqs. 1-4) with o = 1 for pixel centres,
// s(x) = ((2x+1) n_in - n_out) / (2 n_out), and o = 0 for the printed map,
// s(x) = x n_in / n_out: x0 = floor(s(x)); for nearest neighbour the pixel
// whose area holds the point, floor((2x+o) n_in / (2 n_out)).
int64_t base_tap(int64_t x, int64_t n_in, int64_t n_out, int32_t filter = XR_BILINEAR,
                 int32_t mapping = XR_MAP_HALF_PIXEL)
{
    const int64_t o = mapping == XR_MAP_HALF_PIXEL ? 1 : 0;
    if (filter == XR_NEAREST)
        return floor_div((2 * x + o) * n_in, 2 * n_out);
    return floor_div((2 * x + o) * n_in - o * n_out, 2 * n_out);
}

int taps_of(int32_t filter) { return filter == XR_BICUBIC ? 4 : (filter == XR_NEAREST ? 1 : 2); }
int first_offset(int32_t filter) { return filter == XR_BICUBIC ? -1 : 0; }

void aa_taps(int64_t x, int64_t n_in, int64_t n_out, int32_t r, int64_t *lo, int64_t *hi)
{
    const int64_t num = (2 * x + 1) * n_in - n_out;
    const int64_t reach = 2 * r * std::max(n_in, n_out);
    *lo = std::max<int64_t>(floor_div(num - reach, 2 * n_out) + 1, 0);
    *hi = std::min<int64_t>(floor_div(num + reach, 2 * n_out), n_in - 1);
}

void needed_rows(int32_t in_h, int32_t out_h, int32_t row0, int32_t rows, int32_t filter,
                 int32_t *first, int32_t *last, int32_t mapping = XR_MAP_HALF_PIXEL)
{
    if (is_aa(filter)) {
        int64_t lo, hi, lo2, hi2;
        aa_taps(row0, in_h, out_h, aa_radius(filter), &lo, &hi);
        aa_taps(row0 + rows - 1, in_h, out_h, aa_radius(filter), &lo2, &hi2);
        *first = static_cast<int32_t>(lo);
        *last = static_cast<int32_t>(hi2);
        return;
    }
    const int64_t lo = base_tap(row0, in_h, out_h, filter, mapping) + first_offset(filter);
    const int64_t hi = base_tap(row0 + rows - 1, in_h, out_h, filter, mapping) + first_offset(filter) +
                       taps_of(filter) - 1;
    *first = static_cast<int32_t>(std::min<int64_t>(std::max<int64_t>(lo, 0), in_h - 1));
    *last = static_cast<int32_t>(std::min<int64_t>(std::max<int64_t>(hi, 0), in_h - 1));
}

// ---- validation ---------------------------------------------------------

int64_t image_extent(const xr_image &im)
{
    const int64_t row_bytes = static_cast<int64_t>(im.width) * im.channels * elem_size(im.dtype);
    return static_cast<int64_t>(im.planes - 1) * im.plane_pitch +
           static_cast<int64_t>(im.rows - 1) * im.row_pitch + row_bytes;
}

int check_image(const xr_image *im, const char *name)
{
    if (!im)
        return fail(XR_ERR_NULL, "%s descriptor is NULL", name);
    if (!im->data)
        return fail(XR_ERR_NULL, "%s.data is NULL", name);
    if (im->width < 1 || im->height < 1 || im->width > XR_MAX_SIDE || im->height > XR_MAX_SIDE)
        return fail(XR_ERR_SHAPE, "%s size %dx%d outside 1..%d", name, im->width, im->height,
                    XR_MAX_SIDE);
    if (im->planes < 1 || im->planes > 65535)
        return fail(XR_ERR_SHAPE, "%s.planes = %d outside 1..65535", name, im->planes);
    const int es = elem_size(im->dtype);
    if (es == 0)
        return fail(XR_ERR_DTYPE, "%s.dtype = %d is not XR_U8, XR_F16 or XR_F32", name, im->dtype);
    if (im->channels != 1 && im->channels != 4)
        return fail(XR_ERR_CHANNELS, "%s.channels = %d (must be 1 or 4)", name, im->channels);
    if (im->rows < 1 || im->row0 < 0 || static_cast<int64_t>(im->row0) + im->rows > im->height)
        return fail(XR_ERR_RANGE, "%s band rows [%d, %d) outside [0, %d)", name, im->row0,
                    im->row0 + im->rows, im->height);
    const int64_t px = static_cast<int64_t>(im->channels) * es;
    const int64_t row_bytes = px * im->width;
    if (im->row_pitch < row_bytes || im->row_pitch % px != 0)
        return fail(XR_ERR_PITCH, "%s.row_pitch = %lld (need >= %lld, multiple of %lld)", name,
                    static_cast<long long>(im->row_pitch), static_cast<long long>(row_bytes),
                    static_cast<long long>(px));
    if (im->planes > 1) {
        const int64_t need = static_cast<int64_t>(im->rows - 1) * im->row_pitch + row_bytes;
        if (im->plane_pitch < need || im->plane_pitch % px != 0)
            return fail(XR_ERR_PITCH, "%s.plane_pitch = %lld (need >= %lld, multiple of %lld)", name,
                        static_cast<long long>(im->plane_pitch), static_cast<long long>(need),
                        static_cast<long long>(px));
    }
    if (reinterpret_cast<uintptr_t>(im->data) % static_cast<uintptr_t>(px) != 0)
        return fail(XR_ERR_PITCH, "%s.data is not aligned to the %lld-byte pixel", name,
                    static_cast<long long>(px));
    return XR_OK;
}

bool overlaps(const xr_image &a, const xr_image &b)
{
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a.data);
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(b.data);
    const uintptr_t a1 = a0 + static_cast<uintptr_t>(image_extent(a));
    const uintptr_t b1 = b0 + static_cast<uintptr_t>(image_extent(b));
    return a0 < b1 && b0 < a1;
}

int check_pair(const xr_image *src, const xr_image *dst, int32_t filter,
               int32_t mapping = XR_MAP_HALF_PIXEL)
{
    if (!valid_filter(filter))
        return fail(XR_ERR_ARG, "filter = %d is not one of XR_BILINEAR .. XR_BICUBIC_AA", filter);
    if (!valid_mapping(mapping))
        return fail(XR_ERR_ARG, "mapping = %d is not XR_MAP_HALF_PIXEL or XR_MAP_PAPER", mapping);
    if (is_aa(filter) && mapping != XR_MAP_HALF_PIXEL)
        return fail(XR_ERR_ARG, "the antialiased filters take the pixel-centre map");
    int rc = check_image(src, "src");
    if (rc)
        return rc;
    rc = check_image(dst, "dst");
    if (rc)
        return rc;
    if (src->dtype != dst->dtype)
        return fail(XR_ERR_DTYPE, "src.dtype %d != dst.dtype %d", src->dtype, dst->dtype);
    if (src->channels != dst->channels)
        return fail(XR_ERR_CHANNELS, "src.channels %d != dst.channels %d", src->channels,
                    dst->channels);
    if (src->planes != dst->planes)
        return fail(XR_ERR_SHAPE, "src.planes %d != dst.planes %d", src->planes, dst->planes);
    int32_t first, last;
    needed_rows(src->height, dst->height, dst->row0, dst->rows, filter, &first, &last, mapping);
    if (first < src->row0 || last > src->row0 + src->rows - 1)
        return fail(XR_ERR_RANGE, "output rows [%d, %d) read source rows %d..%d but src holds [%d, %d)",
                    dst->row0, dst->row0 + dst->rows, first, last, src->row0,
                    src->row0 + src->rows);
    if (overlaps(*src, *dst))
        return fail(XR_ERR_ALIAS, "src and dst memory overlap");
    return XR_OK;
}

// The source base and pitches are 4-byte aligned and a row is a whole number
// of 4-byte words (the LDS strip kernel then stages small pixels as words).
bool src_aligned4(const xr_image &src)
{
    const int64_t row_bytes = static_cast<int64_t>(src.width) * src.channels * elem_size(src.dtype);
    return reinterpret_cast<uintptr_t>(src.data) % 4 == 0 && src.row_pitch % 4 == 0 &&
           (src.planes == 1 || src.plane_pitch % 4 == 0) && row_bytes % 4 == 0;
}

xr::ResizeArgs make_args(const xr_image &src, const xr_image &dst, int32_t mapping = XR_MAP_HALF_PIXEL)
{
    xr::ResizeArgs a{};
    a.src = static_cast<const unsigned char *>(src.data);
    a.dst = static_cast<unsigned char *>(dst.data);
    a.src_pitch = src.row_pitch;
    a.src_plane_pitch = src.planes > 1 ? src.plane_pitch : 0;
    a.dst_pitch = dst.row_pitch;
    a.dst_plane_pitch = dst.planes > 1 ? dst.plane_pitch : 0;
    a.in_w = src.width;
    a.in_h = src.height;
    a.out_w = dst.width;
    a.out_h = dst.height;
    a.src_row0 = src.row0;
    a.src_rows = src.rows;
    a.dst_row0 = dst.row0;
    a.dst_rows = dst.rows;
    a.planes = src.planes;
    const auto al = [](const void *p, int64_t v1, int64_t v2) {
        return reinterpret_cast<uintptr_t>(p) % 16 == 0 && v1 % 16 == 0 && v2 % 16 == 0;
    };
    a.aligned16 = al(src.data, a.src_pitch, a.src_plane_pitch) && al(dst.data, a.dst_pitch, a.dst_plane_pitch);
    a.aligned4 = src_aligned4(src);
    a.map_off = mapping == XR_MAP_HALF_PIXEL ? 1 : 0;
    return a;
}

// The exact x2 and x0.5 walks assume pixel centres and 2 or 4 taps.
int32_t axis_mode(const xr_image &src, const xr_image &dst, const xr_tile &t, int32_t filter,
                  int32_t mapping)
{
    if (t.kernel != XR_KERNEL_STRIP || mapping != XR_MAP_HALF_PIXEL || filter == XR_NEAREST ||
        is_aa(filter))
        return xr::kGeneral;
    // the x2 walk moves whole dwords through buffer resources: 4-byte aligned
    // images and pitches
    const auto al4 = [](const xr_image &im) {
        return reinterpret_cast<uintptr_t>(im.data) % 4 == 0 && im.row_pitch % 4 == 0 &&
               (im.planes == 1 || im.plane_pitch % 4 == 0);
    };
    if (dst.width == 2 * src.width && dst.height == 2 * src.height && al4(src) && al4(dst))
        return xr::kUp2;
    if (2 * dst.width == src.width && 2 * dst.height == src.height)
        return xr::kDown2;
    return xr::kGeneral;
}

// ---- launch shapes ------------------------------------------------------

// scale class of one axis: 0 = x2 up exactly, 1 = identity, 2 = other up,
// 3 = x2 down exactly, 4 = other down
int scale_class(int32_t n_in, int32_t n_out)
{
    if (n_out == 2 * n_in)
        return 0;
    if (n_out == n_in)
        return 1;
    if (n_out > n_in)
        return 2;
    if (n_in == 2 * n_out)
        return 3;
    return 4;
}

// size class of the output, out_w x out_h x planes pixels: 0 up to 2^16
// (256^2), 1 up to 2^20 (1024^2), 2 up to 2^24 (4096^2), 3 up to 2^26
// (8192^2), 4 beyond. A shape tuned on a large output fills the GPU with
// long strips that a small one would leave mostly idle.
int size_class(int32_t out_w, int32_t out_h, int32_t planes)
{
    const int64_t px = static_cast<int64_t>(out_w) * out_h * std::max(planes, 1);
    return px <= (int64_t(1) << 16) ? 0 : px <= (int64_t(1) << 20) ? 1 : px <= (int64_t(1) << 24) ? 2
                                                                 : px <= (int64_t(1) << 26) ? 3 : 4;
}

using TuneKey = std::tuple<int, int, int, int, int, int>;

TuneKey tune_key(int32_t filter, int32_t dtype, int32_t channels, int32_t in_w, int32_t in_h,
                 int32_t out_w, int32_t out_h, int32_t planes)
{
    return TuneKey(filter, dtype, channels, scale_class(in_w, out_w), scale_class(in_h, out_h),
                   size_class(out_w, out_h, planes));
}

std::mutex g_tune_mu;
std::map<TuneKey, xr_tile> g_tuned;

// Untuned launch shape, by scale (the tuner's typical winners on MI355X):
//  exact x2     256x1 threads, 4 (RGBA) or 8 (one channel) columns per
//               thread, strips of 24 rows (the x2 walk rounds a strip up to
//               a multiple of 8 rows);
//  exact x0.5   512x1 threads, 2 or 4 columns, strips of 6 rows;
//  other        128x2 threads, 2 or 4 columns, strips of 30 rows when the
//               rows grow, 6 when they shrink (a strip then walks several
//               source rows per output row).
// Strips are shortened (24/30 -> 16 -> 14 -> 8 -> 6 -> 2 -> 1 rows) until the
// launch has about 8 wavefronts per SIMD (2048 x 4); tiny outputs use 64-wide
// workgroups.
xr_tile default_tile(int32_t channels, int32_t in_w, int32_t in_h, int32_t out_w, int32_t rows,
                     int32_t out_h, int32_t planes)
{
    const bool c4 = channels == 4;
    xr_tile t{};
    t.kernel = XR_KERNEL_STRIP;
    t.order = 0;
    int first;
    if (out_w == 2 * in_w && out_h == 2 * in_h) {
        t.block_w = 256;
        t.block_h = 1;
        t.ppt_x = c4 ? 4 : 8;
        first = 24;  // the x2 walk's strips of 12 row pairs (measured best on large images)
    } else if (2 * out_w == in_w && 2 * out_h == in_h) {
        t.block_w = 512;
        t.block_h = 1;
        t.ppt_x = c4 ? 2 : 4;
        first = 6;
    } else {
        t.block_w = 128;
        t.block_h = 2;
        t.ppt_x = c4 ? 2 : 4;
        first = out_h >= in_h ? 30 : 6;
    }
    const auto waves = [&](const xr_tile &u) {
        const int64_t wcols = (static_cast<int64_t>(out_w) + 64 * u.ppt_x - 1) / (64 * u.ppt_x);
        return wcols * ((static_cast<int64_t>(rows) + u.ppt_y - 1) / u.ppt_y) * planes;
    };
    const int64_t target = 8192;
    const int steps[] = {first, 16, 14, 8, 6, 2, 1};
    for (int ppy : steps) {
        if (ppy > first)
            continue;
        t.ppt_y = ppy;
        if (waves(t) >= target)
            return t;
    }
    t.ppt_x = c4 ? 2 : 4;
    t.block_w = 64;
    t.block_h = 1;
    return t;
}

int check_tile(const xr_tile &t, int32_t dtype, int32_t channels)
{
    if (t.kernel == XR_KERNEL_GATHER) {
        if (t.order != 0)
            return fail(XR_ERR_ARG, "the gather kernel takes order = 0");
        if (t.block_w < 1 || t.block_h < 1 || t.block_w * t.block_h > 1024 || t.ppt_x != 1 ||
            t.ppt_y != 1)
            return fail(XR_ERR_ARG, "gather tile %dx%d (ppt %dx%d) invalid: need 1..1024 threads, ppt 1x1",
                        t.block_w, t.block_h, t.ppt_x, t.ppt_y);
        return XR_OK;
    }
    if (t.kernel == XR_KERNEL_STRIP || t.kernel == XR_KERNEL_STRIP_ANY) {
        if (t.block_w < 64 || t.block_w % 64 != 0 || t.block_h < 1 || t.block_w * t.block_h > 512)
            return fail(XR_ERR_ARG,
                        "strip tile block %dx%d invalid: block_w a multiple of 64, at most 512 threads",
                        t.block_w, t.block_h);
        if (t.order != 0 && t.order != 1)
            return fail(XR_ERR_ARG, "tile.order = %d (must be 0 or 1)", t.order);
        if (!xr::strip_ppx_supported(dtype, channels, t.ppt_x))
            return fail(XR_ERR_ARG, "strip ppt_x = %d not built for %d channels", t.ppt_x, channels);
        if (t.ppt_y < 1 || t.ppt_y > 4096)
            return fail(XR_ERR_ARG, "strip ppt_y = %d outside 1..4096", t.ppt_y);
        return XR_OK;
    }
    if (t.kernel == XR_KERNEL_STRIP_LDS) {
        if (t.block_w < 64 || t.block_w % 64 != 0 || t.block_w > 512 || t.block_h != 1)
            return fail(XR_ERR_ARG,
                        "LDS strip tile block %dx%d invalid: block_h 1, block_w a multiple of 64 up to 512",
                        t.block_w, t.block_h);
        if (t.order != 0 && t.order != 1)
            return fail(XR_ERR_ARG, "tile.order = %d (must be 0 or 1)", t.order);
        const int32_t ppx = xr::kLdsPpx[channels == 4 ? 1 : 0];
        if (t.ppt_x != ppx)
            return fail(XR_ERR_ARG, "LDS strip ppt_x = %d (must be %d for %d channels)", t.ppt_x, ppx,
                        channels);
        if (t.ppt_y < 1 || t.ppt_y > 4096)
            return fail(XR_ERR_ARG, "strip ppt_y = %d outside 1..4096", t.ppt_y);
        (void)dtype;
        return XR_OK;
    }
    return fail(XR_ERR_ARG, "tile.kernel = %d unknown", t.kernel);
}

// The LDS-staged strip kernel stages one workgroup's source row segment; it
// must fit the kernel's LDS and register budget for this scale.
// `aligned4` is unknown (taken as true) where only sizes are given.
int check_lds(const xr_tile &t, int32_t filter, int32_t dtype, int32_t channels, int32_t in_w,
              int32_t out_w, bool aligned4 = true)
{
    if (t.kernel != XR_KERNEL_STRIP_LDS)
        return XR_OK;
    if (!xr::strip_lds_fits(filter, dtype, channels, in_w, out_w, t.block_w, aligned4))
        return fail(XR_ERR_ARG,
                    "LDS strip: a %d-thread workgroup's row segment for %d -> %d columns does not fit "
                    "(or one-channel source rows are not 4-byte aligned words); use a narrower "
                    "workgroup or another kernel", t.block_w, in_w, out_w);
    return XR_OK;
}

int64_t aa_lds_bytes(const xr_tile &t, int32_t filter, const xr_image &src, const xr_image &dst)
{
    const int32_t r = aa_radius(filter);
    if (t.kernel == XR_KERNEL_STRIP_LDS)
        return xr::aa_tile_plan(src.width, src.height, dst.width, dst.height, r, t.block_w, t.block_h,
                                elem_size(src.dtype) * src.channels, src.channels)
            .lds_bytes;
    return xr::aa_plan(src.width, src.height, dst.width, dst.height, r, t.block_w, t.block_h).lds_bytes;
}

// The antialiased filters take a gather tile (k_gather_aa) or an LDS tile
// (k_tile_aa): block_w x block_h threads, one output pixel each.
int check_aa(const xr_tile &t, int32_t filter, const xr_image &src, const xr_image &dst)
{
    if (!is_aa(filter))
        return XR_OK;
    if (t.kernel != XR_KERNEL_GATHER && t.kernel != XR_KERNEL_STRIP_LDS)
        return fail(XR_ERR_ARG, "the antialiased filters take XR_KERNEL_GATHER or XR_KERNEL_STRIP_LDS tiles");
    if (t.block_w < 1 || t.block_h < 1 || t.block_w * t.block_h > 1024 || t.ppt_x != 1 || t.ppt_y != 1 ||
        t.order != 0)
        return fail(XR_ERR_ARG,
                    "antialiased tile %dx%d (ppt %dx%d, order %d) invalid: need 1..1024 threads, ppt 1x1, "
                    "order 0", t.block_w, t.block_h, t.ppt_x, t.ppt_y, t.order);
    const int64_t bytes = aa_lds_bytes(t, filter, src, dst);
    if (bytes > xr::kAaLdsBudget)
        return fail(XR_ERR_ARG,
                    "antialiased resize: a %dx%d %s block needs %lld bytes of LDS (limit %lld); use a "
                    "smaller block%s", t.block_w, t.block_h,
                    t.kernel == XR_KERNEL_GATHER ? "gather" : "LDS", static_cast<long long>(bytes),
                    static_cast<long long>(xr::kAaLdsBudget),
                    t.kernel == XR_KERNEL_GATHER ? "" : " or a gather tile");
    return XR_OK;
}

// Default antialiased tile: the LDS kernel with the first block whose
// window fits, else the gather.
xr_tile aa_default_tile(int32_t filter, const xr_image &src, const xr_image &dst)
{
    const int blocks[][2] = {{64, 4}, {64, 2}, {32, 2}, {16, 2}};
    for (const auto &b : blocks) {
        const xr_tile t{XR_KERNEL_STRIP_LDS, b[0], b[1], 1, 1, 0};
        if (aa_lds_bytes(t, filter, src, dst) <= xr::kAaLdsBudget)
            return t;
    }
    return xr_tile{XR_KERNEL_GATHER, 64, 4, 1, 1, 0};
}

bool lds_usable(const xr_tile &t, int32_t filter, const xr_image &src, const xr_image &dst)
{
    return xr::strip_lds_fits(filter, src.dtype, src.channels, src.width, dst.width, t.block_w,
                              src_aligned4(src));
}

xr_tile resolve_tile(const xr_tile *tile, int32_t filter, const xr_image &src, const xr_image &dst)
{
    if (tile && tile->kernel != XR_KERNEL_AUTO)
        return *tile;
    const TuneKey key = tune_key(filter, src.dtype, src.channels, src.width, src.height, dst.width,
                                 dst.height, dst.planes);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tuned.find(key);
    // a tuned LDS shape applies only to sources it can stage (alignment is
    // not part of the key)
    if (it != g_tuned.end()) {
        const xr_tile &tt = it->second;
        if (is_aa(filter) ? aa_lds_bytes(tt, filter, src, dst) <= xr::kAaLdsBudget
                          : (tt.kernel != XR_KERNEL_STRIP_LDS || lds_usable(tt, filter, src, dst)))
            return tt;
    }
    return default_tile(src.channels, src.width, src.height, dst.width, dst.rows, dst.height,
                        dst.planes);
}

int check_grid(const xr_tile &t, const xr_image &dst)
{
    const int64_t rows_per_block = static_cast<int64_t>(t.block_h) * t.ppt_y;
    const int64_t gy = (dst.rows + rows_per_block - 1) / rows_per_block;
    if (gy > 65535)
        return fail(XR_ERR_ARG, "tile too short for %d rows: %lld workgroup rows > 65535", dst.rows,
                    static_cast<long long>(gy));
    return XR_OK;
}

int resize_common(const xr_image *src, const xr_image *dst, const xr_tile *tile, int32_t filter,
                  int32_t mapping, void *stream)
{
    int rc = check_pair(src, dst, filter, mapping);
    if (rc)
        return rc;
    xr_tile t = resolve_tile(tile, filter, *src, *dst);
    if (is_aa(filter)) {
        // strip shapes (and the untuned default) mean the default antialiased tile
        if (t.kernel == XR_KERNEL_STRIP || t.kernel == XR_KERNEL_STRIP_ANY ||
            (t.kernel == XR_KERNEL_STRIP_LDS && (t.ppt_x != 1 || t.ppt_y != 1)))
            t = aa_default_tile(filter, *src, *dst);
        rc = check_aa(t, filter, *src, *dst);
    } else {
        rc = check_tile(t, src->dtype, src->channels);
    }
    if (rc)
        return rc;
    rc = check_grid(t, *dst);
    if (rc)
        return rc;
    if (!is_aa(filter))
        rc = check_lds(t, filter, src->dtype, src->channels, src->width, dst->width, src_aligned4(*src));
    if (rc)
        return rc;
    const xr::ResizeArgs a = make_args(*src, *dst, mapping);
    const hipError_t e = xr::launch_forward(a, filter, src->dtype, src->channels, t,
                                            axis_mode(*src, *dst, t, filter, mapping),
                                            static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, "resize launch");
    return XR_OK;
}

// ---- batched workspaces -------------------------------------------------

struct BatchInfo {
    int32_t n_jobs;
    int32_t dtype;
    int32_t block_w, block_h;
    int32_t grid[xr::kBatchKinds];
};
std::mutex g_batch_mu;
std::map<const void *, BatchInfo> g_batches;
std::map<int32_t, xr_tile> g_batch_tuned;  // dtype -> shape chosen by xr_batch_autotune

// Untuned batched shape: 256-wide workgroups, 14-row strips.
xr_tile batch_default_tile(int32_t dtype)
{
    std::lock_guard<std::mutex> lock(g_batch_mu);
    auto it = g_batch_tuned.find(dtype);
    if (it != g_batch_tuned.end())
        return it->second;
    return xr_tile{XR_KERNEL_STRIP, 256, 1, 0, 14, 0};
}

// The current device's architecture name and compute-unit count (the key of
// persisted launch shapes).
int device_identity(std::string &arch, int &cus)
{
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess)
        return fail_hip(e, "device query");
    arch = prop.gcnArchName;
    for (char &c : arch)
        if (c == ' ')
            c = '_';
    cus = prop.multiProcessorCount;
    return XR_OK;
}

// ---- the batched launch without allocation ------------------------------
//
// xr_resize_batched_static keeps its workspace in `scratch`, a file-scope
// device array that every GPU the library runs on holds until the process
// ends. Host code never uses the array's name as an address: each device's
// address is looked up once (hipGetSymbolAddress, with that device current)
// and kept in g_scratch_ptr.
constexpr int32_t kStaticMaxJobs = 1024;
constexpr size_t kScratchBytes = xr::kBatchHeaderBytes + kStaticMaxJobs * sizeof(xr::BatchJob);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_static_mu;                  // the staging buffers below and g_scratch_ptr
void *g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` per device
unsigned char g_static_stage[kScratchBytes];
int32_t g_static_order[kStaticMaxJobs];

// this device's address of `scratch` (looked up on its first use)
int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail(XR_ERR_ARG, "device %d beyond the %d the static workspace supports", dev, kMaxDevices);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return fail_hip(e, "hipGetSymbolAddress(scratch)");
        if (!p)
            return fail(XR_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return XR_OK;
}

// Median per-launch milliseconds of each of n candidates: `groups` groups of
// `reps` launches, each group between HIP events. Everything is enqueued
// first and read after one synchronisation at the end, behind an untimed
// pre-roll of about 20 ms of the first candidate: the GPU runs 10-20% slower
// for 10-20 ms after it has idled, so waiting on every group would time every
// candidate in that state. run(k) enqueues one launch of candidate k.
template <typename Run>
hipError_t time_candidates(size_t n, int32_t reps, int32_t groups, hipStream_t s, Run run,
                           std::vector<float> &med)
{
    med.assign(n, 0.0f);
    if (n == 0)
        return hipSuccess;
    std::vector<hipEvent_t> ev(2 * n * static_cast<size_t>(groups) + 2, nullptr);
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < ev.size() && e == hipSuccess; ++i)
        e = hipEventCreate(&ev[i]);
    // one timed launch of the first candidate sizes the pre-roll
    if (e == hipSuccess)
        e = run(0);
    if (e == hipSuccess)
        e = hipEventRecord(ev[0], s);
    if (e == hipSuccess)
        e = run(0);
    if (e == hipSuccess)
        e = hipEventRecord(ev[1], s);
    if (e == hipSuccess)
        e = hipEventSynchronize(ev[1]);
    float one = 0.0f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&one, ev[0], ev[1]);
    const int64_t pre = std::min<int64_t>(4096, static_cast<int64_t>(20.0f / std::max(one, 1e-3f)) + 1);
    for (int64_t i = 0; i < pre && e == hipSuccess; ++i)
        e = run(0);
    for (size_t k = 0; k < n && e == hipSuccess; ++k) {
        e = run(k);  // warm-up
        for (int32_t g = 0; g < groups && e == hipSuccess; ++g) {
            hipEvent_t *p = &ev[2 + 2 * (k * groups + g)];
            e = hipEventRecord(p[0], s);
            for (int32_t r = 0; r < reps && e == hipSuccess; ++r)
                e = run(k);
            if (e == hipSuccess)
                e = hipEventRecord(p[1], s);
        }
    }
    if (e == hipSuccess)
        e = hipEventSynchronize(ev.back());
    std::vector<float> per_group(groups);
    for (size_t k = 0; k < n && e == hipSuccess; ++k) {
        for (int32_t g = 0; g < groups && e == hipSuccess; ++g) {
            const hipEvent_t *p = &ev[2 + 2 * (k * groups + g)];
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, p[0], p[1]);
            per_group[g] = ms / static_cast<float>(reps);
        }
        std::sort(per_group.begin(), per_group.end());
        med[k] = per_group[groups / 2];
    }
    for (hipEvent_t x : ev)
        if (x)
            (void)hipEventDestroy(x);
    return e;
}

// Validates a batch and builds its workspace image (header and job table,
// xr_batch_workspace_bytes(n_jobs) bytes) in host memory `host`; `order`
// holds n_jobs indices of scratch. No device memory is touched.
int build_batch(const xr_job *jobs, int32_t n_jobs, const xr_tile *tile, unsigned char *host, int32_t *order,
                BatchInfo &info, void *stream, const char *caller)
{
    const int32_t dtype = jobs[0].src.dtype;
    xr_tile t{};
    if (tile && tile->kernel != XR_KERNEL_AUTO) {
        t = *tile;
        if (t.kernel != XR_KERNEL_STRIP)
            return fail(XR_ERR_ARG, "the batched launch takes a strip tile");
    } else {
        t = batch_default_tile(dtype);
    }
    t.ppt_x = 0;  // fixed per job kind
    if (t.block_w < 64 || t.block_w % 64 != 0 || t.block_h < 1 || t.block_w * t.block_h > 256 ||
        t.ppt_y < 1 || t.ppt_y > xr::kBatchMaxStrip)
        return fail(XR_ERR_ARG, "batched tile block %dx%d ppt_y %d invalid", t.block_w, t.block_h,
                    t.ppt_y);
    for (int32_t k = 0; k < n_jobs; ++k) {
        const int rc = check_pair(&jobs[k].src, &jobs[k].dst, jobs[k].filter);
        if (rc)
            return fail(rc, "job %d: %s", k, g_last_error.c_str());
        if (jobs[k].filter != XR_BILINEAR && jobs[k].filter != XR_BICUBIC)
            return fail(XR_ERR_ARG, "job %d: the batched launch takes XR_BILINEAR or XR_BICUBIC", k);
        if (jobs[k].src.dtype != dtype)
            return fail(XR_ERR_DTYPE, "job %d: dtype %d differs from job 0 (%d)", k, jobs[k].src.dtype,
                        dtype);
    }
    for (int32_t k = 0; k < n_jobs; ++k) {
        const xr_image &d = jobs[k].dst;
        for (int32_t m = 0; m < n_jobs; ++m)
            if (overlaps(d, jobs[m].src) || (m != k && overlaps(d, jobs[m].dst)))
                return fail(XR_ERR_ALIAS, "job %d: dst overlaps job %d's %s", k, m,
                            m == k ? "src" : (overlaps(d, jobs[m].src) ? "src" : "dst"));
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(static_cast<hipStream_t>(stream), &cs);
    if (e != hipSuccess)
        return fail_hip(e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)
        return fail(XR_ERR_CAPTURE, "%s called on a capturing stream", caller);

    // grouped by kind, largest output first within a kind
    const auto fc_of = [&](const xr_job &j) {
        return (j.filter == XR_BICUBIC ? 2 : 0) + (j.src.channels == 4 ? 1 : 0);
    };
    const auto kind_of = [&](const xr_job &j) {
        const int32_t taps = j.filter == XR_BICUBIC ? 4 : 2;
        if (j.src.width < taps || j.dst.width < xr::batch_ppx(j.filter, dtype, j.src.channels))
            return xr::kBatchNarrow;
        return fc_of(j);
    };
    // (std::sort with the job index as the last key: the same order as a
    // stable sort, and no temporary buffer)
    for (int32_t k = 0; k < n_jobs; ++k)
        order[k] = k;
    std::sort(order, order + n_jobs, [&](int32_t p, int32_t q) {
        const int32_t kp = kind_of(jobs[p]), kq = kind_of(jobs[q]);
        if (kp != kq)
            return kp < kq;
        const int64_t wp = static_cast<int64_t>(jobs[p].dst.width) * jobs[p].dst.rows * jobs[p].dst.planes;
        const int64_t wq = static_cast<int64_t>(jobs[q].dst.width) * jobs[q].dst.rows * jobs[q].dst.planes;
        return wp != wq ? wp > wq : p < q;
    });
    std::memset(host, 0, xr_batch_workspace_bytes(n_jobs));
    auto *hdr = reinterpret_cast<xr::BatchHeader *>(host);
    auto *tab = reinterpret_cast<xr::BatchJob *>(host + xr::kBatchHeaderBytes);
    for (int32_t k = 0; k < xr::kBatchKinds; ++k)
        hdr->job_lo[k] = hdr->job_hi[k] = 0;
    for (int32_t k = 0; k < n_jobs; ++k) {
        const xr_job &j = jobs[order[k]];
        xr::BatchJob &b = tab[k];
        const int32_t kind = kind_of(j);
        if (k == 0 || tab[k - 1].kind != kind)
            hdr->job_lo[kind] = k;
        hdr->job_hi[kind] = k + 1;
        b.a = make_args(j.src, j.dst);
        b.kind = kind;
        b.kind_fc = fc_of(j);
        // a strip walks about ppt_y source rows or ppt_y output rows, whichever
        // is fewer output rows, so shrinking jobs do not make long tiles
        int64_t strip = std::max<int64_t>(
            1, std::min<int64_t>(t.ppt_y, (static_cast<int64_t>(t.ppt_y) * j.dst.height + j.src.height - 1) /
                                               j.src.height));
        // the source rows of a strip, (strip - 1) n_in / n_out + K + 1 at most,
        // stay below 2^31 bytes (32-bit buffer offsets)
        const int64_t max_rows = (int64_t(1) << 31) / j.src.row_pitch - 6;
        strip = std::min<int64_t>(strip, std::max<int64_t>(1, max_rows * j.dst.height / j.src.height));
        b.strip_h = static_cast<int32_t>(strip);
        const int64_t tile_w =
            static_cast<int64_t>(t.block_w) * (kind == xr::kBatchNarrow ? 1 : xr::batch_ppx(j.filter, dtype, j.src.channels));
        const int64_t tile_h = static_cast<int64_t>(t.block_h) * b.strip_h;
        b.tiles_x = static_cast<int32_t>((j.dst.width + tile_w - 1) / tile_w);
        b.tiles_y = static_cast<int32_t>((j.dst.rows + tile_h - 1) / tile_h);
        b.tile_begin = hdr->tiles[kind];
        hdr->tiles[kind] += static_cast<int64_t>(b.tiles_x) * b.tiles_y * j.dst.planes;
    }
    for (int32_t k = 0; k < xr::kBatchKinds; ++k)
        if (hdr->tiles[k] >= (int64_t(1) << 31))
            return fail(XR_ERR_ARG, "batch has %lld tiles of one kind (limit 2^31)",
                        static_cast<long long>(hdr->tiles[k]));
    int dev = 0, cus = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess)
        return fail_hip(e, "device query");
    hdr->n_jobs = n_jobs;
    hdr->dtype = dtype;
    hdr->block_w = t.block_w;
    hdr->block_h = t.block_h;
    hdr->ppt_y = t.ppt_y;
    info = BatchInfo{n_jobs, dtype, t.block_w, t.block_h, {}};
    for (int32_t k = 0; k < xr::kBatchKinds; ++k) {
        if (hdr->tiles[k] == 0)
            continue;
        const int32_t per_cu = xr::batched_blocks_per_cu(dtype, k, t.block_w * t.block_h);
        hdr->grid[k] = static_cast<int32_t>(
            std::max<int64_t>(1, std::min<int64_t>(static_cast<int64_t>(per_cu) * cus, hdr->tiles[k])));
        info.grid[k] = hdr->grid[k];
        hdr->ticket[k] = 0;
        hdr->done[k] = 0;
    }
    return XR_OK;
}

}  // namespace

extern "C" {

int xr_resize_bilinear(const xr_image *src, const xr_image *dst, const xr_tile *tile, void *stream)
{
    return resize_common(src, dst, tile, XR_BILINEAR, XR_MAP_HALF_PIXEL, stream);
}

int xr_resize_bicubic(const xr_image *src, const xr_image *dst, const xr_tile *tile, void *stream)
{
    return resize_common(src, dst, tile, XR_BICUBIC, XR_MAP_HALF_PIXEL, stream);
}

int xr_resize(const xr_image *src, const xr_image *dst, int32_t filter, int32_t mapping,
              const xr_tile *tile, void *stream)
{
    return resize_common(src, dst, tile, filter, mapping, stream);
}

size_t xr_batch_workspace_bytes(int32_t n_jobs)
{
    if (n_jobs < 1)
        return 0;
    return xr::kBatchHeaderBytes + static_cast<size_t>(n_jobs) * sizeof(xr::BatchJob);
}

int xr_batch_prepare(const xr_job *jobs, int32_t n_jobs, const xr_tile *tile, void *dev_ws,
                     size_t ws_bytes, void *stream)
{
    if (!jobs)
        return fail(XR_ERR_NULL, "jobs is NULL");
    if (n_jobs < 1)
        return fail(XR_ERR_ARG, "n_jobs = %d (must be >= 1)", n_jobs);
    if (!dev_ws)
        return fail(XR_ERR_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_ws) % 256 != 0)
        return fail(XR_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    if (ws_bytes < xr_batch_workspace_bytes(n_jobs))
        return fail(XR_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes,
                    xr_batch_workspace_bytes(n_jobs));
    std::vector<unsigned char> host(xr_batch_workspace_bytes(n_jobs));
    std::vector<int32_t> order(n_jobs);
    BatchInfo info{};
    const int rc = build_batch(jobs, n_jobs, tile, host.data(), order.data(), info, stream, "xr_batch_prepare");
    if (rc)
        return rc;
    hipError_t e = hipMemcpyAsync(dev_ws, host.data(), host.size(), hipMemcpyHostToDevice,
                                  static_cast<hipStream_t>(stream));
    if (e == hipSuccess)
        e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, "uploading the job table");
    std::lock_guard<std::mutex> lock(g_batch_mu);
    g_batches[dev_ws] = info;
    return XR_OK;
}

int xr_resize_batched(const void *dev_ws, int32_t n_jobs, void *stream)
{
    if (!dev_ws)
        return fail(XR_ERR_WORKSPACE, "workspace is NULL");
    BatchInfo info{};
    {
        std::lock_guard<std::mutex> lock(g_batch_mu);
        auto it = g_batches.find(dev_ws);
        if (it == g_batches.end())
            return fail(XR_ERR_WORKSPACE, "workspace was not prepared by xr_batch_prepare");
        info = it->second;
    }
    if (n_jobs != info.n_jobs)
        return fail(XR_ERR_ARG, "n_jobs = %d but the workspace holds %d jobs", n_jobs, info.n_jobs);
    const hipError_t e = xr::launch_batched(dev_ws, info.dtype, info.block_w, info.block_h, info.grid,
                                            static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, "batched launch");
    return XR_OK;
}

int xr_resize_batched_static(const xr_job *jobs, int32_t n_jobs, const xr_tile *tile, void *stream)
{
    if (!jobs)
        return fail(XR_ERR_NULL, "jobs is NULL");
    if (n_jobs < 1)
        return fail(XR_ERR_ARG, "n_jobs = %d (must be >= 1)", n_jobs);
    if (n_jobs > kStaticMaxJobs)
        return fail(XR_ERR_WORKSPACE, "n_jobs = %d exceeds the static workspace (%d jobs)", n_jobs,
                    kStaticMaxJobs);
    std::lock_guard<std::mutex> lock(g_static_mu);
    BatchInfo info{};
    int rc = build_batch(jobs, n_jobs, tile, g_static_stage, g_static_order, info, stream,
                         "xr_resize_batched_static");
    if (rc)
        return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail_hip(e, "hipGetDevice");
    void *ws = nullptr;
    rc = scratch_address(dev, &ws);
    if (rc)
        return rc;
    // the upload writes the whole header, so the tickets start at zero; the
    // staging buffer is reused by the next call, hence the synchronisation
    e = hipMemcpyAsync(ws, g_static_stage, xr_batch_workspace_bytes(n_jobs), hipMemcpyHostToDevice,
                       static_cast<hipStream_t>(stream));
    if (e == hipSuccess)
        e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, "uploading the job table");
    e = xr::launch_batched(ws, info.dtype, info.block_w, info.block_h, info.grid, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, "batched launch");
    return XR_OK;
}

int xr_batch_autotune(const xr_job *jobs, int32_t n_jobs, const xr_tile *candidates,
                      int32_t n_candidates, int32_t reps, int32_t groups, void *dev_ws,
                      size_t ws_bytes, xr_tile *best, float *best_ms, void *stream)
{
    if (!jobs)
        return fail(XR_ERR_NULL, "jobs is NULL");
    if (n_jobs < 1)
        return fail(XR_ERR_ARG, "n_jobs = %d (must be >= 1)", n_jobs);
    if (reps < 1 || groups < 1)
        return fail(XR_ERR_ARG, "reps = %d, groups = %d (both must be >= 1)", reps, groups);
    std::vector<xr_tile> cand;
    if (candidates) {
        if (n_candidates < 1)
            return fail(XR_ERR_ARG, "n_candidates = %d", n_candidates);
        cand.assign(candidates, candidates + n_candidates);
    } else {
        const int blocks[][2] = {{64, 4}, {128, 2}, {256, 1}};
        const int ppy_list[] = {4, 8, 14, 22, 30, 46, 62, 94, 126, 190};
        for (const auto &b : blocks)
            for (int ppy : ppy_list)
                cand.push_back(xr_tile{XR_KERNEL_STRIP, b[0], b[1], 0, ppy, 0});
    }
    for (size_t k = 0; k < cand.size(); ++k)
        if (cand[k].kernel != XR_KERNEL_STRIP)
            return fail(XR_ERR_ARG, "candidate %zu is not a strip tile", k);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // validates the jobs, the workspace and the capture state once
    int rc = xr_batch_prepare(jobs, n_jobs, &cand[0], dev_ws, ws_bytes, stream);
    if (rc)
        return rc;
    hipEvent_t ev0, ev1;
    hipError_t e = hipEventCreate(&ev0);
    if (e != hipSuccess)
        return fail_hip(e, "hipEventCreate");
    if ((e = hipEventCreate(&ev1)) != hipSuccess) {
        (void)hipEventDestroy(ev0);
        return fail_hip(e, "hipEventCreate");
    }
    std::vector<float> per_group(groups);
    float best_t = 0.0f;
    size_t best_k = 0;
    bool have = false;
    for (size_t k = 0; k < cand.size() && rc == XR_OK && e == hipSuccess; ++k) {
        rc = xr_batch_prepare(jobs, n_jobs, &cand[k], dev_ws, ws_bytes, stream);
        if (rc)
            break;
        rc = xr_resize_batched(dev_ws, n_jobs, stream);  // warm-up
        for (int32_t g = 0; g < groups && rc == XR_OK && e == hipSuccess; ++g) {
            e = hipEventRecord(ev0, s);
            for (int32_t r = 0; r < reps && rc == XR_OK && e == hipSuccess; ++r)
                rc = xr_resize_batched(dev_ws, n_jobs, stream);
            if (rc == XR_OK && e == hipSuccess)
                e = hipEventRecord(ev1, s);
            if (rc == XR_OK && e == hipSuccess)
                e = hipEventSynchronize(ev1);
            float ms = 0.0f;
            if (rc == XR_OK && e == hipSuccess)
                e = hipEventElapsedTime(&ms, ev0, ev1);
            per_group[g] = ms / static_cast<float>(reps);
        }
        if (rc != XR_OK || e != hipSuccess)
            break;
        std::sort(per_group.begin(), per_group.end());
        const float med = per_group[groups / 2];
        if (!have || med < best_t) {
            best_t = med;
            best_k = k;
            have = true;
        }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (rc)
        return rc;
    if (e != hipSuccess)
        return fail_hip(e, "timing a candidate");
    rc = xr_batch_prepare(jobs, n_jobs, &cand[best_k], dev_ws, ws_bytes, stream);
    if (rc)
        return rc;
    {
        std::lock_guard<std::mutex> lock(g_batch_mu);
        g_batch_tuned[jobs[0].src.dtype] = cand[best_k];
    }
    if (best)
        *best = cand[best_k];
    if (best_ms)
        *best_ms = best_t;
    return XR_OK;
}

int xr_resize_backward(const xr_image *grad_dst, const xr_image *grad_src, int32_t filter,
                       void *stream)
{
    if (filter != XR_BILINEAR && filter != XR_BICUBIC)
        return fail(XR_ERR_ARG, "filter = %d is not XR_BILINEAR or XR_BICUBIC", filter);
    int rc = check_image(grad_dst, "grad_dst");
    if (rc)
        return rc;
    rc = check_image(grad_src, "grad_src");
    if (rc)
        return rc;
    if ((grad_dst->dtype != XR_F32 && grad_dst->dtype != XR_F16) || grad_src->dtype != grad_dst->dtype)
        return fail(XR_ERR_DTYPE, "the adjoint takes float32 or float16 gradients, both of one type "
                    "(grad_dst %d, grad_src %d)", grad_dst->dtype, grad_src->dtype);
    if (grad_dst->channels != grad_src->channels)
        return fail(XR_ERR_CHANNELS, "grad_dst.channels %d != grad_src.channels %d",
                    grad_dst->channels, grad_src->channels);
    if (grad_dst->planes != grad_src->planes)
        return fail(XR_ERR_SHAPE, "grad_dst.planes %d != grad_src.planes %d", grad_dst->planes,
                    grad_src->planes);
    if (grad_dst->row0 != 0 || grad_dst->rows != grad_dst->height || grad_src->row0 != 0 ||
        grad_src->rows != grad_src->height)
        return fail(XR_ERR_RANGE, "the adjoint takes whole images (row0 = 0, rows = height)");
    if (overlaps(*grad_dst, *grad_src))
        return fail(XR_ERR_ALIAS, "grad_dst and grad_src memory overlap");
    // forward view: source = grad_src geometry, destination = grad_dst geometry
    xr::ResizeArgs a = make_args(*grad_src, *grad_dst);
    a.src = static_cast<const unsigned char *>(grad_dst->data);
    a.src_pitch = grad_dst->row_pitch;
    a.src_plane_pitch = grad_dst->planes > 1 ? grad_dst->plane_pitch : 0;
    a.dst = static_cast<unsigned char *>(grad_src->data);
    a.dst_pitch = grad_src->row_pitch;
    a.dst_plane_pitch = grad_src->planes > 1 ? grad_src->plane_pitch : 0;
    if (!xr::backward_supported(a, filter, grad_src->channels))
        return fail(XR_ERR_SHAPE, "adjoint: %dx%d -> %dx%d is too strong an upscale for one LDS tile",
                    grad_src->width, grad_src->height, grad_dst->width, grad_dst->height);
    const hipError_t e = xr::launch_backward(a, filter, grad_src->dtype, grad_src->channels,
                                             static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, "backward launch");
    return XR_OK;
}

int32_t xr_tune_candidates(int32_t filter, int32_t dtype, int32_t channels, int32_t in_w,
                           int32_t in_h, int32_t out_w, int32_t out_h, xr_tile *out, int32_t cap)
{
    (void)in_h;
    (void)out_h;
    std::vector<xr_tile> c;
    // the paper's block shapes (W x H threads, one pixel each) and a few wider ones
    const int gather[][2] = {{8, 8}, {32, 4}, {32, 16}, {4, 8}, {8, 4}, {16, 16}, {64, 4}, {64, 1},
                             {128, 2}, {256, 1}};
    for (const auto &g : gather)
        c.push_back(xr_tile{XR_KERNEL_GATHER, g[0], g[1], 1, 1, 0});
    if (is_aa(filter)) {  // the antialiased kernels: gather and LDS block shapes, one pixel each
        const int lds_blocks[][2] = {{16, 16}, {32, 8}, {64, 4}, {128, 2}, {32, 16}, {64, 8},
                                     {128, 4}, {64, 16}, {256, 4}, {64, 2}, {32, 2}, {16, 2}};
        for (const auto &b : lds_blocks)
            c.push_back(xr_tile{XR_KERNEL_STRIP_LDS, b[0], b[1], 1, 1, 0});
        if (out)
            for (int32_t k = 0; k < cap && k < static_cast<int32_t>(c.size()); ++k)
                out[k] = c[k];
        return static_cast<int32_t>(c.size());
    }
    // one RGBA column per thread only for the exact x0.5 walk (more waves on
    // its quarter-size output, so taller strips with less halo)
    const int ppx_c4[4] = {2, 4, 8, 1};
    const int ppx_c1[4] = {4, 8, 16, 0};
    const int *ppx_list = channels == 4 ? ppx_c4 : ppx_c1;
    const int blocks[][2] = {{64, 4}, {128, 2}, {256, 1}, {256, 2}, {512, 1}};
    const bool x2 = out_w == 2 * in_w && out_h == 2 * in_h;
    const bool x05 = 2 * out_w == in_w && 2 * out_h == in_h;
    if ((x2 || x05) && filter != XR_NEAREST) {
        // the exact x2 walk: strips of 8 m rows (m pairs of rows per 4-row
        // group of its loop); the exact x0.5 walk: strips of an even number
        // of rows; both workgroup orders
        const int x2_rows[] = {8, 16, 24, 32, 48, 64};
        const int x05_rows[] = {2, 4, 6, 8, 12, 16, 24, 32};
        for (int k = 0; k < (x05 ? 4 : 3); ++k) {
            const int ppx = ppx_list[k];
            if (!xr::strip_ppx_supported(dtype, channels, ppx))
                continue;
            for (const auto &b : blocks)
                for (int order = 0; order < 2; ++order) {
                    if (x2)
                        for (int ppy : x2_rows)
                            c.push_back(xr_tile{XR_KERNEL_STRIP, b[0], b[1], ppx, ppy, order});
                    else
                        for (int ppy : x05_rows)
                            c.push_back(xr_tile{XR_KERNEL_STRIP, b[0], b[1], ppx, ppy, order});
                }
        }
        if (out)
            for (int32_t k = 0; k < cap && k < static_cast<int32_t>(c.size()); ++k)
                out[k] = c[k];
        return static_cast<int32_t>(c.size());
    }
    // strip heights 8m-2 make the x2 walk's source-row groups come out even;
    // 1 and 2 rows give small images enough workgroups
    const int ppy_list[] = {1, 2, 6, 14, 22, 30, 46, 62};
    for (int k = 0; k < 3; ++k) {
        const int ppx = ppx_list[k];
        if (!xr::strip_ppx_supported(dtype, channels, ppx))
            continue;
        for (const auto &b : blocks)
            for (int ppy : ppy_list)
                for (int order = 0; order < 2; ++order)
                    c.push_back(xr_tile{XR_KERNEL_STRIP, b[0], b[1], ppx, ppy, order});
    }
    // the LDS-staged walk, where one workgroup's row segment fits
    const int lds_ppx = xr::kLdsPpx[channels == 4 ? 1 : 0];
    for (int bw : {64, 128, 256, 512}) {
        if (!xr::strip_lds_fits(filter, dtype, channels, in_w, out_w, bw, true))
            continue;
        for (int ppy : ppy_list)
            for (int order = 0; order < 2; ++order)
                c.push_back(xr_tile{XR_KERNEL_STRIP_LDS, bw, 1, lds_ppx, ppy, order});
    }
    if (out)
        for (int32_t k = 0; k < cap && k < static_cast<int32_t>(c.size()); ++k)
            out[k] = c[k];
    return static_cast<int32_t>(c.size());
}

int xr_autotune(const xr_image *srcs, const xr_image *dsts, int32_t n_pairs, int32_t filter,
                const xr_tile *candidates, int32_t n_candidates, int32_t reps, int32_t groups,
                xr_tile *best, float *best_ms, void *stream)
{
    if (!srcs || !dsts)
        return fail(XR_ERR_NULL, "srcs or dsts is NULL");
    if (n_pairs < 1)
        return fail(XR_ERR_ARG, "n_pairs = %d (must be >= 1)", n_pairs);
    int rc = XR_OK;
    for (int32_t k = 0; k < n_pairs; ++k) {
        rc = check_pair(&srcs[k], &dsts[k], filter);
        if (rc)
            return fail(rc, "pair %d: %s", k, g_last_error.c_str());
        const xr_image &s0 = srcs[0], &d0 = dsts[0], &s = srcs[k], &d = dsts[k];
        if (s.width != s0.width || s.height != s0.height || d.width != d0.width ||
            d.height != d0.height || s.dtype != s0.dtype || s.channels != s0.channels ||
            s.planes != s0.planes || d.rows != d0.rows)
            return fail(XR_ERR_ARG, "pair %d differs in size, dtype, channels or planes from pair 0", k);
    }
    const xr_image *src = &srcs[0];
    const xr_image *dst = &dsts[0];
    if (reps < 1 || groups < 1)
        return fail(XR_ERR_ARG, "reps = %d, groups = %d (both must be >= 1)", reps, groups);
    std::vector<xr_tile> cand;
    if (candidates) {
        if (n_candidates < 1)
            return fail(XR_ERR_ARG, "n_candidates = %d", n_candidates);
        cand.assign(candidates, candidates + n_candidates);
    } else {
        const int32_t n = xr_tune_candidates(filter, src->dtype, src->channels, src->width, src->height,
                                             dst->width, dst->height, nullptr, 0);
        cand.resize(n);
        xr_tune_candidates(filter, src->dtype, src->channels, src->width, src->height, dst->width,
                           dst->height, cand.data(), n);
        // the built-in list assumes aligned sources and narrow weight tables;
        // drop the shapes these sources cannot use
        for (int32_t k = 0; k < n_pairs; ++k)
            cand.erase(std::remove_if(cand.begin(), cand.end(),
                                      [&](const xr_tile &t) {
                                          if (is_aa(filter))
                                              return aa_lds_bytes(t, filter, srcs[k], dsts[k]) >
                                                     xr::kAaLdsBudget;
                                          return t.kernel == XR_KERNEL_STRIP_LDS &&
                                                 !lds_usable(t, filter, srcs[k], dsts[k]);
                                      }),
                       cand.end());
    }
    for (size_t k = 0; k < cand.size(); ++k) {
        if (cand[k].kernel == XR_KERNEL_AUTO)
            return fail(XR_ERR_ARG, "candidate %zu is XR_KERNEL_AUTO", k);
        if (is_aa(filter)) {
            for (int32_t j = 0; j < n_pairs && !rc; ++j)
                rc = check_aa(cand[k], filter, srcs[j], dsts[j]);
        } else {
            rc = check_tile(cand[k], src->dtype, src->channels);
            if (!rc)
                rc = check_lds(cand[k], filter, src->dtype, src->channels, src->width, dst->width,
                               std::all_of(srcs, srcs + n_pairs,
                                           [](const xr_image &i) { return src_aligned4(i); }));
        }
        if (!rc)
            rc = check_grid(cand[k], *dst);
        if (rc)
            return fail(rc, "candidate %zu: %s", k, g_last_error.c_str());
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess)
        return fail_hip(e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)
        return fail(XR_ERR_CAPTURE, "xr_autotune called on a capturing stream");
    std::vector<xr::ResizeArgs> args(n_pairs);
    for (int32_t k = 0; k < n_pairs; ++k)
        args[k] = make_args(srcs[k], dsts[k]);
    int32_t next = 0;
    const auto launch = [&](const xr_tile &t, int32_t mode) {
        const xr::ResizeArgs &a = args[next];
        next = (next + 1) % n_pairs;
        return xr::launch_forward(a, filter, src->dtype, src->channels, t, mode, s);
    };
    std::vector<int32_t> modes(cand.size());
    for (size_t k = 0; k < cand.size(); ++k)
        modes[k] = axis_mode(*src, *dst, cand[k], filter, XR_MAP_HALF_PIXEL);
    std::vector<float> med;
    e = time_candidates(cand.size(), reps, groups, s, [&](size_t k) { return launch(cand[k], modes[k]); }, med);
    if (e != hipSuccess)
        return fail_hip(e, "timing a candidate");
    float best_t = 0.0f;
    size_t best_k = 0;
    for (size_t k = 0; k < cand.size(); ++k) {
        const int threads = cand[k].block_w * cand[k].block_h;
        const int best_threads = cand[best_k].block_w * cand[best_k].block_h;
        if (k == 0 || med[k] < best_t || (med[k] == best_t && threads < best_threads)) {
            best_t = med[k];
            best_k = k;
        }
    }
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[tune_key(filter, src->dtype, src->channels, src->width, src->height, dst->width,
                         dst->height, dst->planes)] = cand[best_k];
    }
    if (best)
        *best = cand[best_k];
    if (best_ms)
        *best_ms = best_t;
    return XR_OK;
}

int xr_get_tile(int32_t filter, int32_t dtype, int32_t channels, int32_t in_w, int32_t in_h,
                int32_t out_w, int32_t out_h, xr_tile *out)
{
    if (!out)
        return fail(XR_ERR_NULL, "out is NULL");
    if (!valid_filter(filter))
        return fail(XR_ERR_ARG, "filter = %d unknown", filter);
    if (elem_size(dtype) == 0)
        return fail(XR_ERR_DTYPE, "dtype = %d unknown", dtype);
    if (channels != 1 && channels != 4)
        return fail(XR_ERR_CHANNELS, "channels = %d", channels);
    if (in_w < 1 || in_h < 1 || out_w < 1 || out_h < 1)
        return fail(XR_ERR_SHAPE, "sizes must be positive");
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tuned.find(tune_key(filter, dtype, channels, in_w, in_h, out_w, out_h, 1));
    *out = it != g_tuned.end() ? it->second
                               : default_tile(channels, in_w, in_h, out_w, out_h, out_h, 1);
    return XR_OK;
}

int xr_set_tile(int32_t filter, int32_t dtype, int32_t channels, int32_t in_w, int32_t in_h,
                int32_t out_w, int32_t out_h, const xr_tile *tile)
{
    if (!tile)
        return fail(XR_ERR_NULL, "tile is NULL");
    if (!valid_filter(filter))
        return fail(XR_ERR_ARG, "filter = %d unknown", filter);
    if (elem_size(dtype) == 0)
        return fail(XR_ERR_DTYPE, "dtype = %d unknown", dtype);
    if (channels != 1 && channels != 4)
        return fail(XR_ERR_CHANNELS, "channels = %d", channels);
    if (in_w < 1 || in_h < 1 || out_w < 1 || out_h < 1)
        return fail(XR_ERR_SHAPE, "sizes must be positive");
    const TuneKey key = tune_key(filter, dtype, channels, in_w, in_h, out_w, out_h, 1);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (tile->kernel == XR_KERNEL_AUTO) {
        g_tuned.erase(key);
        return XR_OK;
    }
    int rc = check_tile(*tile, dtype, channels);
    if (!rc)
        rc = check_lds(*tile, filter, dtype, channels, in_w, out_w);
    if (rc)
        return rc;
    g_tuned[key] = *tile;
    return XR_OK;
}

int xr_tune_save(const char *path)
{
    if (!path)
        return fail(XR_ERR_NULL, "path is NULL");
    std::string arch;
    int cus = 0;
    int rc = device_identity(arch, cus);
    if (rc)
        return rc;
    FILE *f = std::fopen(path, "w");
    if (!f)
        return fail(XR_ERR_ARG, "cannot write %s", path);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    std::fprintf(f, "xresize-tiles 1\narch %s cus %d build %s\n", arch.c_str(), cus, XR_BUILD_ID);
    for (const auto &kv : g_tuned) {
        const TuneKey &k = kv.first;
        const xr_tile &t = kv.second;
        std::fprintf(f, "%d %d %d %d %d %d  %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
                     std::get<3>(k), std::get<4>(k), std::get<5>(k), t.kernel, t.block_w, t.block_h, t.ppt_x,
                     t.ppt_y, t.order);
    }
    const bool ok = std::fclose(f) == 0;
    return ok ? XR_OK : fail(XR_ERR_ARG, "writing %s failed", path);
}

int xr_tune_load(const char *path, int32_t *n_loaded)
{
    if (!path || !n_loaded)
        return fail(XR_ERR_NULL, "path or n_loaded is NULL");
    *n_loaded = 0;
    std::string arch;
    int cus = 0;
    int rc = device_identity(arch, cus);
    if (rc)
        return rc;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return fail(XR_ERR_ARG, "cannot read %s", path);
    char f_arch[256] = {0}, f_build[128] = {0};
    int version = 0, f_cus = 0;
    const bool header = std::fscanf(f, "xresize-tiles %d arch %255s cus %d build %127s", &version, f_arch,
                                    &f_cus, f_build) == 4;
    // shapes tuned on another GPU model, CU count or build of the kernels
    // are not used
    if (!header || version != 1 || arch != f_arch || cus != f_cus || std::strcmp(f_build, XR_BUILD_ID) != 0) {
        std::fclose(f);
        return XR_OK;
    }
    int v[12];
    std::lock_guard<std::mutex> lock(g_tune_mu);
    while (std::fscanf(f, "%d %d %d %d %d %d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6],
                       &v[7], &v[8], &v[9], &v[10], &v[11]) == 12) {
        const xr_tile t{v[6], v[7], v[8], v[9], v[10], v[11]};
        if (!valid_filter(v[0]) || elem_size(v[1]) == 0 || (v[2] != 1 && v[2] != 4) ||
            check_tile(t, v[1], v[2]) != XR_OK)
            continue;
        g_tuned[TuneKey(v[0], v[1], v[2], v[3], v[4], v[5])] = t;
        ++*n_loaded;
    }
    std::fclose(f);
    return XR_OK;
}

int xr_source_taps(int32_t n_in, int32_t n_out, int32_t x, int32_t *x0, int64_t *t_num,
                   int64_t *t_den)
{
    if (!x0 || !t_num || !t_den)
        return fail(XR_ERR_NULL, "output pointer is NULL");
    if (n_in < 1 || n_out < 1 || n_in > XR_MAX_SIDE || n_out > XR_MAX_SIDE)
        return fail(XR_ERR_SHAPE, "sizes %d -> %d outside 1..%d", n_in, n_out, XR_MAX_SIDE);
    if (x < 0 || x >= n_out)
        return fail(XR_ERR_RANGE, "x = %d outside [0, %d)", x, n_out);
    const int64_t num = (2 * static_cast<int64_t>(x) + 1) * n_in - n_out;
    const int64_t den = 2 * static_cast<int64_t>(n_out);
    const int64_t q = floor_div(num, den);
    *x0 = static_cast<int32_t>(q);
    *t_num = num - q * den;
    *t_den = den;
    return XR_OK;
}

int xr_needed_rows_map(int32_t in_h, int32_t out_h, int32_t row0, int32_t rows, int32_t filter,
                       int32_t mapping, int32_t *first, int32_t *last)
{
    if (!first || !last)
        return fail(XR_ERR_NULL, "output pointer is NULL");
    if (!valid_filter(filter))
        return fail(XR_ERR_ARG, "filter = %d unknown", filter);
    if (!valid_mapping(mapping))
        return fail(XR_ERR_ARG, "mapping = %d unknown", mapping);
    if (in_h < 1 || out_h < 1 || in_h > XR_MAX_SIDE || out_h > XR_MAX_SIDE)
        return fail(XR_ERR_SHAPE, "sizes %d -> %d outside 1..%d", in_h, out_h, XR_MAX_SIDE);
    if (rows < 1 || row0 < 0 || static_cast<int64_t>(row0) + rows > out_h)
        return fail(XR_ERR_RANGE, "rows [%d, %d) outside [0, %d)", row0, row0 + rows, out_h);
    needed_rows(in_h, out_h, row0, rows, filter, first, last, mapping);
    return XR_OK;
}

int xr_needed_rows(int32_t in_h, int32_t out_h, int32_t row0, int32_t rows, int32_t filter,
                   int32_t *first, int32_t *last)
{
    if (!first || !last)
        return fail(XR_ERR_NULL, "output pointer is NULL");
    if (filter != XR_BILINEAR && filter != XR_BICUBIC)
        return fail(XR_ERR_ARG, "filter = %d unknown", filter);
    if (in_h < 1 || out_h < 1 || in_h > XR_MAX_SIDE || out_h > XR_MAX_SIDE)
        return fail(XR_ERR_SHAPE, "sizes %d -> %d outside 1..%d", in_h, out_h, XR_MAX_SIDE);
    if (rows < 1 || row0 < 0 || static_cast<int64_t>(row0) + rows > out_h)
        return fail(XR_ERR_RANGE, "rows [%d, %d) outside [0, %d)", row0, row0 + rows, out_h);
    needed_rows(in_h, out_h, row0, rows, filter, first, last);
    return XR_OK;
}

int xr_thread_of_pixel(const xr_tile *tile, int32_t px, int32_t py, int32_t *block_x,
                       int32_t *block_y, int32_t *thread_x, int32_t *thread_y, int32_t *sub_x,
                       int32_t *sub_y)
{
    if (!tile || !block_x || !block_y || !thread_x || !thread_y || !sub_x || !sub_y)
        return fail(XR_ERR_NULL, "NULL pointer");
    if (tile->block_w < 1 || tile->block_h < 1 || tile->ppt_x < 1 || tile->ppt_y < 1)
        return fail(XR_ERR_ARG, "tile fields must be positive");
    if (px < 0 || py < 0)
        return fail(XR_ERR_RANGE, "pixel (%d, %d) is negative", px, py);
    // eq. 6: p = b * b_size + t, with b_size = block * ppt and t = thread * ppt + sub
    const int32_t tw = tile->block_w * tile->ppt_x;
    const int32_t th = tile->block_h * tile->ppt_y;
    *block_x = px / tw;
    *block_y = py / th;
    *thread_x = (px % tw) / tile->ppt_x;
    *thread_y = (py % th) / tile->ppt_y;
    *sub_x = (px % tw) % tile->ppt_x;
    *sub_y = (py % th) % tile->ppt_y;
    return XR_OK;
}

const char *xr_strerror(int code)
{
    switch (code) {
    case XR_OK:
        return "success";
    case XR_ERR_NULL:
        return "null pointer";
    case XR_ERR_SHAPE:
        return "invalid size";
    case XR_ERR_DTYPE:
        return "invalid or mismatched dtype";
    case XR_ERR_CHANNELS:
        return "invalid or mismatched channel count";
    case XR_ERR_PITCH:
        return "invalid pitch or alignment";
    case XR_ERR_RANGE:
        return "row band out of range";
    case XR_ERR_ALIAS:
        return "source and destination overlap";
    case XR_ERR_WORKSPACE:
        return "invalid workspace";
    case XR_ERR_CAPTURE:
        return "call not allowed during stream capture";
    case XR_ERR_HIP:
        return "HIP runtime error";
    case XR_ERR_ARG:
        return "invalid argument";
    default:
        return "unknown error code";
    }
}

const char *xr_last_error(void) { return g_last_error.c_str(); }

int xr_version(void) { return 100; }

}  // extern "C"
