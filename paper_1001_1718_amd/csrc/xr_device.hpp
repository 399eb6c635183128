// Device-side building blocks shared by every kernel of the library: the
// coordinate map, the tap weights, and pixel loads/stores per storage type.
//
// Every kernel evaluates an output value in the same float32 order:
//   h_j = w_x0 * p_j0;  h_j = fma(w_x1, p_j1, h_j); ...   (taps ascending)
//   v   = w_y0 * h_0;   v   = fma(w_y1, h_1, v);   ...   (rows ascending)
// and the weights come from the same functions below, compiled with
// floating-point contraction off, so a pixel's value is a pure function of the
// image and its coordinates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xr {
namespace dev {

constexpr int kBilinear = 0;
constexpr int kBicubic = 1;
constexpr int kNearest = 2;

template <int FILTER>
struct Taps {
    static constexpr int K = (FILTER == kBicubic) ? 4 : (FILTER == kNearest ? 1 : 2);  // taps per axis
    static constexpr int LO = (FILTER == kBicubic) ? -1 : 0;  // first tap relative to x0
};

// Eqs. 1-4: s = ((2x+o) n_in - o n_out) / (2 n_out), with o = 1 for pixel
// centres (s = (x + 1/2) n_in / n_out - 1/2) and o = 0 for the map as eq. 1
// prints it (s = x n_in / n_out); x0 = floor(s), t = s - x0, omt = 1 - t.
// The numerator fits in int32 for sides up to 32768; t and 1 - t are each one
// correctly rounded division of two exact integers, so both carry a relative
// error of at most half an ulp (1 - t is not formed by a subtraction that
// would cancel as t -> 1).
__device__ __forceinline__ void axis_tap(int32_t x, int32_t n_in, int32_t n_out, int32_t o,
                                         int32_t &x0, float &t, float &omt)
{
    const int32_t num = (2 * x + o) * n_in - o * n_out;
    const int32_t den = 2 * n_out;
    int32_t q = num / den;
    int32_t rem = num - q * den;
    if (rem < 0) {  // C division truncates; step down to the floor
        q -= 1;
        rem += den;
    }
    x0 = q;
    t = __fdiv_rn(static_cast<float>(rem), static_cast<float>(den));
    omt = __fdiv_rn(static_cast<float>(den - rem), static_cast<float>(den));
}

// a / b correctly rounded from y = RN(1 / b): q0 = RN(a y), then one
// correction with the exact residual a - q0 b (an FMA). For integers
// 0 <= a <= b <= 65536 the result equals the IEEE quotient (checked
// exhaustively on the host for every such pair), so callers that divide many
// numerators by one denominator share one division.
__device__ __forceinline__ float div_rcp(float a, float b, float y)
{
    const float q0 = a * y;
    const float r = __builtin_fmaf(-q0, b, a);
    return __builtin_fmaf(r, y, q0);
}

// axis_tap with the reciprocal of its denominator 2 n_out supplied
// (rcp = RN(1 / (2 n_out))): the same x0, t and 1 - t bit for bit.
__device__ __forceinline__ void axis_tap_rcp(int32_t x, int32_t n_in, int32_t n_out, int32_t o, float rcp,
                                             int32_t &x0, float &t, float &omt)
{
    const int32_t num = (2 * x + o) * n_in - o * n_out;
    const int32_t den = 2 * n_out;
    int32_t q = num / den;
    int32_t rem = num - q * den;
    if (rem < 0) {
        q -= 1;
        rem += den;
    }
    x0 = q;
    const float d = static_cast<float>(den);
    t = div_rcp(static_cast<float>(rem), d, rcp);
    omt = div_rcp(static_cast<float>(den - rem), d, rcp);
}

// The tap of FILTER for output x: eqs. 1-4 for bilinear and bicubic; for
// nearest neighbour the source pixel whose area contains the mapped point,
// floor(s + o/2) = floor((2x+o) n_in / (2 n_out)) (pixel i covers
// [i - 1/2, i + 1/2) with pixel centres, [i, i + 1) with the printed map),
// with weight 1.
template <int FILTER>
__device__ __forceinline__ void source_tap(int32_t x, int32_t n_in, int32_t n_out, int32_t o,
                                           int32_t &x0, float &t, float &omt)
{
    if constexpr (FILTER == kNearest) {
        x0 = ((2 * x + o) * n_in) / (2 * n_out);  // non-negative: division is floor
        t = 0.0f;
        omt = 1.0f;
    } else {
        axis_tap(x, n_in, n_out, o, x0, t, omt);
    }
}

// source_tap with rcp = RN(1 / (2 n_out)) supplied (per-row callers).
template <int FILTER>
__device__ __forceinline__ void source_tap_rcp(int32_t x, int32_t n_in, int32_t n_out, int32_t o, float rcp,
                                               int32_t &x0, float &t, float &omt)
{
    if constexpr (FILTER == kNearest) {
        (void)rcp;
        source_tap<FILTER>(x, n_in, n_out, o, x0, t, omt);
    } else {
        axis_tap_rcp(x, n_in, n_out, o, rcp, x0, t, omt);
    }
}

// Bilinear weights (1 - t, t) for taps x0, x0+1 (eq. 5).
// Keys cubic weights for a = -1/2 at taps x0-1 .. x0+2, i.e. K(t+1), K(t),
// K(1-t), K(2-t), written in factored forms whose every factor is computed
// without cancellation, so each weight has a small relative error:
//   K(t+1) = -t (1-t)^2 / 2          K(t)   = (1-t) (2 + t (2 - 3t)) / 2
//   K(1-t) =  t (1 + t (4 - 3t)) / 2 K(2-t) = -t^2 (1-t) / 2
template <int FILTER>
__device__ __forceinline__ void weights(float t, float omt, float (&w)[Taps<FILTER>::K])
{
    if constexpr (FILTER == kNearest) {
        (void)t;
        (void)omt;
        w[0] = 1.0f;
    } else if constexpr (FILTER == kBilinear) {
        w[0] = omt;
        w[1] = t;
    } else {
        const float ht = -0.5f * t;
        w[0] = (ht * omt) * omt;
        w[1] = (0.5f * omt) * (2.0f + t * (2.0f - 3.0f * t));
        w[2] = (0.5f * t) * (1.0f + t * (4.0f - 3.0f * t));
        w[3] = (ht * t) * omt;
    }
}

// Keeps a float32 value in a register as float32, so that the compiler
// cannot fold the preceding operation into a conversion that rounds once to a
// narrower type (the library rounds to float32 first, then converts).
__device__ __forceinline__ float opaque(float v)
{
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ int32_t clampi(int32_t v, int32_t lo, int32_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

// ---- storage types ------------------------------------------------------

__device__ __forceinline__ float u8_to_f32(uint32_t word, int byte)
{
    return static_cast<float>((word >> (8 * byte)) & 0xffu);
}

// uint8 storage: round half to even, clamp to [0, 255]. v_cvt_pk_u8_f32 does
// exactly this on gfx950 (it rounds in the default round-to-nearest-even mode
// and saturates), and writes the byte into lane `byte` of `old`.
__device__ __forceinline__ uint32_t u8_insert(float v, int byte, uint32_t old)
{
    return __builtin_amdgcn_cvt_pk_u8_f32(v, byte, old);
}

__device__ __forceinline__ uint32_t f32_to_u8(float v) { return u8_insert(v, 0, 0u); }

template <typename T, int C>
struct Pix;

template <>
struct Pix<uint8_t, 1> {
    static constexpr int kBytes = 1;
    __device__ __forceinline__ static void load(const unsigned char *row, int32_t col, float (&v)[1])
    {
        v[0] = static_cast<float>(row[col]);
    }
    __device__ __forceinline__ static void store(unsigned char *row, int32_t col, const float (&v)[1])
    {
        row[col] = static_cast<unsigned char>(f32_to_u8(v[0]));
    }
};

template <>
struct Pix<uint8_t, 4> {
    static constexpr int kBytes = 4;
    __device__ __forceinline__ static void load(const unsigned char *row, int32_t col, float (&v)[4])
    {
        const uint32_t w = *reinterpret_cast<const uint32_t *>(row + 4 * col);
        v[0] = u8_to_f32(w, 0);
        v[1] = u8_to_f32(w, 1);
        v[2] = u8_to_f32(w, 2);
        v[3] = u8_to_f32(w, 3);
    }
    __device__ __forceinline__ static uint32_t pack(const float (&v)[4])
    {
        uint32_t r = u8_insert(v[0], 0, 0u);
        r = u8_insert(v[1], 1, r);
        r = u8_insert(v[2], 2, r);
        return u8_insert(v[3], 3, r);
    }
    __device__ __forceinline__ static void store(unsigned char *row, int32_t col, const float (&v)[4])
    {
        *reinterpret_cast<uint32_t *>(row + 4 * col) = pack(v);
    }
};

template <>
struct Pix<_Float16, 1> {
    static constexpr int kBytes = 2;
    __device__ __forceinline__ static void load(const unsigned char *row, int32_t col, float (&v)[1])
    {
        v[0] = static_cast<float>(reinterpret_cast<const _Float16 *>(row)[col]);
    }
    __device__ __forceinline__ static void store(unsigned char *row, int32_t col, const float (&v)[1])
    {
        reinterpret_cast<_Float16 *>(row)[col] = static_cast<_Float16>(opaque(v[0]));
    }
};

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

template <>
struct Pix<_Float16, 4> {
    static constexpr int kBytes = 8;
    __device__ __forceinline__ static void load(const unsigned char *row, int32_t col, float (&v)[4])
    {
        const half4_t h = *reinterpret_cast<const half4_t *>(row + 8 * col);
        v[0] = static_cast<float>(h[0]);
        v[1] = static_cast<float>(h[1]);
        v[2] = static_cast<float>(h[2]);
        v[3] = static_cast<float>(h[3]);
    }
    __device__ __forceinline__ static void store(unsigned char *row, int32_t col, const float (&v)[4])
    {
        half4_t h;
        h[0] = static_cast<_Float16>(opaque(v[0]));
        h[1] = static_cast<_Float16>(opaque(v[1]));
        h[2] = static_cast<_Float16>(opaque(v[2]));
        h[3] = static_cast<_Float16>(opaque(v[3]));
        *reinterpret_cast<half4_t *>(row + 8 * col) = h;
    }
};

template <>
struct Pix<float, 1> {
    static constexpr int kBytes = 4;
    __device__ __forceinline__ static void load(const unsigned char *row, int32_t col, float (&v)[1])
    {
        v[0] = reinterpret_cast<const float *>(row)[col];
    }
    __device__ __forceinline__ static void store(unsigned char *row, int32_t col, const float (&v)[1])
    {
        reinterpret_cast<float *>(row)[col] = v[0];
    }
};

template <>
struct Pix<float, 4> {
    static constexpr int kBytes = 16;
    __device__ __forceinline__ static void load(const unsigned char *row, int32_t col, float (&v)[4])
    {
        const float4 f = *reinterpret_cast<const float4 *>(row + 16 * col);
        v[0] = f.x;
        v[1] = f.y;
        v[2] = f.z;
        v[3] = f.w;
    }
    __device__ __forceinline__ static void store(unsigned char *row, int32_t col, const float (&v)[4])
    {
        *reinterpret_cast<float4 *>(row + 16 * col) = make_float4(v[0], v[1], v[2], v[3]);
    }
};

// h = sum_i w[i] * p[i] over one source row, taps ascending (first product is
// a plain multiply, the rest are fused multiply-adds).
template <int C>
__device__ __forceinline__ void fma_first(float (&acc)[C], float w, const float (&p)[C])
{
#pragma unroll
    for (int c = 0; c < C; ++c)
        acc[c] = w * p[c];
}

template <int C>
__device__ __forceinline__ void fma_next(float (&acc)[C], float w, const float (&p)[C])
{
#pragma unroll
    for (int c = 0; c < C; ++c)
        acc[c] = __builtin_fmaf(w, p[c], acc[c]);
}

}  // namespace dev
}  // namespace xr
