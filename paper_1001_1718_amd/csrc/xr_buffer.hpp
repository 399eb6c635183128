// Raw buffer access for the walks: every access goes through a buffer
// resource whose bound drops what falls outside it, so a walk can issue each
// load and store on every step (no branch around memory operations) and let
// the bound discard the rows that are not its own.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xr_device.hpp"

namespace xr {
namespace dev {

// Buffer resource over [base, base + bytes): a load at an offset at or past
// `bytes` reads zero and a store there is dropped. base and bytes must be the
// same on every lane of the wavefront (the resource lives in scalar
// registers); offsets are 32-bit, so a resource spans less than 2 GiB and
// "before the base" is any offset of 2^31 or more.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, uint32_t bytes)
{
    const uint64_t p = reinterpret_cast<uint64_t>(base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(p));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(p >> 32));
    void *u = reinterpret_cast<void *>((static_cast<uint64_t>(hi) << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(u, 0, static_cast<int>(__builtin_amdgcn_readfirstlane(bytes)),
                                             0x00020000);
}

// Cache policy of output stores that nothing in the launch reads back:
// streaming (nt) and written past the L2 (sc1). Measured on the x2 walk:
// 79 -> 70 us against plain non-temporal stores, the L2 then keeping the
// source rows that neighbouring strips re-read.
constexpr int kStoreStream = 2 | 16;

typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// BYTES (a multiple of 4) from byte offset `off` into `dst`, in 16-, 8- and
// 4-byte loads (dword-aligned offsets)
template <int BYTES>
__device__ __forceinline__ void buf_load(unsigned char *dst, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    static_assert(BYTES % 4 == 0, "whole dwords");
    int o = 0;
#pragma unroll
    for (; o + 16 <= BYTES; o += 16)
        *reinterpret_cast<u32x4_t *>(dst + o) =
            __builtin_bit_cast(u32x4_t, __builtin_amdgcn_raw_buffer_load_b128(r, off + o, 0, 0));
    if constexpr (BYTES % 16 >= 8) {
        *reinterpret_cast<u32x2_t *>(dst + o) =
            __builtin_bit_cast(u32x2_t, __builtin_amdgcn_raw_buffer_load_b64(r, off + o, 0, 0));
        o += 8;
    }
    if constexpr (BYTES % 8 >= 4)
        *reinterpret_cast<uint32_t *>(dst + o) = __builtin_amdgcn_raw_buffer_load_b32(r, off + o, 0, 0);
}

// one pixel of PB bytes
template <int PB>
__device__ __forceinline__ void buf_load_px(unsigned char *dst, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    if constexpr (PB == 1)
        *dst = __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
    else if constexpr (PB == 2)
        *reinterpret_cast<uint16_t *>(dst) = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    else
        buf_load<PB>(dst, r, off);
}

// BYTES from `src` to byte offset `off` with cache policy AUX (1- and 2-byte
// stores for single small pixels, else whole dwords)
template <int BYTES, int AUX>
__device__ __forceinline__ void buf_store(const unsigned char *src, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    if constexpr (BYTES == 1) {
        __builtin_amdgcn_raw_buffer_store_b8(*src, r, off, 0, AUX);
    } else if constexpr (BYTES == 2) {
        __builtin_amdgcn_raw_buffer_store_b16(*reinterpret_cast<const uint16_t *>(src), r, off, 0, AUX);
    } else {
        static_assert(BYTES % 4 == 0, "whole dwords");
        int o = 0;
#pragma unroll
        for (; o + 16 <= BYTES; o += 16)
            __builtin_amdgcn_raw_buffer_store_b128(*reinterpret_cast<const u32x4_t *>(src + o), r, off + o, 0, AUX);
        if constexpr (BYTES % 16 >= 8) {
            __builtin_amdgcn_raw_buffer_store_b64(*reinterpret_cast<const u32x2_t *>(src + o), r, off + o, 0, AUX);
            o += 8;
        }
        if constexpr (BYTES % 8 >= 4)
            __builtin_amdgcn_raw_buffer_store_b32(*reinterpret_cast<const uint32_t *>(src + o), r, off + o, 0, AUX);
    }
}

}  // namespace dev

// BYTES bytes held in registers (a run of pixels), aligned to ALIGN.
template <int BYTES, int ALIGN>
struct alignas(ALIGN) RawBuf {
    unsigned char b[BYTES];
};

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }
constexpr int cmin(int a, int b) { return a < b ? a : b; }

using namespace dev;

// Output runs of the walks.
//
// A thread's run of PPX output pixels (OB bytes) goes to byte offset
// row_off + col0 * PB of the store resource (rows outside the resource are
// dropped by its bound). Runs of up to 16 bytes are stored directly: one
// store instruction then writes the wavefront's 64 runs as one contiguous
// span. Wider runs would leave every store instruction writing part of each
// cache line, which the streaming (past-the-L2) policy turns into partial
// writes at the memory (float32 RGBA x2: 1.0 ms); they are exchanged through
// a 64-run LDS area of the wavefront so that store c writes the span's chunks
// 64 c .. 64 c + 63, whole lines (float32 RGBA x2: 0.19 ms). Pixels past the
// right image edge are not stored.
template <typename T, int C, int PPX>
struct RunStore {
    static constexpr int PB = Pix<T, C>::kBytes;
    static constexpr int OB = PPX * PB;
    static constexpr bool kExchange = OB > 16;
    static constexpr int PPC = 16 / PB;  // pixels per 16-byte chunk (exchange)

    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t lane_off;       // direct: col0 * PB, + 2^31 when the run crosses the right edge
    int32_t ncols;           // direct: pixels of the run inside the image
    unsigned char *xlds;     // exchange: the wavefront's area
    int32_t lane, wave_col0, out_w;

    // `tid`: the thread's index in its workgroup (blockDim.x a multiple of 64)
    __device__ __forceinline__ void init(__amdgpu_buffer_rsrc_t r, int32_t col0, int32_t out_w_, int32_t tid,
                                         unsigned char *lds)
    {
        rsrc = r;
        ncols = max(0, min(PPX, out_w_ - col0));
        lane_off = static_cast<uint32_t>(col0 * PB) + (ncols < PPX ? 0x80000000u : 0u);
        lane = tid & 63;
        xlds = lds + (tid >> 6) * 64 * OB;
        wave_col0 = col0 - lane * PPX;
        out_w = out_w_;
    }

    template <int ALIGN>
    __device__ __forceinline__ void store(uint32_t row_off, const RawBuf<OB, ALIGN> &out) const
    {
        if constexpr (kExchange) {
            __builtin_memcpy(xlds + lane * OB, out.b, OB);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int c = 0; c < OB / 16; ++c) {
                const int32_t g = lane + 64 * c;
                const int32_t px = wave_col0 + g * PPC;  // first pixel of chunk g
                unsigned char chunk[16];
                __builtin_memcpy(chunk, xlds + 16 * g, 16);
                const int32_t nv = out_w - px;
                const uint32_t off = row_off + static_cast<uint32_t>(px * PB);
                buf_store<16, kStoreStream>(chunk, rsrc, nv >= PPC ? off : off + 0x80000000u);
                if (nv > 0 && nv < PPC) {
#pragma unroll
                    for (int q = 0; q < PPC; ++q)
                        if (q < nv)
                            buf_store<PB, kStoreStream>(chunk + q * PB, rsrc, off + static_cast<uint32_t>(q * PB));
                }
            }
            __builtin_amdgcn_wave_barrier();
        } else {
            buf_store<OB, kStoreStream>(out.b, rsrc, row_off + lane_off);
            if (ncols < PPX) {
#pragma unroll
                for (int c = 0; c < PPX; ++c)
                    if (c < ncols)
                        buf_store<PB, kStoreStream>(out.b + c * PB, rsrc,
                                                    row_off + lane_off - 0x80000000u + static_cast<uint32_t>(c * PB));
            }
        }
    }
};

// LDS bytes of a workgroup of `threads` for RunStore<T, C, PPX>
template <typename T, int C, int PPX>
constexpr size_t run_store_lds(int32_t threads)
{
    return RunStore<T, C, PPX>::kExchange ? static_cast<size_t>(threads) * RunStore<T, C, PPX>::OB : 0;
}

}  // namespace xr
