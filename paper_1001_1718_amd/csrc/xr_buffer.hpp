// Raw buffer access for the walks: every access goes through a buffer
// resource whose bound drops what falls outside it, so a walk can issue each
// load and store on every step (no branch around memory operations) and let
// the bound discard the rows that are not its own.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
}  // namespace xr
