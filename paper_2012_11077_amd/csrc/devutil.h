// Device helpers shared by the HIP kernels of libcfar2d.so (gfx950, wave64):
// buffer resources with per-row range checks, row loads, and the FP64 DPP
// wave scan.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#define CFAR_GLOBAL __attribute__((address_space(1)))

namespace cfar {
namespace dev {

// Word 3 of a raw buffer resource on CDNA (32-bit data format, no swizzle).
constexpr int kRsrcFlags = 0x00020000;
// A lane offset past every resource: such accesses read zero and store nothing.
constexpr uint32_t kOff = 0x80000000u;

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(uint64_t base, uint32_t bytes)
{
    const uint32_t lo = uni((uint32_t)base), hi = uni((uint32_t)(base >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void *)(uintptr_t)(((uint64_t)hi << 32) | lo), (short)0,
                                             (int)uni(bytes), kRsrcFlags);
}

// K consecutive values of one row at lane byte offset voff (each dword past
// the resource's size reads as zero).
template <int K, typename T>
__device__ __forceinline__ void ld_row(__amdgpu_buffer_rsrc_t rs, uint32_t voff, T (&v)[K])
{
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    if constexpr (K * sizeof(T) == 8) {
        const u32x2 w = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, 0u, 0));
        __builtin_memcpy(v, &w, 8);
    } else {
#pragma unroll
        for (int q = 0; q < (int)(K * sizeof(T) / 16); ++q) {
            const u32x4 w =
                __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16u * q, 0u, 0));
            __builtin_memcpy((char *)v + 16 * q, &w, 16);
        }
    }
}

// ---------------------------------------------------------------------------
// Wave64 inclusive prefix sum of one double per lane (DPP on both halves).
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_into(double old, double v)
{
    const long long b = __double_as_longlong(v), o = __double_as_longlong(old);
    const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffll), (int)(b & 0xffffffffll), CTRL, ROW_MASK,
                                               0xf, true);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ double dpp_shr(double v)
{
    return dpp_into<CTRL, 0xf>(0.0, v);
}
// z15 / z31 carry the broadcast steps' registers from call to call (0.0
// before the first): the rows those steps leave out stay zero in them.
__device__ __forceinline__ double wave_scan(double v, double &z15, double &z31)
{
    v += dpp_shr<0x111>(v);  // row_shr:1
    v += dpp_shr<0x112>(v);  // row_shr:2
    v += dpp_shr<0x114>(v);  // row_shr:4
    v += dpp_shr<0x118>(v);  // row_shr:8
    z15 = dpp_into<0x142, 0xa>(z15, v);  // row_bcast:15 into rows 1 and 3
    v += z15;
    z31 = dpp_into<0x143, 0xc>(z31, v);  // row_bcast:31 into rows 2 and 3
    v += z31;
    return v;
}

__device__ __forceinline__ int clip_len(int c, int h, int n)
{
    const int lo = c - h < 0 ? 0 : c - h;
    const int hi = c + h > n - 1 ? n - 1 : c + h;
    return hi - lo + 1;
}

// LDS layout of one prefix row: position p = l*K + k at [k*64 + l]
// (consecutive lanes, consecutive words: conflict-free).  Position p + o
// for element k of lane l, o = q*K + s (0 <= s < K), is element (k+s) mod K
// of lane l+q, or of lane l+q+1 when k+s >= K; lane indices wrap inside the
// row (wrapped values only reach lanes without outputs).
typedef __attribute__((address_space(3))) char lds_char;
typedef __attribute__((address_space(3))) double lds_double;

template <int K>
struct Corner {
    uint32_t addr[K];  // LDS byte addresses in prefix row buffer 0
    uint32_t own;      // LDS byte address of the lane's own element 0 in buffer 0
    __device__ __forceinline__ uint32_t addr0() const { return own; }
    __device__ __forceinline__ void init(int o, int lane, uint32_t base)
    {
        own = base + 8u * (uint32_t)lane;
        asm volatile("" : "+v"(own));
        const int q = o >= 0 ? o / K : -((-o + K - 1) / K);
        const int s = o - q * K;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = k + s;
            addr[k] = base + 8u * (uint32_t)((e >= K ? e - K : e) * 64 + ((lane + q + (e >= K ? 1 : 0)) & 63));
            // an opaque register: the reads then address LDS through it
            // directly instead of re-adding the LDS base symbol every time
            asm volatile("" : "+v"(addr[k]));
        }
    }
};

}  // namespace dev
}  // namespace cfar
