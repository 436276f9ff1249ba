// Device-side helpers for gfx950: buffer-resource loads/stores, 16-bit message
// storage formats and wave64 lane exchanges.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bpk {

// Raw buffer resource over `bytes` bytes at `p` (stride 0; gfx9-family dword 3).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float ld_f32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__device__ __forceinline__ void st_f32(__amdgpu_buffer_rsrc_t r, float v, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}

// Message storage formats.  Arithmetic is always FP32; a stored value is
// rounded to nearest-even in the storage format.
struct StoreF32 {
    static constexpr int bytes = 4;
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        return ld_f32(r, voff, soff);
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, float v, uint32_t voff, uint32_t soff)
    {
        st_f32(r, v, voff, soff);
    }
};

struct StoreF16 {
    static constexpr int bytes = 2;
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        uint16_t u = __builtin_bit_cast(uint16_t, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
        return (float)__builtin_bit_cast(_Float16, u);
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, float v, uint32_t voff, uint32_t soff)
    {
        _Float16 h = (_Float16)v;  // v_cvt_f16_f32: round to nearest even
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, h), r, voff, soff, 0);
    }
};

struct StoreBF16 {
    static constexpr int bytes = 2;
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        uint16_t u = __builtin_bit_cast(uint16_t, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
        return __builtin_bit_cast(float, (uint32_t)u << 16);
    }
    // Round to nearest even on the upper 16 bits (messages are finite).
    static __device__ __forceinline__ uint16_t encode(float v)
    {
        uint32_t u = __builtin_bit_cast(uint32_t, v);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, float v, uint32_t voff, uint32_t soff)
    {
        __builtin_amdgcn_raw_buffer_store_b16(encode(v), r, voff, soff, 0);
    }
};

// Sum of `v` over aligned groups of G lanes (G = 1, 2, 4) with DPP quad
// permutations; IEEE addition is commutative, so every lane of a group gets
// the bit-identical total.
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
    if constexpr (G == 1) {
        return v;
    } else {
        // quad_perm(1,0,3,2): swap neighbouring lanes.
        float o = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, true));
        float s = v + o;
        if constexpr (G == 4) {
            // quad_perm(2,3,0,1): swap lane pairs.
            float o2 = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, s), 0x4E, 0xF, 0xF, true));
            s = s + o2;
        }
        return s;
    }
}

}  // namespace bpk
