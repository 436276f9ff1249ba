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
// rounded to nearest-even in the storage format.  pack2 rounds two values
// into one 32-bit word (low half first) with gfx950's two-value conversion
// instructions; encode rounds one value the same way.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

struct StoreF32 {
    static constexpr int bytes = 4;
    static constexpr int fmt = 0;
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
    static constexpr int fmt = 1;
    static __device__ __forceinline__ float decode(uint16_t u) { return (float)__builtin_bit_cast(_Float16, u); }
    static __device__ __forceinline__ uint16_t encode(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
    static __device__ __forceinline__ uint32_t pack2(float a, float b)
    {
        const f32x2_t v = {a, b};
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2_t));   // v_cvt_pk_f16_f32
    }
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
    static constexpr int fmt = 2;
    static __device__ __forceinline__ float decode(uint16_t u) { return __builtin_bit_cast(float, (uint32_t)u << 16); }
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        uint16_t u = __builtin_bit_cast(uint16_t, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
        return __builtin_bit_cast(float, (uint32_t)u << 16);
    }
    // Round to nearest even on the upper 16 bits (v_cvt_pk_bf16_f32; the
    // same bits as adding 0x7fff plus the kept part's lowest bit and
    // truncating, for the finite values messages are).
    static __device__ __forceinline__ uint16_t encode(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
    static __device__ __forceinline__ uint32_t pack2(float a, float b)
    {
        const f32x2_t v = {a, b};
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, float v, uint32_t voff, uint32_t soff)
    {
        __builtin_amdgcn_raw_buffer_store_b16(encode(v), r, voff, soff, 0);
    }
};

// ---- R consecutive values at a byte offset (pixel-major rows) ----

typedef unsigned int u32x2 __attribute__((vector_size(8)));
typedef unsigned int u32x4 __attribute__((vector_size(16)));

// Rows are loaded as consecutive 32-bit buffer loads held in scalar
// temporaries; the backend merges them into 8- and 16-byte loads.  (This
// toolchain's b128 load builtin lowers to a single 32-bit load, and 32-bit
// loads written into vector components are folded into one load.)
template <int N>
__device__ __forceinline__ void ld_words(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t (&w)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, voff + 4u * i, 0, 0);
}

// Stores: 16-byte stores for groups of four words, then 8- and 4-byte ones.
template <int N>
__device__ __forceinline__ void st_words(__amdgpu_buffer_rsrc_t r, uint32_t voff, const uint32_t (&w)[N])
{
    constexpr int Q = N / 4, rem = N - 4 * Q;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        u32x4 t;
        t[0] = w[4 * q]; t[1] = w[4 * q + 1]; t[2] = w[4 * q + 2]; t[3] = w[4 * q + 3];
        __builtin_amdgcn_raw_buffer_store_b128(t, r, voff + 16u * q, 0, 0);
    }
    if constexpr (rem >= 2) {
        u32x2 t;
        t[0] = w[4 * Q]; t[1] = w[4 * Q + 1];
        __builtin_amdgcn_raw_buffer_store_b64(t, r, voff + 16u * Q, 0, 0);
    }
    if constexpr (rem % 2 == 1) __builtin_amdgcn_raw_buffer_store_b32(w[N - 1], r, voff + 4u * (N - 1), 0, 0);
}

template <typename S, int R>
__device__ __forceinline__ void ld_row(__amdgpu_buffer_rsrc_t r, uint32_t voff, float (&v)[R])
{
    static_assert(R % 2 == 0, "pixel-major rows hold an even number of labels per lane");
    if constexpr (S::bytes == 4) {
        uint32_t w[R];
        ld_words<R>(r, voff, w);
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = __builtin_bit_cast(float, w[i]);
    } else {
        uint32_t w[R / 2];
        ld_words<R / 2>(r, voff, w);
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            v[2 * i] = S::decode((uint16_t)(w[i] & 0xffffu));
            v[2 * i + 1] = S::decode((uint16_t)(w[i] >> 16));
        }
    }
}

// R cost values of a pixel-major level at element offset e, stored as FP32
// (CF 0), FP16 (CF 1) or unsigned bytes (CF 2, R a multiple of 4).
template <int R, int CF>
__device__ __forceinline__ void ld_cost(__amdgpu_buffer_rsrc_t r, uint32_t e, float (&v)[R])
{
    if constexpr (CF == 1) {
        ld_row<StoreF16, R>(r, e * 2u, v);
    } else if constexpr (CF == 2) {
        static_assert(R % 4 == 0, "byte cost rows are whole words per lane");
        uint32_t w[R / 4];
        ld_words<R / 4>(r, e, w);
#pragma unroll
        for (int i = 0; i < R / 4; ++i)
#pragma unroll
            for (int b = 0; b < 4; ++b) v[4 * i + b] = (float)((w[i] >> (8 * b)) & 255u);
    } else {
        ld_row<StoreF32, R>(r, e * 4u, v);
    }
}

template <typename S, int R>
__device__ __forceinline__ void st_row(__amdgpu_buffer_rsrc_t r, uint32_t voff, const float (&v)[R])
{
    if constexpr (S::bytes == 4) {
        uint32_t w[R];
#pragma unroll
        for (int i = 0; i < R; ++i) w[i] = __builtin_bit_cast(uint32_t, v[i]);
        st_words<R>(r, voff, w);
    } else {
        uint32_t w[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) w[i] = S::pack2(v[2 * i], v[2 * i + 1]);
        st_words<R / 2>(r, voff, w);
    }
}

// ---- DPP exchanges inside segments of SEG lanes (SEG = 2, 4, 8 or 16) ----
// dpp controls: row_shl:n = 0x100 + n, row_shr:n = 0x110 + n,
// quad_perm(1,0,3,2) = 0xB1, quad_perm(2,3,0,1) = 0x4E, row_half_mirror = 0x141,
// row_mirror = 0x140.

template <int CTRL>
__device__ __forceinline__ float dpp_f(float old, float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v),
                                                                 CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int old, int v)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xF, 0xF, false);
}

// x + x[lane ^ D] for D in {2, 4, 8, 16, 32}: both lanes of a pair get the
// same bits (IEEE addition is commutative).  D = 2 is a quad permutation,
// D = 4 composes a quad reversal with a
// half-row mirror, D = 8 is a rotation by 8 within a 16-lane row, D = 16 and
// D = 32 are gfx950's register-only row and half-wave swaps: swapping x with
// a copy of itself leaves one register holding the even rows' (lower
// half's) values and the other the odd rows' (upper half's), so their sum is
// the pair sum in every lane.  The swap is written as inline assembly: with
// ROCm 7.2 the builtins' second result is lost after register coalescing
// (the sum compiles to 2 * r[0]).  The s_nop pairs cover the VALU-write to
// lane-swap-read hazard on both sides, which the compiler cannot see
// through the asm statement.
template <int D>
__device__ __forceinline__ float xor_sum(float x)
{
    static_assert(D == 2 || D == 4 || D == 8 || D == 16 || D == 32, "unsupported lane distance");
    if constexpr (D == 2) {
        return x + dpp_f<0x4E>(x, x);
    } else if constexpr (D == 4) {
        return x + dpp_f<0x141>(x, dpp_f<0x1B>(x, x));
    } else if constexpr (D == 8) {
        return x + dpp_f<0x128>(x, x);
    } else {
        float a = x, b = x;
        if constexpr (D == 16)
            asm volatile("s_nop 2\n\tv_permlane16_swap_b32 %0, %1\n\ts_nop 2" : "+v"(a), "+v"(b));
        else
            asm volatile("s_nop 2\n\tv_permlane32_swap_b32 %0, %1\n\ts_nop 2" : "+v"(a), "+v"(b));
        return a + b;
    }
}

// Value of lane (s - N) of the same segment, or `ident` when s < N.
template <int SEG, int N>
__device__ __forceinline__ float seg_from_lower(float v, float ident, int s)
{
    float r = dpp_f<0x110 + N>(ident, v);
    if constexpr (SEG < 16) r = s < N ? ident : r;
    return r;
}

// Value of lane (s + N) of the same segment, or `ident` when s + N >= SEG.
template <int SEG, int N>
__device__ __forceinline__ float seg_from_upper(float v, float ident, int s)
{
    float r = dpp_f<0x100 + N>(ident, v);
    if constexpr (SEG < 16) r = s + N >= SEG ? ident : r;
    return r;
}

// The three DPP chains of one message's transform over a whole 16-lane row,
// written as DPP minimum instructions and interleaved: p becomes the inclusive
// prefix minimum over lanes 0..s, q the inclusive suffix minimum over lanes
// s..15, and m the row's minimum on every lane.  A lane whose source lane lies
// outside the row is not written by a shifting DPP operation without
// bound_ctrl, so it keeps its own value, which is what an inclusive scan needs
// there; the butterfly's sources are all inside the row.  A DPP read of a
// register written by a VALU instruction needs two wait states, which the
// compiler cannot see inside the asm: within the block the other two chains'
// instructions provide them, an s_nop 1 covers a register written just before
// the block, and another one a DPP read just after it.  The values are never
// NaN.
__device__ __forceinline__ void row_scans16(float &p, float &q, float &m)
{
    asm volatile("s_nop 1\n\t"
                 "v_min_f32_dpp %0, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %1, %1, %1 row_shl:1 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %2, %2, %2 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %0, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %1, %1, %1 row_shl:2 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %2, %2, %2 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %0, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %1, %1, %1 row_shl:4 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %2, %2, %2 row_half_mirror row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %0, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %1, %1, %1 row_shl:8 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %2, %2, %2 row_mirror row_mask:0xf bank_mask:0xf\n\t"
                 "s_nop 1"
                 : "+v"(p), "+v"(q), "+v"(m));
}

// Minimum over aligned groups of SEG lanes (2, 4, 8 or 16), every lane ending
// with the group's minimum: the butterfly of seg_allreduce as DPP minimum
// instructions (all source lanes are inside the row).
template <int SEG>
__device__ __forceinline__ float seg_allmin(float v)
{
    static_assert(SEG == 2 || SEG == 4 || SEG == 8 || SEG == 16, "unsupported segment");
    asm volatile("s_nop 1\n\tv_min_f32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf" : "+v"(v));
    if constexpr (SEG > 2)
        asm volatile("s_nop 1\n\tv_min_f32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf" : "+v"(v));
    if constexpr (SEG > 4)
        asm volatile("s_nop 1\n\tv_min_f32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf" : "+v"(v));
    if constexpr (SEG > 8)
        asm volatile("s_nop 1\n\tv_min_f32_dpp %0, %0, %0 row_mirror row_mask:0xf bank_mask:0xf" : "+v"(v));
    asm volatile("s_nop 1" ::);
    return v;
}

// Inclusive prefix minimum over lanes 0..s of the segment.  A lane with no
// lane N below it in its segment takes its own value (min is idempotent), so
// the exchanges need no identity register.
template <int SEG>
__device__ __forceinline__ float seg_prefix_min(float v, int s)
{
    v = fminf(v, seg_from_lower<SEG, 1>(v, v, s));
    if constexpr (SEG > 2) v = fminf(v, seg_from_lower<SEG, 2>(v, v, s));
    if constexpr (SEG > 4) v = fminf(v, seg_from_lower<SEG, 4>(v, v, s));
    if constexpr (SEG > 8) v = fminf(v, seg_from_lower<SEG, 8>(v, v, s));
    return v;
}

// Inclusive suffix minimum over lanes s..SEG-1 of the segment (own value
// where lane s + N is outside the segment, as above).
template <int SEG>
__device__ __forceinline__ float seg_suffix_min(float v, int s)
{
    v = fminf(v, seg_from_upper<SEG, 1>(v, v, s));
    if constexpr (SEG > 2) v = fminf(v, seg_from_upper<SEG, 2>(v, v, s));
    if constexpr (SEG > 4) v = fminf(v, seg_from_upper<SEG, 4>(v, v, s));
    if constexpr (SEG > 8) v = fminf(v, seg_from_upper<SEG, 8>(v, v, s));
    return v;
}

// The three-label transform's exchanges over a whole 16-lane row, interleaved
// like row_scans16: `first` takes the minimum with `below` of the next lower
// lane, `last` with `above` of the next higher lane (a lane at the row's edge
// has none and keeps its value), and m becomes the row's minimum.
__device__ __forceinline__ void row_near16(float &first, float &last, float &m, float below, float above)
{
    asm volatile("s_nop 1\n\t"
                 "v_min_f32_dpp %2, %2, %2 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %0, %3, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %1, %4, %1 row_shl:1 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %2, %2, %2 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
                 "s_nop 1\n\t"
                 "v_min_f32_dpp %2, %2, %2 row_half_mirror row_mask:0xf bank_mask:0xf\n\t"
                 "s_nop 1\n\t"
                 "v_min_f32_dpp %2, %2, %2 row_mirror row_mask:0xf bank_mask:0xf\n\t"
                 "s_nop 1"
                 : "+v"(first), "+v"(last), "+v"(m)
                 : "v"(below), "v"(above));
}

template <int SEG>
__device__ __forceinline__ void seg_near(float &first, float &last, float &m, float below, float above, int s)
{
    if constexpr (SEG == 16) {
        row_near16(first, last, m, below, above);
    } else {
        const float inf = __builtin_huge_valf();
        first = fminf(first, seg_from_lower<SEG, 1>(below, inf, s));
        last = fminf(last, seg_from_upper<SEG, 1>(above, inf, s));
        m = seg_allmin<SEG>(m);
    }
}

// The five-label transform's exchanges over a whole 16-lane row: e[0] and
// e[1] (the lane's first two labels) take the minimum with b0 and b1 of the
// next lower lane, e[3] and e[2] (its last two) with a0 and a1 of the next
// higher lane, and m becomes the row's minimum; the same wait-state reasoning
// as row_scans16.
__device__ __forceinline__ void row_near2_16(float (&e)[4], float &m, float b0, float b1, float a0, float a1)
{
    asm volatile("s_nop 1\n\t"
                 "v_min_f32_dpp %4, %4, %4 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %0, %5, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %1, %6, %1 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %4, %4, %4 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %3, %7, %3 row_shl:1 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %2, %8, %2 row_shl:1 row_mask:0xf bank_mask:0xf\n\t"
                 "v_min_f32_dpp %4, %4, %4 row_half_mirror row_mask:0xf bank_mask:0xf\n\t"
                 "s_nop 1\n\t"
                 "v_min_f32_dpp %4, %4, %4 row_mirror row_mask:0xf bank_mask:0xf\n\t"
                 "s_nop 1"
                 : "+v"(e[0]), "+v"(e[1]), "+v"(e[2]), "+v"(e[3]), "+v"(m)
                 : "v"(b0), "v"(b1), "v"(a0), "v"(a1));
}

template <int SEG>
__device__ __forceinline__ void seg_near2(float (&e)[4], float &m, float b0, float b1, float a0, float a1, int s)
{
    if constexpr (SEG == 16) {
        row_near2_16(e, m, b0, b1, a0, a1);
    } else {
        const float inf = __builtin_huge_valf();
        e[0] = fminf(e[0], seg_from_lower<SEG, 1>(b0, inf, s));
        e[1] = fminf(e[1], seg_from_lower<SEG, 1>(b1, inf, s));
        e[3] = fminf(e[3], seg_from_upper<SEG, 1>(a0, inf, s));
        e[2] = fminf(e[2], seg_from_upper<SEG, 1>(a1, inf, s));
        m = seg_allmin<SEG>(m);
    }
}

// The transform's three segment reductions at once: p the inclusive prefix
// minimum, q the inclusive suffix minimum, m the segment minimum.
template <int SEG>
__device__ __forceinline__ void seg_scans(float &p, float &q, float &m, int s)
{
    if constexpr (SEG == 16) {
        row_scans16(p, q, m);
    } else {
        p = seg_prefix_min<SEG>(p, s);
        q = seg_suffix_min<SEG>(q, s);
        m = seg_allmin<SEG>(m);
    }
}

// Butterfly combine over the segment: every lane ends with op over all lanes.
template <int SEG, typename Op>
__device__ __forceinline__ float seg_allreduce(float v, Op op)
{
    v = op(v, dpp_f<0xB1>(v, v));
    if constexpr (SEG > 2) v = op(v, dpp_f<0x4E>(v, v));
    if constexpr (SEG > 4) v = op(v, dpp_f<0x141>(v, v));
    if constexpr (SEG > 8) v = op(v, dpp_f<0x140>(v, v));
    return v;
}

// Lowest index attaining the minimum value over the segment (ties: lower index).
template <int SEG>
__device__ __forceinline__ void seg_argmin(float &v, int &i)
{
    auto step = [&](float ov, int oi) {
        if (ov < v || (ov == v && oi < i)) {
            v = ov;
            i = oi;
        }
    };
    step(dpp_f<0xB1>(v, v), dpp_i<0xB1>(i, i));
    if constexpr (SEG > 2) step(dpp_f<0x4E>(v, v), dpp_i<0x4E>(i, i));
    if constexpr (SEG > 4) step(dpp_f<0x141>(v, v), dpp_i<0x141>(i, i));
    if constexpr (SEG > 8) step(dpp_f<0x140>(v, v), dpp_i<0x140>(i, i));
}

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
