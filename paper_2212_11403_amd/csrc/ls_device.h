// Device helpers for gfx950: precision traits, wave64 DPP reductions and
// workgroup reductions through LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ls_internal.h"

namespace lsk {

// ---------------------------------------------------------------------------
// Precision traits. T: arithmetic type of the recursion. ST: type the resident
// vector is kept in (registers and table). IO: type of snapshots, posteriors
// and half distances.
struct PrecF64 {
    using T = double;
    using ST = double;
    using IO = double;
    static constexpr int id = 0;
    static constexpr int vgpr_per_slot = 2;
};
struct PrecF32 {
    using T = float;
    using ST = float;
    using IO = float;
    static constexpr int id = 1;
    static constexpr int vgpr_per_slot = 1;
};
struct PrecF16 {
    using T = float;
    using ST = _Float16;
    using IO = float;
    static constexpr int id = 2;
    static constexpr int vgpr_per_slot = 1;
};

// ---------------------------------------------------------------------------
// Wave64 reductions with DPP. The pattern is fixed, so the summation order
// is the same on every call: butterflies inside each quad, rotations inside
// each 16-lane row, then the two row broadcasts, which leave the total in
// lane 63; that lane is read into a scalar register.

template <int CTRL, int ROWMASK = 0xF, int BANKMASK = 0xF, bool BOUND = true>
__device__ __forceinline__ float dpp_f32(float x) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWMASK, BANKMASK, BOUND));
}

template <int CTRL, int ROWMASK = 0xF, int BANKMASK = 0xF, bool BOUND = true>
__device__ __forceinline__ double dpp_f64(double x) {
    int lo = __double2loint(x), hi = __double2hiint(x);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, BANKMASK, BOUND);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, BANKMASK, BOUND);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float read_lane63(float x) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}
__device__ __forceinline__ double read_lane63(double x) {
    int lo = __builtin_amdgcn_readlane(__double2loint(x), 63);
    int hi = __builtin_amdgcn_readlane(__double2hiint(x), 63);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float wave_sum(float x) {
    x += dpp_f32<0xB1>(x);   // quad_perm [1,0,3,2]
    x += dpp_f32<0x4E>(x);   // quad_perm [2,3,0,1]
    x += dpp_f32<0x124>(x);  // row_ror:4
    x += dpp_f32<0x128>(x);  // row_ror:8
    // Row broadcasts as single DPP adds: rows outside row_mask are not
    // written and keep x (the compiler expresses them as a DPP move into a
    // zeroed register plus an add). s_nop 1 gives the two wait states a DPP
    // read of a just-written VGPR needs.
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "s_nop 1"
        : "+v"(x));
    return read_lane63(x);
}

// Four wave sums at once, each with the additions and order of wave_sum: the
// four chains are interleaved stage by stage, so each DPP read comes three
// instructions after the write it depends on and needs no wait states.
__device__ __forceinline__ void wave_sum4(const float (&x)[4], float (&w)[4]) {
    float a = x[0], b = x[1], c = x[2], d = x[3];
    a += dpp_f32<0xB1>(a);
    b += dpp_f32<0xB1>(b);
    c += dpp_f32<0xB1>(c);
    d += dpp_f32<0xB1>(d);
    a += dpp_f32<0x4E>(a);
    b += dpp_f32<0x4E>(b);
    c += dpp_f32<0x4E>(c);
    d += dpp_f32<0x4E>(d);
    a += dpp_f32<0x124>(a);
    b += dpp_f32<0x124>(b);
    c += dpp_f32<0x124>(c);
    d += dpp_f32<0x124>(d);
    a += dpp_f32<0x128>(a);
    b += dpp_f32<0x128>(b);
    c += dpp_f32<0x128>(c);
    d += dpp_f32<0x128>(d);
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %2, %2 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_add_f32_dpp %3, %3, %3 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %2, %2 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "v_add_f32_dpp %3, %3, %3 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "s_nop 1"
        : "+v"(a), "+v"(b), "+v"(c), "+v"(d));
    w[0] = read_lane63(a);
    w[1] = read_lane63(b);
    w[2] = read_lane63(c);
    w[3] = read_lane63(d);
}
__device__ __forceinline__ double wave_sum(double x) {
    x += dpp_f64<0xB1>(x);
    x += dpp_f64<0x4E>(x);
    x += dpp_f64<0x124>(x);
    x += dpp_f64<0x128>(x);
    x += dpp_f64<0x142, 0xA, 0xF, false>(x);  // row_bcast:15 into rows 1, 3
    x += dpp_f64<0x143, 0xC, 0xF, false>(x);  // row_bcast:31 into rows 2, 3
    return read_lane63(x);
}

__device__ __forceinline__ void wave_sum4(const double (&x)[4], double (&w)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = wave_sum(x[q]);
}

// Sum over the workgroup. Every wave returns the same value: each wave's
// partial goes to its entry of a double-buffered LDS array of kRedStride
// entries per buffer (entries of absent waves stay 0); lane k of every wave
// then reads entry k and the first ceil-pow2(MAXW) lanes are added with the
// same DPP butterflies on every wave, so the result is identical across waves
// and runs. One barrier per call; `parity` alternates so consecutive calls
// never reuse a buffer another wave may still be reading. A single-wave group
// takes the same path (its other entries are 0): a branch on the wave count,
// like a loop over it, makes the register allocator spill the resident vector
// inside the variant loop.
constexpr int kRedStride = 64;

// Sum of lanes 0..MAXW-1 (MAXW <= 16), returned as a scalar. The quad
// butterflies leave each quad's sum in all its lanes; row_ror:12 hands lane
// k the value of lane k+4 (a rotation right by 12 within the 16-lane row),
// which adds quad 1 to quad 0; row_ror:8 then adds lanes 8..15.
template <int MAXW, class T>
__device__ __forceinline__ T lanes_sum(T p) {
    static_assert(MAXW <= 16, "cross-wave sums cover one 16-lane DPP row");
    if constexpr (sizeof(T) == 4) {
        if constexpr (MAXW > 1) p += dpp_f32<0xB1>(p);
        if constexpr (MAXW > 2) p += dpp_f32<0x4E>(p);
        if constexpr (MAXW > 4) p += dpp_f32<0x12C>(p);
        if constexpr (MAXW > 8) p += dpp_f32<0x128>(p);
        return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(p)));
    } else {
        if constexpr (MAXW > 1) p += dpp_f64<0xB1>(p);
        if constexpr (MAXW > 2) p += dpp_f64<0x4E>(p);
        if constexpr (MAXW > 4) p += dpp_f64<0x12C>(p);
        if constexpr (MAXW > 8) p += dpp_f64<0x128>(p);
        int lo = __builtin_amdgcn_readfirstlane(__double2loint(p));
        int hi = __builtin_amdgcn_readfirstlane(__double2hiint(p));
        return __hiloint2double(hi, lo);
    }
}

template <int MAXW, class T>
__device__ __forceinline__ T block_sum(T x, T *red, int &parity, int wave, int nwaves) {
    T w = wave_sum(x);
    if constexpr (MAXW == 1) return w;
    T *buf = red + parity * kRedStride;
    buf[wave] = w;
    __syncthreads();
    T p = buf[threadIdx.x & 63];
    parity ^= 1;
    return lanes_sum<MAXW>(p);
}

// Four sums at once with one barrier (same fixed trees as block_sum). Wave w
// writes its partial of sum q to entry 16 q + w of a double-buffered array
// of kRedStride entries per buffer; lane k of every wave then reads entry k,
// so 16-lane DPP row q holds the partials of sum q, and the butterflies of
// lanes_sum, applied to all four rows at once, leave each total in the first
// lane of its row. The additions and their order are those of a pairwise
// tree over the wave partials.
template <int MAXW, class T>
__device__ __forceinline__ void block_sum4(T (&x)[4], T *red, int &parity, int wave) {
    static_assert(MAXW <= 16, "cross-wave sums cover one 16-lane DPP row");
    T w[4];
    wave_sum4(x, w);
    if constexpr (MAXW == 1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = w[q];
        return;
    }
    T *buf = red + parity * kRedStride;
#pragma unroll
    for (int q = 0; q < 4; ++q) buf[16 * q + wave] = w[q];
    __syncthreads();
    T p = buf[threadIdx.x & 63];
    if constexpr (sizeof(T) == 4) {
        if constexpr (MAXW > 1) p += dpp_f32<0xB1>(p);
        if constexpr (MAXW > 2) p += dpp_f32<0x4E>(p);
        if constexpr (MAXW > 4) p += dpp_f32<0x12C>(p);
        if constexpr (MAXW > 8) p += dpp_f32<0x128>(p);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            x[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(p), 16 * q));
    } else {
        if constexpr (MAXW > 1) p += dpp_f64<0xB1>(p);
        if constexpr (MAXW > 2) p += dpp_f64<0x4E>(p);
        if constexpr (MAXW > 4) p += dpp_f64<0x12C>(p);
        if constexpr (MAXW > 8) p += dpp_f64<0x128>(p);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int lo = __builtin_amdgcn_readlane(__double2loint(p), 16 * q);
            const int hi = __builtin_amdgcn_readlane(__double2hiint(p), 16 * q);
            x[q] = __hiloint2double(hi, lo);
        }
    }
    parity ^= 1;
}

// Zero both buffers of a block_sum or block_sum4 array (2 * kRedStride
// entries); call once before the first use, followed by a barrier.
template <int MAXW, class T>
__device__ __forceinline__ void block_sum_init(T *red) {
    for (int k = threadIdx.x; k < 2 * kRedStride; k += blockDim.x) red[k] = (T)0;
}

// ---------------------------------------------------------------------------
// Raw buffer access. A buffer resource covers one row; the per-lane byte
// offset stays in one VGPR and the per-slot offset is a scalar, so a long run
// of loads or stores does not need one 64-bit VGPR address per access.
using rsrc_t = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             0x00020000);
}

template <class X>
__device__ __forceinline__ X buf_load(rsrc_t rs, int voff, int soff);
template <>
__device__ __forceinline__ float buf_load<float>(rsrc_t rs, int voff, int soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(rsrc_t rs, int voff, int soff) {
    auto u = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0);
    return __hiloint2double((int)u[1], (int)u[0]);
}
template <>
__device__ __forceinline__ _Float16 buf_load<_Float16>(rsrc_t rs, int voff, int soff) {
    unsigned short u = __builtin_amdgcn_raw_buffer_load_b16(rs, voff, soff, 0);
    return __builtin_bit_cast(_Float16, u);
}

// Stores take a cache policy: 0 (default) or kStreaming (the `nt` bit), for
// data written once and read by a later kernel (snapshots), so the streamed
// rows do not displace the haplotype rows the sweep keeps reading.
constexpr int kStreaming = 2;

__device__ __forceinline__ void buf_store(float x, rsrc_t rs, int voff, int soff, int pol = 0) {
    if (pol == kStreaming)
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), rs, voff, soff, kStreaming);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), rs, voff, soff, 0);
}
__device__ __forceinline__ void buf_store(double x, rsrc_t rs, int voff, int soff, int pol = 0) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    u32x2 u;
    u[0] = (unsigned int)__double2loint(x);
    u[1] = (unsigned int)__double2hiint(x);
    if (pol == kStreaming)
        __builtin_amdgcn_raw_buffer_store_b64(u, rs, voff, soff, kStreaming);
    else
        __builtin_amdgcn_raw_buffer_store_b64(u, rs, voff, soff, 0);
}
__device__ __forceinline__ void buf_store(_Float16 x, rsrc_t rs, int voff, int soff, int pol = 0) {
    const unsigned short u = __builtin_bit_cast(unsigned short, x);
    if (pol == kStreaming)
        __builtin_amdgcn_raw_buffer_store_b16(u, rs, voff, soff, kStreaming);
    else
        __builtin_amdgcn_raw_buffer_store_b16(u, rs, voff, soff, 0);
}

__device__ __forceinline__ bool lane_bit(uint64_t mask) {
    return __builtin_amdgcn_inverse_ballot_w64(mask);
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// A wave-uniform value copied into a vector register. A VALU instruction that
// reads a scalar register (other than a lane mask) is not issued in the same
// cycle as another wave's VALU instruction; operands of the per-cell updates
// are therefore kept in VGPRs.
__device__ __forceinline__ float in_vgpr(float x) {
    float y;
    asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "s"(x));
    return y;
}
__device__ __forceinline__ double in_vgpr(double x) {
    int lo = __double2loint(x), hi = __double2hiint(x), ylo, yhi;
    asm volatile("v_mov_b32 %0, %1" : "=v"(ylo) : "v"(lo));
    asm volatile("v_mov_b32 %0, %1" : "=v"(yhi) : "v"(hi));
    return __hiloint2double(yhi, ylo);
}

// A copy of a scalar the compiler cannot see through. Address arithmetic of
// rarely executed stores derives from it, so it is not hoisted out of the
// variant loop (where it would pin one scalar register per slot).
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+s"(x));
    return x;
}

// ---------------------------------------------------------------------------
// Emission by lane mask. With the emission pair divided by its larger member
// (see sweep_emissions), one of the two values is exactly 1, so only the
// lanes whose donor takes the other value r need a multiply. The scalar unit
// sets EXEC to those lanes (the 64-bit row word XOR `flip`, which is all ones
// or all zeros), one vector multiply scales them, and EXEC is restored at the
// end of the block: one vector instruction per 64 cells where a select and a
// multiply would take two. Multiplying by 1 is exact, so the results are the
// bits the select form gives. Each block saves and restores EXEC (all lanes
// are active in the sweep); with NOP it ends with the wait states a DPP
// instruction needs after a scalar write of EXEC (the last block before a
// reduction). The scalar XOR also writes SCC, which the blocks declare as
// clobbered: the compiler keeps the carry of a 64-bit address addition in
// SCC between its two halves and may place such a pair around a block.
#define LS_XM(op, i) \
    "s_xor_b64 exec, %[m" #i "], %[fl]\n\t" op " %[v" #i "], %[r], %[v" #i "]\n\t"
#define LS_XM8(op) \
    LS_XM(op, 0) LS_XM(op, 1) LS_XM(op, 2) LS_XM(op, 3) LS_XM(op, 4) LS_XM(op, 5) LS_XM(op, 6) \
        LS_XM(op, 7)
#define LS_XM4(op) LS_XM(op, 0) LS_XM(op, 1) LS_XM(op, 2) LS_XM(op, 3)
#define LS_XM1(op) LS_XM(op, 0)
#define LS_XM_OUT8                                                                        \
    [v0] "+v"(v[0]), [v1] "+v"(v[1]), [v2] "+v"(v[2]), [v3] "+v"(v[3]), [v4] "+v"(v[4]), \
        [v5] "+v"(v[5]), [v6] "+v"(v[6]), [v7] "+v"(v[7]), [sv] "=&s"(sv)
#define LS_XM_IN8                                                                          \
    [m0] "s"(m[0]), [m1] "s"(m[1]), [m2] "s"(m[2]), [m3] "s"(m[3]), [m4] "s"(m[4]),       \
        [m5] "s"(m[5]), [m6] "s"(m[6]), [m7] "s"(m[7]), [fl] "s"(fl), [r] "v"(r)
#define LS_XM_OUT4 [v0] "+v"(v[0]), [v1] "+v"(v[1]), [v2] "+v"(v[2]), [v3] "+v"(v[3]), [sv] "=&s"(sv)
#define LS_XM_IN4 \
    [m0] "s"(m[0]), [m1] "s"(m[1]), [m2] "s"(m[2]), [m3] "s"(m[3]), [fl] "s"(fl), [r] "v"(r)
#define LS_XM_DEFINE(T, op)                                                                      \
    template <bool NOP>                                                                          \
    __device__ __forceinline__ void masked_scale8(T (&v)[8], const uint64_t (&m)[8], uint64_t fl, \
                                                  T r) {                                         \
        uint64_t sv;                                                                             \
        if constexpr (NOP)                                                                       \
            asm("s_mov_b64 %[sv], exec\n\t" LS_XM8(op) "s_mov_b64 exec, %[sv]\n\ts_nop 4"          \
                : LS_XM_OUT8 : LS_XM_IN8 : "scc");                                               \
        else                                                                                     \
            asm("s_mov_b64 %[sv], exec\n\t" LS_XM8(op) "s_mov_b64 exec, %[sv]"                    \
                : LS_XM_OUT8 : LS_XM_IN8 : "scc");                                               \
    }                                                                                            \
    template <bool NOP>                                                                          \
    __device__ __forceinline__ void masked_scale4(T (&v)[4], const uint64_t (&m)[4], uint64_t fl, \
                                                  T r) {                                         \
        uint64_t sv;                                                                             \
        if constexpr (NOP)                                                                       \
            asm("s_mov_b64 %[sv], exec\n\t" LS_XM4(op) "s_mov_b64 exec, %[sv]\n\ts_nop 4"          \
                : LS_XM_OUT4 : LS_XM_IN4 : "scc");                                               \
        else                                                                                     \
            asm("s_mov_b64 %[sv], exec\n\t" LS_XM4(op) "s_mov_b64 exec, %[sv]"                    \
                : LS_XM_OUT4 : LS_XM_IN4 : "scc");                                               \
    }                                                                                            \
    template <bool NOP>                                                                          \
    __device__ __forceinline__ void masked_scale1(T &v0, uint64_t m0, uint64_t fl, T r) {        \
        uint64_t sv;                                                                             \
        if constexpr (NOP)                                                                       \
            asm("s_mov_b64 %[sv], exec\n\t" LS_XM1(op) "s_mov_b64 exec, %[sv]\n\ts_nop 4"          \
                : [v0] "+v"(v0), [sv] "=&s"(sv)                                                  \
                : [m0] "s"(m0), [fl] "s"(fl), [r] "v"(r)                                         \
                : "scc");                                                                        \
        else                                                                                     \
            asm("s_mov_b64 %[sv], exec\n\t" LS_XM1(op) "s_mov_b64 exec, %[sv]"                    \
                : [v0] "+v"(v0), [sv] "=&s"(sv)                                                  \
                : [m0] "s"(m0), [fl] "s"(fl), [r] "v"(r)                                         \
                : "scc");                                                                        \
    }
LS_XM_DEFINE(float, "v_mul_f32")
LS_XM_DEFINE(double, "v_mul_f64")
#undef LS_XM_DEFINE
#undef LS_XM_OUT8
#undef LS_XM_IN8
#undef LS_XM_OUT4
#undef LS_XM_IN4
#undef LS_XM1
#undef LS_XM4
#undef LS_XM8
#undef LS_XM

// Makes the 24 row words of a group live in scalar registers at this point,
// so that their loads are issued together and waited for once. Scalar loads
// return out of order, so every wait for one of them waits for all; left to
// itself the scheduler of the widest kernels (high vector register pressure)
// issues one 8-word load at a time and waits for each, a round trip per 8
// slots and step.
__device__ __forceinline__ void sgpr_group24(const uint64_t (&m)[24]) {
    asm volatile("" ::"s"(m[0]), "s"(m[1]), "s"(m[2]), "s"(m[3]), "s"(m[4]), "s"(m[5]),
                 "s"(m[6]), "s"(m[7]), "s"(m[8]), "s"(m[9]), "s"(m[10]), "s"(m[11]),
                 "s"(m[12]), "s"(m[13]), "s"(m[14]), "s"(m[15]), "s"(m[16]), "s"(m[17]),
                 "s"(m[18]), "s"(m[19]), "s"(m[20]), "s"(m[21]), "s"(m[22]), "s"(m[23]));
}

// v[s] <- r v[s] on the lanes of (mask(s) ^ flip), s < NS, in blocks of
// 8, 4 and 1 slots; the last block carries the DPP wait states. From 64
// slots up the 8-slot blocks go in groups of three whose row words are
// loaded together (sgpr_group24).
template <int NS, class T, class MaskFn>
__device__ __forceinline__ void masked_scale_all(T (&v)[NS], MaskFn mask, uint64_t flip, T r) {
    constexpr int N8 = NS / 8, N4 = (NS % 8) / 4, N1 = NS % 4;
    constexpr int G = NS >= 64 ? 3 : 1;  // 8-slot blocks per load group
#pragma unroll
    for (int q0 = 0; q0 < N8; q0 += G) {
        const int ng = (N8 - q0) < G ? (N8 - q0) : G;
        uint64_t m[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) m[k] = k < 8 * ng ? mask(8 * q0 + k) : 0ull;
        if (G > 1 && ng == G) sgpr_group24(m);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (g >= ng) break;
            const int q = q0 + g;
            T x[8];
            uint64_t mm[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                x[k] = v[8 * q + k];
                mm[k] = m[8 * g + k];
            }
            if (q == N8 - 1 && N4 == 0 && N1 == 0) masked_scale8<true>(x, mm, flip, r);
            else masked_scale8<false>(x, mm, flip, r);
#pragma unroll
            for (int k = 0; k < 8; ++k) v[8 * q + k] = x[k];
        }
    }
    if constexpr (N4 > 0) {
        T x[4];
        uint64_t m[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[k] = v[8 * N8 + k];
            m[k] = mask(8 * N8 + k);
        }
        if constexpr (N1 == 0) masked_scale4<true>(x, m, flip, r);
        else masked_scale4<false>(x, m, flip, r);
#pragma unroll
        for (int k = 0; k < 4; ++k) v[8 * N8 + k] = x[k];
    }
#pragma unroll
    for (int s = NS - N1; s < NS; ++s) {
        if (s == NS - 1) masked_scale1<true>(v[s], mask(s), flip, r);
        else masked_scale1<false>(v[s], mask(s), flip, r);
    }
}

}  // namespace lsk
