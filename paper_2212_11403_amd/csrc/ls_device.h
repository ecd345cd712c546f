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

}  // namespace lsk
