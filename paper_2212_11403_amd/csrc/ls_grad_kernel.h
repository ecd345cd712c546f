// The adjoint kernel of the gradient and its launcher, shared by the
// translation units that instantiate it (one per precision and variant, so
// that the build compiles them in parallel).
#pragma once

#include <type_traits>

#include "ls_sweep.h"

namespace lsk {

// ---------------------------------------------------------------------------
// Adjoint pass over one segment [s0, s1] of variants, one workgroup per
// recipient, walking from s1 down to s0. Inputs: the forward vectors alpha^l
// of the segment (recomputed from its checkpoint), and the backward vector
// y^{s1+1} = theta^{s1+1} (.) beta^{s1+1} left in ybuf by the segment above
// (the last segment starts from beta^{L-1} = 1). For every variant l it
// forms, with d = sum_j alpha^l_j y^{l+1}_j, Sa = sum_j alpha^l_j and
// Sy = sum_j y^{l+1}_j (all reductions over the donor column),
//   d log P / d rho_l = (pi Sa Sy - d) / ((1 - rho_l) d + rho_l pi Sa Sy)
// (the exact score of the transition; homogeneous in alpha and y, so any
// scaling of the stored vectors cancels, the FP32 emission unit included),
// and, with beta^l = c y^{l+1} + b,
//   M_l = sum_{j mismatching at l} alpha^l_j beta^l_j / sum_j alpha^l_j beta^l_j
//   d log P / d mu += M_l / mu - (1 - M_l) / (1 - mu).
// Per-variant rho terms go to grow[l][r]; the mu term accumulates in gmu[r].
// PI (a prior copying matrix): the kernel keeps pi' = (N-1) Pi_ji beside
// y, as the sweep does; Sy becomes the pi'-weighted sum W' (so c =
// (1 - rho)(N-1) / W' and pi Sa Sy = Sa sum_j Pi_ji y_j, the prior-weighted
// normaliser of the score), and the derived forward step adds b pi'_j.
// MUV (a mutation probability per variant): theta^l is the pair of variant
// l from `emis` (the sweep's table), and d log P / d mu^l = M_l / mu^l -
// (1 - M_l) / (1 - mu^l), with the FP64 pair from `em64`, goes to
// gmul[l][r].
//
// The recompute keeps alpha only at even offsets from s0 (offset 0 is the
// checkpoint) and the c of every forward step. The pass therefore walks the
// segment in pairs: it reads alpha^{l-1} (even offset), derives alpha^l with
// the forward step theta^l (.) (c_l alpha^{l-1} + b_l) in the sweep's own
// arithmetic (the theta select is shared with the adjoint update), and
// handles variant l, then l-1. A segment whose top offset is even starts
// with that variant alone. This halves the alpha bytes written and read.
struct GradSegArgs {
    int64_t hr_stride;
    int32_t N, L, NF, R;
    int32_t s0, s1;
    double inv_mu, inv_omu;   // 1 / mu and 1 / (1 - mu)
    double th_match, th_mis;  // the sweep's emission pair (sweep_emissions)
    double bmul;              // b of the forward step is rho_{l-1} bmul (FP64)
};

// Largest group of the adjoint kernel. The narrow variant reads alpha one
// variant ahead and holds three vectors per slot (y, alpha of this variant
// and of the next), so its limit comes from grad_max_waves; the wide variant
// reads alpha when it is used and takes the sweep's limit, which allows the
// 16-wave groups of the largest N (at the price of register spills).
// (A slot count with no narrow shape still instantiates the narrow kernel,
// with a 4-wave bound, but never launches it.)
__host__ __device__ constexpr int grad_kernel_waves(int nslot, int vgpr_per_slot, bool narrow,
                                                    bool prior = false) {
    return !narrow ? max_waves_for(nslot, sweep_slot_vgprs(vgpr_per_slot, prior), prior)
                   : (grad_max_waves(nslot, vgpr_per_slot, prior) > 0
                          ? grad_max_waves(nslot, vgpr_per_slot, prior)
                          : 4);
}

template <class PT, int NSLOT, bool NARROW, bool MUV = false, bool PI = false>
__global__ void __launch_bounds__(64 * grad_kernel_waves(NSLOT, PT::vgpr_per_slot, NARROW, PI))
grad_seg_kernel(const uint64_t *__restrict__ Hr, const double *__restrict__ rho,
                const float *__restrict__ coef, const float *__restrict__ coefb,
                const int32_t *__restrict__ recipients,
                const typename PT::T *__restrict__ alpha0, const typename PT::T *__restrict__ aseg,
                const typename PT::T *__restrict__ cval, typename PT::T *__restrict__ ybuf,
                double *__restrict__ grow, double *__restrict__ gmu,
                const typename PT::T *__restrict__ emis, const double *__restrict__ em64,
                double *__restrict__ gmul, const double *__restrict__ prior,
                const GradSegArgs a) {
#pragma clang fp contract(off)
    using T = typename PT::T;
    constexpr int K = special_slots(NSLOT);
    constexpr int NR = NSLOT - K;
    constexpr int MAXW = grad_kernel_waves(NSLOT, PT::vgpr_per_slot, NARROW, PI);
    __shared__ T red[2 * kRedStride];

    const int nwaves = uniform(blockDim.x >> 6);
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x;
    const int N = a.N, NF = a.NF;
    const int i = recipients[r];
    if (i < 0 || i >= N) return;
    block_sum_init<MAXW>(red);
    __syncthreads();
    int parity = 0;

    const int sw = i >> 6;
    const uint64_t self_bit = 1ull << (i & 63);
    const bool self_full = sw < NF;
    const int g = self_full ? sw : 0;
    const int reg_base = g + wave * NR;
    const uint64_t m0 = (NR > 0 && wave == 0 && self_full) ? ~self_bit : ~0ull;
    const int self_off = self_full ? sw : 2 * NF;
    const T keep0 = lane_bit(m0) ? (T)1 : (T)0;
    int spec_off[K];
    T spec_keep[K];
    int spec_voff[K];  // element offset in a row; lanes without a donor read element 0
#pragma unroll
    for (int k = 0; k < K; ++k) {
        SpecSlot sp = special_slot(nwaves * NR + wave * K + k, NF, N, g, self_full, sw, self_bit);
        spec_off[k] = sp.off;
        spec_keep[k] = lane_bit(sp.bmask) ? (T)1 : (T)0;
        spec_voff[k] = (sp.word >= 0 && lane_bit(sp.valid)) ? sp.word * 64 + lane : 0;
    }
    const T th_m = (T)a.th_match, th_x = (T)a.th_mis;
    const double pi = 1.0 / (double)(N - 1);
    const int voff = lane * (int)sizeof(T);
    auto word_of = [&](int s) __attribute__((always_inline)) -> int {
        int w = reg_base + s;
        return w >= NF ? w - NF : w;
    };

    // with a prior matrix: pi' = (N-1) Pi_ji per slot, 0 on the recipient's
    // lane and on lanes without a donor (those read element 0, then masked)
    T pv[PI ? NSLOT : 1];
    if constexpr (PI) {
        const double *prow = prior + (int64_t)i * N;
        const double n1 = (double)(N - 1);
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            double x;
            if (s < NR) {
                x = prow[word_of(s) * 64 + lane];
                if (s == 0) x = lane_bit(m0) ? x : 0.0;
            } else {
                x = prow[spec_voff[s - NR]] * (double)spec_keep[s - NR];
            }
            pv[s] = (T)(x * n1);
        }
    }
    T y[NSLOT];
    double gm = 0.0;
    T Sy = (T)0;
    const bool fresh = a.s1 == a.L - 1;
    // alpha at an even offset from s0 (offset 0: the checkpoint)
    auto alpha_row = [&](int ll) __attribute__((always_inline)) -> const T * {
        return ll == a.s0 ? alpha0 + (int64_t)r * N
                          : aseg + ((int64_t)((ll - a.s0) / 2 - 1) * a.R + r) * N;
    };
    // alpha of variant ll, one value per slot (lanes of special slots that
    // hold no donor read element 0; the steps mask them)
    auto load_alpha = [&](int ll, T (&al)[NSLOT]) __attribute__((always_inline)) {
        const rsrc_t rs = make_rsrc(alpha_row(ll), (uint32_t)N * sizeof(T));
#pragma unroll
        for (int s = 0; s < NSLOT; ++s)
            al[s] = (s < NR) ? buf_load<T>(rs, voff, word_of(s) * 64 * (int)sizeof(T))
                             : buf_load<T>(rs, spec_voff[s - NR] * (int)sizeof(T), 0);
    };
    // One variant of the adjoint: returns the {d, Sa, Mn, Sy'} partial sums
    // and updates y. With DERIVE, alpha^ll is formed from alpha^{ll-1} (in
    // `src`) with the forward step of coefficients (cf, bf); otherwise `src`
    // is alpha^ll.
    auto step = [&](auto derive, int ll, T c, T b, const T (&src)[NSLOT], T cf, T bf,
                    T (&out)[4]) __attribute__((always_inline)) {
        constexpr bool DERIVE = decltype(derive)::value;
        const uint64_t *row = Hr + (int64_t)ll * a.hr_stride;
        const bool rb = (row[self_off] & self_bit) != 0;
        const uint64_t flip = rb ? ~0ull : 0ull;
        T ta, tb;
        if constexpr (MUV) {
            // kept in VGPRs, as in the sweep (else the row masks are flipped
            // with scalar xors)
            const T em = emis[2 * ll], ex = emis[2 * ll + 1];
            ta = in_vgpr(rb ? ex : em);
            tb = in_vgpr(rb ? em : ex);
        } else {
            ta = rb ? th_x : th_m;
            tb = rb ? th_m : th_x;
        }
        T d = 0, sa = 0, mn = 0, sy = 0;
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            const uint64_t m = (s < NR) ? row[reg_base + s] : row[spec_off[s - NR]];
            const T th = lane_bit(m) ? tb : ta;
            T al = src[s];
            if constexpr (DERIVE) {
                T bbf;
            if constexpr (PI) bbf = bf * pv[s];
            else bbf = (s < NR) ? (s == 0 ? bf * keep0 : bf) : bf * spec_keep[s - NR];
                al = th * fma(cf, al, bbf);
            }
            if (s >= NR) al = al * spec_keep[s - NR];
            const T bb = (s < NR) ? (s == 0 ? b * keep0 : b) : b * spec_keep[s - NR];
            d = fma(al, y[s], d);
            sa += al;
            const T u = fma(c, y[s], bb);
            mn = fma(lane_bit(m ^ flip) ? al : (T)0, u, mn);
            const T nv = th * u;
            y[s] = nv;
            if constexpr (PI) sy = fma(pv[s], nv, sy);
            else sy += nv;
        }
        out[0] = d;
        out[1] = sa;
        out[2] = mn;
        out[3] = sy;
    };
    using Loaded = std::false_type;
    using Derived = std::true_type;
    // the forward coefficients (c_ll, b_ll) that formed alpha^ll from
    // alpha^{ll-1}: c as the recompute stored it, b as the sweep forms it
    auto fwd_coefs = [&](int ll, T &cf, T &bf) __attribute__((always_inline)) {
        cf = cval[(int64_t)(ll - a.s0 - 1) * a.R + r];
        if constexpr (sizeof(T) == 4) bf = coef[2 * ll + 1];
        else bf = rho[ll - 1] * a.bmul;
    };
    auto mu_term = [&](int ll, double Mn, double Z) __attribute__((always_inline)) {
        const double M = Mn / Z;
        if constexpr (MUV) {
            if (lane == 0)
                gmul[(int64_t)ll * a.R + r] = M / em64[2 * ll + 1] - (1.0 - M) / em64[2 * ll];
        } else {
            gm += M * a.inv_mu - (1.0 - M) * a.inv_omu;
        }
    };
    // variant ll after the first of the pass: the rho term and the mu term.
    // beta^ll = c y^{ll+1} + b with c = (1 - rho_ll)(N-1) / Sy and b = rho_ll;
    // FP32 takes (1 - rho)(N-1) and rho from the backward coefficient table
    // and forms c as the sweep does. Only wave 0's terms are kept (thread 0
    // writes them), so only wave 0 forms them.
    auto variant = [&](auto derive, int ll, const T (&src)[NSLOT]) __attribute__((always_inline)) {
        T c, b;
        if constexpr (sizeof(T) == 4) {
            const float A = coefb[2 * ll];
            b = coefb[2 * ll + 1];
            const float r0 = __builtin_amdgcn_rcpf(Sy);
            const float r1 = fmaf(fmaf(-Sy, r0, 1.0f), r0, r0);
            const float qt = A * r1;
            c = fmaf(fmaf(-Sy, qt, A), r1, qt);
        } else {
            const double rr = rho[ll];
            c = ((1.0 - rr) * (double)(N - 1)) / Sy;
            b = rr;
        }
        T cf = (T)0, bf = (T)0;
        if constexpr (decltype(derive)::value) fwd_coefs(ll, cf, bf);
        T q[4];
        step(derive, ll, c, b, src, cf, bf, q);
        block_sum4<MAXW>(q, red, parity, wave);
        if (wave == 0) {
            const double rr = rho[ll];
            const double d = (double)q[0], Sa = (double)q[1];
            const double pss = pi * Sa * (double)Sy;
            if (lane == 0) grow[(int64_t)ll * a.R + r] = (pss - d) / ((1.0 - rr) * d + rr * pss);
            mu_term(ll, (double)q[2], (double)c * d + (double)b * Sa);
        }
        Sy = q[3];
    };
    // variant L-1: beta = 1, so y^{L-1} = theta^{L-1} and Z = Sa
    auto last_variant = [&](auto derive, int ll, const T (&src)[NSLOT]) __attribute__((always_inline)) {
        T cf = (T)0, bf = (T)0;
        if constexpr (decltype(derive)::value) fwd_coefs(ll, cf, bf);
        T q[4];
        step(derive, ll, (T)0, (T)1, src, cf, bf, q);
        block_sum4<MAXW>(q, red, parity, wave);
        if (wave == 0) mu_term(ll, (double)q[2], (double)q[1]);
        Sy = q[3];
    };

    // `al` holds the alpha the next unit (a lone even variant or a pair)
    // starts from. The narrow kernel reads the following unit's alpha into
    // `nx` before it works on this one, so the loads overlap a whole unit;
    // the wide kernel reads each when its unit starts.
    T al[NSLOT];
    auto advance = [&](T (&nx)[NSLOT]) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) al[s] = nx[s];
    };
    int l = a.s1;
    const bool top_even = ((a.s1 - a.s0) & 1) == 0;
    // alpha the first unit needs: alpha^{s1} if its offset is even, else
    // alpha^{s1-1}
    const int first = top_even ? a.s1 : a.s1 - 1;
    if constexpr (NARROW) load_alpha(first, al);
    if (fresh) {
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) y[s] = (T)0;
    } else {
        const rsrc_t rs = make_rsrc(ybuf + (int64_t)r * N, (uint32_t)N * sizeof(T));
        T sy = 0;
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            T x;
            if (s < NR) {
                x = buf_load<T>(rs, voff, word_of(s) * 64 * (int)sizeof(T));
                if (s == 0) x *= keep0;
            } else {
                x = buf_load<T>(rs, spec_voff[s - NR] * (int)sizeof(T), 0) * spec_keep[s - NR];
            }
            y[s] = x;
            if constexpr (PI) sy = fma(pv[s], x, sy);
            else sy += x;
        }
        T q[4] = {sy, (T)0, (T)0, (T)0};
        block_sum4<MAXW>(q, red, parity, wave);
        Sy = q[0];
    }
    // the first unit, outside the loop (it may be the last variant, and a
    // lone even variant only ever comes first)
    {
        T nx[NSLOT];
        const int nxt = top_even ? a.s1 - 2 : a.s1 - 3;  // alpha the next unit needs
        if constexpr (NARROW) load_alpha(nxt >= a.s0 ? nxt : a.s0, nx);
        else load_alpha(first, al);
        if (top_even) {
            if (fresh) last_variant(Loaded{}, l, al);
            else variant(Loaded{}, l, al);
            l -= 1;
        } else {
            if (fresh) last_variant(Derived{}, l, al);
            else variant(Derived{}, l, al);
            variant(Loaded{}, l - 1, al);
            l -= 2;
        }
        if constexpr (NARROW) advance(nx);
    }
    // pairs (l, l-1): offset of l odd, of l-1 even
    for (; l > a.s0; l -= 2) {
        T nx[NSLOT];
        if constexpr (NARROW) load_alpha(l - 3 >= a.s0 ? l - 3 : a.s0, nx);
        else load_alpha(l - 1, al);
        variant(Derived{}, l, al);
        variant(Loaded{}, l - 1, al);
        if constexpr (NARROW) advance(nx);
    }
    // hand y^{s0} to the segment below
    {
        const rsrc_t rs = make_rsrc(ybuf + (int64_t)r * N, (uint32_t)N * sizeof(T));
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            if (s < NR) {
                buf_store(y[s], rs, voff, word_of(s) * 64 * (int)sizeof(T));
            } else {
                SpecSlot sp = special_slot(nwaves * NR + wave * K + (s - NR), NF, N, g, self_full,
                                           sw, self_bit);
                if (lane_bit(sp.valid)) buf_store(y[s], rs, voff, sp.word * 64 * (int)sizeof(T));
            }
        }
    }
    if (threadIdx.x == 0) gmu[r] = (fresh ? 0.0 : gmu[r]) + gm;
}

// Launch of one instantiated variant (nwaves must fit it).
template <class PT, int NSLOT, bool NARROW>
hipError_t launch_grad_seg(const GradArgs &ga, const GradSegArgs &sa, int nwaves, hipStream_t st) {
    using T = typename PT::T;
    if (nwaves < 1 || nwaves > grad_kernel_waves(NSLOT, PT::vgpr_per_slot, NARROW, ga.prior != nullptr))
        return hipErrorInvalidValue;
    const GradLayout &L = ga.lay;
    char *ws = ga.ws;
    const int k = sa.s0 / ga.seg;
    const T *alpha0 = reinterpret_cast<const T *>(ws + L.off_ckpt) + (size_t)k * ga.R * ga.N;
    const T *aseg = reinterpret_cast<const T *>(ws + L.off_seg);
    const T *cval = reinterpret_cast<const T *>(ws + L.off_cval);
    T *ybuf = reinterpret_cast<T *>(ws + L.off_ybuf);
    double *grow = reinterpret_cast<double *>(ws + L.off_grow);
    double *gmu = reinterpret_cast<double *>(ws + L.off_gmu);
    const float *coef = sizeof(T) == 4 ? ga.coef_fwd32 : nullptr;
    const float *coefb = sizeof(T) == 4 ? ga.coef_bwd32 : nullptr;
    const T *emis = reinterpret_cast<const T *>(ga.emis);
    double *gmul = reinterpret_cast<double *>(ws + L.off_gmul);
    if (ga.emis && ga.prior)
        hipLaunchKernelGGL((grad_seg_kernel<PT, NSLOT, NARROW, true, true>), dim3(ga.R),
                           dim3(64 * nwaves), 0, st, ga.Hr, ga.rho, coef, coefb, ga.recipients,
                           alpha0, aseg, cval, ybuf, grow, gmu, emis, ga.em64, gmul, ga.prior, sa);
    else if (ga.prior)
        hipLaunchKernelGGL((grad_seg_kernel<PT, NSLOT, NARROW, false, true>), dim3(ga.R),
                           dim3(64 * nwaves), 0, st, ga.Hr, ga.rho, coef, coefb, ga.recipients,
                           alpha0, aseg, cval, ybuf, grow, gmu, nullptr, nullptr, nullptr,
                           ga.prior, sa);
    else if (ga.emis)
        hipLaunchKernelGGL((grad_seg_kernel<PT, NSLOT, NARROW, true>), dim3(ga.R),
                           dim3(64 * nwaves), 0, st, ga.Hr, ga.rho, coef, coefb, ga.recipients,
                           alpha0, aseg, cval, ybuf, grow, gmu, emis, ga.em64, gmul, nullptr, sa);
    else
        hipLaunchKernelGGL((grad_seg_kernel<PT, NSLOT, NARROW>), dim3(ga.R), dim3(64 * nwaves), 0,
                           st, ga.Hr, ga.rho, coef, coefb, ga.recipients, alpha0, aseg, cval, ybuf,
                           grow, gmu, nullptr, nullptr, nullptr, nullptr, sa);
    return hipGetLastError();
}

// The wide variant is instantiated only where a group can be wider than the
// narrow one allows.
template <class PT, int NSLOT>
constexpr bool grad_wide_needed() {
    constexpr int v = PT::vgpr_per_slot;
    return grad_max_waves(NSLOT, v) < max_waves_for(NSLOT, v) ||
           grad_max_waves(NSLOT, v, true) < max_waves_for(NSLOT, sweep_slot_vgprs(v, true), true);
}

// Adjoint launchers over the slot menu, one per precision and variant
// (ls_grad_seg_<prec>_<variant>.hip).
hipError_t grad_seg_f32_narrow(const GradArgs &ga, const GradSegArgs &sa, Shape sh, hipStream_t st);
hipError_t grad_seg_f32_wide(const GradArgs &ga, const GradSegArgs &sa, Shape sh, hipStream_t st);
hipError_t grad_seg_f64_narrow(const GradArgs &ga, const GradSegArgs &sa, Shape sh, hipStream_t st);
hipError_t grad_seg_f64_wide(const GradArgs &ga, const GradSegArgs &sa, Shape sh, hipStream_t st);
// The keep-alpha forward sweep of the segment recompute (ls_every_<prec>.hip).
hipError_t launch_every_f32(const SweepPtrs &p, const SweepArgs &a, Shape sh, hipStream_t st);
hipError_t launch_every_f64(const SweepPtrs &p, const SweepArgs &a, Shape sh, hipStream_t st);

}  // namespace lsk
