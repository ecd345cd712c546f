// The sweep kernel: scaled forward (eq. fwd0/fwd1) and backward (eq.
// bck0/bck1) recursions of the LS model for one recipient per workgroup,
// with the posterior (eq. postprob) and half distances (eq. distmat) fused at
// forward targets and beta snapshots written at backward targets.
//
// Both directions run the same update on a resident vector v:
//   v <- theta^l (.) (c v + b),  c = num / sum(v_prev),  b = rho-term,
// where (.) is the elementwise product and theta^l_j is 1-mu on a match of
// donor j with the recipient at variant l and mu on a mismatch, both divided
// by the larger (for mu <= 1/2: 1 and mu/(1-mu), with log(1-mu) per step in
// the log offset), so the emission scales only the donors whose value is
// not 1 (a lane-masked multiply).
//   forward:  v = kappa alpha^l,          c = (1-rho_{l-1}) kappa / S,
//             b = kappa rho_{l-1} / (N-1); log F^l = log F^{l-1} + log(S_l / kappa)
//   backward: v = kappa beta^l theta^l,   c = (1-rho_l) kappa (N-1) / S,
//             b = kappa rho_l;            log G^l = log G^{l+1} + log(S_{l+1} / ((N-1) kappa))
// (the backward form is eq. bck1 multiplied through by theta^l; c v + b is
// kappa beta^l itself, which is what snapshots and tables store).
//
// Layout of one recipient's donor column. Donor j belongs to 64-bit word
// j / 64 of a variant row, lane j % 64. Each wave holds NSLOT words ("slots")
// in registers: slot s, lane x holds one donor. The words are handed out in a
// rotated order that starts at the recipient's own word, so the self lane is
// always in slot 0 of wave 0, and the last K slots of every wave ("special"
// slots) take the remaining full words, the partial last word and empty
// (phantom) slots. Slot 0 and the special slots add the rho-term through a
// per-lane vector that is zero on the self lane and on lanes that hold no
// donor, which keeps those entries exactly 0 with no per-cell cost. The
// internal rows store every full word twice in a row, so the rotated words
// of a wave are contiguous and are read with wide scalar loads; the mask of
// one word drives v_cndmask for 64 donors at once.
#pragma once

#include <type_traits>

#include "ls_device.h"

namespace lsk {

// Placement of one special slot.
struct SpecSlot {
    int off;         // offset of its word in the internal row
    int word;        // donor word index (-1: phantom)
    uint64_t valid;  // lanes that hold a donor (self included)
    uint64_t bmask;  // lanes that hold a donor other than the recipient
};

__device__ __forceinline__ SpecSlot special_slot(int q, int NF, int N, int g, bool self_full,
                                                 int sw, uint64_t self_bit) {
    SpecSlot sp;
    if (q < NF) {
        int word = g + q;
        sp.off = word;
        if (word >= NF) word -= NF;
        sp.word = word;
        sp.valid = ~0ull;
        sp.bmask = (self_full && word == sw) ? ~self_bit : ~0ull;
    } else if ((N & 63) != 0 && q == NF) {
        sp.off = 2 * NF;
        sp.word = NF;
        sp.valid = (1ull << (N & 63)) - 1ull;
        sp.bmask = self_full ? sp.valid : (sp.valid & ~self_bit);
    } else {
        sp.off = 0;
        sp.word = -1;
        sp.valid = 0;
        sp.bmask = 0;
    }
    return sp;
}

// EVERY (forward only, kappa = 1; the segment recompute of the gradient):
// for the variants l0+1 .. t keep alpha at even offsets k = l - l0 (snap row
// tgt_out[0] + k/2 - 1) and the c of every step (at snap + c_off, [k-1][R]);
// the target list is not used.
// MUV: a mutation probability per variant; the emission pair of variant l is
// read from `emis` ([L][2], in the arithmetic type) and, in FP32 arithmetic,
// the logs of the divisors of the pairs emitted by this launch are added to
// the log scale from the prefix table `lu_prefix` ([L+1]).
// PI: a prior copying matrix (section 2.1; eq. transition with Pi_ki in
// place of 1/(N-1)). Row i of `prior` ([N][N] FP64) is the prior column of
// recipient i; the kernel keeps pi' = (N-1) Pi_ji beside the donor column
// (exactly 1 for the uniform prior). The forward jump term becomes b pi'_j,
// and the backward normaliser the pi'-weighted column sum W' in place of S:
// with y = theta^{l+1} (.) beta^{l+1}, beta^l is proportional to
// (1 - rho_l) y / W + rho_l, W = sum_j Pi_ji y_j, so c = (1 - rho) kappa
// (N-1) / W' and log G^l = log G^{l+1} + log(W' / ((N-1) kappa)).
// With FP16-stored vectors the backward normalises by the plain sum S
// instead: it keeps (W/S) beta^l, a positive multiple of beta^l per
// recipient and step, with c = (1 - rho) kappa (N-1) / S and
// b = kappa rho W' / ((N-1) S), whose entries stay below kappa (N-1) for
// any prior; its log scale adds log(S / ((N-1) kappa)) per step, which keeps
// the stored vector times exp(log scale) equal to kappa' beta^l G^l.
template <class PT, int NSLOT, int DIR, bool EVERY = false, bool MUV = false, bool PI = false>
__global__ void __launch_bounds__(64 * max_waves_for(NSLOT, sweep_slot_vgprs(PT::vgpr_per_slot, PI), PI))
__attribute__((amdgpu_waves_per_eu(
    sweep_waves_per_simd(sweep_budget_slots(NSLOT, sweep_slot_vgprs(PT::vgpr_per_slot, PI), EVERY),
                         sweep_slot_vgprs(PT::vgpr_per_slot, PI)))))
sweep_kernel(const uint64_t *__restrict__ Hr, const typename PT::T *__restrict__ emis,
             const double *__restrict__ lu_prefix, const double *__restrict__ prior,
             const double *__restrict__ rho,
             const float *__restrict__ coef, const int32_t *__restrict__ recipients, typename PT::ST *__restrict__ state,
             double *__restrict__ log_scale, uint32_t *__restrict__ status,
             typename PT::IO *__restrict__ snap, const SweepArgs a) {
    // No contraction: the column sums add the rounded entries, exactly as
    // the sum of a table loaded back from memory does, so a sweep resumed
    // from a stored table gives the same bits as an uninterrupted one.
#pragma clang fp contract(off)
    using T = typename PT::T;
    using ST = typename PT::ST;
    using IO = typename PT::IO;
    constexpr int K = special_slots(NSLOT);
    constexpr int NR = NSLOT - K;
    constexpr int MAXW = max_waves_for(NSLOT, sweep_slot_vgprs(PT::vgpr_per_slot, PI), PI);
    // emission as a lane-masked multiply (every sweep whose emission pairs
    // have a member equal to 1: all but FP64 with a per-variant mu), except
    // the gradient's keep-alpha recompute, where the select form measured
    // faster (its 8-slot groups store every step's vector: 0.43 against
    // 0.49 ms per segment in FP32 at N = 2,000, and the same in FP64)
    constexpr bool XMUL = !(MUV && sizeof(T) == 8) && !EVERY;
    // FP16-stored vectors: rounded to half after every update
    constexpr bool QH = std::is_same<ST, _Float16>::value;
    // the FP16-stored backward with a prior matrix normalises by the plain
    // column sum S and carries W'/S in the rho-term (entries stay below
    // kappa, inside half's range, whatever the prior)
    constexpr bool SNORM = QH && PI && DIR == 1;
    static_assert(!QH || XMUL, "FP16-stored sweeps use the masked emission");
    __shared__ T red[2 * kRedStride];

    const int nwaves = uniform(blockDim.x >> 6);
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int r = a.r0 + blockIdx.x;
    const int N = a.N, NF = a.NF;
    const int i = recipients[r];
    if (i < 0 || i >= N) {
        if (threadIdx.x == 0) status[r] |= kFlagBadRecipient;
        return;
    }
    block_sum_init<MAXW>(red);
    __syncthreads();
    // ---- geometry --------------------------------------------------------
    const int sw = i >> 6;
    const uint64_t self_bit = 1ull << (i & 63);
    const bool self_full = sw < NF;
    const int g = self_full ? sw : 0;
    const int reg_base = g + wave * NR;
    const uint64_t m0 = (NR > 0 && wave == 0 && self_full) ? ~self_bit : ~0ull;
    const int self_off = self_full ? sw : 2 * NF;
    // per special slot: row offset of its word (scalar) and a 0/1 multiplier
    // of the rho-term that is 0 on lanes without a donor or with the recipient
    int spec_off[K];
    T spec_keep[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        SpecSlot sp = special_slot(nwaves * NR + wave * K + k, NF, N, g, self_full, sw, self_bit);
        spec_off[k] = sp.off;
        spec_keep[k] = lane_bit(sp.bmask) ? (T)1 : (T)0;
    }
    const T keep0 = lane_bit(m0) ? (T)1 : (T)0;
    // the emission pair (match, mismatch), formed in FP64 by the host and
    // rounded once to the sweep precision
    const T th_m = (T)a.th_match, th_x = (T)a.th_mis;
    // masked emission with a scalar mu: the scaled member is fixed for the
    // whole sweep and held in a vector register
    T r_fix = (T)0;
    if constexpr (XMUL && !MUV && DIR == 1) r_fix = in_vgpr(th_m != (T)1 ? th_m : th_x);
    // with a prior matrix: pi' = (N-1) Pi_ji per slot, 0 on the recipient's
    // lane and on lanes without a donor
    T pv[PI ? NSLOT : 1];
    if constexpr (PI) {
        const rsrc_t rs = make_rsrc(prior + (int64_t)i * N, (uint32_t)N * sizeof(double));
        const int voff = lane * (int)sizeof(double);
        const double n1 = (double)(N - 1);
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            double x;
            if (s < NR) {
                int w = reg_base + s;
                if (w >= NF) w -= NF;
                x = buf_load<double>(rs, voff, w * 64 * (int)sizeof(double));
                if (s == 0) x = lane_bit(m0) ? x : 0.0;
            } else {
                SpecSlot sp = special_slot(nwaves * NR + wave * K + (s - NR), NF, N, g, self_full,
                                           sw, self_bit);
                x = 0.0;
                if (lane_bit(sp.bmask))
                    x = buf_load<double>(rs, voff, sp.word * 64 * (int)sizeof(double));
            }
            pv[s] = (T)(x * n1);
        }
    }

    // resident vector in the arithmetic precision; the table state (ST) is
    // converted only when it is loaded or stored
    T v[NSLOT];
    int parity = 0;
    double prod = 1.0;  // running product of column sums: mantissa part
    int expo = 0;       // and binary exponent
    int nlog = 0;       // number of per-step log offsets to add
    double base = 0.0;  // log scale the table started from
    int kt = 0;         // next target, in travel order
    T S;                // sum of the resident vector
    T part_w = (T)0;    // SNORM: this lane's pi'-weighted partial sum
    T Wsum = (T)0;      // SNORM: the pi'-weighted column sum W'
    // the workgroup sum of a step's partials (with SNORM also W')
    auto reduce = [&](T part) __attribute__((always_inline)) -> T {
        if constexpr (SNORM) {
            T x[4] = {part, part_w, (T)0, (T)0};
            block_sum4<MAXW>(x, red, parity, wave);
            Wsum = x[1];
            return x[0];
        } else {
            return block_sum<MAXW>(part, red, parity, wave, nwaves);
        }
    };

    // the recipient's own word of variant row l (read one step ahead)
    auto self_word = [&](int l) __attribute__((always_inline)) -> uint64_t {
        return Hr[(int64_t)l * a.hr_stride + self_off];
    };
    // emission pair (match, mismatch) of variant l with a per-variant mu;
    // with a scalar mu the pair is (th_m, th_x) and (em, ex) is not used
    auto emis_at = [&](int l, T &em, T &ex) __attribute__((always_inline)) {
        if constexpr (MUV) {
            em = emis[2 * l];
            ex = emis[2 * l + 1];
        } else {
            em = ex = (T)0;
        }
    };
    // theta pair for a variant whose recipient word is `sw_bits` (and whose
    // emission pair is (em, ex)): value where the donor bit is 0, where it is 1
    auto thetas = [&](uint64_t sw_bits, T em, T ex, T &ta, T &tb) __attribute__((always_inline)) {
        const bool rb = (sw_bits & self_bit) != 0;
        if constexpr (MUV) {
            // kept in VGPRs: as a select of two loaded scalars the compiler
            // flips every row mask with a scalar xor instead (one more
            // instruction per slot)
            ta = in_vgpr(rb ? ex : em);
            tb = in_vgpr(rb ? em : ex);
        } else {
            ta = rb ? th_x : th_m;
            tb = rb ? th_m : th_x;
        }
    };
    // Lane partial sums of the column: even slots into acc0, odd into acc1,
    // starting from slots 0 and 1 (the entries are never -0, so this equals
    // adding them to zero).
    auto accumulate = [&](int s, T x, T &acc0, T &acc1) __attribute__((always_inline)) {
        if (s == 0) acc0 = x;
        else if (s == 1) acc1 = x;
        else if (s & 1) acc1 += x;
        else acc0 += x;
    };
    // the column sum a step hands on: the backward with a prior matrix sums
    // pi' v (its normaliser W'), every other sweep v itself; the FP16-stored
    // backward with a prior matrix sums both (SNORM: plain sum in acc0/acc1,
    // the weighted one in aw0/aw1)
    T aw0 = (T)0, aw1 = (T)0;
    auto weighted = [&](int s, T x, T &acc0, T &acc1) __attribute__((always_inline)) {
        if (s == 0) acc0 = pv[0] * x;
        else if (s == 1) acc1 = pv[1] * x;
        else if (s & 1) acc1 = fma(pv[s], x, acc1);
        else acc0 = fma(pv[s], x, acc0);
    };
    auto account_sum = [&](int s, T x, T &acc0, T &acc1) __attribute__((always_inline)) {
        if constexpr (SNORM) {
            accumulate(s, x, acc0, acc1);
            weighted(s, x, aw0, aw1);
        } else if constexpr (PI && DIR == 1) {
            weighted(s, x, acc0, acc1);
        } else {
            accumulate(s, x, acc0, acc1);
        }
    };
    // FP16 storage: each new vector is rounded to half at every step, so the
    // sweep carries exactly the values a half table holds
    auto quantise = [&]() __attribute__((always_inline)) {
        if constexpr (QH) {
#pragma unroll
            for (int s = 0; s < NSLOT; ++s) v[s] = (T)(ST)v[s];
        }
    };
    // x on the lanes that hold a donor other than the recipient, 0 elsewhere
    // (slot 0 and the special slots). Their entries are 0 and stay 0, so
    // c v + b followed by this multiply gives the bits c v + 0 gives.
    auto keep_lanes = [&](int s, T x) __attribute__((always_inline)) -> T {
        if (s == 0 && NR > 0) return x * keep0;
        if (s >= NR) return x * spec_keep[s - NR];
        return x;
    };
    // Row words of slot s at variant row `row`.
    auto mask_of = [&](const uint64_t *row, int s) __attribute__((always_inline)) -> uint64_t {
        return (s < NR) ? row[reg_base + s] : row[spec_off[s - NR]];
    };
    // The emission as a lane-masked multiply (masked_scale4): one member of
    // the pair is exactly 1 (the pair divided by its larger member), so only
    // the donors taking the other value r are scaled. They are the lanes of
    // the row word XOR `flip`: the mismatching donors when r is the mismatch
    // value, the matching ones when it is the match value. Not for the FP64
    // sweep with a per-variant mu, whose pairs are kept as they are.
    auto xmul_params = [&](uint64_t sw_bits, T em, T ex, T &r, uint64_t &flip)
                           __attribute__((always_inline)) {
        const bool rb = (sw_bits & self_bit) != 0;
        T m1;
        if constexpr (MUV) {
            m1 = em;
            r = in_vgpr(em != (T)1 ? em : ex);
        } else if constexpr (DIR == 1) {
            m1 = th_m;
            r = r_fix;
        } else {
            m1 = th_m;
            r = in_vgpr(th_m != (T)1 ? th_m : th_x);
        }
        const bool on_match = m1 != (T)1;
        // a float compare runs on the vector unit; the flag goes back to a
        // scalar register, which the EXEC arithmetic needs
        flip = uniform((int)(rb != on_match)) ? ~0ull : 0ull;
    };
    auto xmul_all = [&](const uint64_t *row, uint64_t flip, T r) __attribute__((always_inline)) {
        masked_scale_all<NSLOT>(
            v, [&](int s) __attribute__((always_inline)) { return mask_of(row, s); }, flip, r);
    };
    // v <- theta^l (.) (c v + b); returns this lane's partial sum
    auto step = [&](int l, uint64_t sw_bits, T em, T ex, T c, T b_s)
                    __attribute__((always_inline)) -> T {
        const uint64_t *row = Hr + (int64_t)l * a.hr_stride;
        const T b = in_vgpr(b_s);
        T acc0, acc1 = (T)0;
        if constexpr (XMUL) {
            T r;
            uint64_t flip;
            xmul_params(sw_bits, em, ex, r, flip);
#pragma unroll
            for (int s = 0; s < NSLOT; ++s) {
                if constexpr (PI && DIR == 0) {
                    v[s] = fma(c, (T)v[s], b * pv[s]);
                } else if constexpr (DIR == 1) {
                    v[s] = keep_lanes(s, fma(c, (T)v[s], b));
                } else {
                    // the forward keeps the rho-term multiplier inside: with
                    // it outside, the scheduler issued the row loads after
                    // this block (forward at N = 10,000: 4% slower)
                    const T bb = (s < NR) ? (s == 0 ? b * keep0 : b) : b * spec_keep[s - NR];
                    v[s] = fma(c, (T)v[s], bb);
                }
            }
            // FP16 storage rounds what a table holds: the backward vector
            // kappa beta^l before its emission, the forward kappa alpha^l
            if constexpr (DIR == 1) quantise();
            xmul_all(row, flip, r);
            if constexpr (DIR == 0) quantise();
#pragma unroll
            for (int s = 0; s < NSLOT; ++s) account_sum(s, v[s], acc0, acc1);
            if constexpr (SNORM) part_w = aw0 + aw1;
            return acc0 + acc1;
        }
        T ta, tb;
        thetas(sw_bits, em, ex, ta, tb);
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            const T th = lane_bit(mask_of(row, s)) ? tb : ta;
            T bb;
            if constexpr (PI && DIR == 0) bb = b * pv[s];
            else bb = (s < NR) ? (s == 0 ? b * keep0 : b) : b * spec_keep[s - NR];
            const T nv = th * fma(c, (T)v[s], bb);
            v[s] = nv;
            account_sum(s, nv, acc0, acc1);
        }
        return acc0 + acc1;
    };
    // v <- c v + b (no emission): the backward vector before theta^l
    auto affine = [&](T c, T b) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) v[s] = keep_lanes(s, fma(c, v[s], b));
        quantise();
    };
    // v <- theta^l (.) v; returns this lane's partial sum
    auto emit = [&](int l) __attribute__((always_inline)) -> T {
        const uint64_t *row = Hr + (int64_t)l * a.hr_stride;
        T em, ex, ta, tb;
        emis_at(l, em, ex);
        T acc0, acc1 = (T)0;
        if constexpr (XMUL) {
            T r;
            uint64_t flip;
            xmul_params(row[self_off], em, ex, r, flip);
            xmul_all(row, flip, r);
#pragma unroll
            for (int s = 0; s < NSLOT; ++s) account_sum(s, v[s], acc0, acc1);
            if constexpr (SNORM) part_w = aw0 + aw1;
            return acc0 + acc1;
        }
        thetas(row[self_off], em, ex, ta, tb);
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            const T th = lane_bit(mask_of(row, s)) ? tb : ta;
            const T nv = th * v[s];
            v[s] = nv;
            account_sum(s, nv, acc0, acc1);
        }
        return acc0 + acc1;
    };
    // write v (times `scale`, as type D) to a row of N elements starting at
    // `dst`; the diagonal entry is written as 0 and lanes past N are skipped
    auto store_row = [&](auto *dst, T scale) __attribute__((always_inline)) {
        using D = typename std::remove_pointer<decltype(dst)>::type;
        const rsrc_t rs = make_rsrc(dst, (uint32_t)N * sizeof(D));
        const int voff = lane * (int)sizeof(D);
        const int rb = opaque(reg_base);
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            if (s < NR) {
                int w = rb + s;
                if (w >= NF) w -= NF;
                T x = (T)v[s] * scale;
                if (s == 0) x = lane_bit(m0) ? x : (T)0;
                buf_store((D)x, rs, voff, w * 64 * (int)sizeof(D), kStreaming);
            } else {
                SpecSlot sp = special_slot(opaque(nwaves * NR + wave * K) + (s - NR), NF, N, g,
                                           self_full, sw, self_bit);
                if (lane_bit(sp.valid)) {
                    T x = lane_bit(sp.bmask) ? (T)v[s] * scale : (T)0;
                    buf_store((D)x, rs, voff, sp.word * 64 * (int)sizeof(D), kStreaming);
                }
            }
        }
    };
    auto store_state = [&]() __attribute__((always_inline)) {
        const rsrc_t rs = make_rsrc(state + (int64_t)r * N, (uint32_t)N * sizeof(ST));
        const int voff = lane * (int)sizeof(ST);
        const int rb = opaque(reg_base);
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            if (s < NR) {
                int w = rb + s;
                if (w >= NF) w -= NF;
                ST x = (ST)v[s];
                if (s == 0) x = lane_bit(m0) ? x : (ST)0;
                buf_store(x, rs, voff, w * 64 * (int)sizeof(ST));
            } else {
                SpecSlot sp = special_slot(opaque(nwaves * NR + wave * K) + (s - NR), NF, N, g,
                                           self_full, sw, self_bit);
                if (lane_bit(sp.valid))
                    buf_store(lane_bit(sp.bmask) ? (ST)v[s] : (ST)0, rs, voff,
                              sp.word * 64 * (int)sizeof(ST));
            }
        }
    };
    auto load_state = [&]() __attribute__((always_inline)) {
        const rsrc_t rs = make_rsrc(state + (int64_t)r * N, (uint32_t)N * sizeof(ST));
        const int voff = lane * (int)sizeof(ST);
        const int rb = opaque(reg_base);
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            if (s < NR) {
                int w = rb + s;
                if (w >= NF) w -= NF;
                ST x = buf_load<ST>(rs, voff, w * 64 * (int)sizeof(ST));
                if (s == 0) x = lane_bit(m0) ? x : (ST)0;
                v[s] = (T)x;
            } else {
                SpecSlot sp = special_slot(opaque(nwaves * NR + wave * K) + (s - NR), NF, N, g,
                                           self_full, sw, self_bit);
                ST x = (ST)0;
                if (lane_bit(sp.bmask)) x = buf_load<ST>(rs, voff, sp.word * 64 * (int)sizeof(ST));
                v[s] = (T)x;
            }
        }
    };
    auto snapshot = [&]() __attribute__((always_inline)) {
        IO *dst = snap + (int64_t)a.tgt_out[kt] * a.snap_ts + (int64_t)r * a.snap_rs;
        store_row(dst, (T)a.inv_kappa);
        ++kt;
    };
    // (A_l, B_l) of variant l, with c = A_l / S and b = B_l. FP32 sweeps read
    // them from the model's coefficient table (formed in FP64, rounded once);
    // the FP64 sweep forms them here. Forward variant l uses rho_{l-1} (and
    // at l = 0 gives c = 0, b = kappa / (N-1), i.e. alpha^0); backward
    // variant l uses rho_l. A decoding forward sweep has the emission
    // divisor in A and B (cnum, bmul), so its vector is kappa alpha^l.
    auto coefs_at = [&](int l, T &A, T &B) __attribute__((always_inline)) {
        if constexpr (sizeof(T) == 4) {
            A = coef[2 * l];
            B = coef[2 * l + 1];
        } else if constexpr (DIR == 0) {
            // the load is unconditional: a branch here costs registers
            const double r0 = rho[l > 0 ? l - 1 : 0];
            const double rr = l > 0 ? r0 : 1.0;
            const double keep = l > 0 ? 1.0 : 0.0;
            A = keep * (1.0 - rr) * a.cnum;
            B = rr * a.bmul;
        } else {
            const double rr = rho[l];
            A = (1.0 - rr) * a.cnum;
            B = rr * a.bmul;
        }
    };
    // c = A / S in the sweep precision. FP64 divides (correctly rounded).
    // FP32 refines the hardware reciprocal (about 1 ulp, and its error has a
    // consistent sign, which the log scale would sum over every step) by one
    // Newton step and corrects the quotient once, which gives A / S rounded
    // to nearest in all but rare ties; a zero or non-finite S gives a NaN or
    // infinite c, as the division would.
    auto coef_c = [&](T A, T sum) __attribute__((always_inline)) -> T {
        if constexpr (sizeof(T) == 4) {
            const float r0 = __builtin_amdgcn_rcpf(sum);
            const float r1 = fmaf(fmaf(-sum, r0, 1.0f), r0, r0);
            const float q = A * r1;
            return fmaf(fmaf(-sum, q, A), r1, q);
        } else {
            return A / sum;
        }
    };
    auto account = [&](T sum) __attribute__((always_inline)) {
        int e;
        prod = frexp(prod * (double)sum, &e);
        expo += e;
        ++nlog;
    };

    // ---- march ------------------------------------------------------------
    // The variant loops below run only fused steps and contain no branches:
    // with the whole donor column live in registers, any control flow inside
    // them makes the register allocator spill. Targets, the first backward
    // step and the last backward step are handled between loop segments.
    const bool fresh = a.l0 < 0;
    if (fresh) {
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) v[s] = (T)0;
    } else {
        base = log_scale[r];
        load_state();
    }
    if constexpr (DIR == 0) {
        // alpha^0 = theta^0 pi (eq. fwd0), then eq. fwd1
        int l;
        S = (T)1;
        if (fresh) {
            l = 0;
        } else {
            l = a.l0 + 1;
            T acc0, acc1 = (T)0;  // same order as in step()
#pragma unroll
            for (int s = 0; s < NSLOT; ++s) accumulate(s, v[s], acc0, acc1);
            S = block_sum<MAXW>(acc0 + acc1, red, parity, wave, nwaves);
        }
        // the coefficients and the recipient's own word are read one variant
        // ahead, so their latency overlaps the previous step, and c of the
        // next variant is formed as soon as the column sum is known
        const int lmax = a.L - 1;
        if constexpr (EVERY) {
            // per special slot, the byte offset of each lane in a snapshot row;
            // lanes that hold no donor get an offset past the row, whose store
            // the buffer range check drops (the entries are exactly 0 anyway)
            int spec_byte[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                SpecSlot sp = special_slot(nwaves * NR + wave * K + k, NF, N, g, self_full, sw,
                                           self_bit);
                spec_byte[k] = (sp.word >= 0 && lane_bit(sp.valid))
                                   ? (sp.word * 64 + lane) * (int)sizeof(IO)
                                   : 0x7ffffff0;
            }
            const int voff = lane * (int)sizeof(IO);
            IO *const seg0 = snap + ((int64_t)a.tgt_out[0] * a.R + r) * N;
            // c of every step, [step][R]; one lane of the group stores it (the
            // others get an offset past the record, so their stores drop)
            const rsrc_t rs_c =
                make_rsrc(snap + a.c_off, (uint32_t)((a.t - a.l0) * a.R * (int)sizeof(IO)));
            const int c_voff = threadIdx.x == 0 ? r * (int)sizeof(IO) : 0x7ffffff0;
            T A_nx, B_nx, em_nx, ex_nx;
            coefs_at(l <= lmax ? l : lmax, A_nx, B_nx);
            emis_at(l <= lmax ? l : lmax, em_nx, ex_nx);
            uint64_t w_nx = self_word(l <= lmax ? l : lmax);
            for (; l <= a.t; ++l) {
                const T A = A_nx, B = B_nx, em = em_nx, ex = ex_nx;
                const uint64_t wb = w_nx;
                const int ln = l < lmax ? l + 1 : lmax;
                coefs_at(ln, A_nx, B_nx);
                emis_at(ln, em_nx, ex_nx);
                w_nx = self_word(ln);
                const T c = coef_c(A, S);
                T part = step(l, wb, em, ex, c, B);
                buf_store((IO)c, rs_c, c_voff, (l - a.l0 - 1) * a.R * (int)sizeof(IO));
                S = block_sum<MAXW>(part, red, parity, wave, nwaves);
                account(S);
                // alpha^l (exactly 0 on the recipient's lane and on lanes
                // without a donor), unscaled: kappa = 1 in this mode. Only
                // even offsets k = l - l0 from the checkpoint are kept, in row
                // k/2 - 1; at odd offsets the record is empty and the stores
                // drop (the adjoint pass derives those vectors with one step)
                const int k = l - a.l0;
                const rsrc_t rs =
                    make_rsrc(seg0 + (int64_t)((k >> 1) - 1 + (k & 1)) * a.R * N,
                              (k & 1) ? 0u : (uint32_t)N * (uint32_t)sizeof(IO));
                const int rb = opaque(reg_base);
#pragma unroll
                for (int s = 0; s < NSLOT; ++s) {
                    if (s < NR) {
                        int w = rb + s;
                        if (w >= NF) w -= NF;
                        buf_store((IO)v[s], rs, voff, w * 64 * (int)sizeof(IO), kStreaming);
                    } else {
                        buf_store((IO)v[s], rs, spec_byte[s - NR], 0, kStreaming);
                    }
                }
                // keep the stores of alpha^l ahead of the next update: moved
                // past it, they would hold a second copy of the column live
                __builtin_amdgcn_sched_barrier(0);
            }
        } else for (;;) {
            const int lend = kt < a.nt ? a.tgt_l[kt] : a.t;
            T A_nx, B_nx, em_nx, ex_nx;
            coefs_at(l <= lmax ? l : lmax, A_nx, B_nx);
            emis_at(l <= lmax ? l : lmax, em_nx, ex_nx);
            uint64_t w_nx = self_word(l <= lmax ? l : lmax);
            for (; l <= lend; ++l) {
                const T A = A_nx, b = B_nx, em = em_nx, ex = ex_nx;
                const uint64_t wb = w_nx;
                const int ln = l < lmax ? l + 1 : lmax;
                coefs_at(ln, A_nx, B_nx);
                emis_at(ln, em_nx, ex_nx);
                w_nx = self_word(ln);
                // c of this variant at the top of the step: its reciprocal
                // chain then overlaps the scalar address work of the step,
                // and the FP64 log-scale update sits after the reduction,
                // where nothing waits for it (forward at N = 10,000: 20.1
                // -> 18.0 ms per 2,048 variants with c formed after the
                // reduction instead)
                const T c = coef_c(A, S);
                T part = step(l, wb, em, ex, c, b);
                S = block_sum<MAXW>(part, red, parity, wave, nwaves);
                account(S);
            }
            if (kt < a.nt) snapshot();
            if (lend >= a.t) break;
        }
    } else {
        // beta^{L-1} = 1 (eq. bck0), then eq. bck1
        const int lstart = fresh ? a.L - 1 : a.l0;
        if (fresh) affine((T)0, (T)a.kappa);
        if (kt < a.nt && a.tgt_l[kt] == lstart) snapshot();
        if (a.t < lstart) {
            // each column sum enters the log scale right after its
            // reduction (off the path to the next step's coefficients)
            T part = emit(lstart);
            S = reduce(part);
            account(S);
            int l = lstart - 1;
            for (;;) {
                const int lend = kt < a.nt ? a.tgt_l[kt] : a.t;
                // the coefficients and the recipient's own word are read one
                // variant ahead
                T A_nx, B_nx, em_nx, ex_nx;
                coefs_at(l, A_nx, B_nx);
                emis_at(l, em_nx, ex_nx);
                uint64_t w_nx = self_word(l);
                for (; l > lend; --l) {
                    const T A = A_nx, B = B_nx, em = em_nx, ex = ex_nx;
                    const uint64_t wb = w_nx;
                    const int ln = l > 0 ? l - 1 : 0;
                    coefs_at(ln, A_nx, B_nx);
                    emis_at(ln, em_nx, ex_nx);
                    w_nx = self_word(ln);
                    const T c = coef_c(A, S);
                    const T b = SNORM ? coef_c(B * Wsum, S) : B;
                    part = step(l, wb, em, ex, c, b);
                    S = reduce(part);
                    account(S);
                }
                // l == lend: a target or the stopping variant; keep beta^l
                T A, B;
                coefs_at(l, A, B);
                const T c = coef_c(A, S);
                const T b = SNORM ? coef_c(B * Wsum, S) : B;
                affine(c, b);
                if (kt < a.nt && a.tgt_l[kt] == l) snapshot();
                if (l <= a.t) break;
                part = emit(l);
                S = reduce(part);
                account(S);
                --l;
            }
        }
    }
    // the keep-alpha recompute reads its start vector from a checkpoint that
    // the adjoint pass needs unchanged, and nothing reads its final vector
    if constexpr (!EVERY) store_state();
    // ---- epilogue: log scale and status ------------------------------------
    if (threadIdx.x == 0) {
        double ls = base + (log(prod) + (double)expo * 0.69314718055994530942) +
                    (double)nlog * a.log_off;
        if constexpr (MUV && sizeof(T) == 4) {
            // logs of the divisors of the emission pairs applied here: the
            // forward applies variants first .. t, the backward lstart .. t+1
            // (a decoding forward sweep has them in its coefficients and
            // passes no prefix table)
            if constexpr (DIR == 0) {
                const int first = a.l0 < 0 ? 0 : a.l0 + 1;
                if (lu_prefix && a.t >= first) ls += lu_prefix[a.t + 1] - lu_prefix[first];
            } else {
                const int lstart = a.l0 < 0 ? a.L - 1 : a.l0;
                if (a.t < lstart) ls += lu_prefix[lstart + 1] - lu_prefix[a.t + 1];
            }
        }
        log_scale[r] = ls;
        if (!isfinite(ls)) status[r] |= kFlagNonfinite;
    }
}

}  // namespace lsk
