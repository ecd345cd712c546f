// Log-likelihood reduction and the gradient of the summed log-likelihood
// with respect to the recombination probabilities and the mutation
// probability.
#include <cmath>
#include <cstring>

#include <algorithm>
#include <vector>

#include "ls_sweep.h"

namespace lsk {

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

size_t grad_workspace_bytes(int32_t N, int32_t L, int32_t R, int prec, GradLayout *lay) {
    GradLayout g;
    const size_t es = prec == 0 ? 8 : (prec == 1 ? 4 : 2);
    const size_t gs = prec == 0 ? 8 : 4;  // checkpoint / segment element
    int32_t seg = 1;
    while ((int64_t)seg * seg < L) ++seg;  // ceil(sqrt(L)) variants per segment
    const int32_t nseg = (L + seg - 1) / seg;
    size_t off = 0;
    g.off_recips = off;
    off = align256(off + sizeof(int32_t) * (size_t)R);
    g.off_state = off;
    off = align256(off + es * (size_t)R * N);
    g.off_ll = off;
    off = align256(off + sizeof(double) * (size_t)R);
    g.off_status = off;
    off = align256(off + sizeof(uint32_t) * (size_t)R);
    g.off_ckpt = off;
    off = align256(off + gs * (size_t)R * nseg * N);
    g.off_seg = off;
    off = align256(off + gs * (size_t)R * seg * N);
    g.off_grow = off;
    off = align256(off + sizeof(double) * (size_t)(L > 1 ? L - 1 : 1) * R);
    g.off_gmu = off;
    off = align256(off + sizeof(double) * (size_t)R);
    g.off_lsc = off;
    off = align256(off + sizeof(double) * (size_t)R);
    g.off_ybuf = off;
    off = align256(off + gs * (size_t)R * N);
    g.total = off;
    g.seg = seg;
    g.nseg = nseg;
    if (lay) *lay = g;
    return g.total;
}

__global__ void iota_kernel(int32_t *p, int32_t n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = i;
}

hipError_t launch_iota(int32_t *p, int32_t n, hipStream_t st) {
    int blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(iota_kernel, dim3(blocks), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

// One workgroup: per-thread strided partial sums in index order, then a
// fixed tree, so the total does not depend on scheduling.
__global__ void __launch_bounds__(256)
loglik_sum_kernel(const double *__restrict__ ll, int32_t R, double *loglik, double *pac) {
    __shared__ double part[256];
    double s = 0.0;
    for (int r = threadIdx.x; r < R; r += 256) {
        s += ll[r];
        if (loglik) loglik[r] = ll[r];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *pac = part[0];
}

hipError_t launch_loglik_sum(const double *ll, int32_t R, double *loglik, double *pac,
                             hipStream_t st) {
    hipLaunchKernelGGL(loglik_sum_kernel, dim3(1), dim3(256), 0, st, ll, R, loglik, pac);
    return hipGetLastError();
}

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
// scaling of the stored vectors cancels, the FP32 emission unit included), and, with beta^l = c y^{l+1} + b,
//   M_l = sum_{j mismatching at l} alpha^l_j beta^l_j / sum_j alpha^l_j beta^l_j
//   d log P / d mu += M_l / mu - (1 - M_l) / (1 - mu).
// Per-variant rho terms go to grow[l][r]; the mu term accumulates in gmu[r].
struct GradSegArgs {
    int64_t hr_stride;
    int32_t N, L, NF, R;
    int32_t s0, s1;
    double mu;
    double th_match, th_mis;  // the sweep's emission pair (sweep_emissions)
};

template <class PT, int NSLOT>
__global__ void __launch_bounds__(64 * max_waves_for(NSLOT, PT::vgpr_per_slot))
grad_seg_kernel(const uint64_t *__restrict__ Hr, const double *__restrict__ rho,
                const int32_t *__restrict__ recipients, const typename PT::T *__restrict__ alpha0,
                const typename PT::T *__restrict__ aseg, typename PT::T *__restrict__ ybuf,
                double *__restrict__ grow, double *__restrict__ gmu, const GradSegArgs a) {
    using T = typename PT::T;
    constexpr int K = special_slots(NSLOT);
    constexpr int NR = NSLOT - K;
    constexpr int MAXW = max_waves_for(NSLOT, PT::vgpr_per_slot);
    __shared__ T red[2 * 4 * MAXW];

    const int nwaves = uniform(blockDim.x >> 6);
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x;
    const int N = a.N, NF = a.NF;
    const int i = recipients[r];
    if (i < 0 || i >= N) return;
    block_sum_init<MAXW, T, 4>(red);
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

    T y[NSLOT];
    double gm = 0.0;
    T Sy = (T)0;
    const bool fresh = a.s1 == a.L - 1;
    int l = a.s1;
    auto alpha_row = [&](int ll) __attribute__((always_inline)) -> const T * {
        return ll == a.s0 ? alpha0 + (int64_t)r * N
                          : aseg + ((int64_t)(ll - a.s0 - 1) * a.R + r) * N;
    };
    // one variant: returns {d, Sa, Mn, Sy'} partial sums; updates y
    auto step = [&](int ll, T c, T b, T (&out)[4]) __attribute__((always_inline)) {
        const uint64_t *row = Hr + (int64_t)ll * a.hr_stride;
        const bool rb = (row[self_off] & self_bit) != 0;
        const uint64_t flip = rb ? ~0ull : 0ull;
        const T ta = rb ? th_x : th_m, tb = rb ? th_m : th_x;
        const rsrc_t rs = make_rsrc(alpha_row(ll), (uint32_t)N * sizeof(T));
        T d = 0, sa = 0, mn = 0, sy = 0;
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            const uint64_t m = (s < NR) ? row[reg_base + s] : row[spec_off[s - NR]];
            T al;
            if (s < NR) {
                al = buf_load<T>(rs, voff, word_of(s) * 64 * (int)sizeof(T));
            } else {
                al = buf_load<T>(rs, spec_voff[s - NR] * (int)sizeof(T), 0) * spec_keep[s - NR];
            }
            const T bb = (s < NR) ? (s == 0 ? b * keep0 : b) : b * spec_keep[s - NR];
            d = fma(al, y[s], d);
            sa += al;
            const T u = fma(c, y[s], bb);
            mn = fma(lane_bit(m ^ flip) ? al : (T)0, u, mn);
            const T nv = (lane_bit(m) ? tb : ta) * u;
            y[s] = nv;
            sy += nv;
        }
        out[0] = d;
        out[1] = sa;
        out[2] = mn;
        out[3] = sy;
    };
    auto mu_term = [&](double Mn, double Z) __attribute__((always_inline)) {
        const double M = Mn / Z;
        gm += M / a.mu - (1.0 - M) / (1.0 - a.mu);
    };

    if (fresh) {
        // variant L-1: beta = 1, so y^{L-1} = theta^{L-1} and Z = Sa
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) y[s] = (T)0;
        T q[4];
        step(l, (T)0, (T)1, q);
        block_sum4<MAXW>(q, red, parity, wave);
        mu_term((double)q[2], (double)q[1]);
        Sy = q[3];
        --l;
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
            sy += x;
        }
        T q[4] = {sy, (T)0, (T)0, (T)0};
        block_sum4<MAXW>(q, red, parity, wave);
        Sy = q[0];
    }
    for (; l >= a.s0; --l) {
        const double rr = rho[l];
        const T c = (T)((1.0 - rr) * (double)(N - 1)) / Sy;
        const T b = (T)rr;
        T q[4];
        step(l, c, b, q);
        block_sum4<MAXW>(q, red, parity, wave);
        const double d = (double)q[0], Sa = (double)q[1];
        const double pss = pi * Sa * (double)Sy;
        if (threadIdx.x == 0) grow[(int64_t)l * a.R + r] = (pss - d) / ((1.0 - rr) * d + rr * pss);
        mu_term((double)q[2], (double)c * d + rr * Sa);
        Sy = q[3];
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

template <class PT, int NSLOT>
static hipError_t launch_grad_seg(const GradArgs &ga, const GradSegArgs &sa, int nwaves,
                                  hipStream_t st) {
    using T = typename PT::T;
    if (nwaves < 1 || nwaves > max_waves_for(NSLOT, PT::vgpr_per_slot)) return hipErrorInvalidValue;
    const GradLayout &L = ga.lay;
    char *ws = ga.ws;
    const int k = sa.s0 / ga.seg;
    const T *alpha0 = reinterpret_cast<const T *>(ws + L.off_ckpt) + (size_t)k * ga.R * ga.N;
    hipLaunchKernelGGL((grad_seg_kernel<PT, NSLOT>), dim3(ga.R), dim3(64 * nwaves), 0, st, ga.Hr,
                       ga.rho, ga.recipients, alpha0,
                       reinterpret_cast<const T *>(ws + L.off_seg),
                       reinterpret_cast<T *>(ws + L.off_ybuf),
                       reinterpret_cast<double *>(ws + L.off_grow),
                       reinterpret_cast<double *>(ws + L.off_gmu), sa);
    return hipGetLastError();
}

template <class PT>
static hipError_t dispatch_grad_seg(const GradArgs &ga, const GradSegArgs &sa, Shape sh,
                                    hipStream_t st);
template <>
hipError_t dispatch_grad_seg<PrecF32>(const GradArgs &ga, const GradSegArgs &sa, Shape sh,
                                      hipStream_t st) {
    switch (sh.nslot) {
#define LS_CASE(n) \
    case n:        \
        return launch_grad_seg<PrecF32, n>(ga, sa, sh.nwaves, st);
        LS_MENU_GRAD(LS_CASE)
#undef LS_CASE
    default:
        return hipErrorInvalidValue;
    }
}
template <>
hipError_t dispatch_grad_seg<PrecF64>(const GradArgs &ga, const GradSegArgs &sa, Shape sh,
                                      hipStream_t st) {
    switch (sh.nslot) {
#define LS_CASE(n) \
    case n:        \
        return launch_grad_seg<PrecF64, n>(ga, sa, sh.nwaves, st);
        LS_MENU_GRAD(LS_CASE)
#undef LS_CASE
    default:
        return hipErrorInvalidValue;
    }
}

// Deterministic sums over recipients: grad_rho[l] = sum_r grow[l][r] (one
// workgroup of 64 per variant, fixed strided order then the DPP tree).
__global__ void __launch_bounds__(64)
sum_rows_kernel(const double *__restrict__ grow, int32_t R, int32_t rows, double *__restrict__ out) {
    const int l = blockIdx.x;
    if (l >= rows) return;
    const double *src = grow + (int64_t)l * R;
    double s = 0.0;
    for (int r = threadIdx.x; r < R; r += 64) s += src[r];
    s = wave_sum(s);
    if (threadIdx.x == 0) out[l] = s;
}

hipError_t launch_grad(const GradArgs &ga, int prec, Shape sh, double *loglik, double *pac,
                       double *grad_rho, double *grad_mu, hipStream_t st);

// Forward sweep keeping alpha at every variant (segment recompute).
template <class PT, int NSLOT>
static hipError_t launch_every_one(const SweepPtrs &p, const SweepArgs &a, int nwaves,
                                   hipStream_t st) {
    if (nwaves < 1 || nwaves > max_waves_for(NSLOT, PT::vgpr_per_slot)) return hipErrorInvalidValue;
    if (a.nblk < 1 || a.r0 < 0 || a.r0 + a.nblk > a.R) return hipErrorInvalidValue;
    hipLaunchKernelGGL((sweep_kernel<PT, NSLOT, 0, true>), dim3(a.nblk), dim3(64 * nwaves), 0, st,
                       p.Hr, p.rho, p.coef, p.recipients, (typename PT::ST *)p.state,
                       p.log_scale, p.status, (typename PT::IO *)p.snap, a);
    return hipGetLastError();
}

template <class PT>
static hipError_t launch_every(const SweepPtrs &p, const SweepArgs &a, Shape sh, hipStream_t st) {
    switch (sh.nslot) {
#define LS_CASE(n) \
    case n:        \
        return launch_every_one<PT, n>(p, a, sh.nwaves, st);
        LS_MENU_GRAD(LS_CASE)
#undef LS_CASE
    default:
        return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Whole gradient: a forward sweep with checkpoints every `seg` variants (its
// table also gives log P per recipient), then, segment by segment from the
// last, a forward recompute of the segment from its checkpoint (sweep kernel
// with a snapshot at every variant) followed by the adjoint pass above.
hipError_t launch_grad(const GradArgs &ga, int prec, Shape sh, double *loglik, double *pac,
                       double *grad_rho, double *grad_mu, hipStream_t st) {
    const GradLayout &Ly = ga.lay;
    char *ws = ga.ws;
    const int64_t RN = (int64_t)ga.R * ga.N;
    const size_t es = prec == 0 ? 8 : 4;
    const Emissions em = sweep_emissions(ga.mu, prec != 0);
    auto sweep = [&](int dir, int l0, int t, const int32_t *tl, int nt, void *state, void *snap,
                     double *lsc, bool every = false) -> hipError_t {
        SweepPtrs p;
        p.Hr = ga.Hr;
        p.rho = ga.rho;
        p.coef = prec == 0 ? nullptr : ga.coef_fwd32;
        p.recipients = ga.recipients;
        p.state = state;
        p.log_scale = lsc;
        p.status = reinterpret_cast<uint32_t *>(ws + Ly.off_status);
        p.snap = snap;
        SweepArgs a;
        std::memset(&a, 0, sizeof a);
        a.hr_stride = ga.hr_stride;
        a.N = ga.N;
        a.L = ga.L;
        a.NF = ga.NF;
        a.R = ga.R;
        a.dir = dir;
        a.l0 = l0;
        a.t = t;
        a.nt = nt;
        a.r0 = 0;
        a.nblk = ga.R;
        a.th_match = em.match;
        a.th_mis = em.mis;
        a.kappa = 1.0;
        a.inv_kappa = 1.0;
        a.cnum = 1.0;
        a.bmul = 1.0 / (double)(ga.N - 1);
        a.log_off = em.log_unit;
        for (int k = 0; k < nt; ++k) {
            a.tgt_l[k] = tl[2 * k];
            a.tgt_out[k] = tl[2 * k + 1];
        }
        if (every) {
            a.nt = 0;
            a.tgt_out[0] = tl[0];
            return prec == 0 ? launch_every<PrecF64>(p, a, sh, st)
                             : launch_every<PrecF32>(p, a, sh, st);
        }
        return prec == 0 ? launch_sweep_f64_fwd(p, a, sh, st) : launch_sweep_f32_fwd(p, a, sh, st);
    };
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(ws + Ly.off_status), 0u, ga.R, st);
    if (e != hipSuccess) return e;
    // 1. forward with checkpoints at l = k * seg; ll = log F^{L-1}
    void *fstate = ws + Ly.off_state;
    double *ll = reinterpret_cast<double *>(ws + Ly.off_ll);
    std::vector<int32_t> tl(2 * kMaxTargets);
    int l0 = -1;
    for (int k0 = 0; k0 < ga.nseg; k0 += kMaxTargets) {
        const int k1 = std::min(ga.nseg, k0 + kMaxTargets);
        for (int k = k0; k < k1; ++k) {
            tl[2 * (k - k0)] = k * ga.seg;
            tl[2 * (k - k0) + 1] = k;
        }
        const int t = k1 == ga.nseg ? ga.L - 1 : (k1 - 1) * ga.seg;
        e = sweep(0, l0, t, tl.data(), k1 - k0, fstate, ws + Ly.off_ckpt, ll);
        if (e != hipSuccess) return e;
        l0 = t;
    }
    // 2. segments from the last to the first
    double *scratch = reinterpret_cast<double *>(ws + Ly.off_lsc);
    for (int k = ga.nseg - 1; k >= 0; --k) {
        const int s0 = k * ga.seg;
        const int s1 = std::min(s0 + ga.seg - 1, ga.L - 1);
        if (s1 > s0) {
            // recompute alpha^{s0+1..s1} from the checkpoint (a copy, so the
            // checkpoint itself stays for the adjoint pass)
            e = hipMemcpyAsync(fstate, ws + Ly.off_ckpt + (size_t)k * RN * es, (size_t)RN * es,
                               hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return e;
            // alpha^{s0+1..s1} into segment rows 0 .. s1-s0-1
            const int32_t out0 = 0;
            e = sweep(0, s0, s1, &out0, 0, fstate, ws + Ly.off_seg, scratch, true);
            if (e != hipSuccess) return e;
        }
        GradSegArgs sa;
        sa.hr_stride = ga.hr_stride;
        sa.N = ga.N;
        sa.L = ga.L;
        sa.NF = ga.NF;
        sa.R = ga.R;
        sa.s0 = s0;
        sa.s1 = s1;
        sa.mu = ga.mu;
        sa.th_match = em.match;
        sa.th_mis = em.mis;
        e = prec == 0 ? dispatch_grad_seg<PrecF64>(ga, sa, sh, st)
                      : dispatch_grad_seg<PrecF32>(ga, sa, sh, st);
        if (e != hipSuccess) return e;
    }
    // 3. fixed-order sums over recipients
    if (ga.L > 1) {
        hipLaunchKernelGGL(sum_rows_kernel, dim3(ga.L - 1), dim3(64), 0, st,
                           reinterpret_cast<const double *>(ws + Ly.off_grow), ga.R, ga.L - 1,
                           grad_rho);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(sum_rows_kernel, dim3(1), dim3(64), 0, st,
                       reinterpret_cast<const double *>(ws + Ly.off_gmu), ga.R, 1, grad_mu);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_loglik_sum(ll, ga.R, loglik, pac, st);
}

}  // namespace lsk
