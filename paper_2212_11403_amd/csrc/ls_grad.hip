// Log-likelihood reduction and the gradient of the summed log-likelihood
// with respect to the recombination probabilities and the mutation
// probability.
#include <cmath>
#include <cstring>

#include <algorithm>
#include <vector>

#include "ls_grad_kernel.h"

namespace lsk {

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

size_t grad_workspace_bytes(int32_t N, int32_t L, int32_t R, int prec, bool muv,
                            GradLayout *lay) {
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
    off = align256(off + gs * (size_t)R * N * (size_t)std::max(1, (seg - 1) / 2));
    g.off_cval = off;
    off = align256(off + gs * (size_t)R * seg);
    g.off_grow = off;
    off = align256(off + sizeof(double) * (size_t)(L > 1 ? L - 1 : 1) * R);
    g.off_gmu = off;
    off = align256(off + sizeof(double) * (size_t)R);
    g.off_gmul = off;
    if (muv) off = align256(off + sizeof(double) * (size_t)L * R);
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

// The adjoint pass of one segment: the narrow kernel when the group fits
// it, else the wide one.
static hipError_t dispatch_grad_seg(int prec, const GradArgs &ga, const GradSegArgs &sa, Shape sh,
                                    hipStream_t st) {
    const int vps = prec == 0 ? 2 : 1;
    const bool narrow = sh.nwaves <= grad_max_waves(sh.nslot, vps, ga.prior != nullptr);
    if (prec == 0)
        return narrow ? grad_seg_f64_narrow(ga, sa, sh, st) : grad_seg_f64_wide(ga, sa, sh, st);
    return narrow ? grad_seg_f32_narrow(ga, sa, sh, st) : grad_seg_f32_wide(ga, sa, sh, st);
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

// ---------------------------------------------------------------------------
// Whole gradient: a forward sweep with checkpoints every `seg` variants (its
// table also gives log P per recipient), then, segment by segment from the
// last, a forward recompute of the segment from its checkpoint (sweep kernel
// in its keep-alpha mode) followed by the adjoint pass (ls_grad_kernel.h).
// The two halves are separate calls (GradPhase), so that a caller can keep
// the checkpoints of a log-likelihood evaluation and run the adjoint later.
hipError_t launch_grad(const GradArgs &ga, int prec, Shape sh, double *loglik, double *pac,
                       double *grad_rho, double *grad_mu, hipStream_t st, GradPhase phase) {
    const GradLayout &Ly = ga.lay;
    char *ws = ga.ws;
    const int64_t RN = (int64_t)ga.R * ga.N;
    const size_t es = prec == 0 ? 8 : 4;
    Emissions em = sweep_emissions(ga.mu);
    if (ga.emis) em.log_unit = 0.0;  // per variant, from the prefix table
    auto sweep = [&](int dir, int l0, int t, const int32_t *tl, int nt, void *state, void *snap,
                     double *lsc, bool every = false) -> hipError_t {
        SweepPtrs p;
        p.Hr = ga.Hr;
        p.emis = ga.emis;
        p.lu_prefix = ga.lu_prefix;
        p.prior = ga.prior;
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
        a.c_off = (int64_t)((Ly.off_cval - Ly.off_seg) / es);
        a.snap_ts = RN;
        a.snap_rs = ga.N;
        for (int k = 0; k < nt; ++k) {
            a.tgt_l[k] = tl[2 * k];
            a.tgt_out[k] = tl[2 * k + 1];
        }
        if (every) {
            a.nt = 0;
            a.tgt_out[0] = tl[0];
            return prec == 0 ? launch_every_f64(p, a, sh, st) : launch_every_f32(p, a, sh, st);
        }
        return prec == 0 ? launch_sweep_f64_fwd(p, a, ga.fwd_shape, st)
                         : launch_sweep_f32_fwd(p, a, ga.fwd_shape, st);
    };
    void *fstate = ws + Ly.off_state;
    double *ll = reinterpret_cast<double *>(ws + Ly.off_ll);
    hipError_t e = hipSuccess;
    if (phase != kGradAdjoint) {
        e = launch_fill_u32(reinterpret_cast<uint32_t *>(ws + Ly.off_status), 0u, ga.R, st);
        if (e != hipSuccess) return e;
        // 1. forward with checkpoints at l = k * seg; ll = log F^{L-1}. It runs
        // with the sweep's own shape and in the launches a plain forward sweep
        // makes (at most ga.chunk variants each, resuming from the table), so
        // log P is bit-identical to that of the log-likelihood alone. A launch
        // holds at most chunk / seg + 1 <= sqrt(chunk) + 1 checkpoints (with an
        // oversized chunk, a launch ends at its 256th checkpoint).
        std::vector<int32_t> tl(2 * kMaxTargets);
        int l0 = -1, knext = 0;
        while (l0 < ga.L - 1) {
            int t = std::min(ga.L - 1, (l0 < 0 ? 0 : l0) + ga.chunk);
            int nt = 0;
            for (; knext < ga.nseg && knext * ga.seg <= t && nt < kMaxTargets; ++knext, ++nt) {
                tl[2 * nt] = knext * ga.seg;
                tl[2 * nt + 1] = knext;
            }
            if (knext < ga.nseg && knext * ga.seg <= t) t = tl[2 * (nt - 1)];
            e = sweep(0, l0, t, tl.data(), nt, fstate, ws + Ly.off_ckpt, ll);
            if (e != hipSuccess) return e;
            l0 = t;
        }
        if (phase == kGradForward) return launch_loglik_sum(ll, ga.R, loglik, pac, st);
    }
    // 2. segments from the last to the first
    double *scratch = reinterpret_cast<double *>(ws + Ly.off_lsc);
    for (int k = ga.nseg - 1; k >= 0; --k) {
        const int s0 = k * ga.seg;
        const int s1 = std::min(s0 + ga.seg - 1, ga.L - 1);
        if (s1 > s0) {
            // recompute alpha^{s0+1..s1} into segment rows 0 .. s1-s0-1,
            // starting from the checkpoint itself (the keep-alpha sweep only
            // reads its table, so the checkpoint stays for the adjoint pass)
            const int32_t out0 = 0;
            e = sweep(0, s0, s1, &out0, 0, ws + Ly.off_ckpt + (size_t)k * RN * es, ws + Ly.off_seg,
                      scratch, true);
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
        sa.bmul = 1.0 / (double)(ga.N - 1);
        sa.inv_mu = 1.0 / ga.mu;
        sa.inv_omu = 1.0 / (1.0 - ga.mu);
        sa.th_match = em.match;
        sa.th_mis = em.mis;
        e = dispatch_grad_seg(prec, ga, sa, sh, st);
        if (e != hipSuccess) return e;
    }
    // 3. fixed-order sums over recipients
    if (ga.L > 1) {
        hipLaunchKernelGGL(sum_rows_kernel, dim3(ga.L - 1), dim3(64), 0, st,
                           reinterpret_cast<const double *>(ws + Ly.off_grow), ga.R, ga.L - 1,
                           grad_rho);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (ga.emis)
        hipLaunchKernelGGL(sum_rows_kernel, dim3(ga.L), dim3(64), 0, st,
                           reinterpret_cast<const double *>(ws + Ly.off_gmul), ga.R, ga.L, grad_mu);
    else
        hipLaunchKernelGGL(sum_rows_kernel, dim3(1), dim3(64), 0, st,
                           reinterpret_cast<const double *>(ws + Ly.off_gmu), ga.R, 1, grad_mu);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (phase == kGradAdjoint) return hipSuccess;
    return launch_loglik_sum(ll, ga.R, loglik, pac, st);
}

}  // namespace lsk
