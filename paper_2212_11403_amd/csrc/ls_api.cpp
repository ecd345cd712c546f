// Host side of the C ABI declared in include/ls.h: argument validation,
// kernel-shape selection, per-call scalar set-up and launches on the
// caller's stream. No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ls.h"
#include "ls_cluster.h"
#include "ls_internal.h"

using lsk::Shape;
using lsk::SweepArgs;
using lsk::SweepPtrs;

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

ls_status dev(hipError_t e) { return e == hipSuccess ? LS_OK : LS_ERR_DEVICE; }

bool valid_prec(int p) { return p == LS_FP64 || p == LS_FP32 || p == LS_FP32_F16STORE; }

size_t state_elem(int prec) { return prec == LS_FP64 ? 8 : (prec == LS_FP32 ? 4 : 2); }
size_t io_elem(int prec) { return prec == LS_FP64 ? 8 : 4; }

int64_t hr_stride_for(int32_t N) {
    const int64_t nf = N / 64;
    const int64_t need = 2 * nf + 1;
    return (need + 7) / 8 * 8;
}

// Byte offset of the coefficient tables in the model workspace (after the
// internal rows, 256-byte aligned).
size_t coef_offset_bytes(int32_t N, int32_t L) {
    const size_t rows = (size_t)L * (size_t)hr_stride_for(N) * sizeof(uint64_t);
    return (rows + 255) / 256 * 256;
}

// Byte offset of the emission tables of a per-variant mu, after the
// coefficient tables: [L][2] double, [L][2] float, [L+1] double.
size_t emis_offset_bytes(int32_t N, int32_t L) {
    return coef_offset_bytes(N, L) + (size_t)lsk::kCoefTables * 2 * (size_t)L * sizeof(float);
}

// Byte offset of the [N][2] checks of a prior matrix, after the emission
// tables.
size_t prior_stats_offset_bytes(int32_t N, int32_t L) {
    return emis_offset_bytes(N, L) + (size_t)L * (2 * sizeof(double) + 2 * sizeof(float)) +
           (size_t)(L + 1) * sizeof(double);
}

uint64_t fnv1a(uint64_t h, const void *data, size_t n) {
    const unsigned char *p = static_cast<const unsigned char *>(data);
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

// ---- kernel shapes ----------------------------------------------------------
int vgpr_per_slot(int prec) { return prec == LS_FP64 ? 2 : 1; }

bool in_menu(int prec, int n) {
#define LS_MATCH(v) \
    if (n == v) return true;
    if (prec == LS_FP64) {
        LS_MENU_F64(LS_MATCH)
    } else {
        LS_MENU_F32(LS_MATCH)
    }
#undef LS_MATCH
    return false;
}

std::vector<int> menu(int prec, bool grad = false) {
    std::vector<int> m;
#define LS_PUSH(v) m.push_back(v);
    if (grad) {
        LS_MENU_GRAD(LS_PUSH)
    } else if (prec == LS_FP64) {
        LS_MENU_F64(LS_PUSH)
    } else {
        LS_MENU_F32(LS_PUSH)
    }
#undef LS_PUSH
    return m;
}

// Does (nslot, nwaves) place every donor word of N haplotypes? Regular
// slots must all hold full words and all words must be placed.
bool shape_fits(int32_t N, int prec, int nslot, int nwaves, bool prior = false) {
    if (!in_menu(prec, nslot)) return false;
    const int vps = lsk::sweep_slot_vgprs(vgpr_per_slot(prec), prior);
    if (nwaves < 1 || nwaves > lsk::max_waves_for(nslot, vps, prior)) return false;
    const int NW = (N + 63) / 64, NF = N / 64;
    const int K = lsk::special_slots(nslot);
    return (int64_t)nwaves * (nslot - K) <= NF && (int64_t)nwaves * nslot >= NW;
}

// Relative time of one recipient step for a shape, from a cost model fitted
// to measured sweep times on MI355X: the VALU work of the step (per slot and
// per wave) over all waves of the group, inflated when a SIMD holds fewer
// waves than it needs to hide the per-step load, reduction and barrier
// latency, and by the uneven spread of the group's waves over the four SIMDs
// of a compute unit (every step ends in a barrier, so the busiest SIMD sets
// the pace). Sweeps with the masked emission were fitted to every shape
// that places N: FP32 arithmetic at N = 1,000 .. 100,000 (130 shapes), FP64
// at N = 1,000 .. 45,000 (111 shapes), forward and backward; sweeps with a
// prior matrix and the gradient keep the parameters fitted to the select
// form (N = 2,000 .. 100,000, 38 shapes).
double shape_cost(int32_t N, int prec, int ns, int nw, int wps = 0, bool sweep = true) {
    const bool f64 = prec == LS_FP64;
    if (wps <= 0) wps = lsk::sweep_waves_per_simd(ns, vgpr_per_slot(prec));
    // waves resident per SIMD when all N recipients are swept
    const double occ = std::min<double>(wps, (double)N * nw / 1024.0);
    double ops, hide, ex;
    if (sweep) {
        ops = 2.5 * ns + 40.0;
        hide = f64 ? 2.5 : 5.0;
        ex = f64 ? 0.5 : 1.5;
    } else {
        ops = (f64 ? 4.19 : 4.0) * ns + 60.7;
        hide = f64 ? 3.34 : 5.57;
        ex = 0.847;
    }
    const double imb = nw >= 4 ? ((nw + 3) / 4) / (nw / 4.0) : 1.0;
    return (double)nw * ops * std::max(1.0, hide / occ) * std::pow(imb, ex);
}

// Cheapest shape by shape_cost; among shapes within 1% of the cheapest, the
// one with the fewest waves (then the fewest slots). Depends on N and the
// precision only, so a given problem always runs with the same summation
// order. The gradient first looks among the groups its prefetching adjoint
// kernel runs (grad_max_waves), costed with that kernel's occupancy; only
// when none of them places N does it take the sweep's wider groups.
bool choose_shape(int32_t N, int prec, Shape *out, bool grad = false, bool prior = false) {
    if (const char *env = std::getenv("LS_FORCE_SHAPE")) {
        int ns = 0, nw = 0;
        if (std::sscanf(env, "%d,%d", &ns, &nw) == 2 && shape_fits(N, prec, ns, nw, prior)) {
            *out = Shape{ns, nw};
            return true;
        }
    }
    const int vps = vgpr_per_slot(prec);
    for (int pass = grad ? 0 : 1; pass < 2; ++pass) {
        auto ok = [&](int ns, int nw) {
            return shape_fits(N, prec, ns, nw, prior) &&
                   (pass == 1 || nw <= lsk::grad_max_waves(ns, vps, prior));
        };
        auto cost = [&](int ns, int nw) {
            const int wps = pass == 0 ? lsk::grad_waves_per_simd(ns, vps, prior)
                                      : lsk::sweep_waves_per_simd(ns, lsk::sweep_slot_vgprs(vps, prior));
            return shape_cost(N, prec, ns, nw, wps, !grad && !prior);
        };
        double best = 1e300;
        for (int nw = 1; nw <= lsk::kMaxWaves; ++nw)
            for (int ns : menu(prec, grad))
                if (ok(ns, nw)) best = std::min(best, cost(ns, nw));
        if (best >= 1e300) continue;
        for (int nw = 1; nw <= lsk::kMaxWaves; ++nw)
            for (int ns : menu(prec, grad))
                if (ok(ns, nw) && cost(ns, nw) <= best * 1.01) {
                    *out = Shape{ns, nw};
                    return true;
                }
    }
    return false;
}

ls_status check_model(const ls_model *m) {
    if (!m || !m->Hr || m->hash == 0 || m->N < 2 || m->L < 1) return LS_ERR_ARG;
    return LS_OK;
}

// `fold`: the forward multiplies the emission divisor back into c and b, so
// that its vector is kappa alpha^l (decoding tables); without it the forward
// keeps the divided pairs' scale and adds the divisor's log per step, as the
// gradient's forward recursion does (see loglik_grad_impl).
void fill_scalars(SweepArgs &a, const ls_model *m, int prec, int dir, bool fold = true) {
    const double n1 = (double)(m->N - 1);
    double kappa = 1.0;
    if (prec == LS_FP32_F16STORE) kappa = dir == 0 ? 16384.0 : 16384.0 / n1;
    a.hr_stride = m->hr_stride;
    a.N = m->N;
    a.L = m->L;
    a.NF = m->N / 64;
    lsk::Emissions em = lsk::sweep_emissions(m->mu);
    if (m->mu_vec) {
        // per variant: in the coefficient tables (forward) or from the
        // prefix table (backward); the FP64 pairs are not divided
        em.log_unit = 0.0;
        em.unit = 1.0;
    }
    a.th_match = em.match;
    a.th_mis = em.mis;
    a.kappa = kappa;
    a.inv_kappa = 1.0 / kappa;
    if (dir == 0) {
        const double u = fold ? em.unit : 1.0;
        a.cnum = kappa * u;
        a.bmul = kappa / n1 * u;
        a.log_off = (fold ? 0.0 : em.log_unit) - std::log(kappa);
    } else {
        a.cnum = kappa * n1;
        a.bmul = kappa;
        a.log_off = em.log_unit - std::log(n1 * kappa);
    }
}

// The coefficient table of a precision and direction (FP32 arithmetic), or
// null for the FP64 sweep, which forms its coefficients per variant.
const float *coef_table(const ls_model *m, int prec, int dir) {
    if (prec == LS_FP64) return nullptr;
    const int k = (prec == LS_FP32 ? lsk::kCoefF32Fwd : lsk::kCoefF16Fwd) + (dir ? 1 : 0);
    const char *base = reinterpret_cast<const char *>(m->Hr) + coef_offset_bytes(m->N, m->L);
    return reinterpret_cast<const float *>(base) + (size_t)k * 2 * (size_t)m->L;
}

// The forward coefficients of the gradient's recursion (divided emission
// pairs' scale), or null for the FP64 sweep.
const float *grad_forward_coefs(const ls_model *m, int prec) {
    if (prec == LS_FP64) return nullptr;
    return reinterpret_cast<const float *>(reinterpret_cast<const char *>(m->Hr) +
                                           coef_offset_bytes(m->N, m->L)) +
           (size_t)lsk::kCoefF32FwdGrad * 2 * (size_t)m->L;
}

// Per-variant mu: the emission pairs in the sweep's arithmetic type and, for
// FP32 arithmetic, the log-unit prefix; null for a scalar mu.
void emission_tables(const ls_model *m, int prec, SweepPtrs &p) {
    p.emis = nullptr;
    p.lu_prefix = nullptr;
    if (!m->mu_vec) return;
    const char *base = reinterpret_cast<const char *>(m->Hr) + emis_offset_bytes(m->N, m->L);
    const size_t L = (size_t)m->L;
    if (prec == LS_FP64) {
        p.emis = base;
    } else {
        p.emis = base + 2 * L * sizeof(double);
        p.lu_prefix = reinterpret_cast<const double *>(base + 2 * L * (sizeof(double) + sizeof(float)));
    }
}

hipError_t launch_sweep(int prec, int dir, const SweepPtrs &p, const SweepArgs &a, Shape sh,
                        hipStream_t st) {
    if (prec == LS_FP64)
        return dir == 0 ? lsk::launch_sweep_f64_fwd(p, a, sh, st)
                        : lsk::launch_sweep_f64_bwd(p, a, sh, st);
    if (prec == LS_FP32)
        return dir == 0 ? lsk::launch_sweep_f32_fwd(p, a, sh, st)
                        : lsk::launch_sweep_f32_bwd(p, a, sh, st);
    return dir == 0 ? lsk::launch_sweep_f16_fwd(p, a, sh, st)
                    : lsk::launch_sweep_f16_bwd(p, a, sh, st);
}

// Variants per sweep launch. A long sweep is split into launches of at most
// this many variants, each resuming from the table the previous one left
// (resumption is exact in every precision). Every launch starts all groups at
// the same variant; within one long launch the groups drift apart, the rows
// they read at any moment spread beyond the L2 cache and the scalar row loads
// fall through to the last-level cache. Measured backward sweep at N = 10,000,
// L = 100,000: one launch 1044 ms; chunks of 8192: 984; 4096: 913; 2048: 882;
// 1024: 883 ms (row fetches beyond L2: 325 GB at 4096, 62 GB at 1024).
// FP16-stored sweeps round the vector to half at every step, so a table
// stored at a launch boundary holds exactly the values the sweep carries on
// with, and they are split the same way.
constexpr int32_t kSweepChunk = 2048;

// The chunk length (LS_SWEEP_CHUNK overrides it, for tuning).
int32_t sweep_chunk() {
    if (const char *env = std::getenv("LS_SWEEP_CHUNK")) {
        const int v = std::atoi(env);
        if (v >= 1) return v;
    }
    return kSweepChunk;
}

hipError_t run_chunks(int prec, int dir, const SweepPtrs &p, const SweepArgs &a, Shape sh,
                      hipStream_t st) {
    SweepArgs c = a;
    int32_t l0 = a.l0;
    int next = 0;  // next target, in travel order
    const int32_t chunk = sweep_chunk();
    for (;;) {
        int32_t tc;
        if (dir == 0) {
            const int32_t from = l0 < 0 ? 0 : l0;
            tc = std::min(a.t, from + chunk);
        } else {
            const int32_t top = l0 < 0 ? a.L - 1 : l0;
            tc = std::max(a.t, top - chunk);
        }
        int n = 0;
        while (next + n < a.nt &&
               (dir == 0 ? a.tgt_l[next + n] <= tc : a.tgt_l[next + n] >= tc)) {
            c.tgt_l[n] = a.tgt_l[next + n];
            c.tgt_out[n] = a.tgt_out[next + n];
            ++n;
        }
        next += n;
        c.nt = n;
        c.l0 = l0;
        c.t = tc;
        const hipError_t e = launch_sweep(prec, dir, p, c, sh, st);
        if (e != hipSuccess || tc == a.t) return e;
        l0 = tc;
    }
}

// A whole sweep over recipients [0, a.R), in chunks. (Splitting the
// recipients over two streams, staggered or not, so that one half fills the
// other's partly filled last round of workgroups, measured slower: the
// concurrent launches cost more than the tail they fill.)
hipError_t launch_sweep_chunked(int prec, int dir, const SweepPtrs &p, const SweepArgs &a,
                                Shape sh, hipStream_t st) {
    SweepArgs b = a;
    b.r0 = 0;
    b.nblk = a.R;
    return run_chunks(prec, dir, p, b, sh, st);
}

ls_status check_table(const ls_table *t, const ls_model *m, int dir) {
    if (!t || !t->state || !t->log_scale || !t->status || !t->recipients || t->R < 1)
        return LS_ERR_ARG;
    if (!valid_prec(t->prec)) return LS_ERR_ARG;
    if (t->direction != dir) return LS_ERR_STATE;
    if (t->model_hash != 0 && t->model_hash != m->hash) return LS_ERR_STATE;
    if (t->l < -1 || t->l >= m->L) return LS_ERR_STATE;
    return LS_OK;
}

}  // namespace

// hipGetLastError() reports the last error of any HIP runtime call made on
// the calling thread, including calls by other libraries that handled their
// own failure (a framework probing devices, for instance). Every entry point
// that launches clears it first, so the check after its own launches sees
// only those launches.
static inline void clear_stale_hip_error() { (void)hipGetLastError(); }

extern "C" {

size_t ls_model_workspace_bytes(int32_t N, int32_t L) {
    if (N < 2 || L < 1) return 0;
    return prior_stats_offset_bytes(N, L) + (size_t)N * 2 * sizeof(double);
}

ls_status ls_model_init(ls_model *m, void *workspace, size_t ws_bytes, void *stream) {
    clear_stale_hip_error();
    if (!m || !m->H || m->N < 2 || m->L < 1) return LS_ERR_ARG;
    if (m->stride_words < (m->N + 31) / 32 || (m->stride_words & 1)) return LS_ERR_ARG;
    if (!(m->mu >= 0.0 && m->mu <= 1.0)) return LS_ERR_ARG;
    if (m->L > 1 && !m->rho) return LS_ERR_ARG;
    const size_t need = ls_model_workspace_bytes(m->N, m->L);
    if (!workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return LS_ERR_WORKSPACE;
    hipStream_t st = as_stream(stream);
    std::vector<double> rho((size_t)std::max(m->L - 1, 0));
    if (!rho.empty()) {
        hipError_t e = hipMemcpyAsync(rho.data(), m->rho, rho.size() * sizeof(double),
                                      hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return LS_ERR_DEVICE;
        for (double r : rho)
            if (!(r >= 0.0 && r <= 1.0)) return LS_ERR_ARG;
    }
    std::vector<double> muv(m->mu_vec ? (size_t)m->L : 0);
    if (!muv.empty()) {
        hipError_t e = hipMemcpyAsync(muv.data(), m->mu_vec, muv.size() * sizeof(double),
                                      hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return LS_ERR_DEVICE;
        for (double x : muv)
            if (!(x >= 0.0 && x <= 1.0)) return LS_ERR_ARG;
    }
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(h, &m->N, sizeof m->N);
    h = fnv1a(h, &m->L, sizeof m->L);
    h = fnv1a(h, &m->mu, sizeof m->mu);
    if (!rho.empty()) h = fnv1a(h, rho.data(), rho.size() * sizeof(double));
    if (!muv.empty()) h = fnv1a(h, muv.data(), muv.size() * sizeof(double));
    if (m->prior) {
        // every column in [0, 1] and summing to 1 off the diagonal; the
        // per-column sums and hashes of the full contents go into the hash
        double *stats = reinterpret_cast<double *>(static_cast<char *>(workspace) +
                                                   prior_stats_offset_bytes(m->N, m->L));
        std::vector<double> hs((size_t)m->N * 2);
        hipError_t e = lsk::launch_prior_stats(m->prior, m->N, stats, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hs.data(), stats, hs.size() * sizeof(double), hipMemcpyDeviceToHost,
                               st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return LS_ERR_DEVICE;
        for (int32_t c = 0; c < m->N; ++c)
            if (!(std::fabs(hs[2 * (size_t)c] - 1.0) <= 1e-9)) return LS_ERR_ARG;
        h = fnv1a(h, hs.data(), hs.size() * sizeof(double));
    }
    if (h == 0) h = 1;
    const int64_t hs = hr_stride_for(m->N);
    uint64_t *Hr = static_cast<uint64_t *>(workspace);
    hipError_t e = lsk::launch_repack(m->H, m->stride_words, m->N, m->L, Hr, hs, st);
    if (e != hipSuccess) return LS_ERR_DEVICE;
    // forward tables: kappa and kappa / (N-1), times the emission divisor
    // (fill_scalars' forward cnum and bmul, with the divisor applied last,
    // so that a constant per-variant mu gives the scalar model's table)
    lsk::CoefScalars cs;
    cs.unit = lsk::sweep_emissions(m->mu).unit;
    for (int k = 0; k < lsk::kCoefTables; ++k) {
        const int dir = k & 1;
        SweepArgs sa;
        fill_scalars(sa, m, (k == 2 || k == 3) ? LS_FP32_F16STORE : LS_FP32, dir);
        cs.cnum[k] = dir ? sa.cnum : sa.kappa;
        cs.bmul[k] = dir ? sa.bmul : sa.kappa / (double)(m->N - 1);
        cs.fold[k] = dir == 0 && k != lsk::kCoefF32FwdGrad;
    }
    float *coef = reinterpret_cast<float *>(static_cast<char *>(workspace) +
                                            coef_offset_bytes(m->N, m->L));
    e = lsk::launch_coef_tables(m->L > 1 ? m->rho : nullptr, m->mu_vec, m->L, cs, coef, st);
    if (e != hipSuccess) return LS_ERR_DEVICE;
    if (m->mu_vec) {
        char *eb = static_cast<char *>(workspace) + emis_offset_bytes(m->N, m->L);
        const size_t L = (size_t)m->L;
        e = lsk::launch_emission_tables(
            m->mu_vec, m->L, reinterpret_cast<double *>(eb),
            reinterpret_cast<float *>(eb + 2 * L * sizeof(double)),
            reinterpret_cast<double *>(eb + 2 * L * (sizeof(double) + sizeof(float))), st);
        if (e != hipSuccess) return LS_ERR_DEVICE;
    }
    m->hash = h;
    m->Hr = Hr;
    m->hr_stride = hs;
    m->nf = m->N / 64;
    m->reserved = 0;
    return LS_OK;
}

ls_status ls_table_init(ls_table *t, int32_t direction, ls_precision prec, void *state,
                        double *log_scale, uint32_t *status, const int32_t *recipients,
                        int32_t R, void *stream) {
    clear_stale_hip_error();
    if (!t || (direction != 0 && direction != 1) || !valid_prec(prec) || !state || !log_scale ||
        !status || !recipients || R < 1)
        return LS_ERR_ARG;
    t->state = state;
    t->log_scale = log_scale;
    t->status = status;
    t->recipients = recipients;
    t->R = R;
    t->l = -1;
    t->direction = direction;
    t->prec = prec;
    t->model_hash = 0;
    return dev(lsk::launch_fill_u32(status, 0u, R, as_stream(stream)));
}

ls_status ls_table_copy(ls_table *dst, const ls_table *src, int32_t N, void *stream) {
    clear_stale_hip_error();
    if (!dst || !src || N < 2 || !dst->state || !src->state || !dst->log_scale ||
        !src->log_scale || !dst->status || !src->status)
        return LS_ERR_ARG;
    if (dst->direction != src->direction || dst->prec != src->prec || dst->R != src->R)
        return LS_ERR_SHAPE;
    hipStream_t st = as_stream(stream);
    const size_t R = (size_t)src->R;
    hipError_t e = hipMemcpyAsync(dst->state, src->state, R * (size_t)N * state_elem(src->prec),
                                  hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dst->log_scale, src->log_scale, R * sizeof(double),
                           hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dst->status, src->status, R * sizeof(uint32_t),
                           hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return LS_ERR_DEVICE;
    dst->recipients = src->recipients;
    dst->l = src->l;
    dst->model_hash = src->model_hash;
    return LS_OK;
}

namespace {

// ls_forward; with `fold` false (FP32 and FP64 only) the sweep keeps the
// divided emission pairs' scale, as the gradient's forward does, so that a
// log-likelihood has the same bits with and without the gradient.
ls_status forward_impl(ls_table *fwd, const ls_model *m, int32_t t, const int32_t *targets,
                       int32_t T, const void *bsnap, void *P, void *E, int64_t out_target_stride,
                       int64_t out_row_stride, void *stream, bool fold) {
    clear_stale_hip_error();
    ls_status s = check_model(m);
    if (s != LS_OK) return s;
    if ((s = check_table(fwd, m, 0)) != LS_OK) return s;
    if (t < 0 || t >= m->L || T < 0 || T > LS_MAX_TARGETS) return LS_ERR_ARG;
    // output layout: row (k, r) of P and E starts at k ts + r rs elements
    const int64_t rs = out_row_stride ? out_row_stride : (int64_t)m->N;
    const int64_t ts = out_target_stride ? out_target_stride : (int64_t)fwd->R * rs;
    if (rs < m->N || (T > 1 && ts < (int64_t)(fwd->R - 1) * rs + m->N) || ts < 0)
        return LS_ERR_SHAPE;
    if (fwd->l >= 0 && t < fwd->l) return LS_ERR_STATE;
    if (T > 0 && !targets) return LS_ERR_ARG;
    const bool want_out = T > 0 && (P || E);
    if (want_out && !bsnap) return LS_ERR_ARG;
    for (int k = 0; k < T; ++k) {
        if (targets[k] <= fwd->l || targets[k] > t) return LS_ERR_ARG;
        if (k > 0 && targets[k] <= targets[k - 1]) return LS_ERR_ARG;
    }
    if (fwd->l == t) return T == 0 ? LS_OK : LS_ERR_ARG;
    Shape sh;
    if (!choose_shape(m->N, fwd->prec, &sh, false, m->prior != nullptr)) return LS_ERR_UNSUPPORTED;
    SweepArgs a;
    std::memset(&a, 0, sizeof a);
    if (fwd->prec == LS_FP32_F16STORE) fold = true;
    fill_scalars(a, m, fwd->prec, 0, fold);
    a.R = fwd->R;
    a.dir = 0;
    a.l0 = fwd->l;
    a.t = t;
    a.nt = want_out ? T : 0;
    a.snap_ts = ts;
    a.snap_rs = rs;
    for (int k = 0; k < a.nt; ++k) {
        a.tgt_l[k] = targets[k];
        a.tgt_out[k] = k;
    }
    // forward vectors at the targets are staged in E (else P) and turned into
    // posteriors / half distances in place afterwards
    void *stage = E ? E : P;
    SweepPtrs p;
    p.Hr = m->Hr;
    p.rho = m->L > 1 ? m->rho : reinterpret_cast<const double *>(m->Hr);  // only a discarded load when L == 1
    emission_tables(m, fwd->prec, p);
    if (fold) {
        p.coef = coef_table(m, fwd->prec, 0);
        p.lu_prefix = nullptr;  // the divisors are in the forward coefficient table
    } else {
        p.coef = grad_forward_coefs(m, fwd->prec);
    }
    p.prior = m->prior;
    p.recipients = fwd->recipients;
    p.state = fwd->state;
    p.log_scale = fwd->log_scale;
    p.status = fwd->status;
    p.snap = want_out ? stage : fwd->state;
    hipStream_t st = as_stream(stream);
    hipError_t e = launch_sweep_chunked(fwd->prec, 0, p, a, sh, st);
    if (e != hipSuccess) return LS_ERR_DEVICE;
    if (want_out) {
        e = lsk::launch_posterior_rows(stage, 0, bsnap, 0, fwd->recipients, fwd->R, T, ts, rs,
                                       m->N, fwd->prec == LS_FP64, P, E, st);
        if (e != hipSuccess) return LS_ERR_DEVICE;
    }
    fwd->l = t;
    fwd->model_hash = m->hash;
    return LS_OK;
}

}  // namespace

ls_status ls_forward(ls_table *fwd, const ls_model *m, int32_t t, const int32_t *targets,
                     int32_t T, const void *bsnap, void *P, void *E, int64_t out_target_stride,
                     int64_t out_row_stride, void *stream) {
    return forward_impl(fwd, m, t, targets, T, bsnap, P, E, out_target_stride, out_row_stride,
                        stream, true);
}

ls_status ls_backward(ls_table *bck, const ls_model *m, int32_t t, const int32_t *targets,
                      int32_t T, void *bsnap, void *stream) {
    clear_stale_hip_error();
    ls_status s = check_model(m);
    if (s != LS_OK) return s;
    if ((s = check_table(bck, m, 1)) != LS_OK) return s;
    if (t < 0 || t >= m->L || T < 0 || T > LS_MAX_TARGETS) return LS_ERR_ARG;
    if (T > 0 && (!targets || !bsnap)) return LS_ERR_ARG;
    const int32_t top = bck->l >= 0 ? bck->l : m->L - 1;
    if (t > top) return LS_ERR_STATE;
    for (int k = 0; k < T; ++k) {
        if (targets[k] < t) return LS_ERR_ARG;
        if (bck->l >= 0 ? targets[k] >= bck->l : targets[k] > m->L - 1) return LS_ERR_ARG;
        if (k > 0 && targets[k] <= targets[k - 1]) return LS_ERR_ARG;
    }
    if (bck->l == t) return T == 0 ? LS_OK : LS_ERR_ARG;
    Shape sh;
    if (!choose_shape(m->N, bck->prec, &sh, false, m->prior != nullptr)) return LS_ERR_UNSUPPORTED;
    SweepArgs a;
    std::memset(&a, 0, sizeof a);
    fill_scalars(a, m, bck->prec, 1);
    a.R = bck->R;
    a.dir = 1;
    a.l0 = bck->l;
    a.t = t;
    a.nt = T;
    a.snap_ts = (int64_t)bck->R * m->N;
    a.snap_rs = m->N;
    for (int k = 0; k < T; ++k) {  // travel order: descending
        a.tgt_l[k] = targets[T - 1 - k];
        a.tgt_out[k] = T - 1 - k;
    }
    SweepPtrs p;
    p.Hr = m->Hr;
    p.rho = m->L > 1 ? m->rho : reinterpret_cast<const double *>(m->Hr);  // only a discarded load when L == 1
    p.coef = coef_table(m, bck->prec, 1);
    emission_tables(m, bck->prec, p);
    p.prior = m->prior;
    p.recipients = bck->recipients;
    p.state = bck->state;
    p.log_scale = bck->log_scale;
    p.status = bck->status;
    p.snap = T > 0 ? bsnap : bck->state;
    hipError_t e = launch_sweep_chunked(bck->prec, 1, p, a, sh, as_stream(stream));
    if (e != hipSuccess) return LS_ERR_DEVICE;
    bck->l = t;
    bck->model_hash = m->hash;
    return LS_OK;
}

ls_status ls_posterior_distance(const ls_table *fwd, const ls_table *bck, const ls_model *m,
                                void *P, void *E, void *stream) {
    clear_stale_hip_error();
    ls_status s = check_model(m);
    if (s != LS_OK) return s;
    if ((s = check_table(fwd, m, 0)) != LS_OK) return s;
    if ((s = check_table(bck, m, 1)) != LS_OK) return s;
    // (the recipient lists themselves are device memory; the caller
    // guarantees both tables hold the same recipients in the same order)
    if (fwd->l < 0 || fwd->l != bck->l || fwd->R != bck->R || fwd->prec != bck->prec ||
        fwd->model_hash != m->hash || bck->model_hash != m->hash)
        return LS_ERR_STATE;
    if (!P && !E) return LS_OK;
    const int half = fwd->prec == LS_FP32_F16STORE;
    return dev(lsk::launch_posterior_rows(fwd->state, half, bck->state, half, fwd->recipients,
                                          fwd->R, 1, 0, m->N, m->N, fwd->prec == LS_FP64, P, E,
                                          as_stream(stream)));
}

ls_status ls_distance_symmetrise(const void *E, void *D, int32_t N, int32_t T,
                                 ls_precision prec, void *stream) {
    clear_stale_hip_error();
    if (!E || !D || N < 1 || T < 0 || !valid_prec(prec)) return LS_ERR_ARG;
    return dev(lsk::launch_symmetrise(E, D, N, T, prec == LS_FP64, as_stream(stream)));
}

size_t ls_average_linkage_workspace_bytes(int32_t N, int32_t T, ls_precision prec) {
    if (N < 1 || T < 1 || !valid_prec(prec)) return 0;
    return lsk::linkage_workspace_bytes(N, T, prec == LS_FP64);
}

ls_status ls_average_linkage(void *D, int32_t N, int32_t T, ls_precision prec, double *Z,
                             int32_t *order, void *workspace, size_t ws_bytes, void *stream) {
    clear_stale_hip_error();
    if (!D || N < 1 || T < 1 || !valid_prec(prec) || (N > 1 && !Z)) return LS_ERR_ARG;
    if (T > 0x7fffffff / 1024) return LS_ERR_ARG;
    const size_t need = lsk::linkage_workspace_bytes(N, T, prec == LS_FP64);
    if (!workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return LS_ERR_WORKSPACE;
    return dev(lsk::launch_linkage(D, N, T, prec == LS_FP64, Z, order, workspace,
                                   as_stream(stream)));
}

ls_status ls_average_linkage_noalloc(void *D, int32_t N, int32_t T, ls_precision prec, double *Z,
                                     int32_t *order, void *stream) {
    clear_stale_hip_error();
    if (!D || N < 1 || T < 1 || !valid_prec(prec) || (N > 1 && !Z)) return LS_ERR_ARG;
    if (T > 0x7fffffff / 1024) return LS_ERR_ARG;
    if (lsk::linkage_workspace_bytes(N, T, prec == LS_FP64) > lsk::kLinkageScratchBytes)
        return LS_ERR_SCRATCH;
    void *ws = nullptr;
    if (lsk::linkage_scratch(&ws) != hipSuccess) return LS_ERR_DEVICE;
    return dev(lsk::launch_linkage(D, N, T, prec == LS_FP64, Z, order, ws, as_stream(stream)));
}

ls_status ls_standardise_rows(void *E, const int32_t *recipients, int32_t R, int32_t T,
                              int32_t N, int64_t out_target_stride, int64_t out_row_stride,
                              ls_precision prec, void *stream) {
    clear_stale_hip_error();
    if (!E || !recipients || R < 1 || T < 1 || T > LS_MAX_TARGETS || N < 2 || !valid_prec(prec))
        return LS_ERR_ARG;
    const int64_t rs = out_row_stride ? out_row_stride : (int64_t)N;
    const int64_t ts = out_target_stride ? out_target_stride : (int64_t)R * rs;
    if (rs < N || (T > 1 && ts < (int64_t)(R - 1) * rs + N) || ts < 0) return LS_ERR_SHAPE;
    return dev(lsk::launch_standardise(E, recipients, R, T, N, ts, rs, prec == LS_FP64,
                                       as_stream(stream)));
}

ls_status ls_calc_rho(const double *cM, int32_t n, double s, double gamma, double *rho,
                      void *stream) {
    clear_stale_hip_error();
    if (n < 0 || (n > 0 && (!cM || !rho)) || !std::isfinite(s) || !std::isfinite(gamma) ||
        s < 0.0 || gamma <= 0.0)
        return LS_ERR_ARG;
    return dev(lsk::launch_calc_rho(cM, n, s, gamma, rho, as_stream(stream)));
}

ls_status ls_rho_map_grad(const double *cM, int32_t n, double s, double gamma,
                          const double *grad_rho, double *grad_s_gamma, void *stream) {
    clear_stale_hip_error();
    if (n < 0 || (n > 0 && (!cM || !grad_rho)) || !grad_s_gamma || !std::isfinite(s) ||
        !std::isfinite(gamma) || s < 0.0 || gamma <= 0.0)
        return LS_ERR_ARG;
    return dev(lsk::launch_rho_map_grad(cM, n, s, gamma, grad_rho, grad_s_gamma,
                                        as_stream(stream)));
}

size_t ls_loglik_grad_workspace_bytes(const ls_model *m, int32_t R, ls_precision prec) {
    if (check_model(m) != LS_OK || R < 1 || !valid_prec(prec)) return 0;
    return lsk::grad_workspace_bytes(m->N, m->L, R, (int)prec, m->mu_vec != nullptr, nullptr);
}

}  // extern "C"

namespace {

// The log-likelihood and gradient entry points share their checks and set-up;
// `phase` picks the passes (lsk::GradPhase), 0 = the log-likelihood alone.
ls_status loglik_grad_impl(const ls_model *m, const int32_t *recipients, int32_t R,
                           ls_precision prec, double *loglik, double *pac, double *grad_rho,
                           double *grad_mu, void *workspace, size_t ws_bytes, void *stream,
                           int phase) {
    clear_stale_hip_error();
    ls_status s = check_model(m);
    if (s != LS_OK) return s;
    if (R < 1 || !valid_prec(prec)) return LS_ERR_ARG;
    if (!recipients && R != m->N) return LS_ERR_ARG;
    if (phase != lsk::kGradAdjoint && !pac) return LS_ERR_ARG;
    const bool grad = phase & lsk::kGradAdjoint;
    if (grad && (!grad_mu || (m->L > 1 && !grad_rho))) return LS_ERR_ARG;
    const bool muv = m->mu_vec != nullptr;
    const size_t need = lsk::grad_workspace_bytes(m->N, m->L, R, (int)prec, muv, nullptr);
    if (!workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return LS_ERR_WORKSPACE;
    if (phase != 0 && prec != LS_FP32 && prec != LS_FP64) return LS_ERR_UNSUPPORTED;
    Shape sh;
    if (!choose_shape(m->N, prec, &sh, phase != 0, m->prior != nullptr)) return LS_ERR_UNSUPPORTED;
    lsk::GradLayout lay;
    lsk::grad_workspace_bytes(m->N, m->L, R, (int)prec, muv, &lay);
    char *ws = static_cast<char *>(workspace);
    hipStream_t st = as_stream(stream);
    const int32_t *rec = recipients;
    if (!rec) {
        int32_t *iota = reinterpret_cast<int32_t *>(ws + lay.off_recips);
        hipError_t e = lsk::launch_iota(iota, R, st);
        if (e != hipSuccess) return LS_ERR_DEVICE;
        rec = iota;
    }
    if (phase == 0) {
        // forward sweep of every recipient to the last variant: log F^{L-1}
        ls_table tab;
        s = ls_table_init(&tab, 0, prec, ws + lay.off_state,
                          reinterpret_cast<double *>(ws + lay.off_ll),
                          reinterpret_cast<uint32_t *>(ws + lay.off_status), rec, R, stream);
        if (s != LS_OK) return s;
        s = forward_impl(&tab, m, m->L - 1, nullptr, 0, nullptr, nullptr, nullptr, 0, 0, stream,
                         false);
        if (s != LS_OK) return s;
        return dev(lsk::launch_loglik_sum(reinterpret_cast<const double *>(ws + lay.off_ll), R,
                                          loglik, pac, st));
    }
    lsk::GradArgs ga;
    std::memset(&ga, 0, sizeof ga);
    ga.Hr = m->Hr;
    ga.rho = m->L > 1 ? m->rho : reinterpret_cast<const double *>(m->Hr);
    ga.coef_fwd32 = grad_forward_coefs(m, LS_FP32);
    ga.coef_bwd32 = coef_table(m, LS_FP32, 1);
    ga.recipients = rec;
    ga.hr_stride = m->hr_stride;
    ga.N = m->N;
    ga.L = m->L;
    ga.NF = m->N / 64;
    ga.R = R;
    ga.seg = lay.seg;
    ga.nseg = lay.nseg;
    ga.mu = m->mu;
    {
        SweepPtrs ep;
        emission_tables(m, prec, ep);
        ga.emis = ep.emis;
        ga.lu_prefix = ep.lu_prefix;
        SweepPtrs e64;
        emission_tables(m, LS_FP64, e64);
        ga.em64 = static_cast<const double *>(e64.emis);
    }
    ga.chunk = sweep_chunk();
    if (!choose_shape(m->N, prec, &ga.fwd_shape, false, m->prior != nullptr))
        return LS_ERR_UNSUPPORTED;
    ga.prior = m->prior;
    ga.ws = ws;
    ga.lay = lay;
    return dev(lsk::launch_grad(ga, (int)prec, sh, loglik, pac, grad_rho, grad_mu, st,
                                static_cast<lsk::GradPhase>(phase)));
}

}  // namespace

extern "C" {

ls_status ls_loglik_grad(const ls_model *m, const int32_t *recipients, int32_t R,
                         ls_precision prec, double *loglik, double *pac, double *grad_rho,
                         double *grad_mu, void *workspace, size_t ws_bytes, void *stream) {
    const bool grad = grad_rho || grad_mu;
    return loglik_grad_impl(m, recipients, R, prec, loglik, pac, grad_rho, grad_mu, workspace,
                            ws_bytes, stream, grad ? lsk::kGradBoth : 0);
}

ls_status ls_loglik_checkpoint(const ls_model *m, const int32_t *recipients, int32_t R,
                               ls_precision prec, double *loglik, double *pac, void *workspace,
                               size_t ws_bytes, void *stream) {
    return loglik_grad_impl(m, recipients, R, prec, loglik, pac, nullptr, nullptr, workspace,
                            ws_bytes, stream, lsk::kGradForward);
}

ls_status ls_loglik_grad_adjoint(const ls_model *m, const int32_t *recipients, int32_t R,
                                 ls_precision prec, double *grad_rho, double *grad_mu,
                                 void *workspace, size_t ws_bytes, void *stream) {
    return loglik_grad_impl(m, recipients, R, prec, nullptr, nullptr, grad_rho, grad_mu,
                            workspace, ws_bytes, stream, lsk::kGradAdjoint);
}

ls_status ls_status_check(const uint32_t *status, int32_t R, void *stream) {
    clear_stale_hip_error();
    if (!status || R < 1) return LS_ERR_ARG;
    std::vector<uint32_t> h((size_t)R);
    hipStream_t st = as_stream(stream);
    hipError_t e = hipMemcpyAsync(h.data(), status, h.size() * sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return LS_ERR_DEVICE;
    uint32_t any = 0;
    for (uint32_t v : h) any |= v;
    if (any & LS_FLAG_BAD_RECIPIENT) return LS_ERR_ARG;
    if (any & LS_FLAG_NONFINITE) return LS_WARN_NONFINITE;
    return LS_OK;
}

ls_status ls_kernel_shape(int32_t N, ls_precision prec, int32_t with_prior,
                          int32_t *slots_per_wave, int32_t *waves_per_recipient) {
    if (N < 2 || !valid_prec(prec)) return LS_ERR_ARG;
    Shape sh;
    if (!choose_shape(N, prec, &sh, false, with_prior != 0)) return LS_ERR_UNSUPPORTED;
    if (slots_per_wave) *slots_per_wave = sh.nslot;
    if (waves_per_recipient) *waves_per_recipient = sh.nwaves;
    return LS_OK;
}

const char *ls_status_string(ls_status s) {
    switch (s) {
    case LS_OK: return "ok";
    case LS_ERR_ARG: return "invalid argument";
    case LS_ERR_SHAPE: return "inconsistent sizes";
    case LS_ERR_STATE: return "table in the wrong state for this call";
    case LS_ERR_UNSUPPORTED: return "N too large for this precision on one GPU, or not offered in it";
    case LS_ERR_DEVICE: return "HIP runtime error";
    case LS_ERR_WORKSPACE: return "workspace missing or too small";
    case LS_ERR_SCRATCH: return "request larger than the fixed scratch of an allocation-free call";
    case LS_WARN_NONFINITE: return "a column sum was zero or non-finite";
    }
    return "unknown status";
}

const char *ls_version(void) { return "libls 0.1 (gfx950)"; }

}  // extern "C"
