// Internal definitions shared by the host C-ABI layer and the kernel
// translation units. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <cmath>

namespace lsk {

constexpr int kWave = 64;
constexpr int kMaxWaves = 16;   // waves per recipient (1024-thread workgroup)
constexpr int kMaxTargets = 256;
constexpr uint32_t kFlagNonfinite = 1u;     // LS_FLAG_NONFINITE
constexpr uint32_t kFlagBadRecipient = 2u;  // LS_FLAG_BAD_RECIPIENT

// Arguments of one sweep launch (forward or backward) over R recipients.
// The pointers travel as separate __restrict__ kernel parameters (so the
// compiler may read the haplotype rows with scalar loads); everything else is
// passed by value in this block.
struct SweepPtrs {
    const uint64_t *Hr;         // [L][hr_stride] internal rows (see ls_model_init)
    const void *emis;           // per-variant mu: [L][2] emission pairs in the sweep's
                                // arithmetic type, else null (scalar mu)
    const double *lu_prefix;    // per-variant mu, FP32 arithmetic: [L+1] log-unit prefix
    const double *prior;        // prior copying matrix, [N][N] (row i: the prior
                                // column of recipient i), or null (uniform)
    const double *rho;          // [L-1]
    const float *coef;          // [L][2] coefficient table of the precision and
                                // direction (FP32 arithmetic), else null
    const int32_t *recipients;  // [R]
    void *state;                // table state [R][N]
    double *log_scale;          // [R]
    uint32_t *status;           // [R]
    void *snap;                 // [T][R][N] vectors written at the targets
};
struct SweepArgs {
    int64_t hr_stride;    // 64-bit words per internal row
    int32_t N, L, NF, R;  // NF = floor(N/64) full words
    int32_t dir;          // 0 forward, 1 backward
    int32_t l0;           // current variant of the table (-1: not propagated)
    int32_t t;            // variant to stop at
    int32_t nt;           // number of targets visited, in travel order
    int32_t r0, nblk;     // this launch: recipients [r0, r0 + nblk) of the R
    double th_match;      // emission where the donor carries the recipient's allele
    double th_mis;        // and where it does not (see sweep_emissions)
    double kappa;         // storage scale of the resident vector
    double inv_kappa;
    double cnum;          // forward: kappa; backward: kappa * (N-1)
    double bmul;          // forward: kappa / (N-1); backward: kappa
    double log_off;       // per-step log offset: fwd -log(kappa), bwd -log((N-1) kappa)
                          // plus the emission unit's log (see sweep_emissions)
    int64_t c_off;        // keep-alpha mode (gradient recompute): element offset, from
                          // the snapshot array, of the [t - l0][R] c of each step
    int64_t snap_ts;      // elements between the snapshot rows of consecutive targets
    int64_t snap_rs;      // elements between the snapshot rows of consecutive recipients
    int32_t tgt_l[kMaxTargets];    // variant of each visited target, travel order
    int32_t tgt_out[kMaxTargets];  // its index k in the [T] output arrays
};

// The emission pair a sweep multiplies by, from the form (1-H)(1-2mu)+mu of
// appendix A.3 evaluated in FP64, divided by its larger member `unit` (the
// match value 1-mu for every mu <= 1/2): that member is then exactly 1, so
// the emission is a multiply of the other donors only (masked_scale_all) and
// adds no rounding to most cells; in FP32 the rounded 1-mu would also bias
// every step's sum the same way (a log-likelihood error growing with L).
// Dividing every step's emissions by one constant only rescales the
// vectors. The backward adds its log (`log_unit`) to the per-step log offset
// in FP64; the forward multiplies it back into the step's coefficients c
// and b instead, so that its vector is alpha^l itself (see fill_scalars).
struct Emissions {
    double match, mis, log_unit, unit;
};
inline Emissions sweep_emissions(double mu) {
    const double omu = (1.0 - 2.0 * mu) + mu;
    if (omu >= mu) return Emissions{1.0, mu / omu, std::log(omu), omu};
    return Emissions{omu / mu, 1.0, std::log(mu), mu};
}

// Kernel shape: 64-donor register slots per wave, waves per recipient.
struct Shape {
    int nslot;
    int nwaves;
};

// Largest workgroup (in waves) a kernel with `nslot` slots may be launched
// with: the register file of one SIMD (512 VGPRs per lane) must hold every
// wave the workgroup places on it. The constant covers the per-wave registers
// besides the resident vector (emission pair, accumulators, special-slot
// multipliers, the division and reduction temporaries). With one register per
// slot it is the allowance the compile budget gives (sweep_waves_per_simd),
// which the widest kernels keep within (about 23 registers beside the slots
// at 128..144 slots), so that 128 and 132 slots run 12-wave groups at three
// waves per SIMD. FP64 sweeps without a prior column use about 33 beside
// their two registers per slot (223..225 VGPRs at 96 slots); above 96 slots
// they are allowed 48, which lets 100 and 104 slots run 8-wave groups at two
// waves per SIMD (N up to 53,248 in FP64). Below that, and with a prior
// column, the allowance stays 64.
__host__ __device__ constexpr int max_waves_for(int nslot, int vgpr_per_slot, bool prior = false) {
    const int allow = vgpr_per_slot == 1 ? 36 : (vgpr_per_slot == 2 && !prior && nslot > 96 ? 48 : 64);
    int need = nslot * vgpr_per_slot + allow;
    need = (need + 7) / 8 * 8;
    int per_simd = 512 / need;
    if (per_simd > 8) per_simd = 8;
    int w = 4 * per_simd;
    return w > kMaxWaves ? kMaxWaves : (w < 1 ? 1 : w);
}

// Registers per slot of the sweep: the donor column and, with a prior
// matrix, the prior column beside it.
__host__ __device__ constexpr int sweep_slot_vgprs(int vgpr_per_slot, bool prior) {
    return prior ? 2 * vgpr_per_slot : vgpr_per_slot;
}

// Largest group of the adjoint kernel that reads alpha ahead: per wave it
// holds y, the alpha of the current pair of variants and of the next, and
// the temporaries of two steps; 7 registers per slot plus 28 (FP32), 14.5
// per slot plus 40 (FP64), fitted to the compiler's allocations, so that
// the occupancy the shape choice assumes is the one the kernel gets. A
// prior matrix adds its column (one more value per slot).
__host__ __device__ constexpr int grad_waves_per_simd(int nslot, int vgpr_per_slot,
                                                      bool prior = false) {
    int need = vgpr_per_slot == 2 ? (29 * nslot + 80) / 2 : 7 * nslot + 28;
    if (prior) need += nslot * vgpr_per_slot;
    need = (need + 7) / 8 * 8;
    int per_simd = 512 / need;  // 0: one wave does not fit, no narrow kernel
    return per_simd > 8 ? 8 : per_simd;
}
__host__ __device__ constexpr int grad_max_waves(int nslot, int vgpr_per_slot, bool prior = false) {
    int w = 4 * grad_waves_per_simd(nslot, vgpr_per_slot, prior);
    return w > kMaxWaves ? kMaxWaves : w;
}

// Waves per SIMD the sweep kernel is compiled for (amdgpu_waves_per_eu): the
// register file of one SIMD (512 VGPRs per lane) over the resident vector
// plus a per-wave allowance. Holding the compiler to it keeps the common
// 40-slot FP32 kernel at 7 resident waves instead of 6 (its scheduler
// otherwise spends registers on longer live ranges) and measured 6-10%
// faster per sweep.
__host__ __device__ constexpr int sweep_waves_per_simd(int nslot, int vgpr_per_slot) {
    int need = nslot * vgpr_per_slot + (vgpr_per_slot >= 2 ? 64 : 36);
    need = (need + 7) / 8 * 8;
    int w = 512 / need;
    return w > 8 ? 8 : (w < 1 ? 1 : w);
}

// Slot count whose sweep_waves_per_simd budget the sweep kernel is compiled
// for. The keep-alpha mode (the gradient's recompute) holds more
// registers: in FP32 about two per slot (measured).
__host__ __device__ constexpr int sweep_budget_slots(int nslot, int vgpr_per_slot, bool every) {
    if (!every) return nslot;
    if (vgpr_per_slot == 1 && 2 * nslot - 12 > nslot + 16) return 2 * nslot - 12;
    return nslot + 16;
}

// Slot counts instantiated per precision. Every shape the host picks uses
// one of these; the menu is dense enough that some number of waves fits
// every N up to the register budget of one compute unit.
#define LS_MENU_F32(X) \
    X(1) X(2) X(3) X(4) X(8) X(12) X(16) X(20) X(24) X(28) X(32) X(40) X(48) X(56) X(64) \
    X(72) X(80) X(88) X(96) X(104) X(112) X(120) X(128) X(132) X(136) X(144) X(152) X(160) X(164) \
    X(168) X(172) X(176) X(180) X(184) X(188) X(192) X(196) X(200)
#define LS_MENU_F64(X) \
    X(1) X(2) X(3) X(4) X(8) X(12) X(16) X(20) X(24) X(28) X(32) X(40) X(48) X(56) X(64) \
    X(68) X(72) X(76) X(80) X(84) X(88) X(92) X(96) X(100) X(104)

// Slot counts of the gradient kernel (two precisions).
#define LS_MENU_GRAD(X) \
    X(1) X(2) X(3) X(4) X(8) X(12) X(16) X(20) X(24) X(28) X(32) X(40) X(48) X(56) X(64) \
    X(72) X(80) X(88) X(96)

// Launchers, one per precision and direction (ls_sweep_<prec>_<dir>.hip).
// Return hipSuccess, hipErrorInvalidValue for a slot count that is not in
// the menu, or the launch error.
#define LS_DECLARE_LAUNCH(P, D)                                                          \
    hipError_t launch_sweep_##P##_##D(const SweepPtrs &p, const SweepArgs &a, Shape shape, \
                                      hipStream_t st);
LS_DECLARE_LAUNCH(f64, fwd)
LS_DECLARE_LAUNCH(f64, bwd)
LS_DECLARE_LAUNCH(f32, fwd)
LS_DECLARE_LAUNCH(f32, bwd)
LS_DECLARE_LAUNCH(f16, fwd)
LS_DECLARE_LAUNCH(f16, bwd)
#undef LS_DECLARE_LAUNCH
// Special (boundary) slots per wave for a given slot count.
__host__ __device__ constexpr int special_slots(int nslot) { return nslot < 4 ? nslot : 4; }

// Per-variant coefficients of the FP32 sweeps, kept in the model workspace
// after the internal rows: kCoefTables tables of L pairs (A_l, B_l), with
// c = A_l / S and b = B_l in the sweep's update v <- theta (c v + b):
//   forward:  l = 0: (0, bmul); l >= 1: ((1 - rho_{l-1}) cnum, rho_{l-1} bmul)
//   backward: l <= L-2: ((1 - rho_l) cnum, rho_l bmul); l = L-1: (0, 0), unused
// Each product is formed in FP64 and rounded once to FP32. The forward
// tables of the decoding sweeps (`fold`) multiply both by the emission
// divisor (sweep_emissions: `unit`, or with a per-variant mu that of variant
// l) last; the gradient's forward recursion keeps the divided pairs' scale
// (kCoefF32FwdGrad) and adds the divisors' logs instead.
enum {
    kCoefF32Fwd = 0,
    kCoefF32Bwd = 1,
    kCoefF16Fwd = 2,
    kCoefF16Bwd = 3,
    kCoefF32FwdGrad = 4,
    kCoefTables = 5
};
struct CoefScalars {
    double cnum[kCoefTables];
    double bmul[kCoefTables];
    int fold[kCoefTables];
    double unit;
};

// Miscellaneous kernels (ls_misc.hip).
hipError_t launch_coef_tables(const double *rho, const double *mu_vec, int32_t L,
                              const CoefScalars &cs, float *out, hipStream_t st);
hipError_t launch_repack(const uint32_t *H, int64_t stride_words, int32_t N, int32_t L,
                         uint64_t *Hr, int64_t hr_stride, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);
// Emission tables of a per-variant mu (ls_misc.hip), after the coefficient
// tables: [L][2] FP64 (match, mismatch) for the FP64 sweep, [L][2] FP32 pairs
// divided by their larger member for sweeps in FP32 arithmetic, and the FP64
// prefix sums [L+1] of the log of that divisor (entry l = sum over variants
// below l).
hipError_t launch_emission_tables(const double *mu_vec, int32_t L, double *em64, float *em32,
                                  double *lu_prefix, hipStream_t st);
// Per row i of a prior matrix ([N][N], row i = prior column of recipient i):
// out[2i] = sum of the row without its diagonal (NaN if any entry is
// negative, above 1 or not finite), in a fixed order; out[2i+1] = the bits
// of a 64-bit hash of the whole row (ls_misc.hip).
hipError_t launch_prior_stats(const double *prior, int32_t N, double *out, hipStream_t st);
// Recombination map (eq. rho) and its chain rule (ls_misc.hip)
hipError_t launch_calc_rho(const double *cM, int32_t n, double s, double gamma, double *rho,
                           hipStream_t st);
hipError_t launch_rho_map_grad(const double *cM, int32_t n, double s, double gamma,
                               const double *g, double *out, hipStream_t st);
hipError_t launch_symmetrise(const void *E, void *D, int32_t N, int32_t T, int is_f64,
                             hipStream_t st);
// Posterior and half distances for T x R rows of length N: row (k, r) pairs
// the forward vector at alpha + k ts + r rs with the backward vector at
// beta + (k R + r) N for recipient recips[r], and writes P and E at the
// same offsets as alpha (elements). P and E may be null; either may alias
// alpha (in place). alpha/beta/P/E element types follow `is_f64` and the
// half flags (half tables hold IEEE half; P and E are then FP32).
hipError_t launch_posterior_rows(const void *alpha, int alpha_half, const void *beta,
                                 int beta_half, const int32_t *recips, int32_t R, int32_t T,
                                 int64_t ts, int64_t rs, int32_t N, int is_f64, void *P, void *E,
                                 hipStream_t st);

// Log-likelihood and gradient (ls_grad.hip).
// Workspace layout of ls_loglik_grad (byte offsets, 256-byte aligned).
struct GradLayout {
    size_t off_recips;  // int32 [R]   recipient indices when the caller passes none
    size_t off_state;   // [R][N]      forward table of the log-likelihood pass
    size_t off_ll;      // double [R]  per-recipient log-likelihood
    size_t off_status;  // uint32 [R]
    size_t off_ckpt;    // [R][nseg][N] forward vectors at checkpoints (gradient)
    size_t off_seg;     // [(seg-1)/2][R][N] forward vectors at even offsets
                        // 2, 4, .. from the segment's checkpoint
    size_t off_cval;    // [seg][R] c of the forward step at each offset 1, 2, ..
    size_t off_grow;    // double [L-1][R] per-recipient d log P / d rho
    size_t off_gmu;     // double [R]
    size_t off_gmul;    // double [L][R] per-recipient d log P / d mu^l (vector mu)
    size_t off_lsc;     // double [R] scratch log scale of the recompute sweeps
    size_t off_ybuf;    // [R][N] backward vector handed between segments
    size_t total;
    int32_t seg, nseg;
};
// Fills *lay (if not null) and returns the workspace size.
size_t grad_workspace_bytes(int32_t N, int32_t L, int32_t R, int prec, bool muv,
                            GradLayout *lay);

struct GradArgs {
    const uint64_t *Hr;
    const double *rho;
    const float *coef_fwd32;  // FP32 forward coefficient table
    const float *coef_bwd32;  // FP32 backward coefficient table
    const int32_t *recipients;
    int64_t hr_stride;
    int32_t N, L, NF, R;
    int32_t seg, nseg;
    int32_t chunk;      // variants per launch of the checkpointing forward sweep
    Shape fwd_shape;    // its shape: the one a plain forward sweep of N uses
    double mu;
    // per-variant mu (else all null): the emission pairs in the arithmetic
    // type, the FP64 pairs (1-mu^l, mu^l) and, for FP32, the log-unit prefix
    const void *emis;
    const double *em64;
    const double *lu_prefix;
    const double *prior;  // prior copying matrix ([N][N], row i = column i), or null
    char *ws;
    GradLayout lay;
};
hipError_t launch_iota(int32_t *p, int32_t n, hipStream_t st);
// loglik[r] = ll[r] (if loglik != null) and *pac = sum_r ll[r] in index order
hipError_t launch_loglik_sum(const double *ll, int32_t R, double *loglik, double *pac,
                             hipStream_t st);
// What launch_grad runs: the checkpointing forward and the log-likelihood
// sum, the adjoint pass over checkpoints a previous kGradForward call left
// in the workspace, or both.
enum GradPhase { kGradForward = 1, kGradAdjoint = 2, kGradBoth = 3 };
hipError_t launch_grad(const GradArgs &a, int prec, Shape shape, double *loglik, double *pac,
                       double *grad_rho, double *grad_mu, hipStream_t st, GradPhase phase);

}  // namespace lsk
