/*
 * ls.h -- C ABI of libls: the Li & Stephens all-vs-all copying model
 * (Li & Stephens 2003, in the reformulation of Aslett & Christ, "kalis",
 * arXiv 2212.11403) on AMD Instinct MI355X (gfx950).
 *
 * For every recipient haplotype i the library runs one hidden Markov model
 * whose hidden state is the donor j != i that i copies at each variant. It
 * propagates the scaled forward and backward recursions of the paper
 * (section 2.2, eq. fwd0/fwd1 and bck0/bck1), decodes posterior copying
 * probabilities (eq. postprob) and local distances (eq. distmat), and
 * returns the per-recipient log-likelihood and its gradient with respect to
 * the recombination probabilities and the mutation probability.
 *
 * Conventions used by every entry point
 * -------------------------------------
 * - Indices are 0-based. Haplotypes 0..N-1, variants 0..L-1. rho[l] is the
 *   recombination probability between variants l and l+1, l = 0..L-2 (the
 *   paper's rho vector of length L-1, section 3.4).
 * - The copying prior is uniform, pi_ji = 1/(N-1) for j != i and 0 for
 *   j == i (the default prior of section 2.1; self copying excluded),
 *   unless the model carries a prior copying matrix (ls_model.prior).
 * - The mutation probability is the scalar ls_model.mu at every variant,
 *   unless the model carries one value per variant (ls_model.mu_vec,
 *   section 3.4).
 * - Every data pointer named "device" is device memory on the current HIP
 *   device. Pointers named "host" are host memory. The caller allocates and
 *   owns every buffer; the library allocates nothing and keeps no global
 *   state.
 * - "stream" is a hipStream_t (NULL = the legacy default stream). Calls that
 *   take a stream only validate arguments on the host, then enqueue kernels
 *   on that stream and return; outputs are valid once the stream has
 *   completed. A validation error returns before anything is enqueued.
 * - Tables are modified in place, as in the paper (section 3.6).
 * - Numerical failure is not an error code: if a column sum of a recipient
 *   becomes 0 or non-finite ("total underflow", appendix A.3), that
 *   recipient's column turns NaN except the diagonal, which stays 0, and
 *   LS_FLAG_NONFINITE is set in its status word. ls_status_check() reads the
 *   status words back.
 */
#ifndef LS_H
#define LS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LS_OK = 0,
    LS_ERR_ARG = 1,         /* NULL pointer, value out of range, bad enum */
    LS_ERR_SHAPE = 2,       /* sizes inconsistent with each other */
    LS_ERR_STATE = 3,       /* table at the wrong variant or direction, or
                               built with another model (hash mismatch) */
    LS_ERR_UNSUPPORTED = 4, /* N too large for this precision on one GPU, or a
                               feature this precision does not offer */
    LS_ERR_DEVICE = 5,      /* the HIP runtime reported an error */
    LS_ERR_WORKSPACE = 6,   /* workspace missing or too small */
    LS_ERR_SCRATCH = 7,     /* request larger than the fixed scratch of an
                               allocation-free call (nothing launched) */
    LS_WARN_NONFINITE = 16  /* returned by ls_status_check only */
} ls_status;

/* Arithmetic of the sweep.
 * LS_FP64: everything in double precision.
 * LS_FP32: single-precision vectors with per-step renormalisation; column
 *   sums reduced in FP32 lanes; the log scale factors and the
 *   log-likelihood accumulate in FP64.
 * LS_FP32_F16STORE: FP16-stored vectors: FP32 arithmetic as LS_FP32, but
 *   the vector is rounded to IEEE half precision after every update, at
 *   every variant, and the tables hold it in half (half their memory). The
 *   per-recipient scale is the FP64 log scale of the table and a fixed
 *   factor kappa per direction that keeps entries inside half's range (see
 *   ls_table); the vectors are renormalised at every step. Snapshots,
 *   posteriors and distances are FP32. A precision-study option: its error
 *   against LS_FP64 is that of half storage. Half holds an entry down to
 *   about 2^-38 of its vector's largest (its smallest subnormal over kappa);
 *   smaller entries round to 0 and stay 0 until a jump refills them. With a
 *   prior whose weights span more than that, a donor can hold a large
 *   posterior as the product of an alpha and a beta entry each below that
 *   range, and half storage loses it (the tables stay finite). */
typedef enum { LS_FP64 = 0, LS_FP32 = 1, LS_FP32_F16STORE = 2 } ls_precision;

/* Status word flags (per recipient, device memory). */
#define LS_FLAG_NONFINITE 1u   /* a column sum was 0, Inf or NaN */
#define LS_FLAG_BAD_RECIPIENT 2u /* recipient index outside [0, N) */

/* Maximum number of targets one ls_forward / ls_backward call can visit.
 * Longer lists are handled by several calls: tables resume where they stop. */
#define LS_MAX_TARGETS 256

/* The model: haplotypes and parameters (cf. the kalis parameter object,
 * section 4.1.2). Fill the input fields, then call ls_model_init. */
typedef struct {
    /* inputs */
    const uint32_t *H;    /* device, [L][stride_words]: haplotype j at
                             variant l is bit (j % 32) of word j / 32 of row l
                             (the variant-major bit cache of section 4.1.1) */
    int64_t stride_words; /* 32-bit words per row; >= ceil(N/32), even */
    int32_t N;            /* haplotypes, >= 2 */
    int32_t L;            /* variants, >= 1 */
    const double *rho;    /* device, [L-1], each in [0, 1]; may be NULL if L == 1 */
    double mu;            /* in [0, 1] */
    /* set by ls_model_init */
    uint64_t hash;        /* hash of (N, L, rho, mu, mu_vec, prior); tables remember it */
    const uint64_t *Hr;   /* device: internal row layout in the workspace */
    int64_t hr_stride;    /* 64-bit words per internal row */
    int32_t nf;           /* number of full 64-haplotype words: floor(N/64) */
    int32_t reserved;
    /* optional, set by the caller before ls_model_init: */
    const double *mu_vec; /* device, [L] mutation probability per variant (the
                             paper's vector mu, section 3.4), each in [0, 1],
                             or NULL: mu at every variant. Used by decoding,
                             the log-likelihood and its gradient (then one
                             d/d mu^l per variant) in every precision that
                             offers them. */
    const double *prior;  /* device, [N][N] prior copying matrix Pi (section
                             2.1), row i = column i of Pi: prior[i*N + j] =
                             Pi_ji, the prior probability that recipient i
                             copies donor j; every entry in [0, 1], each row
                             summing to 1 without its diagonal (which is not
                             used: self copying is excluded), else
                             ls_model_init returns LS_ERR_ARG. NULL: the
                             uniform prior 1/(N-1). Used by decoding, the
                             log-likelihood and its gradient, with a scalar
                             mu or mu_vec, in every precision that offers
                             them. With LS_FP32_F16STORE a backward
                             table with a prior holds a positive multiple
                             of beta per recipient (W/S beta with W the
                             prior-weighted and S the plain column sum of
                             beta theta), which stays inside half's range
                             for any prior; posteriors do not depend on the
                             multiple. The caller
                             keeps it alive and unchanged while the model
                             is in use. */
} ls_model;

/* Device bytes of the workspace ls_model_init lays the internal haplotype
 * rows (about 2 N L / 8 bytes), the per-variant FP32 transition
 * coefficients of the sweeps (40 L bytes), the per-variant emission
 * tables for a vector mu (32 L + 8 bytes) and the checks of a prior matrix
 * (16 N bytes) into. */
size_t ls_model_workspace_bytes(int32_t N, int32_t L);

/* Validates the inputs, computes the hash and builds the internal rows in
 * `workspace` (device, >= ls_model_workspace_bytes(N, L) bytes, 256-byte
 * aligned) on `stream`. Reads rho back to the host (synchronises the
 * stream). The workspace must stay allocated and unchanged while the model
 * is used. Errors: LS_ERR_ARG (NULL H/rho, N < 2, L < 1, mu or rho out of
 * range, short stride), LS_ERR_WORKSPACE, LS_ERR_DEVICE. */
ls_status ls_model_init(ls_model *m, void *workspace, size_t ws_bytes, void *stream);

/* A forward or backward table for R recipients at one variant (cf. the
 * kalis forward/backward table, section 4.1.3).
 *   forward at variant l:  state[r][j] = alpha^l_{j,i} (eq. fwd0/fwd1),
 *                          log_scale[r] = log F^l = sum_{k<=l} log S_k,
 *                          S_k = sum_j alpha^k_j (eq. F).
 *   backward at variant l: state[r][j] = beta^l_{j,i} (eq. bck0/bck1),
 *                          log_scale[r] = log G^l (eq. G).
 * with i = recipients[r]. The diagonal entry j == i is always 0.
 * Element type of state: double (LS_FP64), float (LS_FP32) or IEEE half
 * (LS_FP32_F16STORE). Half tables hold kappa * alpha (kappa = 2^14) or
 * kappa * beta (kappa = 2^14 / (N-1); with a prior matrix kappa times a
 * positive multiple of beta, see ls_model.prior), and their log_scale
 * accounts for the factor; the recursions and posteriors do not depend on
 * it. */
typedef struct {
    void *state;               /* device, [R][N] */
    double *log_scale;         /* device, [R] */
    uint32_t *status;          /* device, [R], LS_FLAG_* bits (cleared by init) */
    const int32_t *recipients; /* device, [R], each in [0, N) */
    int32_t R;
    int32_t l;                 /* current variant; -1 = not yet propagated */
    int32_t direction;         /* 0 forward, 1 backward */
    int32_t prec;              /* ls_precision */
    uint64_t model_hash;       /* 0 until the first propagation */
} ls_table;

/* Resets a table to "not yet propagated" (cf. MakeForwardTable /
 * MakeBackwardTable / ResetTable). Clears the status words on `stream`.
 * Errors: LS_ERR_ARG. */
ls_status ls_table_init(ls_table *t, int32_t direction, ls_precision prec, void *state,
                        double *log_scale, uint32_t *status, const int32_t *recipients,
                        int32_t R, void *stream);

/* Copies the contents of `src` into `dst` (cf. CopyTable, section 3.6).
 * Both must have the same direction, precision and R. Errors: LS_ERR_ARG,
 * LS_ERR_SHAPE, LS_ERR_DEVICE. */
ls_status ls_table_copy(ls_table *dst, const ls_table *src, int32_t N, void *stream);

/* Forward (cf. Forward(fwd, pars, t), section 3.6): moves `fwd` from its
 * current variant to t (t > fwd->l; an unpropagated table starts at variant 0
 * and may stop there, t >= 0).
 * targets: host, [T], strictly increasing, each in (fwd->l, t], T <= 256.
 * At each target k the forward vector is combined with the backward vector
 * bsnap[k] (eq. postprob) and, for the outputs that are not NULL:
 *   P[k][r][j] = p_{j,i}                         posterior (eq. postprob)
 *   E[k][r][j] = -log(max(p_{j,i}, eps)) / 2     half distance, eps = 2^-52
 *                                                (eq. distmat), E[k][r][i] = 0
 * bsnap: device, [T][R][N]; element type double for LS_FP64, float
 * otherwise. bsnap[k] must be a backward table state at targets[k] for the
 * same recipients (as written by ls_backward's snapshots); it may be NULL
 * only if T == 0.
 * P, E: device, same element type; row (k, r) starts at element
 * k * out_target_stride + r * out_row_stride and holds N entries. Strides
 * of 0 mean the contiguous [T][R][N] layout (out_row_stride = N,
 * out_target_stride = R * out_row_stride). Other strides let a window of
 * recipients write its rows into larger arrays, e.g. rows r0 .. r0+R-1 of
 * T resident N x N matrices (pass E + r0 * N, out_target_stride = N * N,
 * out_row_stride = N), the recipient windows of section 3.9. Rows must not
 * overlap: out_row_stride >= N and, for T > 1, out_target_stride >=
 * (R-1) * out_row_stride + N, else LS_ERR_SHAPE. P and E share the layout.
 * Errors: LS_ERR_ARG, LS_ERR_SHAPE, LS_ERR_STATE, LS_ERR_UNSUPPORTED,
 * LS_ERR_DEVICE. */
ls_status ls_forward(ls_table *fwd, const ls_model *m, int32_t t, const int32_t *targets,
                     int32_t T, const void *bsnap, void *P, void *E, int64_t out_target_stride,
                     int64_t out_row_stride, void *stream);

/* Backward (cf. Backward(bck, pars, t), section 3.6): moves `bck` from its
 * current variant down to t (t < bck->l; an unpropagated table starts at
 * variant L-1, where beta = 1, and may stop there, t <= L-1).
 * targets: host, [T], strictly increasing, each in [t, bck->l) (or
 * [t, L-1] for an unpropagated table), T <= 256. At each target k the
 * backward vector beta^{targets[k]} is written to bsnap[k][r][j] (device,
 * [T][R][N], double for LS_FP64 and float otherwise; diagonal 0).
 * Errors: as ls_forward. */
ls_status ls_backward(ls_table *bck, const ls_model *m, int32_t t, const int32_t *targets,
                      int32_t T, void *bsnap, void *stream);

/* Posterior and half distances from a forward and a backward table at the
 * same variant (cf. PostProbs / DistMat, section 3.7). Both tables must hold
 * the same recipients in the same order (not checked: they are device data);
 * the recipient indices are read from fwd->recipients.
 *   P[r][j] = p_{j,i} (eq. postprob), E[r][j] = -log(max(p_{j,i}, eps))/2.
 * P and E: device, [R][N], double for LS_FP64 tables and float otherwise;
 * either may be NULL. Errors: LS_ERR_ARG, LS_ERR_STATE, LS_ERR_DEVICE. */
ls_status ls_posterior_distance(const ls_table *fwd, const ls_table *bck, const ls_model *m,
                                void *P, void *E, void *stream);

/* Symmetrised local distances (eq. distmat) for T targets from half
 * distances of all N recipients in order (recipient r = haplotype r):
 *   D[k][a][b] = E[k][a][b] + E[k][b][a], D[k][a][a] = 0.
 * E, D: device, [T][N][N], double if prec == LS_FP64 else float. D may
 * equal E (in place). Errors: LS_ERR_ARG, LS_ERR_DEVICE. */
ls_status ls_distance_symmetrise(const void *E, void *D, int32_t N, int32_t T,
                                 ls_precision prec, void *stream);

/* Average pairwise linkage (Sokal and Michener's method, with which the paper
 * clusters a distance matrix, section 6) of T symmetric N x N distance
 * matrices, each by one workgroup, side by side.
 * Definition: every haplotype starts as its own cluster; the two clusters
 * at the smallest distance merge, the distance between clusters being the
 * mean of the pairwise distances of their members, kept with the update
 * d(A u B, C) = (|A| d(A,C) + |B| d(B,C)) / (|A| + |B|) evaluated in the
 * matrix's precision (each operation rounded in that order).
 * Slots and ties: cluster k starts in slot k; merging slots a < b keeps the
 * merged cluster in slot a. Among the pairs at the smallest distance the
 * merge takes the smallest slot a, then the smallest b; a NaN distance comes
 * after every number. The merges are those of the plain algorithm that
 * scans every pair at every merge, bit for bit.
 * D: device, [T][N][N], double if prec == LS_FP64 else float, symmetric
 * (its diagonal is not read); overwritten (the rows and columns of merged
 * clusters hold the merged distances).
 * Z: device, [T][N-1][4] double: per merge m, the two cluster ids (leaves
 * 0..N-1, merge m makes id N + m; smaller id first), the merge distance and
 * the size of the merged cluster (the usual linkage-matrix layout).
 * order: device, [T][N] int32, the dendrogram's leaf order (each merge's
 * smaller id first), or NULL.
 * workspace: device, >= ls_average_linkage_workspace_bytes(N, T, prec)
 * bytes (about 21 N T bytes), 256-byte aligned; contents undefined after.
 * Errors: LS_ERR_ARG, LS_ERR_WORKSPACE, LS_ERR_DEVICE. */
size_t ls_average_linkage_workspace_bytes(int32_t N, int32_t T, ls_precision prec);
ls_status ls_average_linkage(void *D, int32_t N, int32_t T, ls_precision prec, double *Z,
                             int32_t *order, void *workspace, size_t ws_bytes, void *stream);

/* ls_average_linkage for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid it):
 * the same kernels and results, with the workspace taken from a fixed
 * 32 MiB scratch array the library holds on each GPU until the process ends
 * (enough for N = 10,000 with up to 150 matrices, or N = 100,000 with up to
 * 15). The call allocates nothing; the caller passes D, Z and order as for
 * ls_average_linkage. Every call on one GPU uses that GPU's array: calls
 * that overlap on one GPU (other streams or threads) race and must be
 * ordered by the caller. The array needs no clearing (every entry a call
 * reads it first writes).
 * Errors: LS_ERR_ARG; LS_ERR_SCRATCH when
 * ls_average_linkage_workspace_bytes(N, T, prec) exceeds 32 MiB (nothing is
 * launched); LS_ERR_DEVICE. */
ls_status ls_average_linkage_noalloc(void *D, int32_t N, int32_t T, ls_precision prec, double *Z,
                                     int32_t *order, void *stream);

/* Standardised half-distance rows (section 2.2: a recipient's column of
 * distances standardised, with 0 where its deviation is 0), in place: row
 * (k, r) of N half distances at E + k * out_target_stride + r *
 * out_row_stride (the layout of ls_forward's E; strides 0 = contiguous
 * [T][R][N]) belongs to recipient i = recipients[r]:
 *   z_j = (e_j - mean) / sd over the donors j != i, with the mean and the
 *   population standard deviation (divisor N - 1), accumulated in FP64;
 *   z_i = 0; a row whose donor entries are all equal (the zero-total case
 *   of eq. postprob gives every donor -log(eps)/2) becomes 0; a NaN row
 *   stays NaN.
 * Symmetrising standardised rows (ls_distance_symmetrise) gives standardised
 * distances. E: device, double for LS_FP64 else float; recipients: device
 * [R]. Errors: LS_ERR_ARG, LS_ERR_SHAPE (overlapping rows), LS_ERR_DEVICE. */
ls_status ls_standardise_rows(void *E, const int32_t *recipients, int32_t R, int32_t T,
                              int32_t N, int64_t out_target_stride, int64_t out_row_stride,
                              ls_precision prec, void *stream);

/* Log-likelihood of each recipient, log P(h_i | h_-i) = log F^{L-1}, their
 * sum (the product-of-approximate-conditionals log-likelihood over all
 * recipients, section 1) and, if grad_rho / grad_mu are not NULL, the
 * gradient of that sum with respect to rho[0..L-2] and mu (with a
 * per-variant mu_vec: with respect to each mu^l).
 * recipients: device, [R] (NULL = all N haplotypes in order, R must be N).
 * loglik: device [R] double (may be NULL); pac: device [1] double;
 * grad_mu: device double, [1] for a scalar mu, [L] with mu_vec;
 * grad_rho: device [L-1] double. The sum over recipients is taken in a fixed
 * order, so results do not depend on scheduling. The gradient is the exact
 * score (not a finite difference), computed with forward checkpoints every
 * ceil(sqrt(L)) variants, a recompute of each segment and an adjoint pass;
 * it is available for LS_FP64 and LS_FP32 (LS_FP32_F16STORE gives the
 * log-likelihood only and returns LS_ERR_UNSUPPORTED if a gradient is
 * asked for). log P and the sum are the same bits with or without the
 * gradient.
 * workspace: device, >= ls_loglik_grad_workspace_bytes(m, R, prec) bytes,
 * 256-byte aligned; owned by the caller, contents undefined after the call.
 * About e R N (1.5 sqrt(L) + 3) + 8 R L bytes (e = 4 for FP32, 8 for FP64):
 * checkpoints, the kept half of one segment's forward vectors, the
 * per-variant rho terms of every recipient (and with mu_vec 8 R L more
 * for the per-variant mu terms).
 * Errors: LS_ERR_ARG, LS_ERR_WORKSPACE (missing, too small or misaligned),
 * LS_ERR_UNSUPPORTED, LS_ERR_DEVICE. */
ls_status ls_loglik_grad(const ls_model *m, const int32_t *recipients, int32_t R,
                         ls_precision prec, double *loglik, double *pac, double *grad_rho,
                         double *grad_mu, void *workspace, size_t ws_bytes, void *stream);

/* The two halves of ls_loglik_grad with a gradient, for callers that
 * evaluate the log-likelihood first and decide later whether they need its
 * gradient (an autograd forward and backward):
 * ls_loglik_checkpoint runs the checkpointing forward sweep and writes
 * loglik (may be NULL) and pac, exactly as ls_loglik_grad does (the same
 * bits); it leaves the forward checkpoints in `workspace`.
 * ls_loglik_grad_adjoint then runs the recompute and adjoint passes over
 * those checkpoints and writes grad_rho and grad_mu, the same bits as
 * ls_loglik_grad. Both calls take the same model, recipients, R,
 * precision and workspace (size from ls_loglik_grad_workspace_bytes); the
 * workspace must not be changed between them (nothing checks this: device
 * memory is not read back). LS_FP64 and LS_FP32 only (LS_ERR_UNSUPPORTED
 * otherwise). Errors as ls_loglik_grad. */
ls_status ls_loglik_checkpoint(const ls_model *m, const int32_t *recipients, int32_t R,
                               ls_precision prec, double *loglik, double *pac, void *workspace,
                               size_t ws_bytes, void *stream);
ls_status ls_loglik_grad_adjoint(const ls_model *m, const int32_t *recipients, int32_t R,
                                 ls_precision prec, double *grad_rho, double *grad_mu,
                                 void *workspace, size_t ws_bytes, void *stream);

/* Recombination probabilities from a genetic map (eq. rho, section 2.1;
 * the paper's CalcRho, section 3.4):
 *   rho[l] = 1 - exp(-s (cM[l] / 100)^gamma),  l = 0 .. n-1,
 * where cM[l] is the map distance between variants l and l+1 in
 * centimorgans (cM / 100 is the distance in Morgans of eq. rho), s the
 * scalar multiple N_e and gamma the power; evaluated with expm1.
 * cM, rho: device, [n] double (n = L - 1 for a model's rho); cM >= 0.
 * Errors: LS_ERR_ARG (n < 0, null pointers, s < 0, gamma <= 0, or a
 * non-finite s or gamma), LS_ERR_DEVICE. */
ls_status ls_calc_rho(const double *cM, int32_t n, double s, double gamma, double *rho,
                      void *stream);

/* Chain rule from a gradient w.r.t. rho (such as ls_loglik_grad's
 * grad_rho) to the map parameters of ls_calc_rho: with x_l = s m_l^gamma,
 * m_l = cM[l] / 100,
 *   grad_s_gamma[0] = sum_l grad_rho[l] m_l^gamma exp(-x_l)
 *   grad_s_gamma[1] = sum_l grad_rho[l] s m_l^gamma log(m_l) exp(-x_l)
 * (terms with m_l = 0 are 0), summed in a fixed order.
 * cM, grad_rho: device, [n] double; grad_s_gamma: device, [2] double.
 * Errors: as ls_calc_rho. */
ls_status ls_rho_map_grad(const double *cM, int32_t n, double s, double gamma,
                          const double *grad_rho, double *grad_s_gamma, void *stream);

/* Workspace bytes ls_loglik_grad needs (0 on bad arguments). */
size_t ls_loglik_grad_workspace_bytes(const ls_model *m, int32_t R, ls_precision prec);

/* Synchronises `stream`, reads `R` status words and returns LS_OK,
 * LS_WARN_NONFINITE if any recipient has LS_FLAG_NONFINITE, or LS_ERR_ARG if
 * any has LS_FLAG_BAD_RECIPIENT. */
ls_status ls_status_check(const uint32_t *status, int32_t R, void *stream);

/* The kernel shape the library uses for the sweeps of N haplotypes at
 * `prec`: slots (64-donor register groups) per wave and waves per
 * recipient. with_prior != 0: the shape of a model with a prior matrix
 * (whose sweeps keep the prior column in registers beside the donor
 * column). Returns LS_ERR_UNSUPPORTED if no shape fits on one compute unit,
 * LS_ERR_ARG for N < 2 or an unknown precision. */
ls_status ls_kernel_shape(int32_t N, ls_precision prec, int32_t with_prior,
                          int32_t *slots_per_wave, int32_t *waves_per_recipient);

const char *ls_status_string(ls_status s);
const char *ls_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LS_H */
