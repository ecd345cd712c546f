/*
 * ls_oracle.c -- plain FP64 CPU reference for the Li & Stephens all-vs-all
 * copying model (Aslett & Christ, "kalis", arXiv 2212.11403).
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library. It shares no code with the GPU
 * path and is written for clarity, not speed: scalar loops, one recipient at
 * a time, every division written out, built with -ffp-contract=off.
 *
 * Notation follows the paper (section 2): h is L x N, recipient i, donor j,
 * variant l. Indices here are 0-based: variants 0..L-1, and rho[l] is the
 * recombination probability between variants l and l+1 (l = 0..L-2).
 *
 * Definitions used (paper section 2.1 and 2.2, appendix A):
 *   emission  theta^l_j = (1 - H)(1 - 2 mu) + mu, H = 1{h_j^l != h_i^l}
 *             (eq. emission, in the form of appendix A.3)
 *   prior     pi_j = Pi_ji, column i of the prior copying matrix Pi (section
 *             2.1; left stochastic, Pi_ii = 0), or by default the uniform
 *             prior pi_j = 1/(N-1) for j != i, pi_i = 0. The transition is
 *             T_jk = rho pi_k + (1-rho) 1{j=k} (eq. transition)
 *   forward   alpha^0 = theta^0 pi                                (eq. fwd0)
 *             alpha^l = theta^l ((1-rho_{l-1}) alpha^{l-1}/sum(alpha^{l-1})
 *                                 + rho_{l-1} pi)                 (eq. fwd1)
 *   backward  beta^{L-1} = 1                                      (eq. bck0)
 *             beta^l = (1-rho_l) beta^{l+1} theta^{l+1}
 *                        / sum(beta^{l+1} theta^{l+1} pi) + rho_l (eq. bck1)
 *   posterior p^l = alpha^l beta^l / sum(alpha^l beta^l); if that sum is 0,
 *             p_j = eps for all j != i                           (eq. postprob)
 *   distance  d_ji = -(log(p_ji v eps) + log(p_ij v eps))/2, d_ii = 0,
 *             eps = 2^-52                                        (eq. distmat)
 * Self copying is excluded: alpha_ii = beta_ii = p_ii = 0 at every variant,
 * as the paper's tables show a zero diagonal.
 *
 * Scale factors (eq. F, eq. G): with S_l = sum_j alpha^l_j the forward scale
 * is F^l = prod_{k<=l} S_k, and with g_l = sum_j pi_j theta^l_j beta^l_j the
 * backward scale is G^l = prod_{k>l} g_k. Both are kept as logarithms. The
 * log-likelihood of recipient i is log P(h_i | h_-i) = log F^{L-1} (forward)
 * = log G^0 + log g_0 (backward).
 *
 * Gradient (not in the paper; the exact score of the HMM). With a_l =
 * sum_j alpha^l_j theta^{l+1}_j beta^{l+1}_j:
 *   d log P / d rho_l = (S_l g_{l+1} - a_l) / ((1-rho_l) a_l + rho_l S_l g_{l+1})
 *   d log P / d mu    = sum_l sum_j p^l_j (H^l_j/mu - (1-H^l_j)/(1-mu))
 * The first follows from d T_jk / d rho = pi_k - 1{j=k} for the transition
 * T_jk = rho pi_k + (1-rho) 1{j=k} (eq. transition); the second from
 * d log theta / d mu = 1/mu on a mismatch and -1/(1-mu) on a match.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LSO_EPS 2.220446049250313080847e-16 /* 2^-52, double machine epsilon */

typedef struct {
    const uint32_t *H; /* [L][stride] bit-packed haplotypes */
    int64_t stride;    /* 32-bit words per variant row */
    int32_t N, L;
    const double *rho; /* [L-1] */
    double mu;
    const double *mu_vec; /* [L] per-variant mu^l, or NULL: mu at every variant */
    const double *Pi;     /* [N][N], Pi[i*N + j] = Pi_ji (column i: the prior of
                             recipient i), or NULL: the uniform prior */
} lso_model;

/* allele of haplotype j at variant l: bit (j mod 32) of word floor(j/32) */
static int allele(const lso_model *m, int l, int j)
{
    return (int)((m->H[(int64_t)l * m->stride + (j >> 5)] >> (j & 31)) & 1u);
}

/* mutation probability at variant l (the paper's mu may be a vector of
 * length L, section 3.4) */
static double mu_at(const lso_model *m, int l)
{
    return m->mu_vec ? m->mu_vec[l] : m->mu;
}

static double theta(const lso_model *m, int l, int j, int i)
{
    int Hm = allele(m, l, j) ^ allele(m, l, i);
    double mu = mu_at(m, l);
    return (double)(1 - Hm) * (1.0 - 2.0 * mu) + mu;
}

/* Pi_ji; the diagonal is 0 by convention (self copying is excluded) */
static double prior(const lso_model *m, int j, int i)
{
    if (j == i)
        return 0.0;
    return m->Pi ? m->Pi[(int64_t)i * m->N + j] : 1.0 / (double)(m->N - 1);
}

static double sum_vec(const double *v, int n)
{
    double s = 0.0;
    for (int j = 0; j < n; ++j)
        s += v[j];
    return s;
}

/* alpha^0 (eq. fwd0) */
static void forward_init(const lso_model *m, int i, double *alpha)
{
    for (int j = 0; j < m->N; ++j)
        alpha[j] = theta(m, 0, j, i) * prior(m, j, i);
}

/* alpha^{l-1} -> alpha^l (eq. fwd1), l >= 1. S = sum_j alpha^{l-1}_j */
static void forward_step(const lso_model *m, int i, int l, const double *prev, double S,
                         double *next)
{
    double r = m->rho[l - 1];
    for (int j = 0; j < m->N; ++j) {
        if (j == i) {
            next[j] = 0.0;
            continue;
        }
        next[j] = theta(m, l, j, i) * ((1.0 - r) * prev[j] / S + r * prior(m, j, i));
    }
}

/* g_l = sum_j pi_j theta^l_j beta^l_j (the denominator of eq. bck1) */
static double backward_norm(const lso_model *m, int i, int l, const double *beta)
{
    double g = 0.0;
    for (int j = 0; j < m->N; ++j)
        g += prior(m, j, i) * theta(m, l, j, i) * beta[j];
    return g;
}

/* beta^{l+1} -> beta^l (eq. bck1), l <= L-2. g = g_{l+1} */
static void backward_step(const lso_model *m, int i, int l, const double *next, double g,
                          double *cur)
{
    double r = m->rho[l];
    for (int j = 0; j < m->N; ++j) {
        if (j == i) {
            cur[j] = 0.0;
            continue;
        }
        cur[j] = (1.0 - r) * next[j] * theta(m, l + 1, j, i) / g + r;
    }
}

/* eq. postprob with the zero-sum rule */
static void posterior(const lso_model *m, int i, const double *alpha, const double *beta,
                      double *p)
{
    double Z = 0.0;
    for (int j = 0; j < m->N; ++j)
        Z += alpha[j] * beta[j];
    for (int j = 0; j < m->N; ++j) {
        if (j == i)
            p[j] = 0.0;
        else if (Z == 0.0)
            p[j] = LSO_EPS;
        else
            p[j] = alpha[j] * beta[j] / Z;
    }
}

/* one half of eq. distmat: -log(p v eps)/2; NaN stays NaN */
static double half_distance(double p)
{
    double q = (p < LSO_EPS) ? LSO_EPS : p;
    return -log(q) / 2.0;
}

/* ------------------------------------------------------------------------ */
/* Per-recipient pass: backward from L-1 (storing beta at the targets), then
 * forward from 0 (storing alpha, posteriors and half distances at targets).
 * Outputs with a NULL pointer are skipped. Target arrays are [T][N]; the
 * scale outputs are per target. Returns a status: bit 0 forward total
 * underflow/non-finite sum, bit 1 backward. */
typedef struct {
    const int32_t *targets;
    int32_t T;
    double *A, *B, *P, *E;      /* [T][N] rows for this recipient */
    double *logF, *logG;        /* [T] */
    double *llf, *llb;          /* scalars */
} lso_out;

static int recipient_pass(const lso_model *m, int i, const lso_out *o, double *buf0,
                          double *buf1, double *bsnap)
{
    const int N = m->N, L = m->L, T = o->T;
    int status = 0;
    /* backward */
    double *cur = buf0, *nxt = buf1;
    for (int j = 0; j < N; ++j)
        cur[j] = (j == i) ? 0.0 : 1.0;
    double logG = 0.0;
    for (int l = L - 1;; --l) {
        for (int k = 0; k < T; ++k)
            if (o->targets[k] == l) {
                memcpy(bsnap + (int64_t)k * N, cur, sizeof(double) * N);
                if (o->B)
                    memcpy(o->B + (int64_t)k * N, cur, sizeof(double) * N);
                if (o->logG)
                    o->logG[k] = logG;
            }
        double g = backward_norm(m, i, l, cur);
        if (!(g > 0.0) || !isfinite(g))
            status |= 2;
        if (l == 0) {
            if (o->llb)
                *o->llb = logG + log(g);
            break;
        }
        logG += log(g);
        backward_step(m, i, l - 1, cur, g, nxt);
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    /* forward */
    double *a = buf0, *an = buf1;
    double *ptmp = (double *)malloc(sizeof(double) * N);
    forward_init(m, i, a);
    double logF = 0.0;
    for (int l = 0;; ++l) {
        double S = sum_vec(a, N);
        if (!(S > 0.0) || !isfinite(S))
            status |= 1;
        logF += log(S);
        for (int k = 0; k < T; ++k)
            if (o->targets[k] == l) {
                const double *bt = bsnap + (int64_t)k * N;
                if (o->A)
                    memcpy(o->A + (int64_t)k * N, a, sizeof(double) * N);
                if (o->logF)
                    o->logF[k] = logF;
                posterior(m, i, a, bt, ptmp);
                if (o->P)
                    memcpy(o->P + (int64_t)k * N, ptmp, sizeof(double) * N);
                if (o->E)
                    for (int j = 0; j < N; ++j)
                        o->E[(int64_t)k * N + j] = (j == i) ? 0.0 : half_distance(ptmp[j]);
            }
        if (l == L - 1)
            break;
        forward_step(m, i, l + 1, a, S, an);
        double *t = a;
        a = an;
        an = t;
    }
    if (o->llf)
        *o->llf = logF;
    free(ptmp);
    return status;
}

/* Gradient of log P(h_i | h_-i) w.r.t. rho[0..L-2] and mu; with grad_mu_l
 * (may be NULL) also the derivative w.r.t. each mu^l, l = 0..L-1 (their sum
 * is *grad_mu). Stores the full forward table (L x N) for this recipient.
 * Returns the status bits. */
static int recipient_gradient(const lso_model *m, int i, double *grad_rho, double *grad_mu,
                              double *grad_mu_l, double *loglik)
{
    const int N = m->N, L = m->L;
    int status = 0;
    double *alpha = (double *)malloc(sizeof(double) * (size_t)L * N);
    double *S = (double *)malloc(sizeof(double) * L);
    double *beta = (double *)malloc(sizeof(double) * N);
    double *bprev = (double *)malloc(sizeof(double) * N);
    double *p = (double *)malloc(sizeof(double) * N);
    forward_init(m, i, alpha);
    for (int l = 0; l < L; ++l) {
        S[l] = sum_vec(alpha + (int64_t)l * N, N);
        if (!(S[l] > 0.0) || !isfinite(S[l]))
            status |= 1;
        if (l + 1 < L)
            forward_step(m, i, l + 1, alpha + (int64_t)l * N, S[l], alpha + (int64_t)(l + 1) * N);
    }
    double ll = 0.0;
    for (int l = 0; l < L; ++l)
        ll += log(S[l]);
    *loglik = ll;
    double gmu = 0.0;
    for (int j = 0; j < N; ++j)
        beta[j] = (j == i) ? 0.0 : 1.0;
    for (int l = L - 1; l >= 0; --l) {
        /* mu term at l from p^l */
        posterior(m, i, alpha + (int64_t)l * N, beta, p);
        double gl = 0.0;
        for (int j = 0; j < N; ++j) {
            if (j == i)
                continue;
            int Hm = allele(m, l, j) ^ allele(m, l, i);
            double t = Hm ? p[j] / mu_at(m, l) : -p[j] / (1.0 - mu_at(m, l));
            gmu += t;
            gl += t;
        }
        if (grad_mu_l)
            grad_mu_l[l] = gl;
        if (l == 0)
            break;
        /* rho_{l-1} term uses alpha^{l-1}, theta^l, beta^l */
        const double *al = alpha + (int64_t)(l - 1) * N;
        double g = backward_norm(m, i, l, beta);
        double a = 0.0;
        for (int j = 0; j < N; ++j)
            a += al[j] * theta(m, l, j, i) * beta[j];
        double r = m->rho[l - 1];
        double Sg = S[l - 1] * g;
        grad_rho[l - 1] = (Sg - a) / ((1.0 - r) * a + r * Sg);
        if (!(g > 0.0) || !isfinite(g))
            status |= 2;
        backward_step(m, i, l - 1, beta, g, bprev);
        double *t = beta;
        beta = bprev;
        bprev = t;
    }
    *grad_mu = gmu;
    free(alpha);
    free(S);
    free(beta);
    free(bprev);
    free(p);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Threaded drivers: recipients recips[0..R-1] are dealt round-robin to
 * nthreads threads. Every output row belongs to one recipient, so results do
 * not depend on the thread count. */

typedef struct {
    const lso_model *m;
    const int32_t *recips;
    int32_t R, T, tid, nth;
    const int32_t *targets;
    double *A, *B, *P, *E, *logF, *logG, *llf, *llb;
    int32_t *status;
    /* gradient */
    double *grad_rho_rows; /* [R][L-1] */
    double *grad_mu;       /* [R] */
    double *grad_mu_rows;  /* [R][L] per-variant mu terms, or NULL */
} lso_job;

static void *pass_worker(void *arg)
{
    lso_job *jb = (lso_job *)arg;
    const lso_model *m = jb->m;
    const int N = m->N, T = jb->T, R = jb->R;
    double *b0 = (double *)malloc(sizeof(double) * N);
    double *b1 = (double *)malloc(sizeof(double) * N);
    double *bs = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1) * N);
    double *rowA = jb->A ? (double *)malloc(sizeof(double) * (size_t)(T ? T : 1) * N) : NULL;
    double *rowB = jb->B ? (double *)malloc(sizeof(double) * (size_t)(T ? T : 1) * N) : NULL;
    double *rowP = jb->P ? (double *)malloc(sizeof(double) * (size_t)(T ? T : 1) * N) : NULL;
    double *rowE = jb->E ? (double *)malloc(sizeof(double) * (size_t)(T ? T : 1) * N) : NULL;
    double *lF = (double *)malloc(sizeof(double) * (T ? T : 1));
    double *lG = (double *)malloc(sizeof(double) * (T ? T : 1));
    for (int r = jb->tid; r < R; r += jb->nth) {
        lso_out o;
        double llf = 0, llb = 0;
        o.targets = jb->targets;
        o.T = T;
        o.A = rowA;
        o.B = rowB;
        o.P = rowP;
        o.E = rowE;
        o.logF = lF;
        o.logG = lG;
        o.llf = &llf;
        o.llb = &llb;
        int st = recipient_pass(m, jb->recips[r], &o, b0, b1, bs);
        /* scatter [T][N] rows into the [T][R][N] outputs */
        for (int k = 0; k < T; ++k) {
            int64_t dst = ((int64_t)k * R + r) * N;
            if (jb->A)
                memcpy(jb->A + dst, rowA + (int64_t)k * N, sizeof(double) * N);
            if (jb->B)
                memcpy(jb->B + dst, rowB + (int64_t)k * N, sizeof(double) * N);
            if (jb->P)
                memcpy(jb->P + dst, rowP + (int64_t)k * N, sizeof(double) * N);
            if (jb->E)
                memcpy(jb->E + dst, rowE + (int64_t)k * N, sizeof(double) * N);
            if (jb->logF)
                jb->logF[(int64_t)k * R + r] = lF[k];
            if (jb->logG)
                jb->logG[(int64_t)k * R + r] = lG[k];
        }
        if (jb->llf)
            jb->llf[r] = llf;
        if (jb->llb)
            jb->llb[r] = llb;
        if (jb->status)
            jb->status[r] = st;
    }
    free(b0);
    free(b1);
    free(bs);
    free(rowA);
    free(rowB);
    free(rowP);
    free(rowE);
    free(lF);
    free(lG);
    return NULL;
}

static void *grad_worker(void *arg)
{
    lso_job *jb = (lso_job *)arg;
    const lso_model *m = jb->m;
    for (int r = jb->tid; r < jb->R; r += jb->nth) {
        double gm = 0, ll = 0;
        int st = recipient_gradient(m, jb->recips[r], jb->grad_rho_rows + (int64_t)r * (m->L - 1),
                                    &gm, jb->grad_mu_rows ? jb->grad_mu_rows + (int64_t)r * m->L : NULL,
                                    &ll);
        jb->grad_mu[r] = gm;
        if (jb->llf)
            jb->llf[r] = ll;
        if (jb->status)
            jb->status[r] = st;
    }
    return NULL;
}

static int run_jobs(lso_job *proto, int nthreads, void *(*fn)(void *))
{
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > proto->R && proto->R > 0)
        nthreads = proto->R;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
    lso_job *jobs = (lso_job *)malloc(sizeof(lso_job) * nthreads);
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *proto;
        jobs[t].tid = t;
        jobs[t].nth = nthreads;
        pthread_create(&th[t], NULL, fn, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t)
        pthread_join(th[t], NULL);
    free(th);
    free(jobs);
    return 0;
}

static int check_model(const lso_model *m)
{
    if (!m || !m->H || m->N < 2 || m->L < 1 || m->stride < (m->N + 31) / 32)
        return 1;
    if (m->L > 1 && !m->rho)
        return 1;
    return 0;
}

/* Forward/backward/posterior/distance pass for recipients recips[0..R-1].
 * Target outputs are [T][R][N]; logF/logG are [T][R]; llf/llb/status [R].
 * Any output pointer may be NULL. Returns 0, or 1 on a bad argument. */
static int pass_model(const lso_model *mp, const int32_t *recips, int32_t R,
                      const int32_t *targets, int32_t T, double *A, double *B, double *P,
                      double *E, double *logF, double *logG, double *llf, double *llb,
                      int32_t *status, int32_t nthreads);

int lso_pass(const uint32_t *H, int64_t stride, int32_t N, int32_t L, const double *rho,
             double mu, const int32_t *recips, int32_t R, const int32_t *targets, int32_t T,
             double *A, double *B, double *P, double *E, double *logF, double *logG,
             double *llf, double *llb, int32_t *status, int32_t nthreads)
{
    lso_model m = {H, stride, N, L, rho, mu, NULL};
    return pass_model(&m, recips, R, targets, T, A, B, P, E, logF, logG, llf, llb, status,
                      nthreads);
}

/* As lso_pass with a per-variant mutation probability mu_vec[0..L-1]. */
int lso_pass_v(const uint32_t *H, int64_t stride, int32_t N, int32_t L, const double *rho,
               const double *mu_vec, const int32_t *recips, int32_t R, const int32_t *targets,
               int32_t T, double *A, double *B, double *P, double *E, double *logF,
               double *logG, double *llf, double *llb, int32_t *status, int32_t nthreads)
{
    if (!mu_vec)
        return 1;
    lso_model m = {H, stride, N, L, rho, 0.0, mu_vec};
    return pass_model(&m, recips, R, targets, T, A, B, P, E, logF, logG, llf, llb, status,
                      nthreads);
}

/* The general pass: a scalar mu or mu_vec (if not NULL), and the prior
 * matrix Pi (NULL: uniform). */
int lso_pass_x(const uint32_t *H, int64_t stride, int32_t N, int32_t L, const double *rho,
               double mu, const double *mu_vec, const double *Pi, const int32_t *recips,
               int32_t R, const int32_t *targets, int32_t T, double *A, double *B, double *P,
               double *E, double *logF, double *logG, double *llf, double *llb, int32_t *status,
               int32_t nthreads)
{
    lso_model m = {H, stride, N, L, rho, mu, mu_vec, Pi};
    return pass_model(&m, recips, R, targets, T, A, B, P, E, logF, logG, llf, llb, status,
                      nthreads);
}

static int pass_model(const lso_model *mp, const int32_t *recips, int32_t R,
                      const int32_t *targets, int32_t T, double *A, double *B, double *P,
                      double *E, double *logF, double *logG, double *llf, double *llb,
                      int32_t *status, int32_t nthreads)
{
    const lso_model m = *mp;
    const int32_t L = m.L, N = m.N;
    if (check_model(&m) || R < 0 || (R > 0 && !recips) || T < 0 || (T > 0 && !targets))
        return 1;
    for (int k = 0; k < T; ++k)
        if (targets[k] < 0 || targets[k] >= L)
            return 1;
    for (int r = 0; r < R; ++r)
        if (recips[r] < 0 || recips[r] >= N)
            return 1;
    lso_job proto;
    memset(&proto, 0, sizeof proto);
    proto.m = &m;
    proto.recips = recips;
    proto.R = R;
    proto.T = T;
    proto.targets = targets;
    proto.A = A;
    proto.B = B;
    proto.P = P;
    proto.E = E;
    proto.logF = logF;
    proto.logG = logG;
    proto.llf = llf;
    proto.llb = llb;
    proto.status = status;
    return run_jobs(&proto, nthreads, pass_worker);
}

/* Per-recipient gradients: grad_rho_rows [R][L-1], grad_mu [R], loglik [R]. */
int lso_gradient(const uint32_t *H, int64_t stride, int32_t N, int32_t L, const double *rho,
                 double mu, const int32_t *recips, int32_t R, double *grad_rho_rows,
                 double *grad_mu, double *loglik, int32_t *status, int32_t nthreads)
{
    lso_model m = {H, stride, N, L, rho, mu, NULL};
    if (check_model(&m) || R < 0 || (R > 0 && (!recips || !grad_mu || !loglik)) ||
        (L > 1 && !grad_rho_rows))
        return 1;
    for (int r = 0; r < R; ++r)
        if (recips[r] < 0 || recips[r] >= N)
            return 1;
    lso_job proto;
    memset(&proto, 0, sizeof proto);
    proto.m = &m;
    proto.recips = recips;
    proto.R = R;
    proto.grad_rho_rows = grad_rho_rows;
    proto.grad_mu = grad_mu;
    proto.llf = loglik;
    proto.status = status;
    return run_jobs(&proto, nthreads, grad_worker);
}

/* As lso_gradient with a per-variant mutation probability mu_vec[0..L-1];
 * grad_mu_rows [R][L] receives d log P / d mu^l per recipient and grad_mu [R]
 * their sum over l. */
int lso_gradient_v(const uint32_t *H, int64_t stride, int32_t N, int32_t L, const double *rho,
                   const double *mu_vec, const int32_t *recips, int32_t R, double *grad_rho_rows,
                   double *grad_mu_rows, double *grad_mu, double *loglik, int32_t *status,
                   int32_t nthreads)
{
    lso_model m = {H, stride, N, L, rho, 0.0, mu_vec};
    if (!mu_vec || check_model(&m) || R < 0 ||
        (R > 0 && (!recips || !grad_mu || !grad_mu_rows || !loglik)) || (L > 1 && !grad_rho_rows))
        return 1;
    for (int r = 0; r < R; ++r)
        if (recips[r] < 0 || recips[r] >= N)
            return 1;
    lso_job proto;
    memset(&proto, 0, sizeof proto);
    proto.m = &m;
    proto.recips = recips;
    proto.R = R;
    proto.grad_rho_rows = grad_rho_rows;
    proto.grad_mu = grad_mu;
    proto.grad_mu_rows = grad_mu_rows;
    proto.llf = loglik;
    proto.status = status;
    return run_jobs(&proto, nthreads, grad_worker);
}

/* The general gradient: a scalar mu or mu_vec (if not NULL; then
 * grad_mu_rows [R][L] is required), and the prior matrix Pi (NULL:
 * uniform). */
int lso_gradient_x(const uint32_t *H, int64_t stride, int32_t N, int32_t L, const double *rho,
                   double mu, const double *mu_vec, const double *Pi, const int32_t *recips,
                   int32_t R, double *grad_rho_rows, double *grad_mu_rows, double *grad_mu,
                   double *loglik, int32_t *status, int32_t nthreads)
{
    lso_model m = {H, stride, N, L, rho, mu, mu_vec, Pi};
    if (check_model(&m) || R < 0 || (R > 0 && (!recips || !grad_mu || !loglik)) ||
        (L > 1 && !grad_rho_rows) || (mu_vec && R > 0 && !grad_mu_rows))
        return 1;
    for (int r = 0; r < R; ++r)
        if (recips[r] < 0 || recips[r] >= N)
            return 1;
    lso_job proto;
    memset(&proto, 0, sizeof proto);
    proto.m = &m;
    proto.recips = recips;
    proto.R = R;
    proto.grad_rho_rows = grad_rho_rows;
    proto.grad_mu = grad_mu;
    proto.grad_mu_rows = mu_vec ? grad_mu_rows : NULL;
    proto.llf = loglik;
    proto.status = status;
    return run_jobs(&proto, nthreads, grad_worker);
}

/* Symmetrised distance from half distances: D[a][b] = E[a][b] + E[b][a],
 * D[a][a] = 0 (eq. distmat). E and D are N x N, recipient-major. */
void lso_symmetrise(const double *E, int32_t N, double *D)
{
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b)
            D[(int64_t)a * N + b] = (a == b) ? 0.0 : E[(int64_t)a * N + b] + E[(int64_t)b * N + a];
}

/* Recombination probabilities from map distances (eq. rho):
 *   rho_l = 1 - exp(-s m_l^gamma),  m_l = cM_l / 100,
 * the distance in Morgans (the paper's CalcRho takes centimorgans), with s
 * the scalar multiple N_e and gamma the power; evaluated with expm1. */
void lso_calc_rho(const double *cM, int32_t n, double s, double gamma, double *rho)
{
    for (int l = 0; l < n; ++l) {
        double m = cM[l] / 100.0;
        rho[l] = -expm1(-s * pow(m, gamma));
    }
}

/* Chain rule from d/d rho_l to the map parameters. With x_l = s m_l^gamma:
 *   d rho_l / d s     = m_l^gamma exp(-x_l)
 *   d rho_l / d gamma = s m_l^gamma log(m_l) exp(-x_l)   (0 where m_l = 0)
 * grad_s = sum_l grad_rho[l] d rho_l / d s, grad_gamma likewise. */
void lso_rho_map_grad(const double *cM, int32_t n, double s, double gamma,
                      const double *grad_rho, double *grad_s, double *grad_gamma)
{
    double gs = 0.0, gg = 0.0;
    for (int l = 0; l < n; ++l) {
        double m = cM[l] / 100.0;
        if (!(m > 0.0))
            continue;
        double mg = pow(m, gamma);
        double e = exp(-s * mg);
        gs += grad_rho[l] * mg * e;
        gg += grad_rho[l] * s * mg * log(m) * e;
    }
    *grad_s = gs;
    *grad_gamma = gg;
}

const char *lso_version(void) { return "ls_oracle 1.0 (FP64 reference, test infrastructure)"; }
