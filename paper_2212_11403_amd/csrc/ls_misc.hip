// Small kernels around the sweep: the internal row layout, the posterior /
// half-distance pass over stored forward and backward vectors (eq. postprob,
// eq. distmat) and the tiled symmetrisation of the distance matrix.
#include <type_traits>

#include "ls_device.h"

namespace lsk {

// Internal rows: row l holds the full 64-haplotype words W_0..W_{NF-1} twice
// in a row, then the partial last word (bits past N cleared), then zeros:
//   Hr[l][q] = W_{q mod NF}  (q < 2 NF),  Hr[l][2 NF] = partial word.
// The sweep reads a recipient's rotated words as one contiguous run.
__global__ void repack_kernel(const uint32_t *__restrict__ H, int64_t stride_words, int32_t N,
                              int32_t L, uint64_t *__restrict__ Hr, int64_t hr_stride) {
    const int64_t total = (int64_t)L * hr_stride;
    const int NF = N >> 6;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = idx / hr_stride;
        const int q = (int)(idx - l * hr_stride);
        const uint32_t *row = H + l * stride_words;
        uint64_t w = 0;
        if (q < 2 * NF) {
            const int wi = q < NF ? q : q - NF;
            w = (uint64_t)row[2 * wi] | ((uint64_t)row[2 * wi + 1] << 32);
        } else if (q == 2 * NF && (N & 63) != 0) {
            const int rem = N & 63;
            w = (uint64_t)row[2 * NF];
            if (rem > 32) w |= (uint64_t)row[2 * NF + 1] << 32;
            w &= (rem == 64) ? ~0ull : ((1ull << rem) - 1ull);
        }
        Hr[idx] = w;
    }
}

hipError_t launch_repack(const uint32_t *H, int64_t stride_words, int32_t N, int32_t L,
                         uint64_t *Hr, int64_t hr_stride, hipStream_t st) {
    const int64_t total = (int64_t)L * hr_stride;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(repack_kernel, dim3((unsigned)blocks), dim3(256), 0, st, H, stride_words,
                       N, L, Hr, hr_stride);
    return hipGetLastError();
}

// One thread per variant writes its pair in all coefficient tables.
__global__ void __launch_bounds__(256)
coef_tables_kernel(const double *__restrict__ rho, const double *__restrict__ mu_vec, int32_t L,
                   CoefScalars cs, float *__restrict__ out) {
#pragma clang fp contract(off)
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L) return;
    // the divisor of this variant's emission pair (as in sweep_emissions)
    double unit = cs.unit;
    if (mu_vec) {
        const double mu = mu_vec[l];
        const double omu = (1.0 - 2.0 * mu) + mu;
        unit = omu >= mu ? omu : mu;
    }
#pragma unroll
    for (int k = 0; k < kCoefTables; ++k) {
        double A = 0.0, B = 0.0;
        if ((k & 1) == 0) {  // forward: variant l uses rho_{l-1}
            if (l == 0) {
                B = cs.bmul[k];
            } else {
                const double rr = rho[l - 1];
                A = (1.0 - rr) * cs.cnum[k];
                B = rr * cs.bmul[k];
            }
            if (cs.fold[k]) {
                A *= unit;
                B *= unit;
            }
        } else if (l <= L - 2) {  // backward: variant l uses rho_l
            const double rr = rho[l];
            A = (1.0 - rr) * cs.cnum[k];
            B = rr * cs.bmul[k];
        }
        out[(int64_t)k * 2 * L + 2 * l] = (float)A;
        out[(int64_t)k * 2 * L + 2 * l + 1] = (float)B;
    }
}

hipError_t launch_coef_tables(const double *rho, const double *mu_vec, int32_t L,
                              const CoefScalars &cs, float *out, hipStream_t st) {
    if (L < 1) return hipSuccess;
    hipLaunchKernelGGL(coef_tables_kernel, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, st,
                       rho, mu_vec, L, cs, out);
    return hipGetLastError();
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

// 16-byte vectors (native vector types: loads, stores and the streaming-store
// builtin take them directly)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Posterior rows. One workgroup per row (k, r) = (blockIdx.y, blockIdx.x) of
// recipient i = recips[r]; the forward row and the outputs sit at
// k ts + r rs, the backward row at (k R + r) N:
//   Z = sum_j alpha_j beta_j,  p_j = alpha_j beta_j / Z (eps for all j != i
//   when Z == 0), E_j = -log(max(p_j, eps)) / 2, p_i = E_i = 0.
// The row is read twice (once for Z, once for the outputs), so P or E may
// overwrite alpha in place: every thread writes only entries it has read.
template <class T, class A, class B, class O>
__global__ void __launch_bounds__(256)
posterior_rows_kernel(const A *alpha, const B *__restrict__ beta, const int32_t *__restrict__ recips,
                      int32_t R, int64_t ts, int64_t rs, int32_t N, O *P, O *E) {
    __shared__ T red[256 / 64];
    const int r = blockIdx.x;
    const int64_t k = blockIdx.y;
    const int i = recips[r];
    const int64_t off = k * ts + (int64_t)r * rs;
    const A *ar = alpha + off;
    const B *br = beta + (k * R + r) * (int64_t)N;
    T z = 0;
    for (int j = threadIdx.x; j < N; j += 256) z = fma((T)ar[j], (T)br[j], z);
    z = wave_sum(z);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wave] = z;
    __syncthreads();
    const T Z = (red[0] + red[1]) + (red[2] + red[3]);
    const T eps = (T)2.220446049250313080847e-16;
    const T invZ = (T)1 / Z;
    O *Pr = P ? P + off : nullptr;
    O *Er = E ? E + off : nullptr;
    for (int j = threadIdx.x; j < N; j += 256) {
        T p = (Z == (T)0) ? eps : (T)ar[j] * (T)br[j] * invZ;
        if (j == i) p = 0;
        const T qv = (p < eps) ? eps : p;  // NaN passes through
        const T e = (j == i) ? (T)0 : (T)-0.5 * log(qv);
        if (Pr) Pr[j] = (O)p;
        if (Er) Er[j] = (O)e;
    }
}

// The same rows with the products alpha_j beta_j held in registers, for
// N <= 1024 K W (W = 16 / sizeof(T) elements per 16-byte vector, N, ts and
// rs multiples of W): alpha and beta are read once, with 16-byte loads, and
// P / E are written with streaming stores. One workgroup of 1024 threads per
// row; each thread keeps the products of the entries it writes.
template <class T, int K>
__global__ void __launch_bounds__(1024)
posterior_rows_reg_kernel(const T *alpha, const T *__restrict__ beta,
                          const int32_t *__restrict__ recips, int32_t R, int64_t ts, int64_t rs,
                          int32_t N, T *P, T *E) {
    using V = typename std::conditional<sizeof(T) == 4, f32x4, f64x2>::type;
    constexpr int W = 16 / (int)sizeof(T);
    __shared__ T red[16];
    const int r = blockIdx.x;
    const int64_t k = blockIdx.y;
    const int i = recips[r];
    const int64_t off = k * ts + (int64_t)r * rs;
    const T *ar = alpha + off;
    const T *br = beta + (k * R + r) * (int64_t)N;
    T w[K][W];
    T z = 0;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const int j0 = ((int)threadIdx.x + 1024 * q) * W;
        V a = {}, b = {};
        if (j0 < N) {
            a = *reinterpret_cast<const V *>(ar + j0);
            b = *reinterpret_cast<const V *>(br + j0);
        }
        const T *xa = reinterpret_cast<const T *>(&a);
        const T *xb = reinterpret_cast<const T *>(&b);
#pragma unroll
        for (int e = 0; e < W; ++e) {
            w[q][e] = xa[e] * xb[e];
            z += w[q][e];
        }
    }
    z = wave_sum(z);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wave] = z;
    __syncthreads();
    T t[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) t[q] = red[q];
#pragma unroll
    for (int h = 1; h < 16; h *= 2)
#pragma unroll
        for (int q = 0; q + h < 16; q += 2 * h) t[q] += t[q + h];
    const T Z = t[0];
    const T eps = (T)2.220446049250313080847e-16;
    const T invZ = (T)1 / Z;
    T *Pr = P ? P + off : nullptr;
    T *Er = E ? E + off : nullptr;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const int j0 = ((int)threadIdx.x + 1024 * q) * W;
        if (j0 >= N) continue;
        V vp, ve;
        T *xp = reinterpret_cast<T *>(&vp);
        T *xe = reinterpret_cast<T *>(&ve);
#pragma unroll
        for (int e = 0; e < W; ++e) {
            const int j = j0 + e;
            T pv = (Z == (T)0) ? eps : w[q][e] * invZ;
            if (j == i) pv = 0;
            const T qv = (pv < eps) ? eps : pv;  // NaN passes through
            xp[e] = pv;
            xe[e] = (j == i) ? (T)0 : (T)-0.5 * log(qv);
        }
        if (Pr) __builtin_nontemporal_store(vp, reinterpret_cast<V *>(Pr + j0));
        if (Er) __builtin_nontemporal_store(ve, reinterpret_cast<V *>(Er + j0));
    }
}

hipError_t launch_posterior_rows(const void *alpha, int alpha_half, const void *beta,
                                 int beta_half, const int32_t *recips, int32_t R, int32_t T,
                                 int64_t ts, int64_t rs, int32_t N, int is_f64, void *P, void *E,
                                 hipStream_t st) {
    if (R <= 0 || T <= 0) return hipSuccess;
    if (T > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)R, (unsigned)T), block(256);
    // rows that fit the register kernel: full-precision inputs, N and the
    // strides multiples of the vector width, at most 16 elements per thread,
    // 16-byte aligned
    auto aligned = [](const void *x) { return (reinterpret_cast<uintptr_t>(x) & 15) == 0; };
    const int w = is_f64 ? 2 : 4;
    const bool reg = !alpha_half && !beta_half && N % w == 0 && ts % w == 0 && rs % w == 0 &&
                     N <= 1024 * 16 && aligned(alpha) && aligned(beta) && aligned(P) &&
                     aligned(E);
    if (reg) {
        if (is_f64)
            hipLaunchKernelGGL((posterior_rows_reg_kernel<double, 8>), grid, dim3(1024), 0, st,
                               (const double *)alpha, (const double *)beta, recips, R, ts, rs, N,
                               (double *)P, (double *)E);
        else
            hipLaunchKernelGGL((posterior_rows_reg_kernel<float, 4>), grid, dim3(1024), 0, st,
                               (const float *)alpha, (const float *)beta, recips, R, ts, rs, N,
                               (float *)P, (float *)E);
        return hipGetLastError();
    }
    if (is_f64) {
        hipLaunchKernelGGL((posterior_rows_kernel<double, double, double, double>), grid, block, 0,
                           st, (const double *)alpha, (const double *)beta, recips, R, ts, rs, N,
                           (double *)P, (double *)E);
    } else if (alpha_half && beta_half) {
        hipLaunchKernelGGL((posterior_rows_kernel<float, _Float16, _Float16, float>), grid, block,
                           0, st, (const _Float16 *)alpha, (const _Float16 *)beta, recips, R, ts,
                           rs, N, (float *)P, (float *)E);
    } else {
        hipLaunchKernelGGL((posterior_rows_kernel<float, float, float, float>), grid, block, 0, st,
                           (const float *)alpha, (const float *)beta, recips, R, ts, rs, N,
                           (float *)P, (float *)E);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// D = E + E^T with a zero diagonal, T matrices of N x N, in place allowed.
// Workgroup (p, k) owns the tile pair (by, bx) / (bx, by), by <= bx, of
// matrix k, where p counts the pairs of the upper triangle row by row: it
// reads both 64 x 64 tiles into LDS before writing either, so no other
// workgroup touches them and D may alias E. With VEC (N a multiple of the
// 16-byte vector) every lane moves 16 bytes per load and store; D is written
// with streaming stores (it is not read again here).
__device__ __forceinline__ void tile_pair(int64_t p, int nb, int &by, int &bx) {
    // first pair of row b: b nb - b (b - 1) / 2
    const double a = 2.0 * nb + 1.0;
    int b = (int)((a - sqrt(a * a - 8.0 * (double)p)) * 0.5);
    auto first = [&](int r) { return (int64_t)r * nb - (int64_t)r * (r - 1) / 2; };
    while (b > 0 && first(b) > p) --b;
    while (b + 1 < nb && first(b + 1) <= p) ++b;
    by = b;
    bx = b + (int)(p - first(b));
}

template <class X, bool VEC>
__global__ void __launch_bounds__(256)
symmetrise_kernel(const X *E, X *D, int32_t N, int32_t nb) {
    using V = typename std::conditional<sizeof(X) == 4, f32x4, f64x2>::type;
    constexpr int W = 16 / (int)sizeof(X);  // elements per vector
    int by, bx;
    tile_pair(blockIdx.x, nb, by, bx);
    __shared__ X ta[64][65];
    __shared__ X tb[VEC ? 1 : 64][65];
    const int64_t base = (int64_t)blockIdx.y * N * N;
    const int r0 = by * 64, c0 = bx * 64;
    if constexpr (VEC) {
        // lane: W consecutive columns of one row; RP rows per pass, IT passes.
        // All loads of a lane are issued before the first wait; tiles fully
        // inside the matrix (all but the last tile row and column) skip the
        // bounds checks.
        constexpr int CV = 64 / W, RP = 256 / CV, IT = 64 / RP;
        const int cv = threadIdx.x % CV, rp = threadIdx.x / CV, cc = cv * W;
        const bool full = r0 + 64 <= N && c0 + 64 <= N;
        const X *ea = E + base + (int64_t)(r0 + rp) * N + c0 + cc;
        const X *eb = E + base + (int64_t)(c0 + rp) * N + r0 + cc;
        V va[IT], vb[IT];
        if (full) {
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                va[it] = *reinterpret_cast<const V *>(ea + (int64_t)it * RP * N);
                vb[it] = *reinterpret_cast<const V *>(eb + (int64_t)it * RP * N);
            }
        } else {
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int rr = rp + it * RP;
                va[it] = (r0 + rr < N && c0 + cc < N)
                             ? *reinterpret_cast<const V *>(ea + (int64_t)it * RP * N)
                             : V{};
                vb[it] = (c0 + rr < N && r0 + cc < N)
                             ? *reinterpret_cast<const V *>(eb + (int64_t)it * RP * N)
                             : V{};
            }
        }
        // Both tiles are now in registers, so D (which may alias E) can be
        // written at once. The transposed operand goes through one LDS tile
        // used twice: tile b for the first output, then tile a.
#pragma unroll
        for (int it = 0; it < IT; ++it)
#pragma unroll
            for (int k = 0; k < W; ++k) ta[rp + it * RP][cc + k] = vb[it][k];
        __syncthreads();
        X *da = D + base + (int64_t)(r0 + rp) * N + c0 + cc;
        X *db = D + base + (int64_t)(c0 + rp) * N + r0 + cc;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int rr = rp + it * RP;
            V o;
#pragma unroll
            for (int k = 0; k < W; ++k)
                o[k] = (r0 + rr == c0 + cc + k) ? (X)0 : va[it][k] + ta[cc + k][rr];
            if (full || (r0 + rr < N && c0 + cc < N))
                __builtin_nontemporal_store(o, reinterpret_cast<V *>(da + (int64_t)it * RP * N));
        }
        if (by != bx) {
            __syncthreads();
#pragma unroll
            for (int it = 0; it < IT; ++it)
#pragma unroll
                for (int k = 0; k < W; ++k) ta[rp + it * RP][cc + k] = va[it][k];
            __syncthreads();
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int rr = rp + it * RP;
                V o;
#pragma unroll
                for (int k = 0; k < W; ++k) o[k] = vb[it][k] + ta[cc + k][rr];
                if (full || (c0 + rr < N && r0 + cc < N))
                    __builtin_nontemporal_store(o,
                                                reinterpret_cast<V *>(db + (int64_t)it * RP * N));
            }
        }
    } else {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
        // ta = E[r0.., c0..], tb = E[c0.., r0..]
        for (int rr = ty; rr < 64; rr += 4) {
            const int r = r0 + rr, c = c0 + tx;
            ta[rr][tx] = (r < N && c < N) ? E[base + (int64_t)r * N + c] : (X)0;
            const int r2 = c0 + rr, c2 = r0 + tx;
            tb[rr][tx] = (r2 < N && c2 < N) ? E[base + (int64_t)r2 * N + c2] : (X)0;
        }
        __syncthreads();
        for (int rr = ty; rr < 64; rr += 4) {
            const int r = r0 + rr, c = c0 + tx;
            if (r < N && c < N) D[base + (int64_t)r * N + c] = (r == c) ? (X)0 : ta[rr][tx] + tb[tx][rr];
            const int r2 = c0 + rr, c2 = r0 + tx;
            if (by != bx && r2 < N && c2 < N)
                D[base + (int64_t)r2 * N + c2] = tb[rr][tx] + ta[tx][rr];
        }
    }
}

hipError_t launch_symmetrise(const void *E, void *D, int32_t N, int32_t T, int is_f64,
                             hipStream_t st) {
    if (T <= 0 || N <= 0) return hipSuccess;
    if (T > 65535) return hipErrorInvalidValue;
    const int nb = (N + 63) / 64;
    const int64_t pairs = (int64_t)nb * (nb + 1) / 2;
    if (pairs > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid((unsigned)pairs, (unsigned)T), block(256);
    // vectors need rows that start on 16 bytes: N a multiple of the vector
    // width and a 16-byte aligned base
    const int w = is_f64 ? 2 : 4;
    const bool vec = N % w == 0 && (reinterpret_cast<uintptr_t>(E) & 15) == 0 &&
                     (reinterpret_cast<uintptr_t>(D) & 15) == 0;
    if (is_f64) {
        if (vec)
            hipLaunchKernelGGL((symmetrise_kernel<double, true>), grid, block, 0, st,
                               (const double *)E, (double *)D, N, nb);
        else
            hipLaunchKernelGGL((symmetrise_kernel<double, false>), grid, block, 0, st,
                               (const double *)E, (double *)D, N, nb);
    } else {
        if (vec)
            hipLaunchKernelGGL((symmetrise_kernel<float, true>), grid, block, 0, st,
                               (const float *)E, (float *)D, N, nb);
        else
            hipLaunchKernelGGL((symmetrise_kernel<float, false>), grid, block, 0, st,
                               (const float *)E, (float *)D, N, nb);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Emission tables of a per-variant mu, from (1-H)(1-2mu)+mu (appendix A.3) in
// FP64: the FP64 pair as is; the FP32 pair divided by its larger member and
// rounded once, with the log of that divisor (all threads, into
// lu_prefix[l+1]); then the prefix sums of those logs in index order (one
// thread, so the sums are fixed).
__global__ void __launch_bounds__(256)
emission_tables_kernel(const double *__restrict__ mu_vec, int32_t L, double *__restrict__ em64,
                       float *__restrict__ em32, double *__restrict__ lu_prefix) {
    for (int l = threadIdx.x; l < L; l += 256) {
        const double mu = mu_vec[l];
        const double omu = (1.0 - 2.0 * mu) + mu;
        em64[2 * l] = omu;
        em64[2 * l + 1] = mu;
        const double unit = omu >= mu ? omu : mu;
        em32[2 * l] = (float)(omu / unit);
        em32[2 * l + 1] = (float)(mu / unit);
        lu_prefix[l + 1] = log(unit);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        lu_prefix[0] = 0.0;
        for (int l = 0; l < L; ++l) {
            acc += lu_prefix[l + 1];
            lu_prefix[l + 1] = acc;
        }
    }
}

hipError_t launch_emission_tables(const double *mu_vec, int32_t L, double *em64, float *em32,
                                  double *lu_prefix, hipStream_t st) {
    hipLaunchKernelGGL(emission_tables_kernel, dim3(1), dim3(256), 0, st, mu_vec, L, em64, em32,
                       lu_prefix);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Checks of a prior copying matrix (one workgroup per recipient's column):
// the sum of the column without its diagonal (NaN if any entry is negative,
// above 1 or not finite), strided per-thread sums in index order, then a
// fixed tree; and a 64-bit hash of the whole column: the wrap-around sum
// over entries of a mixed (value bits, index) word. Integer sums do not
// depend on their order, and two columns that differ in any entry (a
// change that keeps every moment of the column included) differ in the
// hash with overwhelming probability.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256)
prior_stats_kernel(const double *__restrict__ prior, int32_t N, double *__restrict__ out) {
    __shared__ double ps[256];
    __shared__ uint64_t ph[256];
    __shared__ int pbad[256];
    const int i = blockIdx.x;
    const double *row = prior + (int64_t)i * N;
    double s = 0.0;
    uint64_t h = 0;
    int bad = 0;
    for (int j = threadIdx.x; j < N; j += 256) {
        const double x = row[j];
        if (!(x >= 0.0 && x <= 1.0)) bad = 1;
        if (j != i) s += x;
        h += mix64((uint64_t)__double_as_longlong(x) ^ ((uint64_t)(j + 1) * 0x9e3779b97f4a7c15ull));
    }
    ps[threadIdx.x] = s;
    ph[threadIdx.x] = h;
    pbad[threadIdx.x] = bad;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            ps[threadIdx.x] += ps[threadIdx.x + k];
            ph[threadIdx.x] += ph[threadIdx.x + k];
            pbad[threadIdx.x] |= pbad[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * i] = pbad[0] ? __builtin_nan("") : ps[0];
        out[2 * i + 1] = __longlong_as_double((long long)ph[0]);
    }
}

hipError_t launch_prior_stats(const double *prior, int32_t N, double *out, hipStream_t st) {
    hipLaunchKernelGGL(prior_stats_kernel, dim3(N), dim3(256), 0, st, prior, N, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Recombination map (eq. rho): rho_l = 1 - exp(-s m_l^gamma) with m_l =
// cM_l / 100 the distance in Morgans (the argument is in centimorgans, as
// the paper's CalcRho takes it), evaluated with expm1.
__global__ void calc_rho_kernel(const double *__restrict__ cM, int32_t n, double s, double gamma,
                                double *__restrict__ rho) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double m = cM[i] / 100.0;
        rho[i] = -expm1(-s * pow(m, gamma));
    }
}

hipError_t launch_calc_rho(const double *cM, int32_t n, double s, double gamma, double *rho,
                           hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(calc_rho_kernel, dim3(blocks), dim3(256), 0, st, cM, n, s, gamma, rho);
    return hipGetLastError();
}

// Chain rule to the map parameters: with x_l = s m_l^gamma,
//   d rho_l / d s = m_l^gamma e^{-x_l},  d rho_l / d gamma = s m_l^gamma log(m_l) e^{-x_l}
// (0 where m_l = 0); out = {sum_l g_l d rho_l / d s, sum_l g_l d rho_l / d gamma}.
// One workgroup: per-thread strided sums in index order, then a fixed tree,
// so the result does not depend on scheduling.
__global__ void __launch_bounds__(256)
rho_map_grad_kernel(const double *__restrict__ cM, int32_t n, double s, double gamma,
                    const double *__restrict__ g, double *__restrict__ out) {
    __shared__ double ps[256], pg[256];
    double as = 0.0, ag = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double m = cM[i] / 100.0;
        if (m > 0.0) {
            const double mg = pow(m, gamma);
            const double e = exp(-s * mg);
            as += g[i] * mg * e;
            ag += g[i] * s * mg * log(m) * e;
        }
    }
    ps[threadIdx.x] = as;
    pg[threadIdx.x] = ag;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            ps[threadIdx.x] += ps[threadIdx.x + h];
            pg[threadIdx.x] += pg[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = ps[0];
        out[1] = pg[0];
    }
}

hipError_t launch_rho_map_grad(const double *cM, int32_t n, double s, double gamma,
                               const double *g, double *out, hipStream_t st) {
    hipLaunchKernelGGL(rho_map_grad_kernel, dim3(1), dim3(256), 0, st, cM, n, s, gamma, g, out);
    return hipGetLastError();
}

}  // namespace lsk
