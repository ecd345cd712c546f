// Small kernels around the sweep: the internal row layout, the posterior /
// half-distance pass over stored forward and backward vectors (eq. postprob,
// eq. distmat) and the tiled symmetrisation of the distance matrix.
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
coef_tables_kernel(const double *__restrict__ rho, int32_t L, CoefScalars cs,
                   float *__restrict__ out) {
#pragma clang fp contract(off)
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L) return;
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
        } else if (l <= L - 2) {  // backward: variant l uses rho_l
            const double rr = rho[l];
            A = (1.0 - rr) * cs.cnum[k];
            B = rr * cs.bmul[k];
        }
        out[(int64_t)k * 2 * L + 2 * l] = (float)A;
        out[(int64_t)k * 2 * L + 2 * l + 1] = (float)B;
    }
}

hipError_t launch_coef_tables(const double *rho, int32_t L, const CoefScalars &cs, float *out,
                              hipStream_t st) {
    if (L < 1) return hipSuccess;
    hipLaunchKernelGGL(coef_tables_kernel, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, st,
                       rho, L, cs, out);
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

// ---------------------------------------------------------------------------
// Posterior rows. One workgroup per row q (recipient recips[q % R]):
//   Z = sum_j alpha_j beta_j,  p_j = alpha_j beta_j / Z (eps for all j != i
//   when Z == 0), E_j = -log(max(p_j, eps)) / 2, p_i = E_i = 0.
// The row is read twice (once for Z, once for the outputs), so P or E may
// overwrite alpha in place: every thread writes only entries it has read.
template <class T, class A, class B, class O>
__global__ void __launch_bounds__(256)
posterior_rows_kernel(const A *alpha, const B *__restrict__ beta, const int32_t *__restrict__ recips,
                      int32_t R, int32_t N, O *P, O *E) {
    __shared__ T red[256 / 64];
    const int64_t q = blockIdx.x;
    const int i = recips[q % R];
    const A *ar = alpha + q * N;
    const B *br = beta + q * N;
    T z = 0;
    for (int j = threadIdx.x; j < N; j += 256) z = fma((T)ar[j], (T)br[j], z);
    z = wave_sum(z);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wave] = z;
    __syncthreads();
    const T Z = (red[0] + red[1]) + (red[2] + red[3]);
    const T eps = (T)2.220446049250313080847e-16;
    const T invZ = (T)1 / Z;
    O *Pr = P ? P + q * N : nullptr;
    O *Er = E ? E + q * N : nullptr;
    for (int j = threadIdx.x; j < N; j += 256) {
        T p = (Z == (T)0) ? eps : (T)ar[j] * (T)br[j] * invZ;
        if (j == i) p = 0;
        const T qv = (p < eps) ? eps : p;  // NaN passes through
        const T e = (j == i) ? (T)0 : (T)-0.5 * log(qv);
        if (Pr) Pr[j] = (O)p;
        if (Er) Er[j] = (O)e;
    }
}

hipError_t launch_posterior_rows(const void *alpha, int alpha_half, const void *beta,
                                 int beta_half, const int32_t *recips, int32_t R, int64_t rows,
                                 int32_t N, int is_f64, void *P, void *E, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    const dim3 grid((unsigned)rows), block(256);
    if (is_f64) {
        hipLaunchKernelGGL((posterior_rows_kernel<double, double, double, double>), grid, block, 0,
                           st, (const double *)alpha, (const double *)beta, recips, R, N,
                           (double *)P, (double *)E);
    } else if (alpha_half && beta_half) {
        hipLaunchKernelGGL((posterior_rows_kernel<float, _Float16, _Float16, float>), grid, block,
                           0, st, (const _Float16 *)alpha, (const _Float16 *)beta, recips, R, N,
                           (float *)P, (float *)E);
    } else {
        hipLaunchKernelGGL((posterior_rows_kernel<float, float, float, float>), grid, block, 0, st,
                           (const float *)alpha, (const float *)beta, recips, R, N, (float *)P,
                           (float *)E);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// D = E + E^T with a zero diagonal, T matrices of N x N, in place allowed.
// Workgroup (bx, by, k) with by <= bx owns the tile pair (by, bx) / (bx, by):
// it reads both 64 x 64 tiles into LDS before writing either, so no other
// workgroup touches them and D may alias E.
template <class X>
__global__ void __launch_bounds__(256)
symmetrise_kernel(const X *E, X *D, int32_t N) {
    const int bx = blockIdx.x, by = blockIdx.y;
    if (by > bx) return;
    __shared__ X ta[64][65];
    __shared__ X tb[64][65];
    const int64_t base = (int64_t)blockIdx.z * N * N;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    const int r0 = by * 64, c0 = bx * 64;
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

hipError_t launch_symmetrise(const void *E, void *D, int32_t N, int32_t T, int is_f64,
                             hipStream_t st) {
    if (T <= 0 || N <= 0) return hipSuccess;
    const int nb = (N + 63) / 64;
    const dim3 grid(nb, nb, T), block(256);
    if (is_f64)
        hipLaunchKernelGGL((symmetrise_kernel<double>), grid, block, 0, st, (const double *)E,
                           (double *)D, N);
    else
        hipLaunchKernelGGL((symmetrise_kernel<float>), grid, block, 0, st, (const float *)E,
                           (float *)D, N);
    return hipGetLastError();
}

}  // namespace lsk
