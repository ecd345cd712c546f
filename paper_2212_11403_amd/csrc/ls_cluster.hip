// Consumers of the distance matrix: average pairwise linkage (the paper
// clusters a distance matrix with Sokal and Michener's method, section 6)
// and the standardisation of a recipient's half-distance row with the
// zero-deviation rule of section 2.2.
//
// Average linkage is a sequence of N-1 dependent merges, each cheap (a few
// passes over rows of N entries), so one workgroup runs all merges of one
// matrix and T matrices run side by side. The first nearest-neighbour pass
// reads every entry once and runs as its own kernel over all rows of all
// matrices, at full memory bandwidth.
//
// State per occupied slot k: nn[k], the occupied slot nearest to k (ties: the
// smallest slot), and nd[k], its distance. A merge takes the slot pair at the
// smallest distance (ties: the smallest slot pair; a NaN distance after every
// number), keeps the merged cluster in the smaller slot a, empties b, and
// updates row a and column a with d = (|A| d_a + |B| d_b) / (|A| + |B|)
// (each operation rounded in that order). Rows whose nearest slot was a or b
// are rescanned; every other row only compares its new distance to a.
#include <math.h>

#include <cstdlib>
#include <mutex>

#include "ls_cluster.h"
#include "ls_device.h"

namespace lsk {

namespace {

// (d1, p1, q1) before (d2, p2, q2): by distance, NaN after every number,
// then by slot pair.
template <class T>
__device__ __forceinline__ bool before(T d1, int p1, int q1, T d2, int p2, int q2) {
    const bool n1 = isnan(d1), n2 = isnan(d2);
    if (n1 != n2) return n2;
    if (!n1 && d1 != d2) return d1 < d2;
    return p1 < p2 || (p1 == p2 && q1 < q2);
}

template <class T>
struct Cand {
    T d;
    int p, q;
};

template <class T>
__device__ __forceinline__ Cand<T> pick(Cand<T> x, Cand<T> y) {
    if (y.p < 0) return x;
    if (x.p < 0) return y;
    return before(y.d, y.p, y.q, x.d, x.p, x.q) ? y : x;
}

template <class T>
__device__ __forceinline__ Cand<T> shfl_cand(Cand<T> c, int src) {
    Cand<T> o;
    if constexpr (sizeof(T) == 4) {
        o.d = __shfl(c.d, src);
    } else {
        const int lo = __shfl(__double2loint(c.d), src), hi = __shfl(__double2hiint(c.d), src);
        o.d = __hiloint2double(hi, lo);
    }
    o.p = __shfl(c.p, src);
    o.q = __shfl(c.q, src);
    return o;
}

// The first of the candidates of one wave (every lane gets it).
template <class T>
__device__ __forceinline__ Cand<T> wave_pick(Cand<T> c) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        Cand<T> o = shfl_cand(c, lane ^ off);
        c = pick(c, o);
    }
    return c;
}

// The first candidate of the workgroup (every thread gets it). `buf` holds
// one candidate per wave.
template <class T>
__device__ __forceinline__ Cand<T> block_pick(Cand<T> c, Cand<T> *buf) {
    c = wave_pick(c);
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) buf[wave] = c;
    __syncthreads();
    Cand<T> r{(T)0, -1, -1};
    for (int w = 0; w < nw; ++w) r = pick(r, buf[w]);
    return r;
}

// Nearest occupied slot of row i over the slots a thread visits.
template <class T>
__device__ __forceinline__ Cand<T> row_nearest(const T *row, const uint8_t *live, int N, int i,
                                               int t0, int step) {
    Cand<T> c{(T)0, -1, -1};
    for (int k = t0; k < N; k += step) {
        if (k == i || !live[k]) continue;
        Cand<T> x{row[k], k, 0};
        c = pick(c, x);
    }
    return c;
}

}  // namespace

// One wave per row: nn[k] and nd[k] of every row of every matrix.
template <class T>
__global__ void __launch_bounds__(256)
linkage_init_kernel(const T *__restrict__ D, int32_t N, int32_t T_, size_t ws_stride, char *ws) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= (int64_t)N * T_) return;
    const int t = (int)(row / N), i = (int)(row - (int64_t)t * N);
    char *w = ws + (size_t)t * ws_stride;
    int32_t *nn = reinterpret_cast<int32_t *>(w);
    T *nd = reinterpret_cast<T *>(w + 256 * (((size_t)N * 4 + 255) / 256));
    const T *r = D + ((int64_t)t * N + i) * N;
    Cand<T> c{(T)0, -1, -1};
    for (int k = threadIdx.x & 63; k < N; k += 64) {
        if (k == i) continue;
        Cand<T> x{r[k], k, 0};
        c = pick(c, x);
    }
    c = wave_pick(c);
    if ((threadIdx.x & 63) == 0) {
        nn[i] = c.p;
        nd[i] = c.d;
    }
}

// Bytes of local memory the merge kernel keeps nn, nd and the occupancy
// flags of one matrix in (the rest of its state stays in the workspace).
__host__ __device__ constexpr size_t linkage_lds_bytes(int32_t N, size_t tsize) {
    return 16 * (((size_t)N * 4 + 15) / 16) + 16 * (((size_t)N * tsize + 15) / 16) + (size_t)N;
}

// All N-1 merges of matrix blockIdx.x, then its leaf order. With SMEM the
// per-slot state every merge scans (nearest slot, its distance, occupancy)
// lives in local memory (linkage_lds_bytes), copied from the workspace the
// first pass filled; the candidate search then reads no global memory.
template <class T, bool SMEM>
__global__ void __launch_bounds__(1024)
linkage_kernel(T *__restrict__ D, int32_t N, size_t ws_stride, char *ws, double *__restrict__ Z,
               int32_t *__restrict__ order) {
#pragma clang fp contract(off)
    __shared__ Cand<T> buf[16];
    __shared__ int nflag;
    extern __shared__ __align__(16) char lds[];
    const int t = blockIdx.x;
    T *Dm = D + (int64_t)t * N * N;
    char *w = ws + (size_t)t * ws_stride;
    const size_t a4 = 256 * (((size_t)N * 4 + 255) / 256);
    const size_t aT = 256 * (((size_t)N * sizeof(T) + 255) / 256);
    int32_t *size = reinterpret_cast<int32_t *>(w + a4 + aT);
    int32_t *id = reinterpret_cast<int32_t *>(w + 2 * a4 + aT);
    int32_t *flag = reinterpret_cast<int32_t *>(w + 3 * a4 + aT);
    int32_t *nn;
    T *nd;
    uint8_t *live;
    const int tid = threadIdx.x, nth = blockDim.x;
    if constexpr (SMEM) {
        const size_t s4 = 16 * (((size_t)N * 4 + 15) / 16);
        const size_t sT = 16 * (((size_t)N * sizeof(T) + 15) / 16);
        nn = reinterpret_cast<int32_t *>(lds);
        nd = reinterpret_cast<T *>(lds + s4);
        live = reinterpret_cast<uint8_t *>(lds + s4 + sT);
        const int32_t *gnn = reinterpret_cast<const int32_t *>(w);
        const T *gnd = reinterpret_cast<const T *>(w + a4);
        for (int k = tid; k < N; k += nth) {
            nn[k] = gnn[k];
            nd[k] = gnd[k];
        }
    } else {
        nn = reinterpret_cast<int32_t *>(w);
        nd = reinterpret_cast<T *>(w + a4);
        live = reinterpret_cast<uint8_t *>(w + 4 * a4 + aT);
    }
    double *Zm = Z + (int64_t)t * (N - 1) * 4;
    for (int k = tid; k < N; k += nth) {
        size[k] = 1;
        id[k] = k;
        live[k] = 1;
    }
    __syncthreads();
    for (int m = 0; m + 1 < N; ++m) {
        // the first candidate pair over all occupied slots
        Cand<T> c{(T)0, -1, -1};
        for (int i = tid; i < N; i += nth) {
            if (!live[i]) continue;
            const int j = nn[i];
            Cand<T> x{nd[i], i < j ? i : j, i < j ? j : i};
            c = pick(c, x);
        }
        c = block_pick(c, buf);
        const int a = c.p, b = c.q;
        // (two occupied slots always give a candidate; the check keeps every
        // index below in range whatever D holds)
        if (a < 0 || b <= a || b >= N) break;
        const int na = size[a], nb = size[b];
        const T fa = (T)na, fb = (T)nb, fn = (T)(na + nb);
        if (tid == 0) nflag = 0;
        __syncthreads();
        // row and column a of the merged cluster; rows whose nearest slot was
        // a or b are listed for a rescan, the others compare with the new
        // distance to a
        T *ra = Dm + (int64_t)a * N;
        const T *rb = Dm + (int64_t)b * N;
        for (int k = tid; k < N; k += nth) {
            if (!live[k] || k == a || k == b) continue;
            const T x = fa * ra[k];
            const T y = fb * rb[k];
            const T s = x + y;
            const T d = s / fn;
            ra[k] = d;
            Dm[(int64_t)k * N + a] = d;
            const int j = nn[k];
            if (j == a || j == b) {
                flag[atomicAdd(&nflag, 1)] = k;
            } else if (before(d, a, 0, nd[k], j, 0)) {
                nn[k] = a;
                nd[k] = d;
            }
        }
        __syncthreads();
        if (tid == 0) {
            Zm[4 * m + 0] = (double)(id[a] < id[b] ? id[a] : id[b]);
            Zm[4 * m + 1] = (double)(id[a] < id[b] ? id[b] : id[a]);
            Zm[4 * m + 2] = (double)c.d;
            Zm[4 * m + 3] = (double)(na + nb);
            live[b] = 0;
            size[a] = na + nb;
            id[a] = N + m;
            flag[nflag] = a;
        }
        __syncthreads();
        const int nf = nflag + 1;
        // rescan the listed rows (the merged row last); the writes to
        // nn/nd of a row are made by thread 0 after the whole workgroup
        // agreed on the candidate
        for (int f = 0; f < nf; ++f) {
            const int k = flag[f];
            Cand<T> r = row_nearest(Dm + (int64_t)k * N, live, N, k, tid, nth);
            r = block_pick(r, buf);
            if (tid == 0) {
                nn[k] = r.p;
                nd[k] = r.d;
            }
        }
        __syncthreads();
    }
    // leaf order: depth first from the last merge, the smaller id first
    if (order && tid == 0) {
        int32_t *ord = order + (int64_t)t * N;
        if (N == 1) {
            ord[0] = 0;
        } else {
            int32_t *stack = flag;  // N entries suffice: the depth of the pending list
            int top = 0, out = 0;
            stack[top++] = 2 * N - 2;
            // ids in Z are below 2N-1 and every merge id appears once, so at
            // most N entries are pending and N leaves come out; the bounds
            // only guard the indices
            while (top > 0 && out < N) {
                const int cl = stack[--top];
                if (cl < N) {
                    ord[out++] = cl;
                    continue;
                }
                if (cl > 2 * N - 2 || top + 2 > N) break;
                const double *z = Zm + 4 * (int64_t)(cl - N);
                stack[top++] = (int32_t)z[1];
                stack[top++] = (int32_t)z[0];
            }
        }
    }
}

size_t linkage_workspace_bytes(int32_t N, int32_t T, int is_f64) {
    const size_t a4 = 256 * (((size_t)N * 4 + 255) / 256);
    const size_t aT = 256 * (((size_t)N * (is_f64 ? 8 : 4) + 255) / 256);
    const size_t a1 = 256 * (((size_t)N + 255) / 256);
    return (size_t)T * (4 * a4 + aT + a1);
}

namespace {

// Local memory a workgroup may allocate on the current device (0 if the
// runtime does not say), asked once per device.
size_t max_group_lds() {
    static std::mutex mu;
    static int known[64] = {};
    static size_t bytes[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lock(mu);
    if (!known[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 0;
        bytes[dev] = v > 0 ? (size_t)v : 0;
        known[dev] = 1;
    }
    return bytes[dev];
}

template <class T>
hipError_t launch_linkage_t(T *D, int32_t N, int32_t T_, double *Z, int32_t *order, char *w,
                            hipStream_t st) {
    const size_t stride = linkage_workspace_bytes(N, 1, sizeof(T) == 8);
    const int64_t rows = (int64_t)N * T_;
    const int64_t blocks = (rows + 3) / 4;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (N > 1)
        hipLaunchKernelGGL(linkage_init_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st,
                           (const T *)D, N, T_, stride, w);
    // threads per merge workgroup: 1024, or LS_LINKAGE_THREADS (a multiple
    // of 64 up to 1024)
    int threads = 1024;
    if (const char *env = std::getenv("LS_LINKAGE_THREADS")) {
        const int v = std::atoi(env);
        if (v >= 64 && v <= 1024 && v % 64 == 0) threads = v;
    }
    // the static part of the kernel's local memory: 16 candidates and a count
    const size_t lds = linkage_lds_bytes(N, sizeof(T));
    const size_t fixed = 16 * sizeof(Cand<T>) + 64;
    if (lds + fixed <= max_group_lds()) {
        hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&linkage_kernel<T, true>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((linkage_kernel<T, true>), dim3(T_), dim3(threads), lds, st, D, N,
                           stride, w, Z, order);
    } else {
        hipLaunchKernelGGL((linkage_kernel<T, false>), dim3(T_), dim3(threads), 0, st, D, N,
                           stride, w, Z, order);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_linkage(void *D, int32_t N, int32_t T, int is_f64, double *Z, int32_t *order,
                          void *ws, hipStream_t st) {
    if (N < 1 || T < 1) return hipSuccess;
    char *w = static_cast<char *>(ws);
    if (is_f64) return launch_linkage_t<double>((double *)D, N, T, Z, order, w, st);
    return launch_linkage_t<float>((float *)D, N, T, Z, order, w, st);
}

// ---------------------------------------------------------------------------
// Standardised half-distance rows (section 2.2): row (k, r) at E + k ts +
// r rs, recipient i = recips[r]; over the donors j != i, z = (e - mean) / sd
// with the population deviation (divisor N - 1), accumulated in FP64 in a
// fixed order; z_i = 0; a row whose donor entries are all equal becomes 0.
// In place. One workgroup of 256 per row.
template <class X>
__global__ void __launch_bounds__(256)
standardise_kernel(X *E, const int32_t *__restrict__ recips, int32_t N, int64_t ts, int64_t rs) {
    __shared__ double part[4];
    __shared__ int diff[4];
    const int r = blockIdx.x;
    const int64_t k = blockIdx.y;
    const int i = recips[r];
    X *row = E + k * ts + (int64_t)r * rs;
    const int first = i == 0 ? 1 : 0;
    const X x0 = row[first];
    double s = 0.0;
    int neq = 0;
    for (int j = threadIdx.x; j < N; j += 256) {
        if (j == i) continue;
        const X x = row[j];
        s += (double)x;
        neq |= !(x == x0);
    }
    const int wave = threadIdx.x >> 6;
    s = wave_sum(s);
    const int any = __any(neq);
    if ((threadIdx.x & 63) == 0) {
        part[wave] = s;
        diff[wave] = any;
    }
    __syncthreads();
    const double mean = ((part[0] + part[1]) + (part[2] + part[3])) / (double)(N - 1);
    const bool equal = !(diff[0] | diff[1] | diff[2] | diff[3]);
    double v = 0.0;
    for (int j = threadIdx.x; j < N; j += 256) {
        if (j == i) continue;
        const double d = (double)row[j] - mean;
        v += d * d;
    }
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) part[wave] = v;
    __syncthreads();
    const double sd = sqrt(((part[0] + part[1]) + (part[2] + part[3])) / (double)(N - 1));
    for (int j = threadIdx.x; j < N; j += 256)
        row[j] = (j == i || equal) ? (X)0 : (X)(((double)row[j] - mean) / sd);
}

hipError_t launch_standardise(void *E, const int32_t *recips, int32_t R, int32_t T, int32_t N,
                              int64_t ts, int64_t rs, int is_f64, hipStream_t st) {
    if (R < 1 || T < 1 || N < 2) return hipSuccess;
    if (T > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)R, (unsigned)T);
    if (is_f64)
        hipLaunchKernelGGL(standardise_kernel<double>, grid, dim3(256), 0, st, (double *)E,
                           recips, N, ts, rs);
    else
        hipLaunchKernelGGL(standardise_kernel<float>, grid, dim3(256), 0, st, (float *)E, recips,
                           N, ts, rs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed scratch of the allocation-free linkage entry point: a file-scope
// device array, one copy per GPU, held until the process ends. In host code
// its name is not a device address; the address of each GPU's copy comes
// from hipGetSymbolAddress with that GPU current, taken once per GPU on its
// first use and kept.
static __device__ __align__(256) char scratch[kLinkageScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t linkage_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace lsk
