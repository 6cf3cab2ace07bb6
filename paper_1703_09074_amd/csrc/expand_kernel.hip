// Back-projection of the core factors (eq. qbs, Algorithm 2's factor recovery) and the
// final renormalisation: A_n = Q_n Ã_n, unit columns with the
// norms folded into lambda, components sorted by lambda (descending, stable)
// and each column of modes 0..N-2 signed so that its largest-magnitude entry
// (first index on ties) is positive, the sign moved into mode N-1.

#include "rcp_device.h"
#include "rcp_kernels.h"

namespace rcp {

constexpr int ENT = 256;

// raw_n[i, r] = sum_c Q_n[i, c] At_n[c, r]   (float64 accumulation)
__device__ __forceinline__ void expand_raw_body(const ExpandArgs& a, double* raw, int n, int64_t e) {
    const int64_t In = a.I[n];
    const int ln = a.l[n], R = a.R;
    int64_t off = 0;
    for (int m = 0; m < n; ++m) off += a.I[m] * R;
    if (e >= In * R) return;
    const int64_t i = e / R;
    const int r = (int)(e - i * R);
    const float* q = a.Q[n] + i * ln;
    const float* at = a.At[n];
    double s = 0.0;
    for (int c = 0; c < ln; ++c) s += (double)q[c] * (double)at[c * R + r];
    raw[off + e] = s;
}

__global__ __launch_bounds__(ENT) void k_expand_raw(ExpandArgs a, double* raw) {
    expand_raw_body(a, raw, blockIdx.y, (int64_t)blockIdx.x * ENT + threadIdx.x);
}

__global__ __launch_bounds__(ENT) void k_expand_raw_batch(const ExpandArgs* args) {
    const ExpandArgs& a = args[blockIdx.z];
    if ((int)blockIdx.y >= a.N) return;
    expand_raw_body(a, a.raw, blockIdx.y, (int64_t)blockIdx.x * ENT + threadIdx.x);
}

// The final step in three launches.  (1) One wavefront per column (n, r):
// its lanes stride over the rows and combine the sum of squares and the
// first largest-magnitude entry; the norm and the sign go to a.stats.
// (2) One workgroup: lambda (lambda_in times the norms), the sign of mode
// N-1 (the product of the others'), the ranks by lambda (descending,
// stable); lambda_out written, the ranks kept in a.stats.  (3) Every output
// element: A[n][i, rank[r]] = raw / norm * sign.
// a.stats layout (doubles): norms (N x R), signs (N x R), ranks (R).
__device__ __forceinline__ void expand_stats_col(const ExpandArgs& a, const double* raw, int e) {
    const int N = a.N, R = a.R;
    const int lane = threadIdx.x & 63;
    if (e >= N * R) return;
    const int n = e / R, r = e % R;
    int64_t base = 0, In = 0;
#pragma unroll
    for (int m = 0; m < RCP_MAX_NDIM; ++m) {
        if (m < n && m < N) base += a.I[m] * R;
        if (m == n) In = a.I[m];
    }
    const double* col = raw + base + r;
    double s = 0.0, best = -1.0;
    long long bi = 0;
    for (int64_t i = lane; i < In; i += 64) {
        const double v = col[i * R];
        s += v * v;
        if (fabs(v) > best) { best = fabs(v); bi = i; }
    }
    s = warp_sum(s);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const long long oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) {
        a.stats[e] = sqrt(s);
        a.stats[N * R + e] = (col[bi * R] < 0.0) ? -1.0 : 1.0;
    }
}

__global__ __launch_bounds__(64) void k_expand_stats(ExpandArgs a, const double* raw) {
    expand_stats_col(a, raw, (int)blockIdx.x);
}

__global__ __launch_bounds__(64) void k_expand_stats_batch(const ExpandArgs* args) {
    const ExpandArgs& a = args[blockIdx.z];
    expand_stats_col(a, a.raw, (int)blockIdx.x);
}

__device__ __forceinline__ void expand_order_body(const ExpandArgs& a) {
    __shared__ double lam[RCP_MAX_RANK];
    const int N = a.N, R = a.R, tid = threadIdx.x;
    const double* nu = a.stats;
    double* sgn = a.stats + N * R;
    double* rank = a.stats + 2 * N * R;
    for (int r = tid; r < R; r += ENT) {
        double l = (double)a.lambda_in[r];
        for (int n = 0; n < N; ++n) {
            const double v = nu[n * R + r];
            if (v > 0.0) l *= v;
        }
        lam[r] = l;
        double sg = 1.0;
        for (int n = 0; n < N - 1; ++n) sg *= sgn[n * R + r];
        sgn[(N - 1) * R + r] = sg;
    }
    __syncthreads();
    for (int r = tid; r < R; r += ENT) {
        int k = 0;
        for (int t = 0; t < R; ++t)
            if (lam[t] > lam[r] || (lam[t] == lam[r] && t < r)) ++k;
        rank[r] = (double)k;
        a.lambda_out[k] = (float)lam[r];
    }
}

__global__ __launch_bounds__(ENT) void k_expand_order(ExpandArgs a) { expand_order_body(a); }

__global__ __launch_bounds__(ENT) void k_expand_order_batch(const ExpandArgs* args) {
    expand_order_body(args[blockIdx.x]);
}

__device__ __forceinline__ void expand_write_elem(const ExpandArgs& a, const double* raw, int n,
                                                  int64_t e) {
    const int N = a.N, R = a.R;
    if (n >= N) return;
    int64_t off = 0, In = 0;
#pragma unroll
    for (int m = 0; m < RCP_MAX_NDIM; ++m) {
        if (m < n && m < N) off += a.I[m] * R;
        if (m == n) In = a.I[m];
    }
    if (e >= In * R) return;
    const int64_t i = e / R;
    const int r = (int)(e - i * R);
    const double v = a.stats[n * R + r];
    double x = raw[off + e];
    if (v > 0.0) x /= v;
    const int k = (int)a.stats[2 * N * R + r];
    a.A[n][i * R + k] = (float)(x * a.stats[N * R + n * R + r]);
}

__global__ __launch_bounds__(ENT) void k_expand_write(ExpandArgs a, const double* raw) {
    expand_write_elem(a, raw, (int)blockIdx.y, (int64_t)blockIdx.x * ENT + threadIdx.x);
}

__global__ __launch_bounds__(ENT) void k_expand_write_batch(const ExpandArgs* args) {
    const ExpandArgs& a = args[blockIdx.z];
    expand_write_elem(a, a.raw, (int)blockIdx.y, (int64_t)blockIdx.x * ENT + threadIdx.x);
}

static hipError_t launch_expand_tail(const ExpandArgs& a, const double* raw, hipStream_t s) {
    hipLaunchKernelGGL(k_expand_stats, dim3((unsigned)(a.N * a.R)), dim3(64), 0, s, a, raw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_expand_order, dim3(1), dim3(ENT), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int64_t maxc = 0;
    for (int n = 0; n < a.N; ++n) maxc = (a.I[n] * a.R > maxc) ? a.I[n] * a.R : maxc;
    hipLaunchKernelGGL(k_expand_write, dim3((unsigned)((maxc + ENT - 1) / ENT), (unsigned)a.N), dim3(ENT), 0,
                       s, a, raw);
    return hipGetLastError();
}

hipError_t launch_expand(const ExpandArgs& a, hipStream_t s) {
    int64_t maxc = 0;
    for (int n = 0; n < a.N; ++n) maxc = (a.I[n] * a.R > maxc) ? a.I[n] * a.R : maxc;
    double* raw = a.raw;
    const dim3 grid((unsigned)((maxc + ENT - 1) / ENT), (unsigned)a.N);
    hipLaunchKernelGGL(k_expand_raw, grid, dim3(ENT), 0, s, a, raw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_expand_tail(a, raw, s);
}

hipError_t launch_expand_finish(const ExpandArgs& a, hipStream_t s) {
    return launch_expand_tail(a, a.raw, s);
}

hipError_t launch_expand_batch(const ExpandArgs* dargs, const ExpandArgs* hargs, int count,
                               hipStream_t s) {
    if (count < 1) return hipSuccess;
    int64_t maxc = 0;
    int maxN = 0;
    for (int b = 0; b < count; ++b) {
        for (int n = 0; n < hargs[b].N; ++n)
            maxc = (hargs[b].I[n] * hargs[b].R > maxc) ? hargs[b].I[n] * hargs[b].R : maxc;
        maxN = hargs[b].N > maxN ? hargs[b].N : maxN;
    }
    const dim3 grid((unsigned)((maxc + ENT - 1) / ENT), (unsigned)maxN, (unsigned)count);
    hipLaunchKernelGGL(k_expand_raw_batch, grid, dim3(ENT), 0, s, dargs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int maxNR = 0;
    for (int b = 0; b < count; ++b) maxNR = hargs[b].N * hargs[b].R > maxNR ? hargs[b].N * hargs[b].R : maxNR;
    hipLaunchKernelGGL(k_expand_stats_batch, dim3((unsigned)maxNR, 1, (unsigned)count), dim3(64), 0, s, dargs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_expand_order_batch, dim3((unsigned)count), dim3(ENT), 0, s, dargs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_expand_write_batch, dim3((unsigned)((maxc + ENT - 1) / ENT), (unsigned)maxN, (unsigned)count),
                       dim3(ENT), 0, s, dargs);
    return hipGetLastError();
}

}  // namespace rcp
