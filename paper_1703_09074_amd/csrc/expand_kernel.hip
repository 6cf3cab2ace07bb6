// Back-projection of the core factors (eq. qbs, Algorithm 2 step 12) and the
// final renormalisation (step 13): A_n = Q_n Ã_n, unit columns with the
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

// Column norms, signs, lambda, ranks and the final factors.  Wavefront w
// takes columns (n, r) = w, w + 4, ...: its lanes stride over the rows and
// combine the sum of squares and the first largest-magnitude entry.
__device__ __forceinline__ void expand_finish_body(const ExpandArgs& a, const double* raw) {
    __shared__ double nu[RCP_MAX_NDIM * RCP_MAX_RANK];
    __shared__ float sgn[RCP_MAX_NDIM * RCP_MAX_RANK];
    __shared__ double lam[RCP_MAX_RANK];
    __shared__ int rank[RCP_MAX_RANK];
    const int N = a.N, R = a.R, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    int64_t off[RCP_MAX_NDIM];
    {
        int64_t o = 0;
#pragma unroll
        for (int n = 0; n < RCP_MAX_NDIM; ++n) {
            off[n] = o;
            if (n < N) o += a.I[n] * R;
        }
    }
    for (int e = wave; e < N * R; e += ENT / 64) {
        const int n = e / R, r = e % R;
        int64_t base = 0, In = 0;
#pragma unroll
        for (int m = 0; m < RCP_MAX_NDIM; ++m)
            if (m == n) { base = off[m]; In = a.I[m]; }
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
            nu[e] = sqrt(s);
            sgn[e] = (col[bi * R] < 0.0) ? -1.0f : 1.0f;
        }
    }
    __syncthreads();
    for (int r = tid; r < R; r += ENT) {
        double l = (double)a.lambda_in[r];
        for (int n = 0; n < N; ++n) {
            const double v = nu[n * R + r];
            if (v > 0.0) l *= v;
        }
        lam[r] = l;
        float sg = 1.0f;
        for (int n = 0; n < N - 1; ++n) sg *= sgn[n * R + r];
        sgn[(N - 1) * R + r] = sg;
    }
    __syncthreads();
    for (int r = tid; r < R; r += ENT) {
        int k = 0;
        for (int t = 0; t < R; ++t)
            if (lam[t] > lam[r] || (lam[t] == lam[r] && t < r)) ++k;
        rank[r] = k;
    }
    __syncthreads();
    for (int r = tid; r < R; r += ENT) a.lambda_out[rank[r]] = (float)lam[r];
    for (int n = 0; n < N; ++n) {
        const int64_t cnt = a.I[n] * R;
        float* An = a.A[n];
        for (int64_t e = tid; e < cnt; e += ENT) {
            const int64_t i = e / R;
            const int r = (int)(e - i * R);
            const double v = nu[n * R + r];
            double x = raw[off[n] + e];
            if (v > 0.0) x /= v;
            An[i * R + rank[r]] = (float)(x * sgn[n * R + r]);
        }
    }
}

__global__ __launch_bounds__(ENT) void k_expand_finish(ExpandArgs a, const double* raw) {
    expand_finish_body(a, raw);
}

__global__ __launch_bounds__(ENT) void k_expand_finish_batch(const ExpandArgs* args) {
    const ExpandArgs& a = args[blockIdx.x];
    expand_finish_body(a, a.raw);
}

hipError_t launch_expand(const ExpandArgs& a, hipStream_t s) {
    int64_t maxc = 0;
    for (int n = 0; n < a.N; ++n) maxc = (a.I[n] * a.R > maxc) ? a.I[n] * a.R : maxc;
    double* raw = a.raw;
    const dim3 grid((unsigned)((maxc + ENT - 1) / ENT), (unsigned)a.N);
    hipLaunchKernelGGL(k_expand_raw, grid, dim3(ENT), 0, s, a, raw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_expand_finish, dim3(1), dim3(ENT), 0, s, a, (const double*)raw);
    return hipGetLastError();
}

hipError_t launch_expand_finish(const ExpandArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_expand_finish, dim3(1), dim3(ENT), 0, s, a, (const double*)a.raw);
    return hipGetLastError();
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
    hipLaunchKernelGGL(k_expand_finish_batch, dim3((unsigned)count), dim3(ENT), 0, s, dargs);
    return hipGetLastError();
}

}  // namespace rcp
