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
__global__ __launch_bounds__(ENT) void k_expand_raw(ExpandArgs a, double* raw) {
    const int n = blockIdx.y;
    const int64_t In = a.I[n];
    const int ln = a.l[n], R = a.R;
    int64_t off = 0;
    for (int m = 0; m < n; ++m) off += a.I[m] * R;
    const int64_t e = (int64_t)blockIdx.x * ENT + threadIdx.x;
    if (e >= In * R) return;
    const int64_t i = e / R;
    const int r = (int)(e - i * R);
    const float* q = a.Q[n] + i * ln;
    const float* at = a.At[n];
    double s = 0.0;
    for (int c = 0; c < ln; ++c) s += (double)q[c] * (double)at[c * R + r];
    raw[off + e] = s;
}

__global__ __launch_bounds__(ENT) void k_expand_finish(ExpandArgs a, const double* raw) {
    __shared__ double nu[RCP_MAX_NDIM * RCP_MAX_RANK];
    __shared__ float sgn[RCP_MAX_NDIM * RCP_MAX_RANK];
    __shared__ double lam[RCP_MAX_RANK];
    __shared__ int rank[RCP_MAX_RANK];
    const int N = a.N, R = a.R, tid = threadIdx.x;
    int64_t off[RCP_MAX_NDIM];
    {
        int64_t o = 0;
        for (int n = 0; n < N; ++n) { off[n] = o; o += a.I[n] * R; }
    }
    for (int e = tid; e < N * R; e += ENT) {
        const int n = e / R, r = e % R;
        const double* col = raw + off[n] + r;
        double s = 0.0, best = -1.0;
        int64_t bi = 0;
        for (int64_t i = 0; i < a.I[n]; ++i) {
            const double v = col[i * R];
            s += v * v;
            if (fabs(v) > best) { best = fabs(v); bi = i; }
        }
        nu[e] = sqrt(s);
        sgn[e] = (col[bi * R] < 0.0) ? -1.0f : 1.0f;
    }
    __syncthreads();
    for (int r = tid; r < R; r += ENT) {
        double l = (double)a.lambda_in[r];
        for (int n = 0; n < N; ++n) {
            const double v = nu[n * R + r];
            if (v > 0.0) l *= v;
        }
        lam[r] = l;
        float s = 1.0f;
        for (int n = 0; n < N - 1; ++n) s *= sgn[n * R + r];
        sgn[(N - 1) * R + r] = s;
    }
    __syncthreads();
    for (int r = tid; r < R; r += ENT) {
        int k = 0;
        for (int s = 0; s < R; ++s)
            if (lam[s] > lam[r] || (lam[s] == lam[r] && s < r)) ++k;
        rank[r] = k;
    }
    __syncthreads();
    for (int r = tid; r < R; r += ENT) a.lambda_out[rank[r]] = (float)lam[r];
    for (int n = 0; n < N; ++n) {
        const int64_t cnt = a.I[n] * R;
        for (int64_t e = tid; e < cnt; e += ENT) {
            const int64_t i = e / R;
            const int r = (int)(e - i * R);
            const double v = nu[n * R + r];
            double x = raw[off[n] + e];
            if (v > 0.0) x /= v;
            a.A[n][i * R + rank[r]] = (float)(x * sgn[n * R + r]);
        }
    }
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

}  // namespace rcp
