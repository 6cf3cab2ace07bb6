// Orthonormal basis of a tall sketch (Algorithm 1 steps 8 and 12, the
// economic QR Y = Q R of Section 3.1) in float64 on one workgroup.
//
// Householder reflections H_k = I - tau_k v_k v_k^T with v_k(k) = 1 (the
// elementary reflector of the LAPACK convention), then the explicit
// Q = H_0 ... H_{n-1} [I_n; 0] formed in place, then column k of Q negated
// when R_kk < 0 so that diag(R) >= 0.  Householder keeps Q orthonormal when Y
// is rank deficient (noise-free low-rank inputs with l > R), which a Cholesky
// based QR would not.  The matrix lives in LDS when it fits (m*n <= 18432),
// else in the caller's float64 buffer (L2 resident at these sizes).
//
// Thread layout: lane j of a column group owns column j (CL = 32 or 64
// columns), the G = QNT / CL groups split the rows, so the column dot
// products and the rank-1 updates need no integer division and one LDS
// exchange of G partial sums per column.

#include "rcp_device.h"
#include "rcp_kernels.h"

namespace rcp {

constexpr int QNT = 1024;
constexpr int QR_LDS_ELEMS = 18432;          // 144 KiB of float64

// Apply H_k (stored in column k, v_k = 1) to columns k+1..n-1, rows k..m-1.
__device__ __forceinline__ void apply_reflector(double* A, int lda, int m, int n, int k,
                                                double tau, double* wp, int CL, int G) {
    const int j = threadIdx.x % CL, g = threadIdx.x / CL;
    const bool active = (j > k) && (j < n);
    if (active) {
        double s0 = 0.0, s1 = 0.0;
        // row k carries v_k = 1
        if (g == 0) s0 = A[k * lda + j];
        int i = k + 1 + g;
        for (; i + G < m; i += 2 * G) {
            s0 += A[i * lda + k] * A[i * lda + j];
            s1 += A[(i + G) * lda + k] * A[(i + G) * lda + j];
        }
        if (i < m) s0 += A[i * lda + k] * A[i * lda + j];
        wp[g * CL + j] = s0 + s1;
    }
    __syncthreads();
    if (active) {
        double w = 0.0;
        for (int gg = 0; gg < G; ++gg) w += wp[gg * CL + j];
        const double tw = tau * w;
        if (g == 0) A[k * lda + j] -= tw;
        int i = k + 1 + g;
        for (; i + G < m; i += 2 * G) {
            const double v0 = A[i * lda + k], v1 = A[(i + G) * lda + k];
            A[i * lda + j] -= v0 * tw;
            A[(i + G) * lda + j] -= v1 * tw;
        }
        if (i < m) A[i * lda + j] -= A[i * lda + k] * tw;
    }
    __syncthreads();
}

template <bool USE_LDS>
__global__ __launch_bounds__(QNT) void k_qr(double* Yg, int m, int n, int ldy, float* Qpad,
                                            int ldq, float* Qout) {
    extern __shared__ double qsm[];
    __shared__ double wp[QNT];              // G x CL partial dot products
    __shared__ double taus[64];
    __shared__ double betas[64];
    __shared__ double red[QNT / 64];
    const int tid = threadIdx.x;
    const int CL = (n <= 32) ? 32 : 64;
    const int G = QNT / CL;
    const int j = tid % CL, g = tid / CL;
    // USE_LDS is a template parameter so that every access below compiles to
    // LDS (ds_*) or global instructions, never to generic (flat) ones.
    double* A = USE_LDS ? qsm : Yg;
    const int lda = USE_LDS ? n : ldy;
    if (USE_LDS) {
        if (j < n)
            for (int i = g; i < m; i += G) A[i * n + j] = Yg[i * ldy + j];
        __syncthreads();
    }

    // --- factorisation
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int i = k + 1 + tid; i < m; i += QNT) {
            const double v = A[i * lda + k];
            s += v * v;
        }
        const double sigma = block_sum(s, red);
        const double alpha = A[k * lda + k];
        double tau = 0.0, beta = alpha, scale = 0.0;
        if (sigma > 0.0) {
            const double nrm = sqrt(alpha * alpha + sigma);
            beta = (alpha >= 0.0) ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        if (tau != 0.0)
            for (int i = k + 1 + tid; i < m; i += QNT) A[i * lda + k] *= scale;
        if (tid == 0) {
            taus[k] = tau;
            betas[k] = beta;
        }
        __syncthreads();
        if (tau != 0.0 && k + 1 < n) apply_reflector(A, lda, m, n, k, tau, wp, CL, G);
    }

    // --- explicit Q, in place, last reflector first
    for (int k = n - 1; k >= 0; --k) {
        const double tau = taus[k];
        if (k + 1 < n && tau != 0.0) apply_reflector(A, lda, m, n, k, tau, wp, CL, G);
        for (int i = tid; i < m; i += QNT) {
            double* p = A + i * lda + k;
            if (i > k) *p = -tau * (*p);
            else if (i == k) *p = 1.0 - tau;
            else *p = 0.0;
        }
        __syncthreads();
    }

    // --- sign convention diag(R) >= 0, float32 outputs
    for (int i = g; i < m; i += G) {
        for (int c = j; c < ldq; c += CL) {
            float v = 0.0f;
            if (c < n) {
                const double d = A[i * lda + c];
                v = (float)(betas[c] < 0.0 ? -d : d);
                if (Qout != nullptr) Qout[(int64_t)i * n + c] = v;
            }
            Qpad[(int64_t)i * ldq + c] = v;
        }
    }
}

hipError_t launch_qr(double* Y, int64_t m, int n, int ldy, float* Qpad, int ldq, float* Qout,
                     hipStream_t s) {
    if (m * n <= QR_LDS_ELEMS) {
        const size_t smem = (size_t)m * n * sizeof(double);
        hipError_t e = hipFuncSetAttribute((const void*)k_qr<true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(QR_LDS_ELEMS * sizeof(double)));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_qr<true>, dim3(1), dim3(QNT), smem, s, Y, (int)m, n, ldy, Qpad, ldq, Qout);
    } else {
        hipLaunchKernelGGL(k_qr<false>, dim3(1), dim3(QNT), 0, s, Y, (int)m, n, ldy, Qpad, ldq, Qout);
    }
    return hipGetLastError();
}

}  // namespace rcp
