// Orthonormal basis of a tall sketch (Algorithm 1 steps 8 and 12, the
// economic QR Y = Q R of Section 3.1) in float64 on one workgroup.
//
// Householder reflections H_k = I - tau_k v_k v_k^T with v_k(k) = 1 (the
// elementary reflector of the LAPACK convention), then the explicit Q =
// H_0 ... H_{n-1} [I_n; 0] formed in place, then column k of Q negated when
// R_kk < 0 so that diag(R) >= 0.  Householder keeps Q orthonormal when Y is
// rank deficient (noise-free low-rank inputs with l > R), which a Cholesky
// based QR would not.  The matrix lives in LDS when it fits (m*n <= 18432),
// else in the caller's float64 buffer (L2 resident at these sizes).

#include "rcp_device.h"
#include "rcp_kernels.h"

namespace rcp {

constexpr int QNT = 256;
constexpr int QR_LDS_ELEMS = 18432;          // 144 KiB of float64

__device__ __forceinline__ void apply_reflector(double* A, int lda, int m, int n, int k,
                                                double tau, double* wbuf) {
    // w_j = v^T A[k:m, j] for j in (k, n), v = (1, A[k+1:m, k])
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = k + 1 + wave; j < n; j += QNT / 64) {
        double s = 0.0;
        for (int i = k + lane; i < m; i += 64) {
            const double v = (i == k) ? 1.0 : A[(int64_t)i * lda + k];
            s += v * A[(int64_t)i * lda + j];
        }
        s = warp_sum(s);
        if (lane == 0) wbuf[j] = s;
    }
    __syncthreads();
    const int cols = n - k - 1;
    const int64_t total = (int64_t)(m - k) * cols;
    for (int64_t e = threadIdx.x; e < total; e += QNT) {
        const int i = k + (int)(e / cols);
        const int j = k + 1 + (int)(e % cols);
        const double v = (i == k) ? 1.0 : A[(int64_t)i * lda + k];
        A[(int64_t)i * lda + j] -= tau * v * wbuf[j];
    }
    __syncthreads();
}

__global__ __launch_bounds__(QNT) void k_qr(double* Yg, int64_t m64, int n, int ldy,
                                            float* Qpad, int ldq, float* Qout, int use_lds) {
    extern __shared__ double qsm[];
    __shared__ double wbuf[64];
    __shared__ double taus[64];
    __shared__ double betas[64];
    __shared__ double red[QNT / 64];
    const int m = (int)m64;
    double* A = Yg;
    int lda = ldy;
    if (use_lds) {
        A = qsm;
        lda = n;
        for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += QNT) {
            const int i = (int)(e / n), j = (int)(e % n);
            A[e] = Yg[(int64_t)i * ldy + j];
        }
        __syncthreads();
    }

    // --- factorisation
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int i = k + 1 + threadIdx.x; i < m; i += QNT) {
            const double v = A[(int64_t)i * lda + k];
            s += v * v;
        }
        const double sigma = block_sum(s, red);
        const double alpha = A[(int64_t)k * lda + k];
        double tau = 0.0, beta = alpha, scale = 0.0;
        if (sigma > 0.0) {
            const double nrm = sqrt(alpha * alpha + sigma);
            beta = (alpha >= 0.0) ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        __syncthreads();                    // everyone has read alpha
        if (tau != 0.0) {
            for (int i = k + 1 + threadIdx.x; i < m; i += QNT) A[(int64_t)i * lda + k] *= scale;
        }
        if (threadIdx.x == 0) {
            taus[k] = tau;
            betas[k] = beta;
        }
        __syncthreads();
        if (tau != 0.0 && k + 1 < n) apply_reflector(A, lda, m, n, k, tau, wbuf);
    }

    // --- explicit Q, in place, last reflector first
    for (int k = n - 1; k >= 0; --k) {
        const double tau = taus[k];
        if (k + 1 < n && tau != 0.0) apply_reflector(A, lda, m, n, k, tau, wbuf);
        for (int i = threadIdx.x; i < m; i += QNT) {
            double* p = A + (int64_t)i * lda + k;
            if (i > k) *p = -tau * (*p);
            else if (i == k) *p = 1.0 - tau;
            else *p = 0.0;
        }
        __syncthreads();
    }

    // --- sign convention diag(R) >= 0, float32 outputs
    for (int64_t e = threadIdx.x; e < (int64_t)m * ldq; e += QNT) {
        const int i = (int)(e / ldq), c = (int)(e % ldq);
        float v = 0.0f;
        if (c < n) {
            double d = A[(int64_t)i * lda + c];
            if (betas[c] < 0.0) d = -d;
            v = (float)d;
            if (Qout != nullptr) Qout[(int64_t)i * n + c] = v;
        }
        Qpad[e] = v;
    }
}

hipError_t launch_qr(double* Y, int64_t m, int n, int ldy, float* Qpad, int ldq, float* Qout,
                     hipStream_t s) {
    const int use_lds = (m * n <= QR_LDS_ELEMS) ? 1 : 0;
    const size_t smem = use_lds ? (size_t)m * n * sizeof(double) : 0;
    hipError_t e = hipFuncSetAttribute((const void*)k_qr, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(QR_LDS_ELEMS * sizeof(double)));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_qr, dim3(1), dim3(QNT), smem, s, Y, m, n, ldy, Qpad, ldq, Qout, use_lds);
    return hipGetLastError();
}

}  // namespace rcp
