// Orthonormal basis of a tall sketch Y (m x n, n <= 64, float64): the
// economic QR Y = Q R with diag(R) > 0 of Algorithm 1's orthonormalisations
// (Section 3.1), on one workgroup.
//
// Cholesky QR passes: G = A^T A (float64 matrix cores), G = R^T R (Cholesky),
// A <- A R^{-1} (matrix cores).  Every pass keeps span(A) and multiplies R by
// an upper-triangular factor with positive diagonal, so the result is the
// unique Q of Y = Q R with diag(R) > 0, as from Householder QR, up to
// rounding.  Inside the power iteration the sketch is as ill-conditioned as
// (T T^T) restricted to it, far beyond plain Cholesky QR, hence:
//   1. a shifted pass (shifted Cholesky QR, Fukaya, Kannan, Nakatsukasa,
//      Yamamoto and Yanagisawa, SIAM J. Sci. Comput. 2020): G + s I with
//      s = 11 (m n + n (n + 1)) u ||Y||_F^2, which makes the Cholesky succeed
//      for any full-rank Y and leaves a factor with condition number of order
//      u^{-1/2};
//   2. a plain pass, after which the basis is orthonormal to O(cond^2 u),
//      enough for the next power step (only its span matters there);
//   3. for the returned Q_n a third pass: its Gram is I + E with E small, and
//      R3 = I + triu(E) (diagonal halved) is exact to O(|E|^2), used when
//      max|E| <= 1e-8, else a full Cholesky.
// A Cholesky pivot that is not positive (an exactly rank-deficient sketch)
// switches the kernel to Householder QR on the current basis (same span, same
// Q): reflections H_k = I - tau_k v_k v_k^T with v_k(k) = 1, the explicit Q
// formed in place, columns negated so that diag(R) >= 0.
// The matrix lives in LDS when it fits, else in the caller's buffer (L2
// resident at these sizes), updated in place.

#include "rcp_device.h"
#include "rcp_kernels.h"

namespace rcp {

constexpr int QNT = 1024;                      // threads of the largest QR workgroup
constexpr int QNW = QNT / 64;
// threads and wavefronts of the running workgroup: 512 for bases of at most
// 32 columns (their Cholesky runs in one wavefront's registers, which needs
// more than the 128 VGPRs of a 1024-thread workgroup), 1024 otherwise
__device__ __forceinline__ int qnt() { return (int)blockDim.x; }
__device__ __forceinline__ int qnw() { return (int)(blockDim.x >> 6); }
template <int NB>
constexpr int qr_threads() { return NB <= 2 ? 512 : QNT; }
constexpr size_t kQrLds = 160 * 1024;
constexpr int kQrScratch = QNW * 256;         // doubles: Gram partials / Householder partial dots
constexpr double kCqrPivot = 1e-15;           // relative pivot floor of the unshifted passes
constexpr double kCqrFirstOrder = 1e-8;
constexpr double kUnitRoundoff = 1.1102230246251565e-16;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ double qr_block_max(double v, double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = red[0];
    for (int i = 1; i < qnw(); ++i) t = fmax(t, red[i]);
    return t;
}

// G (np x np, row-major) = A^T A over the first n columns (the rest zero),
// on the float64 matrix cores.  16 x 16 blocks of the upper triangle, the
// rows split over the wavefronts, partial blocks summed through `part`.
// Lane layout of v_mfma_f64_16x16x4: A operand [i][k] in lane i + 16 k,
// B operand [k][j] in lane j + 16 k, result element v of lane l is
// [l / 16 + 4 v][l % 16].
__device__ __forceinline__ void gram64(const double* A, int lda, int m, int n, int np, double* G,
                                       double* part, int max_units) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nb = np >> 4;
    const int U = nb * (nb + 1) / 2;
    const int kp = (max_units / U) > 0 ? max_units / U : 1;
    const int per = (((m + kp - 1) / kp) + 3) & ~3;
    for (int u = wave; u < U * kp; u += qnw()) {
        const int blk = u % U, p = u / U;
        int bi = 0, rem = blk;
        while (rem >= nb - bi) { rem -= nb - bi; ++bi; }
        const int bj = bi + rem;
        const int c1 = bi * 16 + li, c2 = bj * 16 + li;
        const int r0 = p * per, r1 = min(m, r0 + per);
        // four steps of 4 rows per iteration, loads first (independent of
        // the accumulators), over two accumulation chains
        f64x4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = r0; k0 < r1; k0 += 16) {
            double a[4], b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int r = k0 + 4 * t + lk;
                const bool rv = r < r1;
                const int rc = rv ? r : r0;
                a[t] = A[rc * lda + (c1 < n ? c1 : 0)];
                b[t] = A[rc * lda + (c2 < n ? c2 : 0)];
                if (!rv || c1 >= n) a[t] = 0.0;
                if (!rv || c2 >= n) b[t] = 0.0;
            }
            acc = mfma64(a[0], b[0], acc);
            acc2 = mfma64(a[1], b[1], acc2);
            acc = mfma64(a[2], b[2], acc);
            acc2 = mfma64(a[3], b[3], acc2);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += acc2[v];
        double* dst = part + u * 256;
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[(lk + 4 * v) * 16 + li] = acc[v];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < np * np; e += qnt()) {
        int i = e / np, j = e - (e / np) * np;
        if ((i >> 4) > (j >> 4)) { const int t = i; i = j; j = t; }
        const int bi = i >> 4, bj = j >> 4;
        const int blk = bi * nb - bi * (bi - 1) / 2 + (bj - bi);
        double s = 0.0;
        for (int p = 0; p < kp; ++p) s += part[(p * U + blk) * 256 + (i & 15) * 16 + (j & 15)];
        G[e] = s;
    }
    __syncthreads();
}

// The upper Cholesky factor R of G + shift I (n x n, n <= NP <= 32, G row
// stride ldg) and its inverse X = R^{-1} (stride ldx, upper, zero
// elsewhere), in one wavefront from registers: lane c holds column c of
// [G + shift I | I] (2 NP <= 64 columns, identity beyond n), and the rows
// rotate through the registers so that the pivot row is
// always register 0 (steps unrolled: static indices).  Step k subtracts
// multiples of the pivot row from the rows below it (their entries in the
// pivot column come from lane k by readlane) and moves it to the back; after
// NP steps the rows read [U | L^{-1}] with G + shift I = L U, U = D L^T.  Then
// R = D^{1/2} L^T, so R^{-1}[i][j] = L^{-1}[j][i] / sqrt(d_j): lane NP + i
// holds column i of L^{-1} and writes row i of X; isd (NP doubles, LDS)
// receives 1 / R_jj.  Wavefront 0 runs it; it returns 0 when a pivot is not
// above thr.  Callers synchronise the workgroup before using X.
template <int NP>
__device__ __forceinline__ int chol_inverse_wave_s(const double* G, int ldg, double* X, int ldx, int n,
                                                   double shift, double thr, double* isd) {
    const int lane = threadIdx.x & 63;
    double col[NP];
    const int c = lane;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        double v;
        if (c < NP) {
            v = (i < n && c < n) ? G[i * ldg + c] : 0.0;
            if (i == c) v = (i < n) ? v + shift : 1.0;
        } else {
            v = (i == c - NP) ? 1.0 : 0.0;
        }
        col[i] = v;
    }
    int ok = 1;
    double mypiv = 1.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        // pivot column first, into distinct scalar registers, then the updates
        double s[NP];
        s[0] = readlane_f64(col[0], k);
        const double u = div_pivot(col[0], s[0]);
#pragma unroll
        for (int i = 1; i < NP - k; ++i) s[i] = readlane_f64(col[i], k);
        __builtin_amdgcn_sched_barrier(0);
        const double piv = s[0];
        if (k < n && !(piv > thr)) ok = 0;
        mypiv = (lane == k) ? piv : mypiv;                       // d_k = U[k][k], kept by lane k
#pragma unroll
        for (int i = 1; i < NP - k; ++i) col[i] -= s[i] * u;
        const double p0 = col[0];
#pragma unroll
        for (int i = 0; i < NP - 1; ++i) col[i] = col[i + 1];
        col[NP - 1] = p0;
    }
    if (lane < NP) isd[lane] = 1.0 / sqrt(fmax(mypiv, thr));
    // the isd stores before the other lanes' reads (one wavefront)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (c >= NP && c < 2 * NP) {
        const int i = c - NP;
#pragma unroll
        for (int j = 0; j < NP; ++j)
            X[i * ldx + j] = (i < n && j < n && j >= i) ? col[j] * isd[j] : 0.0;
    }
    return ok;
}


// chol_inverse_wave_s on G (stride NP) with the shift and pivot floor of
// G's own first n rows, X stride NP.
template <int NP>
__device__ __forceinline__ int chol_inverse_wave(const double* G, double* X, int n,
                                                 double shift_coef, double* isd) {
    double gm = 0.0, tr = 0.0;
    for (int j = 0; j < n; ++j) {
        const double d = G[j * NP + j];
        gm = fmax(gm, d);
        tr += d;
    }
    const double shift = shift_coef * tr;
    const double thr = kCqrPivot * (gm + shift);
    return chol_inverse_wave_s<NP>(G, NP, X, NP, n, shift, thr, isd);
}

// The same result (up to rounding) for 32 < n <= np <= 64 as a 2 x 2 block
// Cholesky, the diagonal blocks factored and inverted by the register
// elimination above (wavefront 0), the off-diagonal products over the
// workgroup:  G + sI = [A B; B^T C],  A = R1^T R1,  R12 = R1^{-T} B,
// S = C + sI - R12^T R12 = R2^T R2,  R^{-1} = [R1^{-1}, -R1^{-1} R12 R2^{-1};
// 0, R2^{-1}].  The shift s = shift_coef trace(G) and the pivot floor are
// those of the whole matrix; S's pivots are the whole elimination's trailing
// ones.  Two register eliminations and four barriers in place of one
// barrier per pivot.  scratch: 4096 doubles.  On return X = R^{-1} (upper,
// zero elsewhere, stride np); G is left as it was.  Returns 0 when a pivot
// is not above the floor.  Callers synchronise the workgroup before using X.
__device__ __forceinline__ int chol_inverse_blk(const double* G, double* X, double* scratch,
                                                double* isd, double* red, int n, int np,
                                                double shift_coef) {
    __shared__ int okf[2];
    const int tid = threadIdx.x;
    const int n2 = n > 32 ? n - 32 : 0;
    double gm = 0.0, tr = 0.0;
    for (int j = tid; j < n; j += qnt()) { gm = fmax(gm, G[j * np + j]); tr += G[j * np + j]; }
    tr = block_sum(tr, red);
    gm = qr_block_max(gm, red);
    const double shift = shift_coef * tr;
    const double thr = kCqrPivot * (gm + shift);
    double* R12 = scratch;          // 32 x 32
    double* S = R12 + 1024;         // 32 x 32
    double* X22 = S + 1024;         // 32 x 32
    double* W = X22 + 1024;         // 32 x 32
    if (tid < 64) {
        const int ok = chol_inverse_wave_s<32>(G, np, X, np, n < 32 ? n : 32, shift, thr, isd);
        if (tid == 0) okf[0] = ok;
    }
    __syncthreads();
    // R12 = R1^{-T} B (X holds R1^{-1}, upper)
    for (int e = tid; e < 1024; e += qnt()) {
        const int i = e >> 5, j = e & 31;
        double v = 0.0;
        if (j < n2)
            for (int k = 0; k <= i; ++k) v += X[k * np + i] * G[k * np + 32 + j];
        R12[e] = v;
    }
    __syncthreads();
    for (int e = tid; e < 1024; e += qnt()) {
        const int i = e >> 5, j = e & 31;
        double v = 0.0;
        if (i < n2 && j < n2) {
            v = G[(32 + i) * np + 32 + j] + ((i == j) ? shift : 0.0);
            for (int k = 0; k < 32; ++k) v -= R12[k * 32 + i] * R12[k * 32 + j];
        }
        S[e] = v;
    }
    __syncthreads();
    if (tid < 64) {
        const int ok = chol_inverse_wave_s<32>(S, 32, X22, 32, n2, 0.0, thr, isd);
        if (tid == 0) okf[1] = ok;
    }
    __syncthreads();
    // W = R12 R2^{-1}
    for (int e = tid; e < 1024; e += qnt()) {
        const int i = e >> 5, j = e & 31;
        double v = 0.0;
        if (j < n2)
            for (int k = 0; k <= j; ++k) v += R12[i * 32 + k] * X22[k * 32 + j];
        W[e] = v;
    }
    __syncthreads();
    // X12 = -R1^{-1} W, X22 into place, zero below
    for (int e = tid; e < 32 * (np - 32); e += qnt()) {
        const int i = e / (np - 32), j = e - i * (np - 32);
        double v = 0.0;
        if (j < n2)
            for (int k = i; k < 32; ++k) v -= X[i * np + k] * W[k * 32 + j];
        X[i * np + 32 + j] = v;
    }
    for (int e = tid; e < (np - 32) * np; e += qnt()) {
        const int i = e / np, c = e - i * np;
        X[(32 + i) * np + c] = (c < 32) ? 0.0 : X22[i * 32 + (c - 32)];
    }
    __syncthreads();
    return okf[0] && okf[1];
}

// A <- A X for upper triangular X (n x n, stride np = 16 NB), on the matrix
// cores.  Wavefront w owns row blocks w, w + 16, ...: it reads its rows
// completely before writing them, so the update is in place.
template <int NB>
__device__ __forceinline__ void apply_upper(double* A, int lda, int m, int n, const double* X) {
    constexpr int np = 16 * NB;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int mb = (m + 15) >> 4;
    for (int rb = wave; rb < mb; rb += qnw()) {
        f64x4 acc[NB];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[cb] = f64x4{0.0, 0.0, 0.0, 0.0};
        const int r = rb * 16 + li;
        const int rc = (r < m) ? r : 0;
        // four steps of 4 columns per iteration, the row loads first
        for (int k0 = 0; k0 < n; k0 += 16) {
            double a[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int kk = k0 + 4 * t + lk;
                a[t] = A[rc * lda + (kk < n ? kk : 0)];
                if (r >= m || kk >= n) a[t] = 0.0;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (k0 + 4 * t < n) {
                    const int kk = k0 + 4 * t + lk;
#pragma unroll
                    for (int cb = 0; cb < NB; ++cb) {
                        const int c = cb * 16 + li;
                        const double b = (kk < n && c < n) ? X[kk * np + c] : 0.0;
                        acc[cb] = mfma64(a[t], b, acc[cb]);
                    }
                }
            }
        }
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = rb * 16 + lk + 4 * v, col = cb * 16 + li;
                if (row < m && col < n) A[row * lda + col] = acc[cb][v];
            }
    }
}

// Householder QR of A (m x n, stride lda) in place: A <- Q with diag(R) >= 0.
__device__ __forceinline__ void apply_reflector(double* A, int lda, int m, int n, int k, double tau,
                                                double* wp, int CL, int G) {
    const int j = threadIdx.x % CL, g = threadIdx.x / CL;
    const bool active = (j > k) && (j < n);
    if (active) {
        double s0 = 0.0, s1 = 0.0;
        if (g == 0) s0 = A[k * lda + j];            // row k carries v_k = 1
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

__device__ __forceinline__ void householder_q(double* A, int lda, int m, int n, double* wp,
                                              double* taus, double* betas, double* red) {
    const int tid = threadIdx.x;
    const int CL = (n <= 32) ? 32 : 64;
    const int G = qnt() / CL;
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int i = k + 1 + tid; i < m; i += qnt()) {
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
            for (int i = k + 1 + tid; i < m; i += qnt()) A[i * lda + k] *= scale;
        if (tid == 0) { taus[k] = tau; betas[k] = beta; }
        __syncthreads();
        if (tau != 0.0 && k + 1 < n) apply_reflector(A, lda, m, n, k, tau, wp, CL, G);
    }
    for (int k = n - 1; k >= 0; --k) {
        const double tau = taus[k];
        if (k + 1 < n && tau != 0.0) apply_reflector(A, lda, m, n, k, tau, wp, CL, G);
        for (int i = tid; i < m; i += qnt()) {
            double* p = A + i * lda + k;
            if (i > k) *p = -tau * (*p);
            else if (i == k) *p = 1.0 - tau;
            else *p = 0.0;
        }
        __syncthreads();
    }
    // diag(R) >= 0: R_kk = beta_k, so negate column k where beta_k < 0
    for (int e = tid; e < m * n; e += qnt()) {
        const int i = e / n, c = e - (e / n) * n;
        if (betas[c] < 0.0) A[i * lda + c] = -A[i * lda + c];
    }
    __syncthreads();
}

template <bool USE_LDS, int NB>
__device__ __forceinline__ void qr_body(double* Yg, int m, int n, int ldy, float* Qpad, int ldq,
                                        float* Qout, int second_pass, int* status) {
    extern __shared__ double qsm[];
    __shared__ double taus[64];
    __shared__ double betas[64];
    __shared__ double dinv[64];
    __shared__ double red[QNW];
    int flag;
    const int tid = threadIdx.x;
    constexpr int np = 16 * NB;
    // USE_LDS is a template parameter so that every access compiles to LDS
    // (ds_*) or global instructions, never to generic (flat) ones.
    const int lda = USE_LDS ? np + 1 : ldy;           // odd stride: no bank conflicts across rows
    double* A = USE_LDS ? qsm : Yg;
    double* G = USE_LDS ? qsm + (size_t)m * lda : qsm;
    double* X = G + np * np;
    double* scratch = X + np * np;
    if (USE_LDS) {
        // eight loads in flight per thread before their stores
        const int total = m * np, nt = qnt();
        for (int e0 = tid; e0 < total; e0 += 8 * nt) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * nt;
                const int i = e / np, c = e - (e / np) * np;
                const bool ok = e < total && c < n;
                v[u] = Yg[ok ? (size_t)i * ldy + c : 0];
                if (!ok) v[u] = 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * nt;
                if (e < total) {
                    const int i = e / np, c = e - (e / np) * np;
                    A[i * lda + c] = v[u];
                }
            }
        }
    }
    __syncthreads();

    // pass 1 (shifted), pass 2, and for the returned basis pass 3
    const double shift_coef = 11.0 * ((double)m * n + (double)n * (n + 1)) * kUnitRoundoff;
    const int passes = second_pass ? 3 : 2;
    for (int pass = 0; pass < passes; ++pass) {
        gram64(A, lda, m, n, np, G, scratch, USE_LDS ? QNW : 2 * QNW);
        bool first_order = false;
        if (pass == 2) {
            double e = 0.0;
            for (int t = tid; t < n * n; t += qnt()) {
                const int i = t / n, j = t - (t / n) * n;
                e = fmax(e, fabs(G[i * np + j] - (i == j ? 1.0 : 0.0)));
            }
            first_order = qr_block_max(e, red) <= kCqrFirstOrder;
        }
        if (first_order) {
            // R3^{-1} = I - F to first order, F = triu(G - I) with the diagonal halved
            for (int t = tid; t < np * np; t += qnt()) {
                const int i = t / np, j = t - (t / np) * np;
                double v = 0.0;
                if (i < n && j < n && i <= j) {
                    const double f = (i == j) ? 0.5 * (G[t] - 1.0) : G[t];
                    v = ((i == j) ? 1.0 : 0.0) - f;
                }
                X[t] = v;
            }
            __syncthreads();
            apply_upper<NB>(A, lda, m, n, X);
        } else {
            const double sc = pass == 0 ? shift_coef : 0.0;
            if (np <= 32) {
                if (tid < 64) {
                    const int okw = (np == 16) ? chol_inverse_wave<16>(G, X, n, sc, dinv)
                                               : chol_inverse_wave<32>(G, X, n, sc, dinv);
                    if (tid == 0) red[0] = okw ? 1.0 : 0.0;
                }
                __syncthreads();
                flag = red[0] != 0.0;
                __syncthreads();
            } else {
                flag = chol_inverse_blk(G, X, scratch, dinv, red, n, np, sc);
            }
            if (!flag) {
                householder_q(A, lda, m, n, scratch, taus, betas, red);
                if (tid == 0 && status != nullptr) *status |= RCP_INFO_QR_HOUSEHOLDER;
                break;
            }
            apply_upper<NB>(A, lda, m, n, X);
        }
        __syncthreads();
    }

    // float32 outputs, zero padding columns; eight reads in flight per thread
    {
        const int total = m * ldq, nt = qnt();
        for (int e0 = tid; e0 < total; e0 += 8 * nt) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * nt;
                const int i = e / ldq, c = e - (e / ldq) * ldq;
                const bool ok = e < total && c < n;
                v[u] = A[ok ? i * lda + c : 0];
                if (!ok) v[u] = 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * nt;
                if (e < total) {
                    const int i = e / ldq, c = e - (e / ldq) * ldq;
                    const float f = (float)v[u];
                    if (Qout != nullptr && c < n) Qout[(int64_t)i * n + c] = f;
                    Qpad[(int64_t)i * ldq + c] = f;
                }
            }
        }
    }
}

template <bool USE_LDS, int NB>
__global__ __launch_bounds__(qr_threads<NB>()) void k_qr(double* Yg, int m, int n, int ldy, float* Qpad, int ldq,
                                            float* Qout, int second_pass, int* status) {
    qr_body<USE_LDS, NB>(Yg, m, n, ldy, Qpad, ldq, Qout, second_pass, status);
}

// One workgroup per problem of a group (same template instantiation).
template <bool USE_LDS, int NB>
__global__ __launch_bounds__(qr_threads<NB>()) void k_qr_grp(const QrDesc* d) {
    const QrDesc& D = d[blockIdx.x];
    qr_body<USE_LDS, NB>(D.Y, D.m, D.n, D.ldy, D.Qpad, D.ldq, D.Qout, D.second_pass, D.status);
}

// ---------------------------------------------------------------------------
// Tall bases (Y too large for one workgroup's LDS): the same Cholesky QR
// passes with the O(m n^2) work spread over row blocks of kTqRows rows.
// Per pass: partial Grams per row block (k_tqr_gram), their sum in block
// order with the Cholesky factor and its inverse in one workgroup
// (k_tqr_chol), and Y <- Y R^{-1} per row block (k_tqr_apply, which also
// writes the float32 outputs after the last pass).  A failed Cholesky sets
// the flag at work[0]; the later launches then return and k_tqr_fallback
// runs the one-workgroup kernel (Householder) on Y as it stands: Y times
// upper-triangular factors with positive diagonal has the same Q.
constexpr int kTqRows = 64;
constexpr int kTqThreads = 512;

__device__ __forceinline__ int* tqr_flag(double* work) { return (int*)work; }
__device__ __forceinline__ double* tqr_X(double* work) { return work + 8; }
__device__ __forceinline__ double* tqr_G(double* work, int np) { return work + 8 + np * np; }

template <int NB>
__global__ __launch_bounds__(kTqThreads) void k_tqr_gram(const double* Y, int m, int n, int ldy,
                                                         double* work) {
    extern __shared__ double qsm[];
    constexpr int np = 16 * NB;
    if (*tqr_flag(work) != 0) return;
    const int r0 = blockIdx.x * kTqRows;
    const int rows = min(kTqRows, m - r0);
    double* G = qsm;
    double* part = qsm + np * np;
    gram64(Y + (size_t)r0 * ldy, ldy, rows, n, np, G, part, 2 * (kTqThreads / 64));
    double* dst = tqr_G(work, np) + (size_t)blockIdx.x * np * np;
    for (int e = threadIdx.x; e < np * np; e += kTqThreads) dst[e] = G[e];
}

template <int NB>
__global__ __launch_bounds__(qr_threads<NB>()) void k_tqr_chol(int m, int n, int nblk, int pass,
                                                               double* work) {
    extern __shared__ double qsm[];
    __shared__ double dinv[64];
    __shared__ double red[QNW];
    constexpr int np = 16 * NB;
    const int tid = threadIdx.x;
    if (*tqr_flag(work) != 0) return;
    double* G = qsm;
    double* X = G + np * np;
    double* scratch = X + np * np;
    const double* Gp = tqr_G(work, np);
    // G = sum of the nblk partial Grams in block order; a thread's loads of
    // eight blocks for four elements are in flight together
    for (int e0 = 0; e0 < np * np; e0 += 4 * qnt()) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        int b = 0;
        for (; b + 8 <= nblk; b += 8) {
            double g[8][4];
#pragma unroll
            for (int bb = 0; bb < 8; ++bb)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int e = e0 + tid + j * qnt();
                    g[bb][j] = (e < np * np) ? Gp[(size_t)(b + bb) * np * np + e] : 0.0;
                }
#pragma unroll
            for (int bb = 0; bb < 8; ++bb)
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] += g[bb][j];
        }
        for (; b < nblk; ++b)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = e0 + tid + j * qnt();
                if (e < np * np) v[j] += Gp[(size_t)b * np * np + e];
            }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = e0 + tid + j * qnt();
            if (e < np * np) G[e] = v[j];
        }
    }
    __syncthreads();
    bool first_order = false;
    if (pass == 2) {
        double e = 0.0;
        for (int t = tid; t < n * n; t += qnt()) {
            const int i = t / n, j = t - (t / n) * n;
            e = fmax(e, fabs(G[i * np + j] - (i == j ? 1.0 : 0.0)));
        }
        first_order = qr_block_max(e, red) <= kCqrFirstOrder;
    }
    int flag = 1;
    if (first_order) {
        for (int t = tid; t < np * np; t += qnt()) {
            const int i = t / np, j = t - (t / np) * np;
            double v = 0.0;
            if (i < n && j < n && i <= j) {
                const double f = (i == j) ? 0.5 * (G[t] - 1.0) : G[t];
                v = ((i == j) ? 1.0 : 0.0) - f;
            }
            X[t] = v;
        }
    } else {
        const double sc = pass == 0 ? 11.0 * ((double)m * n + (double)n * (n + 1)) * kUnitRoundoff : 0.0;
        if (np <= 32) {
            if (tid < 64) {
                const int okw = (np == 16) ? chol_inverse_wave<16>(G, X, n, sc, dinv)
                                           : chol_inverse_wave<32>(G, X, n, sc, dinv);
                if (tid == 0) red[0] = okw ? 1.0 : 0.0;
            }
            __syncthreads();
            flag = red[0] != 0.0;
            __syncthreads();
        } else {
            flag = chol_inverse_blk(G, X, scratch, dinv, red, n, np, sc);
        }
    }
    __syncthreads();
    if (!flag) {
        if (tid == 0) *tqr_flag(work) = 1;
        return;
    }
    double* Xg = tqr_X(work);
    for (int e = tid; e < np * np; e += qnt()) Xg[e] = X[e];
}

template <int NB>
__global__ __launch_bounds__(kTqThreads) void k_tqr_apply(double* Y, int m, int n, int ldy,
                                                          double* work, float* Qpad, int ldq,
                                                          float* Qout, int last) {
    __shared__ double Xs[16 * NB * 16 * NB];
    constexpr int np = 16 * NB;
    if (*tqr_flag(work) != 0) return;
    const double* Xg = tqr_X(work);
    for (int e = threadIdx.x; e < np * np; e += kTqThreads) Xs[e] = Xg[e];
    __syncthreads();
    const int r0 = blockIdx.x * kTqRows;
    const int rows = min(kTqRows, m - r0);
    double* A = Y + (size_t)r0 * ldy;
    apply_upper<NB>(A, ldy, rows, n, Xs);
    if (!last) return;
    __syncthreads();
    for (int e = threadIdx.x; e < rows * ldq; e += kTqThreads) {
        const int i = e / ldq, c = e - (e / ldq) * ldq;
        const float f = (c < n) ? (float)A[(size_t)i * ldy + c] : 0.0f;
        if (Qout != nullptr && c < n) Qout[(int64_t)(r0 + i) * n + c] = f;
        Qpad[(int64_t)(r0 + i) * ldq + c] = f;
    }
}

template <int NB>
__global__ __launch_bounds__(qr_threads<NB>()) void k_tqr_fallback(double* Yg, int m, int n, int ldy,
                                                                   float* Qpad, int ldq, float* Qout,
                                                                   int second_pass, int* status,
                                                                   double* work) {
    if (*tqr_flag(work) == 0) return;
    qr_body<false, NB>(Yg, m, n, ldy, Qpad, ldq, Qout, second_pass, status);
}

template <int NB>
static hipError_t launch_tqr_t(double* Y, int m, int n, int ldy, float* Qpad, int ldq, float* Qout,
                               bool final_basis, int* status, double* work, hipStream_t s) {
    constexpr int np = 16 * NB;
    const int nblk = (m + kTqRows - 1) / kTqRows;
    hipError_t e = launch_fill_i32((int*)work, 0, 2, s);
    if (e != hipSuccess) return e;
    const size_t gsm = (size_t)(np * np + 2 * (kTqThreads / 64) * 256) * sizeof(double);
    const size_t csm = (size_t)(2 * np * np + 2 * kQrScratch) * sizeof(double);
    if ((e = hipFuncSetAttribute((const void*)k_tqr_gram<NB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)gsm)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void*)k_tqr_chol<NB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)csm)) != hipSuccess)
        return e;
    const int passes = final_basis ? 3 : 2;
    for (int pass = 0; pass < passes; ++pass) {
        hipLaunchKernelGGL(k_tqr_gram<NB>, dim3((unsigned)nblk), dim3(kTqThreads), gsm, s, Y, m, n, ldy, work);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_tqr_chol<NB>, dim3(1), dim3(qr_threads<NB>()), csm, s, m, n, nblk, pass, work);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_tqr_apply<NB>, dim3((unsigned)nblk), dim3(kTqThreads), 0, s, Y, m, n, ldy, work,
                           Qpad, ldq, Qout, pass == passes - 1 ? 1 : 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const size_t fsm = (2 * (size_t)np * np + 2 * kQrScratch) * sizeof(double);
    if ((e = hipFuncSetAttribute((const void*)k_tqr_fallback<NB>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)fsm)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_tqr_fallback<NB>, dim3(1), dim3(qr_threads<NB>()), fsm, s, Y, m, n, ldy, Qpad, ldq,
                       Qout, final_basis ? 1 : 0, status, work);
    return hipGetLastError();
}

// doubles of work space the tall form needs
size_t qr_tall_work_doubles(int64_t m, int n) {
    const int np = (n + 15) & ~15;
    return 8 + (size_t)np * np + (size_t)((m + kTqRows - 1) / kTqRows) * np * np;
}

static size_t qr_lds_bytes(int64_t m, int n) {
    const int np = (n + 15) & ~15;
    return ((size_t)m * (np + 1) + 2 * (size_t)np * np + kQrScratch) * sizeof(double);
}

template <bool L, int NB>
static hipError_t launch_qr_t(double* Y, int m, int n, int ldy, float* Qpad, int ldq, float* Qout,
                              int sp, int* status, size_t lds, hipStream_t s) {
    hipError_t e = hipFuncSetAttribute((const void*)k_qr<L, NB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_qr<L, NB>), dim3(1), dim3(qr_threads<NB>()), lds, s, Y, m, n, ldy, Qpad, ldq,
                       Qout, sp, status);
    return hipGetLastError();
}

template <bool L>
static hipError_t launch_qr_l(double* Y, int m, int n, int ldy, float* Qpad, int ldq, float* Qout,
                              int sp, int* status, size_t lds, hipStream_t s) {
    switch ((n + 15) >> 4) {
        case 1: return launch_qr_t<L, 1>(Y, m, n, ldy, Qpad, ldq, Qout, sp, status, lds, s);
        case 2: return launch_qr_t<L, 2>(Y, m, n, ldy, Qpad, ldq, Qout, sp, status, lds, s);
        case 3: return launch_qr_t<L, 3>(Y, m, n, ldy, Qpad, ldq, Qout, sp, status, lds, s);
        default: return launch_qr_t<L, 4>(Y, m, n, ldy, Qpad, ldq, Qout, sp, status, lds, s);
    }
}

// the dynamic LDS a problem's QR takes (0: too tall for the LDS form)
size_t qr_group_lds(int64_t m, int n) {
    const size_t lds = qr_lds_bytes(m, n);
    return lds <= kQrLds - 4096 ? lds : 0;
}

hipError_t launch_qr_group(const QrDesc* d, int count, int NBv, bool use_lds, size_t lds,
                           hipStream_t s) {
    if (count < 1) return hipSuccess;
    if (!use_lds) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    auto go = [&](auto kern, int threads) {
        e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return;
        hipLaunchKernelGGL(kern, dim3((unsigned)count), dim3(threads), lds, s, d);
        e = hipGetLastError();
    };
    switch (NBv) {
        case 1: go(k_qr_grp<true, 1>, qr_threads<1>()); break;
        case 2: go(k_qr_grp<true, 2>, qr_threads<2>()); break;
        case 3: go(k_qr_grp<true, 3>, qr_threads<3>()); break;
        default: go(k_qr_grp<true, 4>, qr_threads<4>()); break;
    }
    return e;
}

hipError_t launch_qr(double* Y, int64_t m, int n, int ldy, float* Qpad, int ldq, float* Qout,
                     bool final_basis, int* status, hipStream_t s, double* work) {
    const int np = (n + 15) & ~15;
    if (n < 1 || n > 64 || ldy < np || ldq < n || m < n || m > ((int64_t)1 << 24)) return hipErrorInvalidValue;
    const int sp = final_basis ? 1 : 0;
    const size_t lds = qr_lds_bytes(m, n);
    if (lds <= kQrLds - 4096)
        return launch_qr_l<true>(Y, (int)m, n, ldy, Qpad, ldq, Qout, sp, status, lds, s);
    if (work != nullptr) {
        switch (np >> 4) {
            case 1: return launch_tqr_t<1>(Y, (int)m, n, ldy, Qpad, ldq, Qout, final_basis, status, work, s);
            case 2: return launch_tqr_t<2>(Y, (int)m, n, ldy, Qpad, ldq, Qout, final_basis, status, work, s);
            case 3: return launch_tqr_t<3>(Y, (int)m, n, ldy, Qpad, ldq, Qout, final_basis, status, work, s);
            default: return launch_tqr_t<4>(Y, (int)m, n, ldy, Qpad, ldq, Qout, final_basis, status, work, s);
        }
    }
    const size_t small = (2 * (size_t)np * np + 2 * kQrScratch) * sizeof(double);
    return launch_qr_l<false>(Y, (int)m, n, ldy, Qpad, ldq, Qout, sp, status, small, s);
}

}  // namespace rcp
