// CP-ALS on the compressed tensor B (Section 3.2.1, Algorithm 2 steps 2-11)
// in one workgroup.  The core is small (l^N elements) and a sweep is a strict
// sequence of dependent least-squares updates, so the whole sweep loop runs
// in one persistent workgroup, with the stopping rule on the device.
//
// Per sweep the mode products B_(n) KR(Ã_{m != n}) use one split of the
// modes, H1 = {0..N-2} and the last mode, so that only two contractions of
// the full core are needed per sweep (instead of N):
//   W[rho, r]     = sum_k B[rho, k] Ã_{N-1}[k, r]                (rho over H1)
//   M_n[i, r]     = sum_{rho: i_n(rho)=i} W[rho, r] prod_{m in H1, m!=n} Ã_m[i_m(rho), r]
//   M_{N-1}[i, r] = sum_rho B[rho, i] prod_{m in H1} Ã_m[i_m(rho), r]
// Each M_n is exactly the mode-n product of the definition, computed with
// the factors Algorithm 2 uses at that point (earlier modes already updated).
// The two core contractions run on the matrix cores (FP32 operands, FP32
// accumulation); Grams, solves, norms and the fit are float64.

#include "rcp_device.h"
#include "rcp_kernels.h"

namespace rcp {

#ifdef RCP_ALS_TIMING
__device__ unsigned long long g_als_stamps[64];
#define ALS_STAMP(slot)                                                                    \
    do {                                                                                   \
        __syncthreads();                                                                   \
        if (threadIdx.x == 0 && it_dbg < 3) g_als_stamps[it_dbg * 16 + (slot)] = wall_clock64(); \
    } while (0)
#else
#define ALS_STAMP(slot) do {} while (0)
#endif

constexpr int ANT = 512;
constexpr int ANW = ANT / 64;
constexpr double kPivotRtol = 1e-13;
constexpr int kJacobiMaxSweeps = 40;
constexpr int kEigLd = 64;
constexpr size_t kAlsLds = 160 * 1024 - 4096;   // dynamic LDS budget

struct AlsCtx {
    int N, R;
    int S, Lh, lN;
    const int* l;                  // LDS: mode sizes l_0..l_{N-1}
    const int* foff;               // LDS: offset of factor n inside fbase
    float* fbase;                  // LDS: l_n x R working factors (matrix-core operands)
    double* red;                   // ANW doubles (LDS)
    double* sh;                    // 128 doubles (LDS)
    __device__ __forceinline__ float* fac(int n) const { return fbase + foff[n]; }
};

// ---------------------------------------------------------------------------
// Parallel cyclic Jacobi eigen-decomposition of the symmetric n x n matrix
// A (row stride kEigLd, overwritten; eigenvalues end on the diagonal), with
// the eigenvectors accumulated in the columns of V.  Round-robin (circle
// method) ordering: each round rotates n/2 disjoint (p, q) pairs.  Returns
// false if the off-diagonal mass did not fall below 1e-30 of the diagonal's.
__device__ __forceinline__ bool jacobi_eig(double* A, double* V, int n, double* red, double* sh) {
    const int tid = threadIdx.x;
    const int np = (n + 1) & ~1;
    double* cs = sh;
    double* sn = sh + 32;
    int* pp = (int*)(sh + 64);
    int* qq = pp + 32;
    for (int i = tid / 64; i < n; i += ANW)
        for (int j = tid % 64; j < n; j += 64) V[i * kEigLd + j] = (i == j) ? 1.0 : 0.0;
    __syncthreads();
    bool converged = false;
    for (int sweep = 0; sweep < kJacobiMaxSweeps; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int i = tid / 64; i < n; i += ANW)
            for (int j = tid % 64; j < n; j += 64) {
                const double v = A[i * kEigLd + j];
                if (i == j) dia += v * v; else off += v * v;
            }
        off = block_sum(off, red);
        dia = block_sum(dia, red);
        if (off <= 1e-30 * dia || off == 0.0) { converged = true; break; }
        for (int round = 0; round < np - 1; ++round) {
            if (tid < np / 2) {
                const int k = tid;
                int a = (k == 0) ? 0 : ((k - 1 + round) % (np - 1)) + 1;
                int b = ((np - 2 - k + round) % (np - 1)) + 1;
                if (a > b) { const int t = a; a = b; b = t; }
                double c = 1.0, s = 0.0;
                if (b < n) {
                    const double apq = A[a * kEigLd + b];
                    if (apq != 0.0) {
                        const double app = A[a * kEigLd + a], aqq = A[b * kEigLd + b];
                        const double th = (aqq - app) / (2.0 * apq);
                        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                    }
                }
                cs[k] = c; sn[k] = s; pp[k] = a; qq[k] = b;
            }
            __syncthreads();
            // rows: A <- J^T A   (thread = (pair k, column j))
            for (int k = tid / 64; k < np / 2; k += ANW) {
                const int p = pp[k], q = qq[k];
                if (q < n && sn[k] != 0.0) {
                    const double c = cs[k], s = sn[k];
                    for (int j = tid % 64; j < n; j += 64) {
                        const double ap = A[p * kEigLd + j], aq = A[q * kEigLd + j];
                        A[p * kEigLd + j] = c * ap - s * aq;
                        A[q * kEigLd + j] = s * ap + c * aq;
                    }
                }
            }
            __syncthreads();
            // columns: A <- A J, V <- V J   (thread = (pair k, row i))
            for (int k = tid / 64; k < np / 2; k += ANW) {
                const int p = pp[k], q = qq[k];
                if (q < n && sn[k] != 0.0) {
                    const double c = cs[k], s = sn[k];
                    for (int i = tid % 64; i < n; i += 64) {
                        const double ap = A[i * kEigLd + p], aq = A[i * kEigLd + q];
                        A[i * kEigLd + p] = c * ap - s * aq;
                        A[i * kEigLd + q] = s * ap + c * aq;
                        const double vp = V[i * kEigLd + p], vq = V[i * kEigLd + q];
                        V[i * kEigLd + p] = c * vp - s * vq;
                        V[i * kEigLd + q] = s * vp + c * vq;
                    }
                }
            }
            __syncthreads();
        }
    }
    return converged;
}

__device__ __forceinline__ int desc_rank(const double* A, int n, int e) {
    const double w = A[e * kEigLd + e];
    int r = 0;
    for (int f = 0; f < n; ++f) {
        const double v = A[f * kEigLd + f];
        if (v > w || (v == w && f < e)) ++r;
    }
    return r;
}

// Algorithm 2 step 2: leading R eigenvectors of B_(n) B_(n)^T.
__device__ __forceinline__ bool eig_init(const AlsCtx& c, const float* Bg, int n, double* E,
                                         double* V) {
    const int tid = threadIdx.x;
    const int ln = c.l[n];
    int Ln = 1, Rn = 1;
    for (int m = 0; m < n; ++m) Ln *= c.l[m];
    for (int m = n + 1; m < c.N; ++m) Rn *= c.l[m];
    const int npairs = ln * (ln + 1) / 2;
    for (int e = tid; e < npairs; e += ANT) {
        int i = 0, rem = e;
        while (rem >= ln - i) { rem -= ln - i; ++i; }
        const int i2 = i + rem;
        double s = 0.0;
        for (int a = 0; a < Ln; ++a) {
            const float* r1 = Bg + ((int64_t)a * ln + i) * Rn;
            const float* r2 = Bg + ((int64_t)a * ln + i2) * Rn;
            for (int b = 0; b < Rn; ++b) s += (double)r1[b] * (double)r2[b];
        }
        E[i * kEigLd + i2] = s;
        E[i2 * kEigLd + i] = s;
    }
    __syncthreads();
    const bool ok = jacobi_eig(E, V, ln, c.red, c.sh);
    for (int e = tid; e < ln; e += ANT) {
        const int r = desc_rank(E, ln, e);
        if (r < c.R) {
            int best = 0;
            double bv = -1.0;
            for (int i = 0; i < ln; ++i) {
                const double v = fabs(V[i * kEigLd + e]);
                if (v > bv) { bv = v; best = i; }
            }
            const double sg = (V[best * kEigLd + e] < 0.0) ? -1.0 : 1.0;
            for (int i = 0; i < ln; ++i) c.fac(n)[i * c.R + r] = (float)(sg * V[i * kEigLd + e]);
        }
    }
    __syncthreads();
    return ok;
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// G_n = Ã_n^T Ã_n in float64 from the float32 factor.
__device__ __forceinline__ void gram_of(const AlsCtx& c, int n, double* G) {
    const int R = c.R, ln = c.l[n];
    const float* A = c.fac(n);
    for (int e = threadIdx.x; e < R * R; e += ANT) {
        const int r = e / R, s = e - r * R;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int i = 0;
        for (; i + 4 <= ln; i += 4) {
            a0 += (double)A[i * R + r] * (double)A[i * R + s];
            a1 += (double)A[(i + 1) * R + r] * (double)A[(i + 1) * R + s];
            a2 += (double)A[(i + 2) * R + r] * (double)A[(i + 2) * R + s];
            a3 += (double)A[(i + 3) * R + r] * (double)A[(i + 3) * R + s];
        }
        for (; i < ln; ++i) a0 += (double)A[i * R + r] * (double)A[i * R + s];
        G[e] = (a0 + a1) + (a2 + a3);
    }
}

// Wavefront 0 solves V X^T = M^T (V symmetric positive definite, R x R) by
// Gauss-Jordan elimination on the augmented matrix [V | M^T] held in LDS
// (row stride 128): lane c owns columns c and c + 64, rows are processed
// four at a time so their LDS accesses overlap.  The loop form keeps the
// code small (this kernel is one workgroup walking long sequences, so
// instruction-cache misses matter more than unrolling).  On return X
// (ln x R, row-major) is in Xo.  Returns 0 when a pivot falls below
// kPivotRtol times the largest diagonal entry of V (the caller then takes
// the pseudo-inverse).
__device__ __forceinline__ int wave_gj_solve(double* V, const double* M, double* Aug, double* Xo,
                                             int R, int ln) {
    const int lane = threadIdx.x;
    const int W = R + ln;
    for (int i = 0; i < R; ++i)
        for (int cc = lane; cc < W; cc += 64)
            Aug[i * 128 + cc] = (cc < R) ? V[i * R + cc] : M[(cc - R) * R + i];
    double maxd = (lane < R) ? V[lane * R + lane] : 0.0;
    for (int o = 32; o > 0; o >>= 1) maxd = fmax(maxd, __shfl_xor(maxd, o, 64));
    const double thr = kPivotRtol * maxd;
    wave_lds_sync();
    int ok = 1;
    for (int j = 0; j < R; ++j) {
        const double piv = Aug[j * 128 + j];
        ok &= (piv > thr) ? 1 : 0;
        const double ip = 1.0 / fmax(piv, thr);
        for (int cc = lane; cc < W; cc += 64) {
            if (cc <= j) continue;
            const double pr = Aug[j * 128 + cc] * ip;
            int i = 0;
            for (; i + 4 <= R; i += 4) {
                const double f0 = Aug[i * 128 + j], f1 = Aug[(i + 1) * 128 + j];
                const double f2 = Aug[(i + 2) * 128 + j], f3 = Aug[(i + 3) * 128 + j];
                const double a0 = Aug[i * 128 + cc], a1 = Aug[(i + 1) * 128 + cc];
                const double a2 = Aug[(i + 2) * 128 + cc], a3 = Aug[(i + 3) * 128 + cc];
                Aug[i * 128 + cc] = (i == j) ? pr : a0 - f0 * pr;
                Aug[(i + 1) * 128 + cc] = (i + 1 == j) ? pr : a1 - f1 * pr;
                Aug[(i + 2) * 128 + cc] = (i + 2 == j) ? pr : a2 - f2 * pr;
                Aug[(i + 3) * 128 + cc] = (i + 3 == j) ? pr : a3 - f3 * pr;
            }
            for (; i < R; ++i) {
                const double f = Aug[i * 128 + j], av = Aug[i * 128 + cc];
                Aug[i * 128 + cc] = (i == j) ? pr : av - f * pr;
            }
        }
        wave_lds_sync();
    }
    if (!ok) return 0;
    for (int cc = 0; cc < R; ++cc)
        for (int i = lane; i < ln; i += 64) Xo[i * R + cc] = Aug[cc * 128 + R + i];
    return 1;
}

// Exact quotient of a non-negative int below 2^31 by a positive divisor,
// from a float64 reciprocal and one correction step.
__device__ __forceinline__ int div_exact(int a, int d, double inv_d) {
    int q = (int)((double)a * inv_d);
    const int r = a - q * d;
    if (r < 0) --q;
    else if (r >= d) ++q;
    return q;
}

// C = A (R x R) * Bm (R x R), float64, all threads; row-major, LDS.
__device__ __forceinline__ void small_gemm(const double* A, const double* Bm, double* C, int R) {
    for (int e = threadIdx.x; e < R * R; e += ANT) {
        const int i = e / R, j = e - (e / R) * R;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int k = 0;
        for (; k + 4 <= R; k += 4) {
            s0 += A[i * R + k] * Bm[k * R + j];
            s1 += A[i * R + k + 1] * Bm[(k + 1) * R + j];
            s2 += A[i * R + k + 2] * Bm[(k + 2) * R + j];
            s3 += A[i * R + k + 3] * Bm[(k + 3) * R + j];
        }
        for (; k < R; ++k) s0 += A[i * R + k] * Bm[k * R + j];
        C[e] = (s0 + s1) + (s2 + s3);
    }
}

__device__ __forceinline__ double block_max(double v, double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = red[0];
    for (int i = 1; i < ANW; ++i) t = fmax(t, red[i]);
    return t;
}

constexpr int kNsMaxIters = 60;
constexpr double kNsTol = 1e-11;

// V^{-1} for the symmetric positive definite V (R x R, LDS) by Newton-Schulz
// iteration X <- X (2I - V X) (Schulz 1933), started from Xi when `warm`
// (the previous sweep's inverse for the same mode) and otherwise from
// V / ||V||_inf^2, which converges for every non-singular V.  Stops once
// max |V X - I| <= kNsTol, after one more step.  Returns 1 and the inverse in
// Xi on convergence, 0 otherwise.  All threads; T, X2 are R x R scratch.
__device__ __forceinline__ int ns_inverse(const double* V, double* Xi, double* T, double* X2, int R,
                                          bool warm, double* red) {
    const int tid = threadIdx.x;
    double rs = 0.0;
    for (int i = tid; i < R; i += ANT) {
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += fabs(V[i * R + k]);
        rs = fmax(rs, s);
    }
    const double ninf = block_max(rs, red);
    if (!(ninf > 0.0) || !isfinite(ninf)) return 0;
    const double scale = 1.0 / (ninf * ninf);
    if (!warm)
        for (int e = tid; e < R * R; e += ANT) Xi[e] = V[e] * scale;
    __syncthreads();
    bool restarted = !warm;
    for (int k = 0; k < kNsMaxIters; ++k) {
        small_gemm(V, Xi, T, R);
        __syncthreads();
        double dev = 0.0;
        for (int e = tid; e < R * R; e += ANT) {
            const int i = e / R, j = e - (e / R) * R;
            dev = fmax(dev, fabs(T[e] - (i == j ? 1.0 : 0.0)));
        }
        const double r = block_max(dev, red);
        if (!isfinite(r)) return 0;
        if (!restarted && r > 0.5) {
            // warm start too far from the new inverse: restart from the scaled V
            for (int e = tid; e < R * R; e += ANT) Xi[e] = V[e] * scale;
            restarted = true;
            __syncthreads();
            continue;
        }
        // X2 = 2 X - X T
        small_gemm(Xi, T, X2, R);
        __syncthreads();
        for (int e = tid; e < R * R; e += ANT) Xi[e] = 2.0 * Xi[e] - X2[e];
        __syncthreads();
        if (r <= kNsTol) return 1;
    }
    return 0;
}

// Ã_n = M V^+ with V = *_{m != n} G_m, then column normalisation; the factor
// lands in c.fac(n) and its Gram in G_n.  Returns RCP_INFO_* bits.
__device__ __forceinline__ int solve_update(const AlsCtx& c, int n, double* G, const double* M,
                                            double* X, double* V, double* Xi, double* T,
                                            double* X2, int* ns_valid, double* Aug, double* E,
                                            double* Ev, double* lam, int* flag) {
    const int tid = threadIdx.x, R = c.R, ln = c.l[n];
    int status = 0;
    for (int e = tid; e < R * R; e += ANT) {
        double v = 1.0;
        for (int m = 0; m < c.N; ++m)
            if (m != n) v *= G[m * R * R + e];
        V[e] = v;
    }
    __syncthreads();
    double* Xin = Xi + n * R * R;
    int ok = ns_inverse(V, Xin, T, X2, R, ns_valid[n] != 0, c.red);
    __syncthreads();
    if (ok) {
        if (tid == 0) ns_valid[n] = 1;
        // X = M V^{-1}
        for (int e = tid; e < ln * R; e += ANT) {
            const int i = e / R, s = e - (e / R) * R;
            double a0 = 0.0, a1 = 0.0;
            int r = 0;
            for (; r + 2 <= R; r += 2) {
                a0 += M[i * R + r] * Xin[r * R + s];
                a1 += M[i * R + r + 1] * Xin[(r + 1) * R + s];
            }
            if (r < R) a0 += M[i * R + r] * Xin[r * R + s];
            X[e] = a0 + a1;
        }
    } else {
        if (tid == 0) ns_valid[n] = 0;
        if (tid < 64) {
            const int okg = wave_gj_solve(V, M, Aug, X, R, ln);
            if (tid == 0) *flag = okg;
        }
        __syncthreads();
        if (!*flag) {
            // Moore-Penrose pseudo-inverse through the eigen-decomposition
            status |= RCP_INFO_PINV_FALLBACK;
            for (int e = tid; e < R * R; e += ANT) E[(e / R) * kEigLd + (e % R)] = V[e];
            __syncthreads();
            jacobi_eig(E, Ev, R, c.red, c.sh);
            double wmax = 0.0;
            for (int f = 0; f < R; ++f) wmax = fmax(wmax, fabs(E[f * kEigLd + f]));
            const double cut = kPivotRtol * wmax;
            for (int e = tid; e < R * R; e += ANT) {
                const int r = e / R, s = e % R;
                double acc = 0.0;
                for (int f = 0; f < R; ++f) {
                    const double w = E[f * kEigLd + f];
                    if (w > cut) acc += Ev[r * kEigLd + f] * Ev[s * kEigLd + f] / w;
                }
                V[e] = acc;                                     // V <- V^+
            }
            __syncthreads();
            for (int e = tid; e < ln * R; e += ANT) {
                const int i = e / R, s = e % R;
                double acc = 0.0;
                for (int r = 0; r < R; ++r) acc += M[i * R + r] * V[r * R + s];
                X[e] = acc;
            }
        }
    }
    __syncthreads();
    // unit columns; wavefront w takes columns r = w, w + 8, ...
    {
        const int lane = tid & 63, wave = tid >> 6;
        for (int r = wave; r < R; r += ANW) {
            double ss = 0.0;
            for (int i = lane; i < ln; i += 64) ss += X[i * R + r] * X[i * R + r];
            ss = warp_sum(ss);
            if (lane == 0) lam[r] = sqrt(ss);
        }
    }
    __syncthreads();
    {
        float* fn = c.fac(n);
        for (int e = tid; e < ln * R; e += ANT) {
            const double nu = lam[e % R];
            fn[e] = (float)((nu > 0.0) ? X[e] / nu : X[e]);
        }
    }
    __syncthreads();
    gram_of(c, n, G + n * R * R);
    __syncthreads();
    return status;
}

// Per-wavefront partial products Mpart[wave] (l_n x R, row stride 64) of the
// mode-n product B_(n) KR(Ã_{m != n}) on the matrix cores.  The core is
// viewed as (Ln, l_n, Rn); the contraction index k = a * Rn + b runs over the
// other modes and is split evenly over the wavefronts; the Khatri-Rao
// operand KR[k, r] = prod_{m != n} Ã_m[i_m(k), r] is formed on the fly from
// the factors in LDS.
__device__ __forceinline__ void mttkrp_mfma(const AlsCtx& c, int n, const float* B, float* Mpart) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int N = c.N, R = c.R, ln = c.l[n];
    int lm[RCP_MAX_NDIM];
    double inv_l[RCP_MAX_NDIM];
    const float* fm[RCP_MAX_NDIM];
    int Ln = 1, Rn = 1;
#pragma unroll
    for (int m = 0; m < RCP_MAX_NDIM; ++m) {
        lm[m] = (m < N) ? c.l[m] : 1;
        inv_l[m] = 1.0 / (double)lm[m];
        fm[m] = c.fac(m < N ? m : 0);
        if (m < n) Ln *= lm[m];
        if (m > n && m < N) Rn *= lm[m];
    }
    const double inv_Rn = 1.0 / (double)Rn;
    const int K = Ln * Rn;
    const int nib = (ln + 15) / 16, ncb = (R + 15) / 16;
    const int per = ((K + ANW - 1) / ANW + 3) & ~3;
    const int k_lo = wave * per;
    const int k_hi = min(K, k_lo + per);
    f32x4 acc[4][4];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[ib][cb] = f32x4{0, 0, 0, 0};
    for (int k0 = k_lo; k0 < k_hi; k0 += 4) {
        const int k = k0 + lk;
        const bool kv = k < k_hi;
        const int kk = kv ? k : 0;
        const int ai = div_exact(kk, Rn, inv_Rn);
        const int bi = kk - ai * Rn;
        int base[RCP_MAX_NDIM];
        int rem = bi;
#pragma unroll
        for (int m = RCP_MAX_NDIM - 1; m >= 0; --m) {
            base[m] = 0;
            if (m > n && m < N) {
                const int q = div_exact(rem, lm[m], inv_l[m]);
                base[m] = (rem - q * lm[m]) * R;
                rem = q;
            }
        }
        rem = ai;
#pragma unroll
        for (int m = RCP_MAX_NDIM - 1; m >= 0; --m) {
            if (m < n) {
                const int q = div_exact(rem, lm[m], inv_l[m]);
                base[m] = (rem - q * lm[m]) * R;
                rem = q;
            }
        }
        const int row0 = ai * ln * Rn + bi;
        float a[4], b[4];
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
            const int i = ib * 16 + lr;
            a[ib] = (kv && ib < nib && i < ln) ? B[row0 + i * Rn] : 0.0f;
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int col = cb * 16 + lr;
            float w = 0.0f;
            if (kv && cb < ncb && col < R) {
                w = 1.0f;
#pragma unroll
                for (int m = 0; m < RCP_MAX_NDIM; ++m)
                    if (m < N && m != n) w *= fm[m][base[m] + col];
            }
            b[cb] = w;
        }
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
            if (ib < nib)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    if (cb < ncb) acc[ib][cb] = mfma16x16x4(a[ib], b[cb], acc[ib][cb]);
    }
    float* mine = Mpart + wave * 64 * 64;
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
        if (ib < nib)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                if (cb < ncb)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        mine[(ib * 16 + 4 * lk + v) * 64 + cb * 16 + lr] = acc[ib][cb][v];
}

template <bool B_IN_LDS, bool EIG_IN_LDS>
__global__ __launch_bounds__(ANT) void k_als(AlsArgs a) {
    extern __shared__ __align__(16) unsigned char als_smem[];
    __shared__ double red[ANW];
    __shared__ double sh[128];
    __shared__ double lam[RCP_MAX_RANK];
    __shared__ double lam_tmp[RCP_MAX_RANK];
    __shared__ int flag;
    __shared__ int ns_valid[RCP_MAX_NDIM];
    __shared__ int sl[RCP_MAX_NDIM];
    __shared__ int sfoff[RCP_MAX_NDIM];
    const int tid = threadIdx.x;
    const int N = a.N, R = a.R;

    AlsCtx c;
    c.N = N;
    c.R = R;
    c.S = 1;
    int lmax = 0;
    size_t fbytes = 0;
#pragma unroll
    for (int n = 0; n < RCP_MAX_NDIM; ++n) {
        if (n < N) {
            c.S *= a.l[n];
            lmax = max(lmax, a.l[n]);
            if (tid == 0) { sl[n] = a.l[n]; sfoff[n] = (int)(fbytes / sizeof(float)); ns_valid[n] = 0; }
            fbytes += ((size_t)a.l[n] * R * sizeof(float) + 15) & ~(size_t)15;
        }
    }
    c.lN = a.l[N - 1];
    c.Lh = c.S / c.lN;
    c.red = red;
    c.sh = sh;
    c.l = sl;
    c.foff = sfoff;

    // dynamic LDS: [factors | G | V | M | X | Xinv (N R^2) | T | X2 | big: E,V (init) then the core]
    unsigned char* p = als_smem;
    c.fbase = (float*)p;
    p += fbytes;
    double* G = (double*)p;  p += (size_t)N * R * R * sizeof(double);
    double* V = (double*)p;  p += (size_t)R * R * sizeof(double);
    double* M = (double*)p;  p += (size_t)lmax * R * sizeof(double);
    double* X = (double*)p;  p += (size_t)lmax * R * sizeof(double);
    double* Xi = (double*)p; p += (size_t)N * R * R * sizeof(double);
    double* T = (double*)p;  p += (size_t)R * R * sizeof(double);
    double* X2 = (double*)p; p += (size_t)R * R * sizeof(double);
    double* E = EIG_IN_LDS ? (double*)p : a.Ebuf;
    double* Ev = E + kEigLd * kEigLd;
    double* Es = a.Ebuf;
    double* Evs = a.Ebuf + kEigLd * kEigLd;
    double* Aug = a.Ebuf + 2 * kEigLd * kEigLd;         // 64 x 128 Gauss-Jordan scratch
    float* Bl = (float*)p;
    float* Mpart = a.Mpart;
    __syncthreads();

    double s = 0.0;
    for (int e = tid; e < c.S; e += ANT) { const double v = a.B[e]; s += v * v; }
    const double normB2 = block_sum(s, red);
    const double normX2 = (a.normX2 != nullptr) ? *a.normX2 : normB2;

    int status = 0;
    for (int n = 1; n < N; ++n) {
        if (!eig_init(c, a.B, n, E, Ev)) status |= RCP_INFO_EIG_NOT_CONVERGED;
        gram_of(c, n, G + n * R * R);
    }
    __syncthreads();
    if (B_IN_LDS)
        for (int e = tid; e < c.S; e += ANT) Bl[e] = a.B[e];
    __syncthreads();
    const float* Bs = B_IN_LDS ? Bl : a.B;

    double rho = 0.0, rho_prev = 0.0;
    int it;
    for (it = 1; it <= a.max_iters; ++it) {
#ifdef RCP_ALS_TIMING
        const int it_dbg = it - 1;
#endif
        ALS_STAMP(0);
        for (int n = 0; n < N; ++n) {
            mttkrp_mfma(c, n, Bs, Mpart);
            __syncthreads();
            const int ln = c.l[n];
            for (int e = tid; e < ln * R; e += ANT) {
                const int i = e / R, r = e - (e / R) * R;
                double acc = 0.0;
#pragma unroll
                for (int w = 0; w < ANW; ++w) acc += (double)Mpart[w * 64 * 64 + i * 64 + r];
                M[e] = acc;
            }
            __syncthreads();
            ALS_STAMP(2 + 2 * n);
            status |= solve_update(c, n, G, M, X, V, Xi, T, X2, ns_valid, Aug, Es, Evs,
                                   (n == N - 1) ? lam : lam_tmp, &flag);
            ALS_STAMP(3 + 2 * n);
        }
        // ---- fit (Section 3.3): rho = 1 - (||X||^2 + ||Xhat||^2 - 2 <Xhat, X>) / ||X||^2
        double pi = 0.0;
        const float* AN = c.fac(N - 1);
        for (int e = tid; e < c.lN * R; e += ANT) pi += lam[e % R] * M[e] * (double)AN[e];
        double pm = 0.0;
        for (int e = tid; e < R * R; e += ANT) {
            double v = lam[e / R] * lam[e % R];
            for (int m = 0; m < N; ++m) v *= G[m * R * R + e];
            pm += v;
        }
        const double inner = block_sum(pi, red);
        const double model = block_sum(pm, red);
        const double err2 = normX2 - 2.0 * inner + model;
        rho = (normX2 > 0.0) ? 1.0 - err2 / normX2 : 0.0;
        ALS_STAMP(15);
        if (!isfinite(rho)) { status |= RCP_INFO_NONFINITE; break; }
        if (a.tol > 0.0 && it >= 2 && fabs(rho - rho_prev) < a.tol) break;
        rho_prev = rho;
    }
    if (it > a.max_iters) it = a.max_iters;

#pragma unroll
    for (int n = 0; n < RCP_MAX_NDIM; ++n)
        if (n < N)
            for (int e = tid; e < a.l[n] * R; e += ANT) a.At[n][e] = c.fac(n)[e];
    for (int r = tid; r < R; r += ANT) a.lambda[r] = (float)lam[r];
    if (tid == 0) {
        a.info->iters = it;
        a.info->status = status;
        a.info->rho = rho;
        a.info->rel_err = sqrt(fmax(0.0, 1.0 - rho));
        a.info->normX2 = normX2;
    }
}

static size_t als_lds_fixed(int N, const int* l, int R) {
    size_t b = 0;
    int lmax = 0;
    for (int n = 0; n < N; ++n) {
        b += ((size_t)l[n] * R * sizeof(float) + 15) & ~(size_t)15;
        lmax = lmax > l[n] ? lmax : l[n];
    }
    b += (size_t)N * R * R * sizeof(double);          // G
    b += (size_t)R * R * sizeof(double);              // V
    b += 2 * (size_t)lmax * R * sizeof(double);       // M, X
    b += (size_t)N * R * R * sizeof(double);          // inverses (Newton-Schulz warm starts)
    b += 2 * (size_t)R * R * sizeof(double);          // T, X2
    return b;
}

// workspace: Mpart (ANW x 64 x 64 floats), then (doubles) Jacobi scratch
// (2 x 64 x 64) and the Gauss-Jordan scratch (64 x 128)
size_t als_workspace_floats(int N, const int* l, int R) {
    (void)N; (void)l; (void)R;
    return (size_t)ANW * 64 * 64;
}

size_t als_workspace_doubles(int N, const int* l, int R) {
    const size_t f = als_workspace_floats(N, l, R);
    return (f + 1) / 2 + 2 * kEigLd * kEigLd + 64 * 128 + 64;
}

bool als_supported(int N, const int* l, int R) {
    int64_t S = 1;
    for (int n = 0; n < N; ++n) S *= l[n];
    return S < ((int64_t)1 << 31) && als_lds_fixed(N, l, R) <= kAlsLds;
}

template <bool BL, bool EL>
static hipError_t launch_als_t(const AlsArgs& a, size_t smem, hipStream_t s) {
    auto k = k_als<BL, EL>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kAlsLds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(1), dim3(ANT), smem, s, a);
    return hipGetLastError();
}

hipError_t launch_als(const AlsArgs& a, hipStream_t s) {
    const size_t fixed = als_lds_fixed(a.N, a.l, a.R);
    int64_t S = 1;
    for (int n = 0; n < a.N; ++n) S *= a.l[n];
    const size_t eig = 2 * kEigLd * kEigLd * sizeof(double);
    const size_t bsz = (size_t)S * sizeof(float);
    const bool bl = fixed + bsz <= kAlsLds;
    const bool el = fixed + eig <= kAlsLds;
    size_t big = 0;
    if (bl) big = bsz;
    if (el && eig > big) big = eig;
    const size_t smem = fixed + big;
    if (bl && el) return launch_als_t<true, true>(a, smem, s);
    if (bl) return launch_als_t<true, false>(a, smem, s);
    if (el) return launch_als_t<false, true>(a, smem, s);
    return launch_als_t<false, false>(a, smem, s);
}

}  // namespace rcp

#ifdef RCP_ALS_TIMING
extern "C" int rcp_debug_als_stamps(unsigned long long* host_out) {
    return (int)hipMemcpyFromSymbol(host_out, HIP_SYMBOL(rcp::g_als_stamps), sizeof(rcp::g_als_stamps));
}
#endif
