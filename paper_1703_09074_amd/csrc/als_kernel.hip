// CP-ALS on the compressed tensor B (Section 3.2.1, Algorithm 2 steps 2-11)
// in one workgroup: the core is small (l^N elements) and the sweep loop is
// a strict sequence of dependent least-squares updates, so it runs as one
// persistent workgroup with the whole sweep loop on the device (no host
// round trip per sweep, device-side stopping rule).
//
// Arithmetic is float64 on the vector ALU (on MI355X the float64 vector rate
// equals the non-packed float32 rate); the core itself is float32.
//
// Per sweep the mode-n products B_(n) KR(Ã_{m != n}) are computed with one
// split of the modes into H1 = {0..N-2} and H2 = {N-1}:
//   W[rho, r]   = sum_k B[rho, k] Ã_{N-1}[k, r]            (rho over H1)
//   M_n[i, r]   = sum_{rho: i_n(rho) = i} W[rho, r] prod_{m in H1, m != n} Ã_m[i_m, r]
//   M_{N-1}[i,r]= sum_rho B[rho, i] prod_{m in H1} Ã_m[i_m(rho), r]
// which equals the definition mode by mode (the updated Ã_m of earlier
// modes enter the later products exactly as in Algorithm 2).

#include "rcp_device.h"
#include "rcp_kernels.h"

namespace rcp {

constexpr int ANT = 512;
constexpr double kPivotRtol = 1e-13;
constexpr int kJacobiMaxSweeps = 40;
constexpr int kEigLd = 64;

struct AlsCtx {
    const float* B;
    int N, R;
    int l[RCP_MAX_NDIM];
    int64_t S, Lh;
    double* fac[RCP_MAX_NDIM];     // l_n x R, float64 working factors
    double* red;                   // ANT/64 doubles (LDS)
    double* sh;                    // 128 doubles (LDS)
};

// ---------------------------------------------------------------------------
// Parallel cyclic Jacobi eigen-decomposition of the symmetric n x n matrix
// A (row stride kEigLd, overwritten; eigenvalues end on the diagonal), with
// the eigenvectors accumulated in the columns of V.  Round-robin ordering:
// each round rotates n/2 disjoint (p, q) pairs.  Returns false when the
// off-diagonal mass did not fall below 1e-30 of the diagonal mass.
__device__ bool jacobi_eig(double* A, double* V, int n, double* red, double* sh) {
    const int tid = threadIdx.x;
    const int np = (n + 1) & ~1;                 // even player count (dummy if n odd)
    double* cs = sh;                             // 32 cosines
    double* sn = sh + 32;                        // 32 sines
    int* pp = (int*)(sh + 64);                   // 32 p indices
    int* qq = pp + 32;                           // 32 q indices
    for (int e = tid; e < n * n; e += ANT) {
        const int i = e / n, j = e % n;
        V[i * kEigLd + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    bool converged = false;
    for (int sweep = 0; sweep < kJacobiMaxSweeps; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int e = tid; e < n * n; e += ANT) {
            const int i = e / n, j = e % n;
            const double v = A[i * kEigLd + j];
            if (i == j) dia += v * v; else off += v * v;
        }
        off = block_sum(off, red);
        dia = block_sum(dia, red);
        if (off <= 1e-30 * dia || off == 0.0) { converged = true; break; }
        for (int round = 0; round < np - 1; ++round) {
            if (tid < np / 2) {
                // circle method: player 0 fixed, the others rotate
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
            // rows: A <- J^T A
            for (int e = tid; e < (np / 2) * n; e += ANT) {
                const int k = e / n, j = e % n;
                const int p = pp[k], q = qq[k];
                if (q < n && sn[k] != 0.0) {
                    const double c = cs[k], s = sn[k];
                    const double ap = A[p * kEigLd + j], aq = A[q * kEigLd + j];
                    A[p * kEigLd + j] = c * ap - s * aq;
                    A[q * kEigLd + j] = s * ap + c * aq;
                }
            }
            __syncthreads();
            // columns: A <- A J, V <- V J
            for (int e = tid; e < (np / 2) * n; e += ANT) {
                const int k = e / n, i = e % n;
                const int p = pp[k], q = qq[k];
                if (q < n && sn[k] != 0.0) {
                    const double c = cs[k], s = sn[k];
                    const double ap = A[i * kEigLd + p], aq = A[i * kEigLd + q];
                    A[i * kEigLd + p] = c * ap - s * aq;
                    A[i * kEigLd + q] = s * ap + c * aq;
                    const double vp = V[i * kEigLd + p], vq = V[i * kEigLd + q];
                    V[i * kEigLd + p] = c * vp - s * vq;
                    V[i * kEigLd + q] = s * vp + c * vq;
                }
            }
            __syncthreads();
        }
    }
    return converged;
}

// rank of eigenvalue e among the n diagonal entries, descending, ties by index
__device__ __forceinline__ int desc_rank(const double* A, int n, int e) {
    const double w = A[e * kEigLd + e];
    int r = 0;
    for (int f = 0; f < n; ++f) {
        const double v = A[f * kEigLd + f];
        if (v > w || (v == w && f < e)) ++r;
    }
    return r;
}

// ---------------------------------------------------------------------------

__device__ __forceinline__ void decode(int64_t rho, const int* l, int nm, int* idx) {
    for (int m = nm - 1; m >= 0; --m) {
        idx[m] = (int)(rho % l[m]);
        rho /= l[m];
    }
}

// Algorithm 2 step 2: leading R eigenvectors of B_(n) B_(n)^T.
__device__ bool eig_init(const AlsCtx& c, int n, double* E, double* V) {
    const int tid = threadIdx.x;
    const int ln = c.l[n];
    int64_t Ln = 1, Rn = 1;
    for (int m = 0; m < n; ++m) Ln *= c.l[m];
    for (int m = n + 1; m < c.N; ++m) Rn *= c.l[m];
    const int npairs = ln * (ln + 1) / 2;
    for (int e = tid; e < npairs; e += ANT) {
        // unrank (i, i2) with i <= i2
        int i = 0, rem = e;
        while (rem >= ln - i) { rem -= ln - i; ++i; }
        const int i2 = i + rem;
        double s = 0.0;
        for (int64_t a = 0; a < Ln; ++a) {
            const float* r1 = c.B + (a * ln + i) * Rn;
            const float* r2 = c.B + (a * ln + i2) * Rn;
            for (int64_t b = 0; b < Rn; ++b) s += (double)r1[b] * (double)r2[b];
        }
        E[i * kEigLd + i2] = s;
        E[i2 * kEigLd + i] = s;
    }
    __syncthreads();
    const bool ok = jacobi_eig(E, V, ln, c.red, c.sh);
    // pick the R largest, order descending, sign rule
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
            for (int i = 0; i < ln; ++i) c.fac[n][i * c.R + r] = sg * V[i * kEigLd + e];
        }
    }
    __syncthreads();
    return ok;
}

__device__ void gram(const AlsCtx& c, int n, double* G) {
    const int R = c.R, ln = c.l[n];
    const double* A = c.fac[n];
    for (int e = threadIdx.x; e < R * R; e += ANT) {
        const int r = e / R, s = e % R;
        double acc = 0.0;
        for (int i = 0; i < ln; ++i) acc += A[i * R + r] * A[i * R + s];
        G[e] = acc;
    }
}

// Ã_n = M V^+ with V = *_{m != n} G_m, then column normalisation.
// Returns the status bits; lam receives the column norms.
__device__ int solve_update(const AlsCtx& c, int n, const double* G, double* M, double* X,
                            double* V, double* Lc, double* E, double* Ev, double* lam) {
    const int tid = threadIdx.x, R = c.R, ln = c.l[n];
    int status = 0;
    for (int e = tid; e < R * R; e += ANT) {
        double v = 1.0;
        for (int m = 0; m < c.N; ++m)
            if (m != n) v *= G[(int64_t)m * R * R + e];
        V[e] = v;
    }
    __syncthreads();
    // Cholesky V = L L^T on one wavefront (lanes own rows)
    __shared__ int chol_ok;
    if (tid < 64) {
        const int lane = tid;
        double maxd = 0.0;
        for (int j = 0; j < R; ++j) maxd = fmax(maxd, V[j * R + j]);
        int ok = 1;
        for (int j = 0; j < R; ++j) {
            // diagonal
            double d = V[j * R + j];
            for (int p = 0; p < j; ++p) d -= Lc[j * R + p] * Lc[j * R + p];
            if (!(d > kPivotRtol * maxd)) { ok = 0; break; }
            const double ljj = sqrt(d);
            // column j below the diagonal: lanes own rows i = j+1+lane, +64
            for (int i = j + 1 + lane; i < R; i += 64) {
                double s = V[i * R + j];
                for (int p = 0; p < j; ++p) s -= Lc[i * R + p] * Lc[j * R + p];
                Lc[i * R + j] = s / ljj;
            }
            if (lane == 0) Lc[j * R + j] = ljj;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        if (lane == 0) chol_ok = ok;
    }
    __syncthreads();
    if (chol_ok) {
        for (int i = tid; i < ln; i += ANT) {
            double* x = X + (int64_t)i * R;
            const double* mrow = M + (int64_t)i * R;
            for (int j = 0; j < R; ++j) {
                double s = mrow[j];
                for (int p = 0; p < j; ++p) s -= Lc[j * R + p] * x[p];
                x[j] = s / Lc[j * R + j];
            }
            for (int j = R - 1; j >= 0; --j) {
                double s = x[j];
                for (int p = j + 1; p < R; ++p) s -= Lc[p * R + j] * x[p];
                x[j] = s / Lc[j * R + j];
            }
        }
    } else {
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
            Lc[e] = acc;                         // V^+
        }
        __syncthreads();
        for (int e = tid; e < ln * R; e += ANT) {
            const int i = e / R, s = e % R;
            double acc = 0.0;
            for (int r = 0; r < R; ++r) acc += M[(int64_t)i * R + r] * Lc[r * R + s];
            X[e] = acc;
        }
    }
    __syncthreads();
    // column norms, normalisation
    for (int r = tid; r < R; r += ANT) {
        double s = 0.0;
        for (int i = 0; i < ln; ++i) s += X[(int64_t)i * R + r] * X[(int64_t)i * R + r];
        lam[r] = sqrt(s);
    }
    __syncthreads();
    for (int e = tid; e < ln * R; e += ANT) {
        const int r = e % R;
        const double nu = lam[r];
        c.fac[n][e] = (nu > 0.0) ? X[e] / nu : X[e];
    }
    __syncthreads();
    return status;
}

__global__ __launch_bounds__(ANT) void k_als(AlsArgs a, int fac_in_lds) {
    extern __shared__ double asmem[];
    __shared__ double red[ANT / 64];
    __shared__ double sh[128];
    __shared__ double lam[RCP_MAX_RANK];
    __shared__ double lam_tmp[RCP_MAX_RANK];
    __shared__ double Lsh[RCP_MAX_RANK * RCP_MAX_RANK];   // Cholesky factor / V^+
    const int tid = threadIdx.x;
    AlsCtx c;
    c.B = a.B;
    c.N = a.N;
    c.R = a.R;
    c.S = 1;
    for (int n = 0; n < a.N; ++n) { c.l[n] = a.l[n]; c.S *= a.l[n]; }
    const int N = a.N, R = a.R, lN = a.l[N - 1];
    c.Lh = c.S / lN;
    c.red = red;
    c.sh = sh;
    // working factors: LDS when they fit, else the workspace
    {
        int64_t off = 0;
        double* base = fac_in_lds ? asmem : a.misc + 64;
        for (int n = 0; n < N; ++n) { c.fac[n] = base + off; off += (int64_t)a.l[n] * R; }
    }
    double* G = a.G;
    double* M = a.Mbuf;
    double* X = a.Mbuf + (int64_t)64 * RCP_MAX_RANK;
    double* V = a.Vbuf;
    double* Lc = Lsh;
    double* E = a.Ebuf;
    double* Ev = a.Ebuf + kEigLd * kEigLd;
    double* W = a.W;
    double* KR = a.KR;

    double s = 0.0;
    for (int64_t e = tid; e < c.S; e += ANT) { const double v = c.B[e]; s += v * v; }
    const double normB2 = block_sum(s, red);
    const double normX2 = (a.normX2 != nullptr) ? *a.normX2 : normB2;

    int status = 0;
    for (int n = 1; n < N; ++n) {
        if (!eig_init(c, n, E, Ev)) status |= RCP_INFO_EIG_NOT_CONVERGED;
        gram(c, n, G + (int64_t)n * R * R);
    }
    __syncthreads();

    // strides of the H1 modes inside rho
    int64_t stride[RCP_MAX_NDIM];
    {
        int64_t st = 1;
        for (int m = N - 2; m >= 0; --m) { stride[m] = st; st *= c.l[m]; }
    }

    double rho = 0.0, rho_prev = 0.0;
    int it = 0;
    for (it = 1; it <= a.max_iters; ++it) {
        // phase A: W = B_view (Lh x lN) * Ã_{N-1}
        {
            const double* AN = c.fac[N - 1];
            for (int64_t e = tid; e < c.Lh * R; e += ANT) {
                const int64_t rho_i = e / R;
                const int r = (int)(e - rho_i * R);
                const float* brow = c.B + rho_i * lN;
                double acc = 0.0;
                for (int k = 0; k < lN; ++k) acc += (double)brow[k] * AN[k * R + r];
                W[e] = acc;
            }
            __syncthreads();
        }
        for (int n = 0; n < N - 1; ++n) {
            const int ln = c.l[n];
            const int64_t Cn = c.Lh / ln;
            int ol[RCP_MAX_NDIM], om[RCP_MAX_NDIM], no = 0;
            for (int m = 0; m < N - 1; ++m)
                if (m != n) { ol[no] = c.l[m]; om[no] = m; ++no; }
            for (int64_t e = tid; e < (int64_t)ln * R; e += ANT) {
                const int i = (int)(e / R), r = (int)(e % R);
                double acc = 0.0;
                for (int64_t qv = 0; qv < Cn; ++qv) {
                    int idx[RCP_MAX_NDIM];
                    decode(qv, ol, no, idx);
                    int64_t rr = (int64_t)i * stride[n];
                    double w = 1.0;
                    for (int t = 0; t < no; ++t) {
                        rr += (int64_t)idx[t] * stride[om[t]];
                        w *= c.fac[om[t]][idx[t] * R + r];
                    }
                    acc += W[rr * R + r] * w;
                }
                M[e] = acc;
            }
            __syncthreads();
            status |= solve_update(c, n, G, M, X, V, Lc, E, Ev, lam_tmp);
            gram(c, n, G + (int64_t)n * R * R);
            __syncthreads();
        }
        // phase B: M_{N-1} = B_view^T * KR(H1)
        {
            for (int64_t e = tid; e < c.Lh * R; e += ANT) {
                const int64_t rho_i = e / R;
                const int r = (int)(e - rho_i * R);
                int idx[RCP_MAX_NDIM];
                decode(rho_i, c.l, N - 1, idx);
                double w = 1.0;
                for (int m = 0; m < N - 1; ++m) w *= c.fac[m][idx[m] * R + r];
                KR[e] = w;
            }
            __syncthreads();
            for (int64_t e = tid; e < (int64_t)lN * R; e += ANT) {
                const int i = (int)(e / R), r = (int)(e % R);
                double acc = 0.0;
                for (int64_t rr = 0; rr < c.Lh; ++rr) acc += (double)c.B[rr * lN + i] * KR[rr * R + r];
                M[e] = acc;
            }
            __syncthreads();
            status |= solve_update(c, N - 1, G, M, X, V, Lc, E, Ev, lam);
            gram(c, N - 1, G + (int64_t)(N - 1) * R * R);
            __syncthreads();
        }
        // fit (Section 3.3): rho = 1 - (||X||^2 + ||Xhat||^2 - 2 <Xhat, X>) / ||X||^2
        double inner = 0.0, model = 0.0;
        {
            const double* AN = c.fac[N - 1];
            double pi = 0.0;
            for (int64_t e = tid; e < (int64_t)lN * R; e += ANT) {
                const int r = (int)(e % R);
                pi += lam[r] * M[e] * AN[e];
            }
            double pm = 0.0;
            for (int e = tid; e < R * R; e += ANT) {
                double v = lam[e / R] * lam[e % R];
                for (int m = 0; m < N; ++m) v *= G[(int64_t)m * R * R + e];
                pm += v;
            }
            inner = block_sum(pi, red);
            model = block_sum(pm, red);
        }
        const double err2 = normX2 - 2.0 * inner + model;
        rho = (normX2 > 0.0) ? 1.0 - err2 / normX2 : 0.0;
        if (!isfinite(rho)) { status |= RCP_INFO_NONFINITE; break; }
        if (a.tol > 0.0 && it >= 2 && fabs(rho - rho_prev) < a.tol) break;
        rho_prev = rho;
    }
    if (it > a.max_iters) it = a.max_iters;

    // outputs
    for (int n = 0; n < N; ++n)
        for (int64_t e = tid; e < (int64_t)a.l[n] * R; e += ANT) a.At[n][e] = (float)c.fac[n][e];
    for (int r = tid; r < R; r += ANT) a.lambda[r] = (float)lam[r];
    if (tid == 0) {
        a.info->iters = it;
        a.info->status = status;
        a.info->rho = rho;
        a.info->rel_err = sqrt(fmax(0.0, 1.0 - rho));
        a.info->normX2 = normX2;
    }
}

size_t als_workspace_doubles(int N, const int* l, int R) {
    int64_t S = 1;
    for (int n = 0; n < N; ++n) S *= l[n];
    const int64_t Lh = S / l[N - 1];
    int64_t facs = 0;
    for (int n = 0; n < N; ++n) facs += (int64_t)l[n] * R;
    return (size_t)(2 * Lh * R                  // W, KR
                    + (int64_t)N * R * R        // G
                    + 2 * 64 * RCP_MAX_RANK     // M, X
                    + 2 * R * R                 // V, L
                    + 2 * kEigLd * kEigLd       // Jacobi
                    + 64 + facs);               // misc + spill factors
}

hipError_t launch_als(const AlsArgs& a, hipStream_t s) {
    int64_t facs = 0;
    for (int n = 0; n < a.N; ++n) facs += (int64_t)a.l[n] * a.R;
    const size_t bytes = (size_t)facs * sizeof(double);
    const int in_lds = bytes <= 96 * 1024 ? 1 : 0;
    hipError_t e = hipFuncSetAttribute((const void*)k_als, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       96 * 1024);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_als, dim3(1), dim3(ANT), in_lds ? bytes : 0, s, a, in_lds);
    return hipGetLastError();
}

}  // namespace rcp
