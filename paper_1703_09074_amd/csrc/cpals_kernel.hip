// Deterministic CP-ALS on the full tensor: Algorithm 2 with Q_n = I, the
// method the randomized algorithm is measured against (Section 3.3 follows
// the Tensor Toolbox's CP-ALS: unit columns after every update, eigenvector
// start, the change of the fit as the stopping rule).
//
// Per mode n of a sweep, with the tensor too large for anything but a
// streaming pass:
//   M_n = X_(n) KR(A_{m != n})   streamed over the whole GPU (the Khatri-Rao
//                                kind of the streaming mode product), float64
//                                reduction into Y (I_n x ldy);
//   V^-1                         one workgroup: Gauss-Jordan on [V | I] with
//                                V = *_{m != n} G_m, the Moore-Penrose
//                                pseudo-inverse when a pivot falls below
//                                1e-13 of diag(V);
//   raw = M_n V^-1               row blocks over the GPU, each also forming
//                                its partial Gram raw^T raw and the partial
//                                inner products <M_n[:, r], raw[:, r]>;
//   norms, G_n, lambda, fit      one workgroup, in a fixed order (no atomics,
//                                the result does not depend on scheduling);
//   A_n = raw / ||raw||          row blocks: the float64 factor in place and
//                                the float32 copy the next mode products read.
// The sweep state lives in global memory (cp_state_doubles):
//   ints [0] the sweep after which the rule stopped (0: running), [1] sweeps
//        done, [2] RCP_INFO_* bits;  double [2] rho of the last sweep,
//        [3] ||X||^2;  G_0 .. G_{N-1} (R x R) from double kCpG, then lambda,
//        V^-1, the column norms, the partial Grams and partial inner products.
// Every launch carries its sweep number and returns at once when the rule
// stopped at an earlier sweep, so the host enqueues all sweeps up front.

#include "als_common.h"

namespace rcp {

constexpr int kCpG = 4;
constexpr int kCpRows = 64;            // rows per chunk of the row-block kernels
constexpr int kCpMaxBlocks = 256;      // row blocks of the apply kernel
constexpr int CNT = 256;

struct CpLayout {
    double *G, *lam, *vinv, *nu, *pgram, *pin;
};

__host__ __device__ inline CpLayout cp_layout(double* st, int N, int R) {
    CpLayout c;
    c.G = st + kCpG;
    c.lam = c.G + (size_t)N * R * R;
    c.vinv = c.lam + R;
    c.nu = c.vinv + (size_t)R * R;
    c.pgram = c.nu + R;
    c.pin = c.pgram + (size_t)kCpMaxBlocks * R * R;
    return c;
}

size_t cp_state_doubles(int N, int R) {
    return kCpG + (size_t)N * R * R + 2 * (size_t)R + (size_t)R * R +
           (size_t)kCpMaxBlocks * R * R + (size_t)kCpMaxBlocks * R;
}

int cp_row_blocks(int64_t I) {
    const int64_t chunks = (I + kCpRows - 1) / kCpRows;
    return (int)(chunks < kCpMaxBlocks ? chunks : kCpMaxBlocks);
}

__device__ __forceinline__ bool cp_stopped(const CpArgs& a) {
    const int s = ((const int*)a.state)[0];
    return s != 0 && a.sweep > s;
}

// V^-1 (or V^+) for mode n, V = *_{m != n} G_m.
__global__ __launch_bounds__(ANT) void k_cp_inverse(CpArgs a) {
    extern __shared__ __align__(16) unsigned char cp_smem[];
    __shared__ double red[ANW];
    __shared__ double sh[128];
    if (cp_stopped(a)) return;
    const int tid = threadIdx.x, N = a.N, R = a.R, n = a.n;
    const CpLayout c = cp_layout(a.state, N, R);
    const int Rp = (R + 3) / 4 * 4;
    const int ldx = aug_ld(Rp, Rp);
    double* Aug = (double*)cp_smem;
    double* pb = Aug + (size_t)Rp * ldx;
    for (int e = tid; e < Rp * 2 * Rp; e += ANT) {
        const int r = e / (2 * Rp), s = e - r * 2 * Rp;
        double v;
        if (s < Rp) {
            if (r < R && s < R) {
                v = 1.0;
                for (int m = 0; m < N; ++m)
                    if (m != n) v *= c.G[(size_t)m * R * R + r * R + s];
            } else {
                v = (r == s) ? 1.0 : 0.0;
            }
        } else {
            v = (s - Rp == r) ? 1.0 : 0.0;
        }
        Aug[r * ldx + s] = v;
    }
    __syncthreads();
    const int ok = gj_solve(Aug, ldx, R, Rp, 2 * Rp, kPivotRtol, pb);
    if (ok) {
        for (int e = tid; e < R * R; e += ANT) c.vinv[e] = Aug[(e / R) * ldx + Rp + e % R];
        return;
    }
    // Moore-Penrose pseudo-inverse through the eigen-decomposition
    double* E = a.E;
    double* Ev = a.E + kEigLd * kEigLd;
    for (int e = tid; e < R * R; e += ANT) {
        double v = 1.0;
        for (int m = 0; m < N; ++m)
            if (m != n) v *= c.G[(size_t)m * R * R + e];
        E[(e / R) * kEigLd + (e % R)] = v;
    }
    __syncthreads();
    jacobi_eig(E, Ev, R, red, sh);
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
        c.vinv[e] = acc;
    }
    if (tid == 0) ((int*)a.state)[2] |= RCP_INFO_PINV_FALLBACK;
}

// raw = Y V^-1 for this block's rows (update) or raw as given (Gram of a
// start), then the block's partial Gram raw^T raw and, for updates, the
// partial inner products <Y[:, r], raw[:, r]>.
__global__ __launch_bounds__(CNT) void k_cp_apply(CpArgs a, int update) {
    extern __shared__ __align__(16) unsigned char cp_smem[];
    if (cp_stopped(a)) return;
    const int tid = threadIdx.x, R = a.R;
    double* vinv = (double*)cp_smem;                 // R x R
    double* rows = vinv + R * R;                     // kCpRows x R
    double* ys = rows + kCpRows * R;                 // kCpRows x R
    const CpLayout c = cp_layout(a.state, a.N, R);
    if (update)
        for (int e = tid; e < R * R; e += CNT) vinv[e] = c.vinv[e];
    // Gram entries (r, s) of this thread: e = tid + k * CNT over R * R
    double gacc[16], pacc = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) gacc[k] = 0.0;
    const int64_t nchunks = (a.I + kCpRows - 1) / kCpRows;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t i0 = ch * kCpRows;
        const int nr = (int)((a.I - i0) < kCpRows ? (a.I - i0) : kCpRows);
        __syncthreads();
        if (update) {
            for (int e = tid; e < nr * R; e += CNT) {
                const int i = e / R, r = e - (e / R) * R;
                ys[e] = a.Y[(i0 + i) * a.ldy + r];
            }
            __syncthreads();
            for (int e = tid; e < nr * R; e += CNT) {
                const int i = e / R, r = e - (e / R) * R;
                double s = 0.0;
                for (int t = 0; t < R; ++t) s += ys[i * R + t] * vinv[t * R + r];
                rows[e] = s;
                a.raw[(i0 + i) * R + r] = s;
            }
        } else {
            for (int e = tid; e < nr * R; e += CNT) rows[e] = a.raw[i0 * R + e];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int e = tid + k * CNT;
            if (e < R * R) {
                const int r = e / R, s = e - (e / R) * R;
                double acc = gacc[k];
                for (int i = 0; i < nr; ++i) acc += rows[i * R + r] * rows[i * R + s];
                gacc[k] = acc;
            }
        }
        if (update && tid < R)
            for (int i = 0; i < nr; ++i) pacc += ys[i * R + tid] * rows[i * R + tid];
    }
    double* pg = c.pgram + (size_t)blockIdx.x * R * R;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int e = tid + k * CNT;
        if (e < R * R) pg[e] = gacc[k];
    }
    if (tid < R) c.pin[(size_t)blockIdx.x * R + tid] = pacc;
}

// Column norms and G_n from the partial Grams (blocks summed in order); for
// updates of the last mode lambda, the fit of Section 3.3 (exact on the full
// tensor) and the stopping rule.  phase 0: sweep update; 1: Gram of a start
// (G_n = raw^T raw as is, norms 1).
__global__ __launch_bounds__(ANT) void k_cp_norm(CpArgs a, int nblk, int update) {
    __shared__ double red[ANW];
    __shared__ double nu[RCP_MAX_RANK];
    if (cp_stopped(a)) return;
    const int tid = threadIdx.x, N = a.N, R = a.R, n = a.n;
    const CpLayout c = cp_layout(a.state, N, R);
    double* Gn = c.G + (size_t)n * R * R;
    for (int e = tid; e < R * R; e += ANT) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += c.pgram[(size_t)b * R * R + e];
        Gn[e] = s;
    }
    __syncthreads();
    for (int r = tid; r < R; r += ANT) {
        const double v = update ? sqrt(Gn[r * R + r]) : 1.0;
        nu[r] = v;
        c.nu[r] = v;
    }
    __syncthreads();
    if (!update) return;
    for (int e = tid; e < R * R; e += ANT) {
        const int r = e / R, s = e - (e / R) * R;
        const double dr = nu[r] > 0.0 ? nu[r] : 1.0, ds = nu[s] > 0.0 ? nu[s] : 1.0;
        Gn[e] = Gn[e] / (dr * ds);
    }
    __syncthreads();
    int* fl = (int*)a.state;
    if (n < N - 1) return;
    const int it = a.sweep;
    double pi = 0.0;
    for (int r = tid; r < R; r += ANT)
        for (int b = 0; b < nblk; ++b) pi += c.pin[(size_t)b * R + r];
    double pm = 0.0;
    for (int e = tid; e < R * R; e += ANT) {
        double v = nu[e / R] * nu[e % R];
        for (int m = 0; m < N; ++m) v *= c.G[(size_t)m * R * R + e];
        pm += v;
    }
    // <M_N[:, r], A_N[:, r]> lambda_r = <M_N[:, r], raw[:, r]>
    const double inner = block_sum(pi, red);
    const double model = block_sum(pm, red);
    const double normX2 = a.state[3];
    const double err2 = normX2 - 2.0 * inner + model;
    const double rho = (normX2 > 0.0) ? 1.0 - err2 / normX2 : 0.0;
    int status = 0;
    bool stop = it >= a.max_iters;
    if (!isfinite(rho)) {
        status |= RCP_INFO_NONFINITE;
        stop = true;
    } else if (a.tol > 0.0 && it >= 2 && fabs(rho - a.state[2]) < a.tol) {
        stop = true;
    }
    for (int r = tid; r < R; r += ANT) {
        c.lam[r] = nu[r];
        a.lam_f[r] = (float)nu[r];
    }
    __syncthreads();
    if (tid == 0) {
        const int st = fl[2] | status;
        fl[2] = st;
        fl[1] = it;
        a.state[2] = rho;
        a.info->iters = it;
        a.info->status = st;
        a.info->rho = rho;
        a.info->rel_err = sqrt(fmax(0.0, 1.0 - rho));
        a.info->normX2 = normX2;
        if (a.status_word != nullptr && st != 0) *a.status_word |= st;
        if (stop) fl[0] = it;
    }
}

// A_n = raw / nu (a zero column is left as is), in place in float64 and as
// the float32 copy the mode products read.
__global__ __launch_bounds__(CNT) void k_cp_scale(CpArgs a) {
    if (cp_stopped(a)) return;
    const int R = a.R;
    const CpLayout c = cp_layout(a.state, a.N, R);
    const int64_t cnt = a.I * R;
    for (int64_t e = (int64_t)blockIdx.x * CNT + threadIdx.x; e < cnt;
         e += (int64_t)gridDim.x * CNT) {
        const int r = (int)(e % R);
        const double v = c.nu[r];
        double x = a.raw[e];
        if (v > 0.0) x /= v;
        a.raw[e] = x;
        a.fac[e] = (float)x;
    }
}

// The eigenvector start of mode n from the subspace basis: U = Q W (Q the
// I x l orthonormal basis, W the l x R leading eigenvectors of the Gram
// Q^T X_(n) X_(n)^T Q), columns scaled to unit norm and signed so that the
// largest-magnitude entry (first index on ties) is positive.  One workgroup
// per column.
__global__ __launch_bounds__(CNT) void k_cp_start(const float* Q, const float* W, int64_t I, int l,
                                                   int R, double* raw, float* fac) {
    __shared__ double red[CNT / 64];
    __shared__ double sbest[CNT / 64];
    __shared__ double sval[CNT / 64];
    __shared__ long long sidx[CNT / 64];
    const int r = blockIdx.x, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    double ss = 0.0, best = -1.0, bval = 0.0;
    long long bi = 0;
    for (int64_t i = tid; i < I; i += CNT) {
        double u = 0.0;
        for (int k = 0; k < l; ++k) u += (double)Q[i * l + k] * (double)W[k * R + r];
        raw[i * R + r] = u;
        ss += u * u;
        if (fabs(u) > best) { best = fabs(u); bi = i; bval = u; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const double ov = __shfl_xor(bval, o, 64);
        const long long oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; bval = ov; }
    }
    if (lane == 0) { sbest[wave] = best; sidx[wave] = bi; sval[wave] = bval; }
    const double tot = block_sum(ss, red);
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < CNT / 64; ++w)
            if (sbest[w] > sbest[0] || (sbest[w] == sbest[0] && sidx[w] < sidx[0])) {
                sbest[0] = sbest[w];
                sidx[0] = sidx[w];
                sval[0] = sval[w];
            }
    }
    __syncthreads();
    const double sgn = (sval[0] < 0.0) ? -1.0 : 1.0;
    const double scale = (tot > 0.0) ? sgn / sqrt(tot) : sgn;
    for (int64_t i = tid; i < I; i += CNT) {
        const double x = raw[i * R + r] * scale;
        raw[i * R + r] = x;
        fac[i * R + r] = (float)x;
    }
}

// A caller's start for mode n: float64 and float32 working copies.
__global__ __launch_bounds__(CNT) void k_cp_load(const float* A, int64_t cnt, double* raw,
                                                  float* fac) {
    for (int64_t e = (int64_t)blockIdx.x * CNT + threadIdx.x; e < cnt;
         e += (int64_t)gridDim.x * CNT) {
        const float v = A[e];
        raw[e] = (double)v;
        fac[e] = v;
    }
}

static size_t apply_smem(int R) {
    return ((size_t)R * R + 2 * (size_t)kCpRows * R) * sizeof(double);
}

static unsigned elem_blocks(int64_t cnt) {
    const int64_t b = (cnt + CNT - 1) / CNT;
    return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

hipError_t launch_cp_update(const CpArgs& a, hipStream_t s) {
    if (a.R < 1 || a.R > RCP_MAX_RANK || a.I < 1) return hipErrorInvalidValue;
    const int Rp = (a.R + 3) / 4 * 4;
    const size_t smem = ((size_t)Rp * aug_ld(Rp, Rp) + gj_buf_doubles(aug_ld(Rp, Rp), Rp)) *
                        sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void*)k_cp_inverse,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cp_inverse, dim3(1), dim3(ANT), smem, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nblk = cp_row_blocks(a.I);
    const size_t asmem = apply_smem(a.R);
    if ((e = hipFuncSetAttribute((const void*)k_cp_apply,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)asmem)) !=
        hipSuccess)
        return e;
    hipLaunchKernelGGL(k_cp_apply, dim3((unsigned)nblk), dim3(CNT), asmem, s, a, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cp_norm, dim3(1), dim3(ANT), 0, s, a, nblk, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cp_scale, dim3(elem_blocks(a.I * a.R)), dim3(CNT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cp_gram(const CpArgs& a, hipStream_t s) {
    if (a.R < 1 || a.R > RCP_MAX_RANK || a.I < 1) return hipErrorInvalidValue;
    const int nblk = cp_row_blocks(a.I);
    const size_t asmem = apply_smem(a.R);
    hipError_t e = hipFuncSetAttribute((const void*)k_cp_apply,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)asmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cp_apply, dim3((unsigned)nblk), dim3(CNT), asmem, s, a, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cp_norm, dim3(1), dim3(ANT), 0, s, a, nblk, 0);
    return hipGetLastError();
}

hipError_t launch_cp_start(const float* Q, const float* W, int64_t I, int l, int R, double* raw,
                           float* fac, hipStream_t s) {
    if (R < 1 || R > RCP_MAX_RANK || l < 1 || I < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cp_start, dim3((unsigned)R), dim3(CNT), 0, s, Q, W, I, l, R, raw, fac);
    return hipGetLastError();
}

hipError_t launch_cp_load(const float* A, int64_t cnt, double* raw, float* fac, hipStream_t s) {
    hipLaunchKernelGGL(k_cp_load, dim3(elem_blocks(cnt)), dim3(CNT), 0, s, A, cnt, raw, fac);
    return hipGetLastError();
}

}  // namespace rcp
