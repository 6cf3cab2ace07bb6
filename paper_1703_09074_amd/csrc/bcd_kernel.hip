// Block coordinate descent on the compressed tensor B (Section 3.2.2,
// Algorithm 3) in one persistent workgroup.
//
// The components are found one after another.  For component r every sweep
// updates its vectors a_r^(0), ..., a_r^(N-1) in mode order, each the
// least-squares solution of its rank-one block on the residual
// Y = B - sum_{s<r} lam_s a_s^(0) o ... o a_s^(N-1) (the residual update), which is never
// formed: by multilinearity
//   Y_(n) (KR_{m != n} a_r^(m)) = B_(n) (KR_{m != n} a_r^(m))
//                                 - sum_{s<r} lam_s a_s^(n) prod_{m != n} <a_s^(m), a_r^(m)>.
// The first term is a matrix-vector product with the core, formed here on
// the vector ALU (thread (i, p) sums row i of B_(n) over the contraction
// indices k = p mod P, the Khatri-Rao entries built from the factor
// columns in LDS, the P partial sums reduced in a fixed order); the
// corrections use the inner products <a_s^(m), a_r^(m)>, kept per mode in
// LDS and refreshed after each update.  The update is divided by
// prod_{m != n} ||a_r^(m)||^2 (the scalar Gram product of the rank-one updates) and
// scaled to unit norm, its norm becoming lambda_r for the last mode (steps
// 7, 9, 11, 12).  The fit of Section 3.3 is kept for the model of components
// 0..r: <B, Bhat> from the stored <B, rank-one s> of finished components and
// the last mode's product, ||Bhat||^2 from the inner-product tables.
// Starting vectors (the initialisation): column r of the leading eigenvectors of
// B_(n) B_(n)^T for modes 1..N-1 (the Jacobi start shared with CP-ALS), or
// the caller's factors.  Factors are float64 in LDS; the core is float32
// (in LDS when it fits, else read from global memory).

#include "als_common.h"

namespace rcp {

// dynamic LDS budget of k_bcd: its static arrays take about 7.4 KB
constexpr size_t kBcdLds = 160 * 1024 - 8192;

template <int NN, bool B_IN_LDS, bool EIG_IN_LDS>
__global__ __launch_bounds__(ANT) void k_bcd(AlsArgs a) {
    constexpr int D = NN - 1;
    extern __shared__ __align__(16) unsigned char bcd_smem[];
    __shared__ double red[ANW];
    __shared__ double sh[128];
    __shared__ double lam[RCP_MAX_RANK];
    __shared__ double ipB[RCP_MAX_RANK];          // <B, rank-one s> of finished components
    __shared__ double wdef[RCP_MAX_RANK];         // lam_s prod_{m != n} <a_s^(m), a_r^(m)>
    __shared__ double Gs[RCP_MAX_NDIM][RCP_MAX_RANK + 1];   // <a_m[:, s], a_m[:, r]>, s <= r
    __shared__ double vraw[64];
    __shared__ int sl[RCP_MAX_NDIM];
    __shared__ int sfoff[RCP_MAX_NDIM];
    __shared__ int sst[RCP_MAX_NDIM];
    __shared__ double sfit[2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int N = a.N, R = a.R;

    AlsCtx c;
    c.N = N;
    c.R = R;
    c.S = 1;
    size_t fbytes = 0, dbytes = 0;
    int foff64[RCP_MAX_NDIM];
#pragma unroll
    for (int n = 0; n < RCP_MAX_NDIM; ++n) {
        foff64[n] = 0;
        if (n < N) {
            c.S *= a.l[n];
            if (tid == 0) { sl[n] = a.l[n]; sfoff[n] = (int)(fbytes / sizeof(float)); }
            foff64[n] = (int)(dbytes / sizeof(double));
            fbytes += ((size_t)a.l[n] * R * sizeof(float) + 15) & ~(size_t)15;
            dbytes += (size_t)a.l[n] * R * sizeof(double);
        }
    }
    if (tid == 0) {
        int st = 1;
        for (int n = N - 1; n >= 0; --n) { sst[n] = st; st *= a.l[n]; }
    }
    c.lN = a.l[N - 1];
    c.Lh = c.S / c.lN;
    c.red = red;
    c.sh = sh;
    c.l = sl;
    c.foff = sfoff;

    // dynamic LDS: [float64 factors | partial sums (ANT) | ones (64) | big]
    // big: the eigenvector scratch E, V (when in LDS) and the float32 start
    // factors during the initialisation, then the core (when in LDS)
    unsigned char* p = bcd_smem;
    double* F = (double*)p; p += dbytes;
    double* part = (double*)p; p += ANT * sizeof(double);
    double* ones = (double*)p; p += 64 * sizeof(double);
    unsigned char* big = p;
    double* E = EIG_IN_LDS ? (double*)big : a.Ebuf;
    double* Ev = E + kEigLd * kEigLd;
    c.fbase = (float*)(EIG_IN_LDS ? big + 2 * kEigLd * kEigLd * sizeof(double) : big);
    float* Bl = (float*)big;
    for (int e = tid; e < 64; e += ANT) ones[e] = 1.0;
    __syncthreads();
    const double normX2 = *a.normX2;

    int status = 0;
    for (int n = 1; n < N; ++n) {
        if (a.warm) {
            for (int e = tid; e < c.l[n] * R; e += ANT) F[foff64[n] + e] = (double)a.At[n][e];
        } else {
            if (!eig_init(c, a.B, n, E, Ev)) status |= RCP_INFO_EIG_NOT_CONVERGED;
            for (int e = tid; e < c.l[n] * R; e += ANT) F[foff64[n] + e] = (double)c.fac(n)[e];
        }
    }
    for (int e = tid; e < c.l[0] * R; e += ANT) F[foff64[0] + e] = 0.0;
    __syncthreads();
    if (B_IN_LDS)
        for (int e = tid; e < c.S; e += ANT) Bl[e] = a.B[e];
    __syncthreads();
    const float* Bs = B_IN_LDS ? Bl : a.B;

    double Cprev = 0.0;              // ||Bhat||^2 of components 0..r-1
    double rho = 0.0;
    int total = 0;
    for (int r = 0; r < R; ++r) {
        // inner products of the starting vectors with the finished components
        if (wave == 0) {
            for (int m = 0; m < N; ++m) {
                const int lm = sl[m];
                const double* Fm = F + foff64[m];
                for (int s = 0; s <= r; ++s) {
                    double v = (lane < lm) ? Fm[lane * R + s] * Fm[lane * R + r] : 0.0;
                    v = warp_sum(v);
                    if (lane == 0) Gs[m][s] = v;
                }
            }
        }
        __syncthreads();
        double rho_prev = 0.0, ipr = 0.0;
        int it;
        for (it = 1; it <= a.max_iters; ++it) {
            for (int n = 0; n < N; ++n) {
                const int ln = sl[n];
                // the other modes, slowest first (padding slots of size 1 read ones)
                int lo[D], so[D], fo[D];
#pragma unroll
                for (int s2 = 0; s2 < D; ++s2) {
                    const int j = s2 - (NN - N);
                    if (j < 0) {
                        lo[s2] = 1; so[s2] = 0; fo[s2] = (int)(ones - F) - r;
                    } else {
                        const int m = (j < n) ? j : j + 1;
                        lo[s2] = sl[m]; so[s2] = sst[m]; fo[s2] = foff64[m];
                    }
                }
                int K = 1;
#pragma unroll
                for (int s2 = 0; s2 < D; ++s2) K *= lo[s2];
                const int P = ANT / ln;
                // B_(n) (KR column r): thread (i, pp) over k = pp, pp + P, ...
                double acc = 0.0;
                if (tid < ln * P) {
                    const int i = tid / P, pp = tid - (tid / P) * P;
                    int d[D], inc[D];
                    {
                        int rem = pp, ri = P;
#pragma unroll
                        for (int s2 = D - 1; s2 >= 0; --s2) {
                            d[s2] = rem % lo[s2];
                            rem /= lo[s2];
                            inc[s2] = ri % lo[s2];
                            ri /= lo[s2];
                        }
                    }
                    const int ioff = i * sst[n];
                    for (int k = pp; k < K; k += P) {
                        int off = ioff;
                        double w = 1.0;
#pragma unroll
                        for (int s2 = 0; s2 < D; ++s2) {
                            off += d[s2] * so[s2];
                            w *= F[fo[s2] + d[s2] * R + r];
                        }
                        acc += (double)Bs[off] * w;
                        int carry = 0;
#pragma unroll
                        for (int s2 = D - 1; s2 >= 0; --s2) {
                            const int v = d[s2] + inc[s2] + carry;
                            carry = v >= lo[s2] ? 1 : 0;
                            d[s2] = carry ? v - lo[s2] : v;
                        }
                    }
                }
                part[tid] = acc;
                // lam_s prod_{m != n} <a_s^(m), a_r^(m)> for the corrections
                for (int s = tid; s < r; s += ANT) {
                    double w = lam[s];
                    for (int m = 0; m < N; ++m)
                        if (m != n) w *= Gs[m][s];
                    wdef[s] = w;
                }
                __syncthreads();
                if (wave == 0) {
                    const int i = lane;
                    double v = 0.0;
                    if (i < ln) {
                        for (int q = 0; q < P; ++q) v += part[i * P + q];
                        vraw[i] = v;
                        const double* Fn = F + foff64[n];
                        for (int s = 0; s < r; ++s) v -= wdef[s] * Fn[i * R + s];
                    }
                    double den = 1.0;
                    for (int m = 0; m < N; ++m)
                        if (m != n) den *= Gs[m][r];
                    v = (den > 0.0) ? v / den : 0.0;
                    const double nu = sqrt(warp_sum(v * v));
                    const double un = (nu > 0.0) ? v / nu : v;
                    if (i < ln) F[foff64[n] + i * R + r] = un;
                    if (n == N - 1) {
                        if (lane == 0) lam[r] = nu;
                        // <B, rank-one r> with the updated last vector
                        ipr = warp_sum((i < ln) ? vraw[i] * un : 0.0);
                    }
                    // refresh <a_n[:, s], a_n[:, r]>, s <= r
                    const double* Fn = F + foff64[n];
                    for (int s = 0; s <= r; ++s) {
                        const double t = warp_sum((i < ln) ? Fn[i * R + s] * ((s == r) ? un : Fn[i * R + r])
                                                           : 0.0);
                        if (lane == 0) Gs[n][s] = t;
                    }
                }
                __syncthreads();
            }
            // fit (Section 3.3) of components 0..r
            if (wave == 0) {
                double inner = 0.0, cross = 0.0;
                for (int s = 0; s < r; ++s) {
                    inner += lam[s] * ipB[s];
                    double g = lam[s];
                    for (int m = 0; m < N; ++m) g *= Gs[m][s];
                    cross += g;
                }
                const double lr = lam[r];
                double grr = 1.0;
                for (int m = 0; m < N; ++m) grr *= Gs[m][r];
                inner += lr * ipr;
                const double model = Cprev + 2.0 * lr * cross + lr * lr * grr;
                const double err2 = normX2 - 2.0 * inner + model;
                if (lane == 0) {
                    sfit[0] = (normX2 > 0.0) ? 1.0 - err2 / normX2 : 0.0;
                    sfit[1] = model;
                }
            }
            __syncthreads();
            rho = sfit[0];
            if (!isfinite(rho)) { status |= RCP_INFO_NONFINITE; break; }
            if (a.tol > 0.0 && it >= 2 && fabs(rho - rho_prev) < a.tol) break;
            rho_prev = rho;
        }
        if (it > a.max_iters) it = a.max_iters;
        total += it;
        if (wave == 0 && lane == 0) ipB[r] = ipr;
        Cprev = sfit[1];
        __syncthreads();
        if (!isfinite(rho)) break;
    }

#pragma unroll
    for (int n = 0; n < RCP_MAX_NDIM; ++n)
        if (n < N)
            for (int e = tid; e < a.l[n] * R; e += ANT) a.At[n][e] = (float)F[foff64[n] + e];
    for (int r = tid; r < R; r += ANT) a.lambda[r] = (float)lam[r];
    if (tid == 0) {
        a.info->iters = total;
        a.info->status = status;
        a.info->rho = rho;
        a.info->rel_err = sqrt(fmax(0.0, 1.0 - rho));
        a.info->normX2 = normX2;
        if (a.status_word != nullptr && status != 0) *a.status_word |= status;
    }
}

// LDS of k_bcd besides its big region
static size_t bcd_lds_fixed(int N, const int* l, int R) {
    size_t b = 0;
    for (int n = 0; n < N; ++n) b += (size_t)l[n] * R * sizeof(double);
    return b + ANT * sizeof(double) + 64 * sizeof(double);
}

static size_t bcd_init_floats(int N, const int* l, int R) {
    size_t f = 0;
    for (int n = 0; n < N; ++n) f += (((size_t)l[n] * R * sizeof(float) + 15) & ~(size_t)15);
    return f;
}

bool bcd_supported(int N, const int* l, int R) {
    int64_t S = 1;
    int lmax = 0;
    for (int n = 0; n < N; ++n) { S *= l[n]; lmax = lmax > l[n] ? lmax : l[n]; }
    return lmax <= 64 && R <= RCP_MAX_RANK && S < ((int64_t)1 << 31) &&
           bcd_lds_fixed(N, l, R) + bcd_init_floats(N, l, R) <= kBcdLds;
}

template <int NN, bool BL, bool EL>
static hipError_t launch_bcd_t(const AlsArgs& a, size_t smem, hipStream_t s) {
    auto k = k_bcd<NN, BL, EL>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kBcdLds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(1), dim3(ANT), smem, s, a);
    return hipGetLastError();
}

template <int NN>
static hipError_t launch_bcd_n(const AlsArgs& a, bool bl, bool el, size_t smem, hipStream_t s) {
    if (bl && el) return launch_bcd_t<NN, true, true>(a, smem, s);
    if (bl) return launch_bcd_t<NN, true, false>(a, smem, s);
    if (el) return launch_bcd_t<NN, false, true>(a, smem, s);
    return launch_bcd_t<NN, false, false>(a, smem, s);
}

hipError_t launch_bcd(const AlsArgs& a, hipStream_t s) {
    if (a.normX2 == nullptr || !bcd_supported(a.N, a.l, a.R)) return hipErrorInvalidValue;
    const size_t fixed = bcd_lds_fixed(a.N, a.l, a.R);
    int64_t S = 1;
    for (int n = 0; n < a.N; ++n) S *= a.l[n];
    const size_t init32 = bcd_init_floats(a.N, a.l, a.R);
    const size_t eig = 2 * kEigLd * kEigLd * sizeof(double);
    const size_t bsz = (size_t)S * sizeof(float);
    const bool el = fixed + eig + init32 <= kBcdLds;
    const size_t init_big = (el ? eig : 0) + init32;
    const bool bl = fixed + bsz <= kBcdLds;
    const size_t big = bl ? (bsz > init_big ? bsz : init_big) : init_big;
    const size_t smem = fixed + big;
    if (a.N == 3) return launch_bcd_n<3>(a, bl, el, smem, s);
    if (a.N == 4) return launch_bcd_n<4>(a, bl, el, smem, s);
    return launch_bcd_n<RCP_MAX_NDIM>(a, bl, el, smem, s);
}

}  // namespace rcp
