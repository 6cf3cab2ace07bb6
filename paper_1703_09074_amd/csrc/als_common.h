// Device building blocks shared by the core solvers (CP-ALS, Algorithm 2,
// and block coordinate descent, Algorithm 3): launch and LDS constants, the
// solver context, the eigenvector start of Algorithms 2 and 3 (parallel
// cyclic Jacobi) and the float64 matrix-core Gram of a factor.
#pragma once

#include "rcp_device.h"
#include "rcp_kernels.h"

namespace rcp {

constexpr int ANT = 512;
constexpr int ANW = ANT / 64;
constexpr double kPivotRtol = 1e-13;
constexpr int kJacobiMaxSweeps = 40;
constexpr int kEigLd = 64;
constexpr size_t kAlsLds = 160 * 1024 - 4096;   // dynamic LDS budget
constexpr int kMtQuads = 8;                      // inner extents up to 32 take the pipelined path

// Floats of LDS for the partial 16 x 16 blocks of the mode products: a mode
// with `blocks` output blocks splits its contraction over up to
// ANW / blocks wavefronts, all but the first slice of a block go to LDS.
__host__ __device__ inline int als_part_floats(int N, const int* l, int R) {
    int mx = 0;
    const int ncb = (R + 15) / 16;
    for (int n = 0; n < N; ++n) {
        const int blocks = ((l[n] + 15) / 16) * ncb;
        const int kp = (blocks >= ANW) ? 1 : ANW / blocks;
        const int f = (kp - 1) * blocks * 256;
        mx = mx > f ? mx : f;
    }
    return mx;
}

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
// method) ordering: each round rotates n/2 disjoint (p, q) pairs.  A round
// is two phases: the rotation angles of the pairs, then one update in which
// a thread owns a 2 x 2 block of A at (pair u, pair v) and replaces it by
// G_u A_uv G_v^T (G = [[c, -s], [s, c]] of each pair, i.e. the row and the
// column rotation at once, in place since no other thread touches the block)
// or two entries of V's row (V <- V G^T).  Returns false if the off-diagonal
// mass did not fall below 1e-30 of the diagonal's.
__device__ __forceinline__ bool jacobi_eig(double* A, double* V, int n, double* red, double* sh) {
    const int tid = threadIdx.x;
    const int np = (n + 1) & ~1;
    const int half = np / 2;
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
            if (tid < half) {
                // round-robin pairing: a = (k - 1 + round) mod (np - 1) + 1 for
                // k > 0, b = (np - 2 - k + round) mod (np - 1) + 1; both
                // arguments lie in [0, 2 (np - 1)), so one subtraction reduces them
                const int k = tid, m = np - 1;
                int xa = k - 1 + round, xb = np - 2 - k + round;
                if (xa >= m) xa -= m;
                if (xb >= m) xb -= m;
                int a = (k == 0) ? 0 : xa + 1;
                int b = xb + 1;
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
            // A: blocks (u, v); V: (row i, pair v)
            const int nblk = half * half;
            for (int e = tid; e < nblk + n * half; e += ANT) {
                if (e < nblk) {
                    const int u = e / half, v = e - (e / half) * half;
                    const double cu = cs[u], su = sn[u], cv = cs[v], sv = sn[v];
                    if (su == 0.0 && sv == 0.0) continue;
                    const int p = pp[u], q = qq[u], r = pp[v], t = qq[v];
                    const bool qv = q < n, tv = t < n;
                    const double a00 = A[p * kEigLd + r];
                    const double a01 = tv ? A[p * kEigLd + t] : 0.0;
                    const double a10 = qv ? A[q * kEigLd + r] : 0.0;
                    const double a11 = (qv && tv) ? A[q * kEigLd + t] : 0.0;
                    // rows: [b0; b1] = G_u [a0; a1]
                    const double b00 = cu * a00 - su * a10, b01 = cu * a01 - su * a11;
                    const double b10 = su * a00 + cu * a10, b11 = su * a01 + cu * a11;
                    // columns: [d0 d1] = [b0 b1] G_v^T
                    A[p * kEigLd + r] = cv * b00 - sv * b01;
                    if (tv) A[p * kEigLd + t] = sv * b00 + cv * b01;
                    if (qv) A[q * kEigLd + r] = cv * b10 - sv * b11;
                    if (qv && tv) A[q * kEigLd + t] = sv * b10 + cv * b11;
                } else {
                    const int e2 = e - nblk;
                    const int i = e2 / half, v = e2 - (e2 / half) * half;
                    const double sv = sn[v];
                    if (sv == 0.0) continue;
                    const double cv = cs[v];
                    const int r = pp[v], t = qq[v];
                    const double vr = V[i * kEigLd + r], vt = V[i * kEigLd + t];
                    V[i * kEigLd + r] = cv * vr - sv * vt;
                    V[i * kEigLd + t] = sv * vr + cv * vt;
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

// Leading R eigenvectors of the symmetric l_n x l_n matrix in E (stride
// kEigLd, destroyed), in descending eigenvalue order, each with its
// largest-magnitude entry positive, into the factor c.fac(n).
__device__ __forceinline__ bool eig_leading(const AlsCtx& c, int n, double* E, double* V) {
    const int tid = threadIdx.x;
    const int ln = c.l[n];
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

// Algorithm 2's initialisation: leading R eigenvectors of B_(n) B_(n)^T.
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
        // sum over k = a Rn + b (a < Ln, b < Rn) of B[a, i, b] B[a, i2, b],
        // eight products in flight in eight partial sums
        const float* p1 = Bg + (int64_t)i * Rn;
        const float* p2 = Bg + (int64_t)i2 * Rn;
        const int64_t sa = (int64_t)ln * Rn;
        const int K = Ln * Rn;
        double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int a = 0, b = 0, k = 0;
        for (; k + 8 <= K; k += 8) {
            float x[8], y[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t off = a * sa + b;
                x[u] = p1[off];
                y[u] = p2[off];
                if (++b == Rn) { b = 0; ++a; }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += (double)x[u] * (double)y[u];
        }
        for (; k < K; ++k) {
            const int64_t off = a * sa + b;
            acc[0] += (double)p1[off] * (double)p2[off];
            if (++b == Rn) { b = 0; ++a; }
        }
        const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        E[i * kEigLd + i2] = s;
        E[i2 * kEigLd + i] = s;
    }
    __syncthreads();
    return eig_leading(c, n, E, V);
}

// G = F^T F (R x R, float64) of the float32 factor F (l_n x R, LDS) on the
// float64 matrix cores: 16 x 16 blocks of the upper triangle, one wavefront
// per block, mirrored into the lower triangle.
__device__ __forceinline__ void gram_mfma(const float* F, int ln, int R, double* G) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nb = (R + 15) >> 4;
    const int U = nb * (nb + 1) / 2;
    for (int u = wave; u < U; u += ANW) {
        int bi = 0, rem = u;
        while (rem >= nb - bi) { rem -= nb - bi; ++bi; }
        const int bj = bi + rem;
        const int c1 = bi * 16 + li, c2 = bj * 16 + li;
        // two independent accumulation chains (even and odd steps of 4 rows)
        f64x4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < ln; k0 += 8) {
            const int k = k0 + lk, kb = k + 4;
            const double a = (k < ln && c1 < R) ? (double)F[k * R + c1] : 0.0;
            const double b = (k < ln && c2 < R) ? (double)F[k * R + c2] : 0.0;
            const double a2 = (kb < ln && c1 < R) ? (double)F[kb * R + c1] : 0.0;
            const double b2 = (kb < ln && c2 < R) ? (double)F[kb * R + c2] : 0.0;
            acc = mfma64(a, b, acc);
            acc2 = mfma64(a2, b2, acc2);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += acc2[v];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = bi * 16 + lk + 4 * v, s = bj * 16 + li;
            if (r < R && s < R) {
                G[r * R + s] = acc[v];
                if (bi != bj) G[s * R + r] = acc[v];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Gauss-Jordan solves of the symmetric positive definite systems V X = Y of
// the least-squares updates.

// Inverse of the pivot block P = A[0..pbs) x [0..pbs) (row stride lda;
// pbs <= NP <= 16, NP a multiple of 4; P padded with the identity up to NP)
// in one wavefront's registers: Gauss-Jordan on [P | I] with lane c holding
// column c (lanes 0..NP-1 P, 16..16+NP-1 I) and the rows rotating through
// the registers so that the pivot row is always register 0; the pivot
// column is read into scalar registers before each step's updates.  NP
// steps: sized to the block, a short last block costs only its own rows.
// P^{-1} goes to Pinv (16 x 16, identity outside NP x NP).  Returns 0 if a
// pivot of the first rreal rows is not above thr (or is NaN).
template <int NP>
__device__ __forceinline__ int invert_wave(const double* A, int lda, int pbs, int rreal, double thr,
                                           double* Pinv) {
    const int c = threadIdx.x & 63;
    double col[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        double v = 0.0;
        if (c < NP) v = (i < pbs && c < pbs) ? A[i * lda + c] : ((i == c) ? 1.0 : 0.0);
        else if (c >= 16 && c < 16 + NP) v = (c - 16 == i) ? 1.0 : 0.0;
        col[i] = v;
    }
    double pmin = __builtin_huge_val();
    bool pnan = false;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        double sk[NP];
        sk[0] = readlane_f64(col[0], k);
        const double u = div_pivot(col[0], sk[0]);
#pragma unroll
        for (int i = 1; i < NP; ++i) sk[i] = readlane_f64(col[i], k);
        __builtin_amdgcn_sched_barrier(0);
        if (k < rreal) {
            pmin = fmin(pmin, sk[0]);
            pnan = pnan || (sk[0] != sk[0]);
        }
#pragma unroll
        for (int i = 1; i < NP; ++i) col[i] -= sk[i] * u;
#pragma unroll
        for (int i = 0; i < NP - 1; ++i) col[i] = col[i + 1];
        col[NP - 1] = u;
    }
    if (c >= 16 && c < 32) {
        const int cj = c - 16;
#pragma unroll
        for (int i = 0; i < 16; ++i)
            Pinv[i * 16 + cj] = (i < NP && cj < NP) ? col[i < NP ? i : 0] : ((i == cj) ? 1.0 : 0.0);
    }
    return (!pnan && (rreal == 0 || pmin > thr)) ? 1 : 0;
}

// SIZED: one register inverse per block size (4, 8, 12, 16 rows); else the
// 16-row one for every block (less code in kernels short of registers).
template <bool SIZED>
__device__ __forceinline__ int invert16_wave(const double* A, int lda, int pbs, int rreal, double thr,
                                             double* Pinv) {
    if constexpr (SIZED) {
        switch (pbs) {
            case 4: return invert_wave<4>(A, lda, pbs, rreal, thr, Pinv);
            case 8: return invert_wave<8>(A, lda, pbs, rreal, thr, Pinv);
            case 12: return invert_wave<12>(A, lda, pbs, rreal, thr, Pinv);
            default: break;
        }
    }
    return invert_wave<16>(A, lda, pbs, rreal, thr, Pinv);
}

// Blocked Gauss-Jordan elimination without pivoting on the augmented system
// Aug = [V | Xt] (Rp x W, row stride ldx, V symmetric positive definite and
// padded with the identity up to Rp, Rp a multiple of 4): on return columns
// Rp..W-1 hold V^{-1} Xt.  Pivot blocks of up to 16 rows; per block j0 (pbs
// rows):
//   1. wavefront 0 inverts the pivot block P in its registers;
//   2. the pivot rows become P^{-1} [pivot rows] (float64 matrix cores);
//   3. every other row block i loses F_i [pivot rows], F_i its entries in the
//      pivot columns (matrix cores).
// Step 3 looks ahead: wavefront 0 first updates the next pivot block and
// inverts it (step 1 of the next block) while the other wavefronts update the
// rest, so the register inverse, the serial part, overlaps the matrix-core
// work.  The pivots of the inverted blocks are the Schur complements, i.e.
// the pivots of unblocked elimination, and each must exceed rtol times the
// largest of V's first R diagonal entries for the rows < R.  Columns left of
// the pivot block are never read again and are not updated; every column
// block is read whole before it is written, so the updates run in place.
// pb holds 258 doubles (P^{-1} and the flag).  SIZED: the register inverse
// sized to each block (see invert16_wave) and the lookahead; without it, the
// 16-row inverse and no lookahead (less code in kernels short of registers).
template <bool SIZED>
__device__ __forceinline__ int block16_gj(double* Aug, int ldx, int R, int Rp, int W, double rtol,
                                          double* pb) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    double* Pinv = pb;
    double* okp = pb + 256;
    if (threadIdx.x == 0) *okp = 1.0;
    // the pivot threshold, needed by wavefront 0 only (R <= 64 = one lane per row)
    double thr = 0.0;
    if (wave == 0) {
        double d = (lane < R) ? Aug[lane * ldx + lane] : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) d = fmax(d, __shfl_xor(d, o, 64));
        thr = rtol * d;
    }
    // step 1 for the block at jb (wavefront 0)
    auto invert = [&](int jb) {
        const int pbs = min(16, Rp - jb);
        const int rreal = max(0, min(pbs, R - jb));
        const int ok = invert16_wave<SIZED>(Aug + jb * ldx + jb, ldx, pbs, rreal, thr, Pinv);
        if (lane == 0 && !ok) *okp = 0.0;
    };
    const int nrb = (Rp + 15) >> 4;
    if (wave == 0) invert(0);
    __syncthreads();
    for (int j0 = 0; j0 < Rp; j0 += 16) {
        const int pbs = min(16, Rp - j0);
        const int c0 = j0 + pbs;                   // first column to update
        const int ncb = (W - c0 + 15) >> 4;
        // 2. pivot rows <- P^{-1} pivot rows
        for (int cb = wave; cb < ncb; cb += ANW) {
            const int cc = c0 + cb * 16 + li;
            const bool cv = cc < W;
            double bop[4], aop[4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int sr = 4 * kk + lk;
                bop[kk] = (sr < pbs && cv) ? Aug[(j0 + sr) * ldx + cc] : 0.0;
                aop[kk] = Pinv[li * 16 + sr];
            }
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) acc = mfma64(aop[kk], bop[kk], acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int t = lk + 4 * v;
                if (t < pbs && cv) Aug[(j0 + t) * ldx + cc] = acc[v];
            }
        }
        __syncthreads();
        // 3. other row blocks: A_ic -= F_i [pivot rows]; unit u is row block
        // u / ncb (the pivot block skipped) and column block u % ncb
        const int units = (nrb - 1) * ncb;
        auto trail = [&](int u) {
            int rb = u / ncb;
            const int cb = u - rb * ncb;
            if (rb >= (j0 >> 4)) ++rb;            // skip the pivot block
            const int i0 = rb * 16;
            const int cc = c0 + cb * 16 + li;
            const bool cv = cc < W;
            double aop[4], bop[4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int sr = 4 * kk + lk;
                const int ri = i0 + li;
                aop[kk] = (sr < pbs && ri < Rp) ? -Aug[ri * ldx + j0 + sr] : 0.0;
                bop[kk] = (sr < pbs && cv) ? Aug[(j0 + sr) * ldx + cc] : 0.0;
            }
            f64x4 acc;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ri = i0 + lk + 4 * v;
                acc[v] = (ri < Rp && cv) ? Aug[ri * ldx + cc] : 0.0;
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) acc = mfma64(aop[kk], bop[kk], acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ri = i0 + lk + 4 * v;
                if (ri < Rp && cv) Aug[ri * ldx + cc] = acc[v];
            }
        };
        if (SIZED && c0 < Rp) {
            // the next pivot block is row block j0/16 + 1, column block 0:
            // unit (j0/16) * ncb, which no other unit reads or writes; P^{-1}
            // of this block was last read in step 2
            const int un = (j0 >> 4) * ncb;
            if (wave == 0) {
                trail(un);
                invert(c0);
            } else {
                for (int u = wave - 1; u < units; u += ANW - 1)
                    if (u != un) trail(u);
            }
        } else {
            for (int u = wave; u < units; u += ANW) trail(u);
        }
        __syncthreads();
    }
    return *okp != 0.0;
}


// Row stride (doubles) of the augmented system [V | Xt]: odd, so that the 16
// rows one matrix-core operand reads at a time fall in distinct LDS banks.
__host__ __device__ inline int aug_ld(int Rp, int lmax) { return (Rp + lmax) | 1; }

// doubles of LDS the solvers need beside the augmented system (the blocked
// one's pivot-block inverse and flag; the one-wavefront one's flag)
__host__ __device__ inline int gj_buf_doubles(int ldx, int Rp) {
    (void)ldx;
    (void)Rp;
    return 258;
}

// One-wavefront variant for small systems (Rp <= 32 rows, W <= 64 columns):
// lane c holds column c in registers and the rows rotate through them so
// that the pivot row is always register 0 (static indexing): at step k the
// pivot column comes from lane k by readlane, the pivot row is scaled, the
// other rows lose their multiples of it and the finished pivot row moves to
// the back; after Rp steps the rows are in order again (the steps are
// unrolled, so the rotation is register renaming).  No barriers.
template <int RP>
__device__ __forceinline__ int gj_wave(double* Aug, int ldx, int R, int W, double rtol) {
    const int c = threadIdx.x & 63;
    const bool cv = c < W;
    double col[RP];
#pragma unroll
    for (int i = 0; i < RP; ++i) col[i] = cv ? Aug[i * ldx + c] : 0.0;
    const double dg = (c < RP) ? Aug[c * ldx + c] : 0.0;     // V_cc (V itself is not written)
    // The pivot test does not steer the elimination, so it is taken once at
    // the end: every pivot of the first R rows must exceed
    // rtol * max_{r < R} V_rr, i.e. none is NaN and the smallest does.
    double pmin = __builtin_huge_val();
    bool pnan = false;
#pragma unroll
    for (int k = 0; k < RP; ++k) {
        // the whole pivot column is read before the first update: readlanes
        // into distinct scalar registers issue back to back, where one
        // broadcast per update serialises on a single register pair
        double s[RP];
        s[0] = readlane_f64(col[0], k);
        const double u = div_pivot(col[0], s[0]);
#pragma unroll
        for (int i = 1; i < RP; ++i) s[i] = readlane_f64(col[i], k);
        __builtin_amdgcn_sched_barrier(0);
        if (k < R) {
            pmin = fmin(pmin, s[0]);
            pnan = pnan || (s[0] != s[0]);
        }
#pragma unroll
        for (int i = 1; i < RP; ++i) col[i] -= s[i] * u;
#pragma unroll
        for (int i = 0; i < RP - 1; ++i) col[i] = col[i + 1];
        col[RP - 1] = u;
    }
    if (cv && c >= RP) {
#pragma unroll
        for (int i = 0; i < RP; ++i) Aug[i * ldx + c] = col[i];
    }
    double dmax = 0.0;
#pragma unroll
    for (int k = 0; k < RP; ++k) {
        const double v = readlane_f64(dg, k);
        if (k < R) dmax = fmax(dmax, v);
    }
    return (!pnan && pmin > rtol * dmax) ? 1 : 0;
}

// V^{-1} Xt in place for Rp (a multiple of 4) rows and W columns; every
// thread returns the ok flag (0 when a pivot of the first R rows is not above
// rtol * max_{r < R} V_rr).
template <bool SIZED = true>
__device__ __forceinline__ int gj_solve(double* Aug, int ldx, int R, int Rp, int W, double rtol,
                                        double* fbuf) {
    if (Rp <= 32 && W <= 64) {
        if ((threadIdx.x >> 6) == 0) {
            int ok = 0;
            switch (Rp) {
                case 4: ok = gj_wave<4>(Aug, ldx, R, W, rtol); break;
                case 8: ok = gj_wave<8>(Aug, ldx, R, W, rtol); break;
                case 12: ok = gj_wave<12>(Aug, ldx, R, W, rtol); break;
                case 16: ok = gj_wave<16>(Aug, ldx, R, W, rtol); break;
                case 20: ok = gj_wave<20>(Aug, ldx, R, W, rtol); break;
                case 24: ok = gj_wave<24>(Aug, ldx, R, W, rtol); break;
                case 28: ok = gj_wave<28>(Aug, ldx, R, W, rtol); break;
                default: ok = gj_wave<32>(Aug, ldx, R, W, rtol); break;
            }
            if (threadIdx.x == 0) fbuf[0] = ok ? 1.0 : 0.0;
        }
        __syncthreads();
        return fbuf[0] != 0.0;
    }
    return block16_gj<SIZED>(Aug, ldx, R, Rp, W, rtol, fbuf);
}

}  // namespace rcp
