// CP-ALS on the compressed tensor B (Section 3.2.1, Algorithm 2)
// in one workgroup.  The core is small (l^N elements) and a sweep is a strict
// sequence of dependent least-squares updates, so the whole sweep loop runs
// in one persistent workgroup, with the stopping rule on the device.
//
// Per mode n of a sweep:
//   M_n = B_(n) KR(Ã_{m != n})   on the matrix cores (float32 operands and
//                                accumulation), the Khatri-Rao operand formed
//                                on the fly from the factors in LDS;
//   V   = *_{m != n} G_m         (Hadamard product of the Gram matrices);
//   Ã_n = M_n V^{-1}             by Gauss-Jordan elimination on [V | M_n^T]
//                                (V is symmetric positive definite, so no
//                                pivoting), the Moore-Penrose pseudo-inverse
//                                when a pivot falls below 1e-13 of diag(V);
//   columns of Ã_n scaled to unit norm (the norms are lambda), G_n updated.
// Grams, solves, norms and the fit are float64; the factors feeding the
// matrix cores are float32.

#include "als_common.h"

#include <type_traits>

namespace rcp {


// ---------------------------------------------------------------------------
// M_n = B_(n) KR(Ã_{m != n}) on the matrix cores.
//
// The core is row-major over (i_0, ..., i_{N-1}); for mode n the contraction
// index k runs over the other modes in increasing order (the row order of the
// Khatri-Rao product with the first factor slowest, Section 2.3), so
// B_(n)[i, k] sits at  i * st_n + sum_m d_m(k) st_m  with st_m the stride of
// mode m and d_m(k) the mixed-radix digits of k.  k splits into an outer part
// (all other modes but the last) and the inner digit of the last other mode:
// per outer index the Khatri-Rao row is the product of the outer factor rows
// (formed once) and the inner factor row, and the inner loop is a plain
// strided walk.  The output (l_n x R) is tiled in 16 x 16 blocks; a work unit
// is one block over one slice of the outer index, the units are spread over
// the eight wavefronts and slices of one block are summed through LDS.  Lane
// (lr, lk) of a v_mfma_f32_16x16x4_f32 feeds row lr of the B_(n) tile and
// column lr of the Khatri-Rao tile at inner index k0 + lk.
//
// NN - 1 digit slots, N - 1 of them real; the NN - N leading slots are
// padding of size 1 and stride 0 whose factor reads hit a row of ones, so one
// instantiation serves every order up to NN.  Writes M (l_n x R) and its
// transpose into the right part of the augmented system.
template <int NN>
__device__ __forceinline__ void mttkrp(const AlsCtx& c, int n, const float* B, const int* st,
                                       const float* ones, float* P, int pfloats, double* M,
                                       double* Xt, int ldx) {
    constexpr int D = NN - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int N = c.N, R = c.R, ln = c.l[n];
    const int stn = st[n];
    int lo[D], so[D], fo[D];
    int Ko = 1;
#pragma unroll
    for (int s = 0; s < D; ++s) {
        const int j = s - (NN - N);             // index among the real other modes
        if (j < 0) {
            lo[s] = 1; so[s] = 0; fo[s] = (int)(ones - c.fbase);
        } else {
            const int m = (j < n) ? j : j + 1;
            lo[s] = c.l[m]; so[s] = st[m]; fo[s] = c.foff[m];
            if (s < D - 1) Ko *= lo[s];
        }
    }
    const int Kl = lo[D - 1], sl = so[D - 1];
    const float* fin = c.fbase + fo[D - 1];
    const int nib = (ln + 15) >> 4, ncb = (R + 15) >> 4;
    const int blocks = nib * ncb;
    // slices of the outer index per block, as many as idle wavefronts and
    // the pfloats of LDS for their partial blocks allow
    const int kp = (blocks >= ANW) ? 1 : min(min(ANW / blocks, Ko), 1 + pfloats / (blocks * 256));
    const int units = blocks * kp;
    const int per = (Ko + kp - 1) / kp;
    f32x4 keep = {0.f, 0.f, 0.f, 0.f};
    int keep_blk = -1;
    for (int u = wave; u < units; u += ANW) {
        const int blk = u % blocks, part = u / blocks;
        const int ib = blk / ncb, cb = blk - (blk / ncb) * ncb;
        const int o_lo = part * per;
        const int o_hi = min(Ko, o_lo + per);
        const int i = ib * 16 + lr, col = cb * 16 + lr;
        const bool rv = i < ln, cv = col < R;
        const int ioff = (rv ? i : 0) * stn;   // rows past l_n only feed discarded outputs
        const int ccol = cv ? col : 0;
        // outer digits of o_lo
        int d[D];
        {
            int rem = o_lo;
#pragma unroll
            for (int s = D - 2; s >= 0; --s) {
                const int q = rem / lo[s];
                d[s] = rem - q * lo[s];
                rem = q;
            }
        }
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
        const int nq = (Kl + 3) >> 2;
        // offset of the core row and Khatri-Rao weight of the outer part at
        // the current digits; then step the digits to the next outer index
        auto outer = [&](int& boff, float& ob) {
            boff = ioff;
            ob = cv ? 1.0f : 0.0f;
#pragma unroll
            for (int s = 0; s < D - 1; ++s) {
                boff += d[s] * so[s];
                ob *= c.fbase[fo[s] + d[s] * R + ccol];
            }
#pragma unroll
            for (int s = D - 2; s >= 0; --s) {
                d[s] += 1;
                if (d[s] < lo[s]) break;
                d[s] = 0;
            }
        };
        // NQ = 0: quad count nq at run time; otherwise a compile-time count
        // NQ >= nq, so the loop body has no branches (the quads past nq read
        // a clamped in-bounds element and feed zeros to the matrix cores)
        auto pipelined = [&](auto nq_const) {
            constexpr int NQ = decltype(nq_const)::value;
            // software pipelined in half steps of four quads: the operands of
            // the next half are in flight while the matrix cores work on the
            // current one (at most nine LDS reads outstanding, within what the
            // LDS counter can track)
            constexpr int HQ = kMtQuads / 2;
            float alo[HQ], blo[HQ], ahi[HQ], bhi[HQ];
            float ob = 0.0f, ob_next = 0.0f;
            int boff = 0, boff_next = 0;
            auto fetch = [&](float* av, float* bv, int bo, int q0) {
                const float* ap = B + bo;
#pragma unroll
                for (int q = 0; q < HQ; ++q) {
                    const int kl = lk + 4 * (q0 + q);
                    const int kc = (kl < Kl) ? kl : 0;
                    av[q] = ap[kc * sl];
                    bv[q] = fin[kc * R + ccol];
                }
            };
            auto compute = [&](const float* av, const float* bv, float w, int q0) {
#pragma unroll
                for (int q = 0; q < HQ; ++q) {
                    if (q0 + q < (NQ ? NQ : nq)) {
                        const bool kv = lk + 4 * (q0 + q) < Kl;
                        const float x = kv ? av[q] : 0.0f;
                        const float y = kv ? w * bv[q] : 0.0f;
                        if (q & 1) acc1 = mfma16x16x4(x, y, acc1);
                        else acc0 = mfma16x16x4(x, y, acc0);
                    }
                }
            };
            if (o_lo < o_hi) {
                outer(boff, ob);
                fetch(alo, blo, boff, 0);
            }
            for (int o = o_lo; o < o_hi; ++o) {
                if ((NQ ? NQ : nq) > HQ) fetch(ahi, bhi, boff, HQ);
                compute(alo, blo, ob, 0);
                const bool more = o + 1 < o_hi;
                if (more) {
                    outer(boff_next, ob_next);
                    fetch(alo, blo, boff_next, 0);
                }
                if ((NQ ? NQ : nq) > HQ) compute(ahi, bhi, ob, HQ);
                ob = ob_next;
                boff = boff_next;
            }
        };
        if (nq <= kMtQuads && nq >= 7) {
            pipelined(std::integral_constant<int, 8>{});
        } else if (nq == 5 || nq == 6) {
            pipelined(std::integral_constant<int, 6>{});
        } else if (nq == 3 || nq == 4) {
            pipelined(std::integral_constant<int, 4>{});
        } else if (nq <= kMtQuads) {
            pipelined(std::integral_constant<int, 0>{});
        } else {
            for (int o = o_lo; o < o_hi; ++o) {
                int boff;
                float ob;
                outer(boff, ob);
                const float* bp = B + boff;
                // wave-uniform trip counts: the matrix-core instructions run with all lanes
                int k0 = 0;
                for (; k0 + 8 <= Kl; k0 += 8) {
                    const int kl = k0 + lk;
                    const float x0 = bp[kl * sl];
                    const float y0 = fin[kl * R + ccol];
                    const float x1 = bp[(kl + 4) * sl];
                    const float y1 = fin[(kl + 4) * R + ccol];
                    acc0 = mfma16x16x4(x0, ob * y0, acc0);
                    acc1 = mfma16x16x4(x1, ob * y1, acc1);
                }
                for (; k0 < Kl; k0 += 4) {
                    const int kl = k0 + lk;
                    float x0 = 0.0f, y0 = 0.0f;
                    if (kl < Kl) { x0 = bp[kl * sl]; y0 = fin[kl * R + ccol]; }
                    acc0 = mfma16x16x4(x0, ob * y0, acc0);
                }
            }
        }
        f32x4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = acc0[v] + acc1[v];
        if (kp == 1) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = ib * 16 + 4 * lk + v;
                if (row < ln && cv) {
                    M[row * R + col] = (double)acc[v];
                    Xt[col * ldx + row] = (double)acc[v];
                }
            }
        } else if (part > 0) {
            float* dst = P + ((part - 1) * blocks + blk) * 256;
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[(4 * lk + v) * 16 + lr] = acc[v];
        } else {
            keep = acc;
            keep_blk = blk;
        }
    }
    __syncthreads();
    if (keep_blk >= 0) {
        const int ib = keep_blk / ncb, cb = keep_blk - (keep_blk / ncb) * ncb;
        const int col = cb * 16 + lr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float sum = keep[v];
            for (int part = 1; part < kp; ++part)
                sum += P[((part - 1) * blocks + keep_blk) * 256 + (4 * lk + v) * 16 + lr];
            const int row = ib * 16 + 4 * lk + v;
            if (row < ln && col < R) {
                M[row * R + col] = (double)sum;
                Xt[col * ldx + row] = (double)sum;
            }
        }
    }
}

// Left block of the augmented system: V = *_{m != n} G_m, identity padding up
// to Rp, and zero padding rows in the right block.
// With the Grams in global memory (G_GLOBAL) a thread holds its at most KE
// entries (Rp <= 64) in registers and issues each Gram's loads together, so
// a Gram costs one memory latency, not one per entry; with the Grams in LDS
// the plain loop is faster.  Either way the product runs over m in
// increasing order.
constexpr int KE = (RCP_MAX_RANK * RCP_MAX_RANK + ANT - 1) / ANT;

template <bool G_GLOBAL>
__device__ __forceinline__ void hadamard_grams(const AlsCtx& c, int n, const double* G, double* Aug,
                                               int ldx, int Rp, int ln) {
    const int R = c.R;
    if constexpr (!G_GLOBAL) {
        for (int e = threadIdx.x; e < Rp * Rp; e += ANT) {
            const int r = e / Rp, s = e - (e / Rp) * Rp;
            double v;
            if (r < R && s < R) {
                v = 1.0;
                for (int m = 0; m < c.N; ++m)
                    if (m != n) v *= G[m * R * R + r * R + s];
            } else {
                v = (r == s) ? 1.0 : 0.0;
            }
            Aug[r * ldx + s] = v;
        }
        for (int e = threadIdx.x; e < (Rp - R) * ln; e += ANT) {
            const int r = R + e / ln, i = e - (e / ln) * ln;
            Aug[r * ldx + Rp + i] = 0.0;
        }
        return;
    }
    double v[KE];
#pragma unroll
    for (int k = 0; k < KE; ++k) v[k] = 1.0;
    // the Grams m != n two at a time (the q-th is q, or q + 1 past n)
    for (int q = 0; q < c.N - 1; q += 2) {
        const int ma = q < n ? q : q + 1, mb = q + 1 < n ? q + 1 : q + 2;
        const bool has_b = q + 1 < c.N - 1;
        const double* Ga = G + ma * R * R;
        const double* Gb = G + (has_b ? mb : ma) * R * R;
        double ga[KE], gb[KE];
#pragma unroll
        for (int k = 0; k < KE; ++k) {
            const int e = threadIdx.x + k * ANT;
            const int r = e / Rp, s = e - r * Rp;
            const bool in = e < Rp * Rp && r < R && s < R;
            ga[k] = in ? Ga[r * R + s] : 1.0;
            gb[k] = (in && has_b) ? Gb[r * R + s] : 1.0;
        }
#pragma unroll
        for (int k = 0; k < KE; ++k) {
            v[k] *= ga[k];
            v[k] *= gb[k];
        }
    }
#pragma unroll
    for (int k = 0; k < KE; ++k) {
        const int e = threadIdx.x + k * ANT;
        if (e < Rp * Rp) {
            const int r = e / Rp, s = e - r * Rp;
            Aug[r * ldx + s] = (r < R && s < R) ? v[k] : ((r == s) ? 1.0 : 0.0);
        }
    }
    for (int e = threadIdx.x; e < (Rp - R) * ln; e += ANT) {
        const int r = R + e / ln, i = e - (e / ln) * ln;
        Aug[r * ldx + Rp + i] = 0.0;
    }
}

// Unit columns of the solution and their Gram: Xt holds the solution
// transposed (R rows of length l_n, float64, stride ldx).  First wavefront b
// forms the norms of rows 16b .. 16b + 15 (each lane sums a quarter of a
// row, the four quarters meet by shuffles): lambda_r = ||Xt_r||, in lam
// (LDS).  Then every wavefront takes 16 x 16 blocks (bi, bj) of the upper
// triangle of G_n = F^T F, F the float32 factor with columns
// Xt_r / ||Xt_r||, and feeds the matrix cores with exactly the float32
// values of F, so G_n is the float64 Gram of the stored factor; the
// wavefronts of diagonal blocks also store F (l_n x R).
__device__ __forceinline__ void unit_factor_gram(const double* Xt, int ldx, int ln, int R, float* F,
                                                 double* G, double* lam) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nb = (R + 15) >> 4;
    for (int b = wave; b < nb; b += ANW) {
        const int c1 = b * 16 + li;
        const bool v1 = c1 < R;
        const double* x1 = Xt + (v1 ? c1 : 0) * ldx;
        double s1 = 0.0;
#pragma unroll 4
        for (int k = lk; k < ln; k += 4) {
            const double p = x1[k];
            s1 += p * p;
        }
        s1 += __shfl_xor(s1, 16, 64);
        s1 += __shfl_xor(s1, 32, 64);
        if (lk == 0 && v1) lam[c1] = sqrt(s1);
    }
    __syncthreads();
    const int U = nb * (nb + 1) / 2;
    for (int u = wave; u < U; u += ANW) {
        int bi = 0, rem = u;
        while (rem >= nb - bi) { rem -= nb - bi; ++bi; }
        const int bj = bi + rem;
        const bool diag = bi == bj;
        const int c1 = bi * 16 + li, c2 = bj * 16 + li;
        const bool v1 = c1 < R, v2 = c2 < R;
        const double* x1 = Xt + (v1 ? c1 : 0) * ldx;
        const double* x2 = Xt + (v2 ? c2 : 0) * ldx;
        const double nu1 = v1 ? lam[c1] : 0.0, nu2 = v2 ? lam[c2] : 0.0;
        const double i1 = (nu1 > 0.0) ? 1.0 / nu1 : 1.0, i2 = (nu2 > 0.0) ? 1.0 / nu2 : 1.0;
        f64x4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < ln; k0 += 8) {
            const int k = k0 + lk, kb = k + 4;
            const bool ka = k < ln, kbv = kb < ln;
            const float fa = (float)(x1[ka ? k : 0] * i1), fb = (float)(x2[ka ? k : 0] * i2);
            const float fa2 = (float)(x1[kbv ? kb : 0] * i1), fb2 = (float)(x2[kbv ? kb : 0] * i2);
            if (diag && v1) {
                if (ka) F[k * R + c1] = fa;
                if (kbv) F[kb * R + c1] = fa2;
            }
            acc = mfma64((ka && v1) ? (double)fa : 0.0, (ka && v2) ? (double)fb : 0.0, acc);
            acc2 = mfma64((kbv && v1) ? (double)fa2 : 0.0, (kbv && v2) ? (double)fb2 : 0.0, acc2);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += acc2[v];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = bi * 16 + lk + 4 * v, t = bj * 16 + li;
            if (r < R && t < R) {
                G[r * R + t] = acc[v];
                if (!diag) G[t * R + r] = acc[v];
            }
        }
    }
}

// Ã_n = M V^+ (V and M^T already in the augmented system), then unit
// columns: lambda_r = ||column r||, the float32 factor in c.fac(n) and
// G_n = Ã_n^T Ã_n of exactly that float32 factor (matrix cores).  Returns
// RCP_INFO_* bits.
template <bool SIZED>
__device__ __forceinline__ int solve_update(const AlsCtx& c, int n, double* G, const double* M,
                                            double* Aug, int ldx, int Rp, double* pb, double* E,
                                            double* Ev, double* lam) {
    const int tid = threadIdx.x, R = c.R, ln = c.l[n];
    double* Xt = Aug + Rp;
    int status = 0;
    const int ok = gj_solve<SIZED>(Aug, ldx, R, Rp, Rp + ln, kPivotRtol, pb);
    if (!ok) {
        // Moore-Penrose pseudo-inverse through the eigen-decomposition
        status |= RCP_INFO_PINV_FALLBACK;
        for (int e = tid; e < R * R; e += ANT) {
            double v = 1.0;
            for (int m = 0; m < c.N; ++m)
                if (m != n) v *= G[m * R * R + e];
            E[(e / R) * kEigLd + (e % R)] = v;
        }
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
            Aug[r * ldx + s] = acc;                             // V^+ into the left block
        }
        __syncthreads();
        for (int e = tid; e < ln * R; e += ANT) {
            const int r = e / ln, i = e - (e / ln) * ln;
            double acc = 0.0;
            for (int t = 0; t < R; ++t) acc += Aug[r * ldx + t] * M[i * R + t];
            Xt[r * ldx + i] = acc;                              // Xt = (M V^+)^T
        }
        __syncthreads();
    }
    unit_factor_gram(Xt, ldx, ln, R, c.fac(n), G + n * R * R, lam);
    __syncthreads();
    return status;
}

template <int NN, bool B_IN_LDS, bool EIG_IN_LDS>
__device__ __forceinline__ void als_body(const AlsArgs& a) {
    extern __shared__ __align__(16) unsigned char als_smem[];
    __shared__ double red[ANW];
    __shared__ double sh[128];
    __shared__ double lam[RCP_MAX_RANK];
    __shared__ double lam_tmp[RCP_MAX_RANK];
    __shared__ int sl[RCP_MAX_NDIM];
    __shared__ int sfoff[RCP_MAX_NDIM];
    __shared__ int sst[RCP_MAX_NDIM];
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
            if (tid == 0) { sl[n] = a.l[n]; sfoff[n] = (int)(fbytes / sizeof(float)); }
            fbytes += ((size_t)a.l[n] * R * sizeof(float) + 15) & ~(size_t)15;
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

    // dynamic LDS: [factors | ones | G | M | Aug = [V | Xt] | pivot buffers | P | big: E,V (init) then the core]
    const int Rp = (R + 3) / 4 * 4;
    const int ldx = aug_ld(Rp, lmax);
    unsigned char* p = als_smem;
    c.fbase = (float*)p;
    p += fbytes;
    float* ones = (float*)p; p += RCP_MAX_RANK * sizeof(float);
    double* G = (double*)p;  p += (size_t)N * R * R * sizeof(double);
    double* Aug = (double*)p; p += (size_t)Rp * ldx * sizeof(double);
    double* pb = (double*)p; p += (size_t)gj_buf_doubles(ldx, Rp) * sizeof(double);
    const int pfl = als_part_floats(N, a.l, R);
    float* P = (float*)p;    p += (size_t)pfl * sizeof(float);
    double* M = a.Ebuf + 2 * kEigLd * kEigLd;            // l_n x R, global (read by the fit and the fallback)
    double* E = EIG_IN_LDS ? (double*)p : a.Ebuf;
    double* Ev = E + kEigLd * kEigLd;
    double* Es = a.Ebuf;
    double* Evs = a.Ebuf + kEigLd * kEigLd;
    float* Bl = (float*)p;
    for (int r = tid; r < RCP_MAX_RANK; r += ANT) ones[r] = 1.0f;
    __syncthreads();

    double s = 0.0;
    for (int e = tid; e < c.S; e += ANT) { const double v = a.B[e]; s += v * v; }
    const double normB2 = block_sum(s, red);
    const double normX2 = (a.normX2 != nullptr) ? *a.normX2 : normB2;

    int status = 0;
    for (int n = 1; n < N; ++n) {
        if (a.warm) {
            // the caller's starting factors (warm start)
            for (int e = tid; e < c.l[n] * R; e += ANT) c.fac(n)[e] = a.At[n][e];
            __syncthreads();
        } else if (!eig_init(c, a.B, n, E, Ev)) {
            status |= RCP_INFO_EIG_NOT_CONVERGED;
        }
        gram_mfma(c.fac(n), c.l[n], R, G + n * R * R);
    }
    __syncthreads();
    if (B_IN_LDS)
        for (int e = tid; e < c.S; e += ANT) Bl[e] = a.B[e];
    __syncthreads();
    const float* Bs = B_IN_LDS ? Bl : a.B;

    double rho = 0.0, rho_prev = 0.0;
    int it;
    for (it = 1; it <= a.max_iters; ++it) {
        for (int n = 0; n < N; ++n) {
            hadamard_grams<false>(c, n, G, Aug, ldx, Rp, c.l[n]);
            mttkrp<NN>(c, n, Bs, sst, ones, P, pfl, M, Aug + Rp, ldx);
            __syncthreads();
            status |= solve_update<false>(c, n, G, M, Aug, ldx, Rp, pb, Es, Evs,
                                   (n == N - 1) ? lam : lam_tmp);
        }
        // ---- fit (Section 3.3): rho = 1 - (||X||^2 + ||Xhat||^2 - 2 <Xhat, X>) / ||X||^2,
        // needed by the stopping rule (tol > 0), after the last sweep, and to
        // report a non-finite model (seen first in lambda)
        bool need_fit = a.tol > 0.0 || it == a.max_iters;
        if (!need_fit) {
            bool fin = true;
            for (int r = 0; r < R; ++r) fin = fin && isfinite(lam[r]);
            need_fit = !fin;
        }
        if (!need_fit) continue;
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
        if (a.status_word != nullptr && status != 0) *a.status_word |= status;
    }
}

template <int NN, bool B_IN_LDS, bool EIG_IN_LDS>
__global__ __launch_bounds__(ANT) void k_als(AlsArgs a) {
    als_body<NN, B_IN_LDS, EIG_IN_LDS>(a);
}

// One workgroup per problem of a batch; every problem's layout fits the
// launch's LDS size and template choice (the launcher takes the maxima).
template <int NN, bool B_IN_LDS, bool EIG_IN_LDS>
__global__ __launch_bounds__(ANT) void k_als_batch(const AlsArgs* args) {
    const AlsArgs& a = args[blockIdx.x];
    als_body<NN, B_IN_LDS, EIG_IN_LDS>(a);
}

// ---------------------------------------------------------------------------
// Grid-wide form for cores larger than LDS.  Per mode, B_(n) KR runs over the
// whole GPU (the Khatri-Rao kind of the streaming mode product, partials
// reduced in float64 into a.Y); the one-workgroup kernels below take it from
// there with the same solve, normalisation, Gram and fit as the persistent
// kernel.  The sweep state lives in a.state:
//   ints  [0] stop flag, [1] sweeps done, [2] RCP_INFO_* bits
//   double[2] rho of the last sweep
//   double[kStG ..] G_0 .. G_{N-1} (R x R each), then lambda (R)
// The stop flag makes every later launch of the sweep loop (these kernels
// and the mode products) return at once, so the host can enqueue all
// max_iters sweeps up front.
constexpr int kStG = 4;

size_t als_state_doubles(int N, int R) { return kStG + (size_t)N * R * R + R; }

__device__ __forceinline__ void wide_ctx(const AlsArgs& a, AlsCtx& c, int* sl, int* sfoff,
                                         float* fbase, double* red, double* sh) {
    const int tid = threadIdx.x;
    if (tid < RCP_MAX_NDIM) {
        sl[tid] = tid < a.N ? a.l[tid] : 1;
        sfoff[tid] = 0;                       // only factor n is held, at fbase
    }
    c.N = a.N;
    c.R = a.R;
    c.S = 1;
    for (int m = 0; m < a.N; ++m) c.S *= a.l[m];
    c.lN = a.l[a.N - 1];
    c.Lh = c.S / c.lN;
    c.l = sl;
    c.foff = sfoff;
    c.fbase = fbase;
    c.red = red;
    c.sh = sh;
    __syncthreads();
}

// Algorithm 2's initialisation for every mode n >= 1 at once, workgroup n - 1 taking
// mode n: the leading eigenvectors of the Gram B_(n) B_(n)^T (upper triangle
// at a.Y + (n - 1) ystride, row stride l_n rounded up to 16).  The sweep
// state is cleared beforehand by the host; a non-converged Jacobi or-s its
// bit into it.
__global__ __launch_bounds__(ANT) void k_als_wide_init(AlsArgs a, int ystride) {
    extern __shared__ __align__(16) unsigned char als_smem[];
    __shared__ double red[ANW];
    __shared__ double sh[128];
    __shared__ int sl[RCP_MAX_NDIM];
    __shared__ int sfoff[RCP_MAX_NDIM];
    const int tid = threadIdx.x;
    const int n = 1 + (int)blockIdx.x;
    const int R = a.R, ln = a.l[n];
    const int ldy = (ln + 15) & ~15;
    const double* Y = a.Y + (size_t)(n - 1) * ystride;
    double* E = (double*)als_smem;
    double* V = E + kEigLd * kEigLd;
    AlsCtx c;
    wide_ctx(a, c, sl, sfoff, (float*)(V + kEigLd * kEigLd), red, sh);
    for (int e = tid; e < ln * ln; e += ANT) {
        const int i = e / ln, j = e - (e / ln) * ln;
        const int lo = min(i, j), hi = max(i, j);
        E[i * kEigLd + j] = Y[lo * ldy + hi];
    }
    __syncthreads();
    const bool ok = eig_leading(c, n, E, V);
    double* G = a.state + kStG;
    gram_mfma(c.fac(n), ln, R, G + n * R * R);
    for (int e = tid; e < ln * R; e += ANT) a.At[n][e] = c.fac(n)[e];
    if (tid == 0 && !ok) atomicOr((int*)a.state + 2, RCP_INFO_EIG_NOT_CONVERGED);
}

// Algorithm 2's update of mode n in one sweep from M_n in a.Y (row
// stride a.ldy); after the last mode the fit of Section 3.3 and the
// stopping rule, with lambda and info written every sweep.
__global__ __launch_bounds__(ANT) void k_als_wide_step(AlsArgs a, int n) {
    extern __shared__ __align__(16) unsigned char als_smem[];
    __shared__ double red[ANW];
    __shared__ double sh[128];
    __shared__ double lam[RCP_MAX_RANK];
    __shared__ int sl[RCP_MAX_NDIM];
    __shared__ int sfoff[RCP_MAX_NDIM];
    int* fl = (int*)a.state;
    if (fl[0] != 0) return;
    const int tid = threadIdx.x;
    const int N = a.N, R = a.R, ln = a.l[n];
    int lmax = 0;
    for (int m = 0; m < N; ++m) lmax = max(lmax, a.l[m]);
    const int Rp = (R + 3) / 4 * 4;
    const int ldx = aug_ld(Rp, lmax);
    double* Aug = (double*)als_smem;
    double* pb = Aug + Rp * ldx;
    float* fbase = (float*)(pb + gj_buf_doubles(ldx, Rp));
    AlsCtx c;
    wide_ctx(a, c, sl, sfoff, fbase, red, sh);
    double* G = a.state + kStG;
    double* M = a.Ebuf + 2 * kEigLd * kEigLd;      // l_n x R
    double* Es = a.Ebuf;
    double* Evs = a.Ebuf + kEigLd * kEigLd;

    {
        // ln * R <= 4096: all of a thread's loads of M in flight at once,
        // and still in flight while the Grams' are issued
        double v[KE];
#pragma unroll
        for (int k = 0; k < KE; ++k) {
            const int e = tid + k * ANT;
            const int i = e / R, r = e - (e / R) * R;
            v[k] = (e < ln * R) ? a.Y[i * a.ldy + r] : 0.0;
        }
        hadamard_grams<true>(c, n, G, Aug, ldx, Rp, ln);
#pragma unroll
        for (int k = 0; k < KE; ++k) {
            const int e = tid + k * ANT;
            if (e < ln * R) {
                const int i = e / R, r = e - (e / R) * R;
                M[e] = v[k];
                Aug[r * ldx + Rp + i] = v[k];
            }
        }
    }
    __syncthreads();
    int status = solve_update<true>(c, n, G, M, Aug, ldx, Rp, pb, Es, Evs, lam);
    for (int e = tid; e < ln * R; e += ANT) a.At[n][e] = c.fac(n)[e];
    if (n < N - 1) {
        if (tid == 0 && status != 0) fl[2] |= status;
        return;
    }
    // fit (Section 3.3) on the core, as in the persistent kernel, when the
    // stopping rule, the last sweep or a non-finite lambda needs it
    const int it = fl[1] + 1;
    bool need_fit = a.tol > 0.0 || it >= a.max_iters;
    if (!need_fit) {
        bool fin = true;
        for (int r = 0; r < R; ++r) fin = fin && isfinite(lam[r]);
        need_fit = !fin;
    }
    if (!need_fit) {
        for (int r = tid; r < R; r += ANT) a.state[kStG + (size_t)N * R * R + r] = lam[r];
        __syncthreads();
        if (tid == 0) {
            fl[2] |= status;
            fl[1] = it;
            a.info->iters = it;
        }
        return;
    }
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
    const double normX2 = *a.normX2;
    const double err2 = normX2 - 2.0 * inner + model;
    const double rho = (normX2 > 0.0) ? 1.0 - err2 / normX2 : 0.0;
    bool stop = it >= a.max_iters;
    if (!isfinite(rho)) {
        status |= RCP_INFO_NONFINITE;
        stop = true;
    } else if (a.tol > 0.0 && it >= 2 && fabs(rho - a.state[2]) < a.tol) {
        stop = true;
    }
    for (int r = tid; r < R; r += ANT) {
        a.lambda[r] = (float)lam[r];
        a.state[kStG + (size_t)N * R * R + r] = lam[r];
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
        if (stop) fl[0] = 1;
    }
}

// Warm start of the grid-wide form: the Grams of the caller's factors
// At[1..N-1] (left in place: the mode products read them there) and a fresh
// sweep state.
__global__ __launch_bounds__(ANT) void k_als_wide_warm(AlsArgs a) {
    extern __shared__ __align__(16) unsigned char als_smem[];
    float* F = (float*)als_smem;
    const int tid = threadIdx.x;
    const int N = a.N, R = a.R;
    double* G = a.state + kStG;
    for (int n = 1; n < N; ++n) {
        const int ln = a.l[n];
        for (int e = tid; e < ln * R; e += ANT) F[e] = a.At[n][e];
        __syncthreads();
        gram_mfma(F, ln, R, G + n * R * R);
        __syncthreads();
    }
    if (tid == 0) {
        int* fl = (int*)a.state;
        fl[0] = 0;
        fl[1] = 0;
        fl[2] = 0;
        a.state[2] = 0.0;
    }
}

static size_t als_lds_fixed(int N, const int* l, int R) {
    size_t b = 0;
    int lmax = 0;
    for (int n = 0; n < N; ++n) {
        b += ((size_t)l[n] * R * sizeof(float) + 15) & ~(size_t)15;
        lmax = lmax > l[n] ? lmax : l[n];
    }
    const int Rp = (R + 3) / 4 * 4;
    const int ldx = aug_ld(Rp, lmax);
    b += RCP_MAX_RANK * sizeof(float);                        // ones
    b += (size_t)N * R * R * sizeof(double);                  // G
    b += (size_t)Rp * ldx * sizeof(double);                   // augmented system [V | M^T]
    b += (size_t)gj_buf_doubles(ldx, Rp) * sizeof(double);   // pivot buffers
    b += (size_t)als_part_floats(N, l, R) * sizeof(float);    // partial products
    return b;
}

// workspace (doubles): Jacobi scratch (2 x 64 x 64) for the pseudo-inverse
// fallback and for the initialisation when it does not fit in LDS, then the
// mode product M_n (l_n x R)
size_t als_workspace_doubles(int N, const int* l, int R) {
    int lmax = 0;
    for (int n = 0; n < N; ++n) lmax = lmax > l[n] ? lmax : l[n];
    return 2 * kEigLd * kEigLd + (size_t)lmax * R;
}

bool als_core_in_lds(int N, const int* l, int R) {
    int64_t S = 1;
    for (int n = 0; n < N; ++n) S *= l[n];
    return als_lds_fixed(N, l, R) + (size_t)S * sizeof(float) <= kAlsLds;
}

static size_t wide_step_lds(const AlsArgs& a) {
    int lmax = 0;
    for (int m = 0; m < a.N; ++m) lmax = lmax > a.l[m] ? lmax : a.l[m];
    const int Rp = (a.R + 3) / 4 * 4;
    const int ldx = aug_ld(Rp, lmax);
    return (size_t)(Rp * ldx + gj_buf_doubles(ldx, Rp)) * sizeof(double) +
           (size_t)lmax * a.R * sizeof(float);
}

hipError_t launch_als_wide_init(const AlsArgs& a, int ystride, hipStream_t s) {
    if (a.N < 2 || a.Y == nullptr || a.state == nullptr) return hipErrorInvalidValue;
    int lmax = 0;
    for (int m = 0; m < a.N; ++m) lmax = lmax > a.l[m] ? lmax : a.l[m];
    const size_t smem = 2 * kEigLd * kEigLd * sizeof(double) + (size_t)lmax * a.R * sizeof(float);
    hipError_t e = hipFuncSetAttribute((const void*)k_als_wide_init,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kAlsLds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_als_wide_init, dim3((unsigned)(a.N - 1)), dim3(ANT), smem, s, a, ystride);
    return hipGetLastError();
}

hipError_t launch_als_wide_warm(const AlsArgs& a, hipStream_t s) {
    if (a.state == nullptr) return hipErrorInvalidValue;
    int lmax = 0;
    for (int m = 0; m < a.N; ++m) lmax = lmax > a.l[m] ? lmax : a.l[m];
    const size_t smem = (size_t)lmax * a.R * sizeof(float);
    hipLaunchKernelGGL(k_als_wide_warm, dim3(1), dim3(ANT), smem, s, a);
    return hipGetLastError();
}

hipError_t launch_als_wide_step(const AlsArgs& a, int n, hipStream_t s) {
    if (n < 0 || n >= a.N || a.Y == nullptr || a.state == nullptr || a.normX2 == nullptr)
        return hipErrorInvalidValue;
    const size_t smem = wide_step_lds(a);
    if (smem > kAlsLds) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void*)k_als_wide_step,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kAlsLds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_als_wide_step, dim3(1), dim3(ANT), smem, s, a, n);
    return hipGetLastError();
}

bool als_supported(int N, const int* l, int R) {
    int64_t S = 1;
    for (int n = 0; n < N; ++n) S *= l[n];
    return S < ((int64_t)1 << 31) && als_lds_fixed(N, l, R) <= kAlsLds;
}

template <int NN, bool BL, bool EL>
static hipError_t launch_als_t(const AlsArgs& a, size_t smem, hipStream_t s) {
    auto k = k_als<NN, BL, EL>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kAlsLds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(1), dim3(ANT), smem, s, a);
    return hipGetLastError();
}

template <int NN>
static hipError_t launch_als_n(const AlsArgs& a, bool bl, bool el, size_t smem, hipStream_t s) {
    if (bl && el) return launch_als_t<NN, true, true>(a, smem, s);
    if (bl) return launch_als_t<NN, true, false>(a, smem, s);
    if (el) return launch_als_t<NN, false, true>(a, smem, s);
    return launch_als_t<NN, false, false>(a, smem, s);
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
    if (a.N == 3) return launch_als_n<3>(a, bl, el, smem, s);
    if (a.N == 4) return launch_als_n<4>(a, bl, el, smem, s);
    return launch_als_n<RCP_MAX_NDIM>(a, bl, el, smem, s);
}

template <int NN, bool BL, bool EL>
static hipError_t launch_als_batch_t(const AlsArgs* dargs, int count, size_t smem, hipStream_t s) {
    auto k = k_als_batch<NN, BL, EL>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kAlsLds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)count), dim3(ANT), smem, s, dargs);
    return hipGetLastError();
}

template <int NN>
static hipError_t launch_als_batch_n(const AlsArgs* dargs, int count, bool bl, bool el, size_t smem,
                                     hipStream_t s) {
    if (bl && el) return launch_als_batch_t<NN, true, true>(dargs, count, smem, s);
    if (bl) return launch_als_batch_t<NN, true, false>(dargs, count, smem, s);
    if (el) return launch_als_batch_t<NN, false, true>(dargs, count, smem, s);
    return launch_als_batch_t<NN, false, false>(dargs, count, smem, s);
}

hipError_t launch_als_batch(const AlsArgs* dargs, const AlsArgs* hargs, int count, hipStream_t s) {
    if (count < 1) return hipSuccess;
    size_t fixed = 0, bmax = 0;
    int N0 = hargs[0].N;
    bool sameN = true;
    for (int i = 0; i < count; ++i) {
        const AlsArgs& a = hargs[i];
        const size_t f = als_lds_fixed(a.N, a.l, a.R);
        fixed = f > fixed ? f : fixed;
        int64_t S = 1;
        for (int n = 0; n < a.N; ++n) S *= a.l[n];
        const size_t b = (size_t)S * sizeof(float);
        bmax = b > bmax ? b : bmax;
        sameN = sameN && a.N == N0;
    }
    const size_t eig = 2 * kEigLd * kEigLd * sizeof(double);
    const bool bl = fixed + bmax <= kAlsLds;
    const bool el = fixed + eig <= kAlsLds;
    size_t big = 0;
    if (bl) big = bmax;
    if (el && eig > big) big = eig;
    const size_t smem = fixed + big;
    if (sameN && N0 == 3) return launch_als_batch_n<3>(dargs, count, bl, el, smem, s);
    if (sameN && N0 == 4) return launch_als_batch_n<4>(dargs, count, bl, el, smem, s);
    return launch_als_batch_n<RCP_MAX_NDIM>(dargs, count, bl, el, smem, s);
}

}  // namespace rcp

