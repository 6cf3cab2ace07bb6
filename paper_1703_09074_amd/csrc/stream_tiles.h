// Streaming contractions over the current tensor T (Algorithm 1: the sketch,
// the power iterations' two products and the projection), hand-written for
// gfx950.
//
// T is C-order with dims (I_0..I_{N-1}); around mode n it is viewed as a
// 3-D array (L, I, Rr): L = prod of dims before n, Rr = prod after n.  The
// mode-n unfolding T_(n) is I x J with column j = a*Rr + b and is never
// materialised.  Its columns are cut into tiles of JT consecutive j that
// stay contiguous in memory:
//   case A (Rr >= JT): a tile is (fixed a, b in [b0, b0+JT)), one run of
//     JT floats per row i;
//   case B (Rr <  JT): a tile is TA whole a-slabs (all b), i.e. one
//     contiguous block of TA*I*Rr floats.
// A workgroup loads a tile (all rows of its row block) into LDS with
// coalesced loads and feeds the matrix cores (v_mfma_f32_16x16x4_f32) from
// there.  The sketch width l is padded to LP (a multiple of 16) with zero
// columns.

//
// This header holds the tile machinery and the kernel templates, shared by
// the float32 instantiations (stream_kernels.hip) and the 16-bit operand
// ones (stream_kernels_lp.hip).  PR selects the matrix-core operand type:
// float32 (v_mfma_f32_16x16x4_f32), or bfloat16 / float16 rounded from the
// float32 tiles in LDS (v_mfma_f32_16x16x16_bf16 / _f16); accumulation is
// float32 in every case.
#pragma once

#include "rcp_device.h"
#include "rcp_kernels.h"

namespace rcp {


constexpr int JT = 32;            // tile width along the unfolding's columns
constexpr int TS = JT + 4;        // LDS row stride of a tile (16-byte aligned rows)
constexpr int NT = 256;           // threads per workgroup of the small kernels
constexpr int NTS = 512;          // threads per workgroup of the streaming kernels (8 wavefronts)
constexpr int NWS = NTS / 64;
// Row-block height (64-row units) of the sketch and stored-Z passes on
// modes taller than 512 rows: 256 rows keep two workgroups resident per CU
// (124 VGPRs, 45 KB of LDS), so one workgroup's barriers, test-matrix
// generation and tile commits overlap the other's matrix-core work; 512-row
// blocks (195 VGPRs, one workgroup per CU) were 8-24% slower on
// 2048x2048x512.
constexpr int kTallMB = 4;

struct TileInfo {
    int64_t j0;      // first unfolding column of the tile
    int64_t a0;      // first a (case A: the a of the tile)
    int64_t b0;      // first b (case A), 0 in case B
    int width;       // number of valid columns (<= JT)
    int na;          // case B: number of a-slabs in the tile
};

__device__ __forceinline__ TileInfo tile_info(const StreamGeom& g, int64_t t) {
    TileInfo ti;
    if (!g.caseB) {
        const int64_t a = t / g.tiles_per_a;
        const int64_t b0 = (t - a * g.tiles_per_a) * JT;
        ti.a0 = a;
        ti.b0 = b0;
        ti.j0 = a * g.Rr + b0;
        const int64_t w = g.Rr - b0;
        ti.width = (int)(w < JT ? w : JT);
        ti.na = 1;
    } else {
        const int64_t a0 = t * g.TA;
        const int64_t left = g.L - a0;
        ti.na = (int)(left < g.TA ? left : g.TA);
        ti.a0 = a0;
        ti.b0 = 0;
        ti.j0 = a0 * g.Rr;
        ti.width = ti.na * (int)g.Rr;
    }
    return ti;
}

// Register staging of one tile (rows [i_lo, i_lo + nrows) of a row block of
// 64*MB rows): MB float4 slots per thread.  Case A slot f = tid + s*NTS
// covers row f / 8, columns 4*(f % 8) .. +3 (one 16-byte load when aligned);
// case B slot covers 4 consecutive floats of the contiguous slab data.
template <int MB>
struct TileRegs {
    float4 v[MB];
};

// Case A (Rr >= JT) staging: row f / 8, columns 4*(f % 8) .. +3 of slot
// f = tid + s*NTS.  Case B tiles (small trailing modes) use load_tile.
template <int MB>
__device__ __forceinline__ void tile_issue(const StreamGeom& g, const TileInfo& ti, int64_t i_lo,
                                           int nrows, TileRegs<MB>& pf) {
    const int tid = threadIdx.x;
    const float* base = g.T + ((ti.a0 * g.Is + i_lo) * g.Rr + ti.b0);
    if (g.vec4 && ti.width == JT) {
        // full, aligned tile: straight-line 16-byte loads; rows past the end
        // read the last valid row and are zeroed afterwards
#pragma unroll
        for (int s = 0; s < MB; ++s) {
            const int f = tid + s * NTS;
            const int r = f >> 3, c0 = (f & 7) * 4;
            const int rr = (r < nrows) ? r : nrows - 1;
            const float4 v = *reinterpret_cast<const float4*>(base + (int64_t)rr * g.Rr + c0);
            pf.v[s] = (r < nrows) ? v : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        return;
    }
#pragma unroll
    for (int s = 0; s < MB; ++s) {
        const int f = tid + s * NTS;
        const int r = f >> 3, c0 = (f & 7) * 4;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r < nrows && c0 < ti.width) {
            const float* p = base + (int64_t)r * g.Rr + c0;
            if (g.vec4 && c0 + 4 <= ti.width) {
                v = *reinterpret_cast<const float4*>(p);
            } else {
                v.x = p[0];
                if (c0 + 1 < ti.width) v.y = p[1];
                if (c0 + 2 < ti.width) v.z = p[2];
                if (c0 + 3 < ti.width) v.w = p[3];
            }
        }
        pf.v[s] = v;
    }
}

// Writes the staged tile into Ts (64*MB rows x JT, stride TS); every cell is
// written (zeros outside the valid rows / columns).  Returns the float64
// sum of squares of the staged values.
template <int MB>
__device__ __forceinline__ double tile_commit(const TileRegs<MB>& pf, float* Ts, bool want_sq) {
    const int tid = threadIdx.x;
    double sq = 0.0;
#pragma unroll
    for (int s = 0; s < MB; ++s) {
        const int f = tid + s * NTS;
        const int r = f >> 3, c0 = (f & 7) * 4;
        *reinterpret_cast<float4*>(Ts + r * TS + c0) = pf.v[s];
        if (want_sq) {
            const float4 v = pf.v[s];
            sq += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
        }
    }
    return sq;
}

// Unstaged load of rows [i_lo, i_lo + nrows) into Ts (rows_alloc x JT),
// zero-filled outside the valid cells; returns the float64 sum of squares.
__device__ __forceinline__ double load_tile(const StreamGeom& g, const TileInfo& ti, int64_t i_lo,
                                            int nrows, int rows_alloc, float* Ts, bool want_sq) {
    const int tid = threadIdx.x;
    double sq = 0.0;
    if (ti.width < JT || nrows < rows_alloc) {
        for (int e = tid; e < rows_alloc * JT; e += NTS) {
            const int r = e / JT, jj = e % JT;
            if (r >= nrows || jj >= ti.width) Ts[r * TS + jj] = 0.0f;
        }
    }
    if (!g.caseB) {
        const float* base = g.T + ((ti.a0 * g.Is + i_lo) * g.Rr + ti.b0);
        const int total = nrows * JT;
        for (int e = tid; e < total; e += NTS) {
            const int r = e / JT, jj = e % JT;
            if (jj < ti.width) {
                const float v = base[(int64_t)r * g.Rr + jj];
                Ts[r * TS + jj] = v;
                if (want_sq) sq += (double)v * v;
            }
        }
    } else {
        const int rr = (int)g.Rr;
        const int slab = nrows * rr;
        const float inv_slab = 1.0f / (float)slab, inv_rr = 1.0f / (float)rr;
        const int total = ti.na * slab;
        for (int e = tid; e < total; e += NTS) {
            const int arel = small_div(e, slab, inv_slab);
            const int rem = e - arel * slab;
            const int r = small_div(rem, rr, inv_rr);
            const int b = rem - r * rr;
            const float v = g.T[((ti.a0 + arel) * g.Is + i_lo) * g.Rr + rem];
            Ts[r * TS + arel * rr + b] = v;
            if (want_sq) sq += (double)v * v;
        }
    }
    return sq;
}

// Y[rows, 0:16*NB] += Ts[rows, 0:JT] * W[0:JT, 0:16*NB] for the row blocks
// this wavefront owns: rb = wave + 8*m, m < MH = ceil(MB/2) (4*MB row blocks
// of 16 rows in all; blocks past the end are skipped).
template <int MB>
struct MHalf { static constexpr int v = (MB + 1) / 2; };

template <int NB, int MB, int PR>
__device__ __forceinline__ void tile_times_w(const float* Ts, const float* W, int ldw,
                                             f32x4 (&acc)[MHalf<MB>::v][NB]) {
    constexpr int MH = MHalf<MB>::v;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    if constexpr (PR != kPrecFp32) {
        // 16-bit operands: lane (lr, lk) feeds k = 4 lk .. 4 lk + 3 of a 16-deep step
#pragma unroll
        for (int k0 = 0; k0 < JT; k0 += 16) {
            s16x4 b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const float* wp = W + (k0 + 4 * lk) * ldw + nb * 16 + lr;
                b[nb] = to_lp<PR>(make_float4(wp[0], wp[ldw], wp[2 * ldw], wp[3 * ldw]));
            }
#pragma unroll
            for (int m = 0; m < MH; ++m) {
                const int rb = wave + NWS * m;
                if (rb < 4 * MB) {
                    const s16x4 a = to_lp<PR>(
                        *reinterpret_cast<const float4*>(Ts + (rb * 16 + lr) * TS + k0 + 4 * lk));
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) acc[m][nb] = mfma_lp<PR>(a, b[nb], acc[m][nb]);
                }
            }
        }
        return;
    }
#pragma unroll
    for (int k0 = 0; k0 < JT; k0 += 4) {
        float b[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) b[nb] = W[(k0 + lk) * ldw + nb * 16 + lr];
#pragma unroll
        for (int m = 0; m < MH; ++m) {
            const int rb = wave + NWS * m;
            if (rb < 4 * MB) {
                const float a = Ts[(rb * 16 + lr) * TS + k0 + lk];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[m][nb] = mfma16x16x4(a, b[nb], acc[m][nb]);
            }
        }
    }
}

// Partial z[jb*16 .. +16, 0:16*NB] = Ts[r, jb-block]^T Qs[r, :] over one
// quarter of the rows: wavefront w takes column block jb = w / 4 and row
// quarter w % 4 (rows is a multiple of 16).
template <int NB, int PR>
__device__ __forceinline__ void tile_t_times_q(const float* Ts, const float* Qs, int ldq,
                                               int rows, f32x4 (&zacc)[NB]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int jb = wave >> 2, quarter = wave & 3;
    const int per = rows / 4;
    const int r_lo = quarter * per, r_hi = r_lo + per;
    if constexpr (PR != kPrecFp32) {
        // per is a multiple of 16 (rows = 64 MB or IC)
        for (int k0 = r_lo; k0 < r_hi; k0 += 16) {
            const float* tp = Ts + (k0 + 4 * lk) * TS + jb * 16 + lr;
            const s16x4 a = to_lp<PR>(make_float4(tp[0], tp[TS], tp[2 * TS], tp[3 * TS]));
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const float* qp = Qs + (k0 + 4 * lk) * ldq + nb * 16 + lr;
                zacc[nb] = mfma_lp<PR>(a, to_lp<PR>(make_float4(qp[0], qp[ldq], qp[2 * ldq], qp[3 * ldq])),
                                       zacc[nb]);
            }
        }
        return;
    }
#pragma unroll 2
    for (int k0 = r_lo; k0 < r_hi; k0 += 4) {
        const float a = Ts[(k0 + lk) * TS + jb * 16 + lr];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
            zacc[nb] = mfma16x16x4(a, Qs[(k0 + lk) * ldq + nb * 16 + lr], zacc[nb]);
    }
}

// Store the wavefronts' partial z into zp[quarter][jj][c] and sum into zs.
template <int NB>
__device__ __forceinline__ void reduce_z(const f32x4 (&zacc)[NB], float* zp, float* zs) {
    constexpr int LPc = NB * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int jb = wave >> 2, quarter = wave & 3;
    float* my = zp + quarter * JT * LPc;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            my[(jb * 16 + 4 * lk + v) * LPc + nb * 16 + lr] = zacc[nb][v];
    __syncthreads();
    for (int e = threadIdx.x; e < JT * LPc; e += NTS)
        zs[e] = zp[e] + zp[JT * LPc + e] + zp[2 * JT * LPc + e] + zp[3 * JT * LPc + e];
    __syncthreads();
}

template <int NB, int MB>
__device__ __forceinline__ void store_partial(const f32x4 (&acc)[MHalf<MB>::v][NB], float* part,
                                              int64_t I, int64_t row0) {
    constexpr int LPc = NB * 16;
    constexpr int MH = MHalf<MB>::v;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int m = 0; m < MH; ++m) {
        const int rb = wave + NWS * m;
        if (rb < 4 * MB) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = row0 + rb * 16 + 4 * lk + v;
                if (row < I) {
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) part[row * LPc + nb * 16 + lr] = acc[m][nb][v];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// contract_out: partial Y = T_(n) W over the tiles of this workgroup, for
// the row block blockIdx.y (64*MB rows).  W (J x LP) is never stored whole;
// per tile its JT rows are
//   WK = kWStored: read from a stored matrix in the layout (L, LP, Rr)
//                  (power iteration with a stored Z),
//   WK = kWOmega:  the Gaussian test matrix, generated in registers,
//   WK = kWKr:     the Khatri-Rao product of the other modes' factors (the
//                  mode product of CP-ALS, Algorithm 2's factor updates), formed
//                  from a packed copy of the factors in LDS,
//   WK = kWKrG:    the same product with the factor rows read from global
//                  memory (through the caches): the full tensor's factors,
//                  too large for LDS.
// Optional float64 partial sum of squares of T (used for ||X||^2 in the
// first pass).

constexpr int kWStored = 0;
constexpr int kWOmega = 1;
constexpr int kWKr = 2;
constexpr int kWKrG = 3;

__device__ __forceinline__ uint32_t fast_udiv(uint32_t x, uint32_t mul, uint32_t shr) {
    return (uint32_t)(((uint64_t)__umulhi(x, mul) + x) >> shr);
}

// Khatri-Rao entry (column c) for the unfolding column with outer index a
// (modes before n) and inner index b (modes after n): digits come out
// least significant first, i.e. from the last mode down.
__device__ __forceinline__ float kr_entry(const KrSpec& kr, const float* Fs, uint32_t a, uint32_t b,
                                          int c) {
    float p = 1.0f;
#pragma unroll
    for (int m = RCP_MAX_NDIM - 1; m >= 0; --m) {
        if (m < kr.N && m != kr.n) {
            const bool inner = m > kr.n;
            const uint32_t x = inner ? b : a;
            const uint32_t q = fast_udiv(x, kr.mul[m], kr.shr[m]);
            const uint32_t d = x - q * (uint32_t)kr.l[m];
            if (inner) b = q; else a = q;
            p *= Fs[kr.foff[m] + (int)d * kr.R + c];
        }
    }
    return p;
}

__device__ __forceinline__ float kr_entry_global(const KrSpec& kr, uint32_t a, uint32_t b, int c) {
    float p = 1.0f;
#pragma unroll
    for (int m = RCP_MAX_NDIM - 1; m >= 0; --m) {
        if (m < kr.N && m != kr.n) {
            const bool inner = m > kr.n;
            const uint32_t x = inner ? b : a;
            const uint32_t q = fast_udiv(x, kr.mul[m], kr.shr[m]);
            const uint32_t d = x - q * (uint32_t)kr.l[m];
            if (inner) b = q; else a = q;
            p *= kr.fac[m][(size_t)d * kr.R + c];
        }
    }
    return p;
}

// The body takes its workgroup's position (bx of nbx along the tiles, row
// block by) as arguments, so that a grouped launch can run it for many
// problems at once.
template <int NB, int MB, int WK, bool CB, int PR>
__device__ __forceinline__ void contract_out_body(const StreamGeom& g, int l, const float* Z,
                                                  uint64_t seed, uint32_t tag, int okind,
                                                  float* part, double* sq_part, const KrSpec& kr,
                                                  int bx, int nbx, int by) {
    constexpr int LPc = NB * 16;
    constexpr int IB = 64 * MB;
    extern __shared__ __align__(16) float smem[];
    float* Ts = smem;                       // IB x TS
    float* Ws = Ts + IB * TS;               // JT x LPc
    float* Fs = Ws + JT * LPc;              // kWKr: the packed factors
    __shared__ double red[NWS];

    if (WK == kWKr || WK == kWKrG) {
        if (kr.skip != nullptr && *kr.skip != 0 && kr.sweep > *kr.skip) return;
    }
    if (WK == kWKr) {
        // l_m * R <= 4096 floats per factor: a thread's loads of one factor
        // are issued together (one memory latency per factor)
        constexpr int KF = (RCP_MAX_L * RCP_MAX_RANK + NTS - 1) / NTS;
#pragma unroll
        for (int m = 0; m < RCP_MAX_NDIM; ++m) {
            if (m < kr.N && m != kr.n) {
                const int cnt = kr.l[m] * kr.R;
                float f[KF];
#pragma unroll
                for (int k = 0; k < KF; ++k) {
                    const int e = threadIdx.x + k * NTS;
                    f[k] = (e < cnt) ? kr.fac[m][e] : 0.0f;
                }
#pragma unroll
                for (int k = 0; k < KF; ++k) {
                    const int e = threadIdx.x + k * NTS;
                    if (e < cnt) Fs[kr.foff[m] + e] = f[k];
                }
            }
        }
    }

    const int64_t row0 = (int64_t)by * IB;
    const int64_t rows_left = g.I - row0;
    const int nrows = (int)(rows_left < IB ? rows_left : IB);

    f32x4 acc[MHalf<MB>::v][NB];
#pragma unroll
    for (int m = 0; m < MHalf<MB>::v; ++m)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[m][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

    double sq = 0.0;
    const bool want_sq = sq_part != nullptr;
    TileRegs<MB> pf;
    int64_t t = bx;
    if (!CB && t < g.ntiles) tile_issue<MB>(g, tile_info(g, t), row0, nrows, pf);
    for (; t < g.ntiles; t += nbx) {
        const TileInfo ti = tile_info(g, t);
        __syncthreads();
        if (CB) sq += load_tile(g, ti, row0, nrows, IB, Ts, want_sq);
        else sq += tile_commit<MB>(pf, Ts, want_sq);
        if (WK == kWKr || WK == kWKrG) {
            const float inv_rr = 1.0f / (float)g.Rr;
            for (int e = threadIdx.x; e < JT * LPc; e += NTS) {
                const int jj = e / LPc, c = e % LPc;
                float v = 0.0f;
                if (jj < ti.width && c < kr.R) {
                    uint32_t a, b;
                    if (!g.caseB) {
                        a = (uint32_t)ti.a0;
                        b = (uint32_t)(ti.b0 + jj);
                    } else {
                        const int q = small_div(jj, (int)g.Rr, inv_rr);
                        a = (uint32_t)(ti.a0 + q);
                        b = (uint32_t)(jj - q * (int)g.Rr);
                    }
                    v = (WK == kWKr) ? kr_entry(kr, Fs, a, b, c) : kr_entry_global(kr, a, b, c);
                }
                Ws[jj * LPc + c] = v;
            }
        } else if (WK == kWOmega) {
            constexpr int NG = LPc / 4;
            for (int e = threadIdx.x; e < JT * NG; e += NTS) {
                const int jj = e / NG, gi = e % NG;
                float z[4] = {0.f, 0.f, 0.f, 0.f};
                if (jj < ti.width) omega4k(okind, seed, tag, (uint64_t)(ti.j0 + jj), (uint32_t)gi, z);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = 4 * gi + v;
                    Ws[jj * LPc + c] = (c < l) ? z[v] : 0.0f;
                }
            }
        } else if (!g.caseB && g.vec4 && ti.width == JT) {
            // full, aligned tile: 16-byte loads of four consecutive rows j
            for (int e = threadIdx.x; e < (JT / 4) * LPc; e += NTS) {
                const int j4 = (e % (JT / 4)) * 4, c = e / (JT / 4);
                const float4 v = *reinterpret_cast<const float4*>(
                    Z + (ti.a0 * LPc + c) * g.Rr + ti.b0 + j4);
                Ws[(j4 + 0) * LPc + c] = v.x;
                Ws[(j4 + 1) * LPc + c] = v.y;
                Ws[(j4 + 2) * LPc + c] = v.z;
                Ws[(j4 + 3) * LPc + c] = v.w;
            }
        } else {
            for (int e = threadIdx.x; e < JT * LPc; e += NTS) {
                const int jj = e % JT, c = e / JT;
                float v = 0.0f;
                if (jj < ti.width) {
                    int64_t a, b;
                    if (!g.caseB) { a = ti.a0; b = ti.b0 + jj; }
                    else { a = ti.a0 + jj / g.Rr; b = jj % g.Rr; }
                    v = Z[(a * LPc + c) * g.Rr + b];
                }
                Ws[jj * LPc + c] = v;
            }
        }
        const int64_t tn = t + nbx;
        if (!CB && tn < g.ntiles) tile_issue<MB>(g, tile_info(g, tn), row0, nrows, pf);
        __syncthreads();
        tile_times_w<NB, MB, PR>(Ts, Ws, LPc, acc);
    }
    store_partial<NB, MB>(acc, part + (int64_t)bx * g.I * LPc, g.I, row0);
    if (want_sq) {
        const double s = block_sum(sq, red);
        if (threadIdx.x == 0) sq_part[(int64_t)by * nbx + bx] = s;
    }
}

template <int NB, int MB, int WK, bool CB, int PR>
__global__ __launch_bounds__(NTS) void k_contract_out(StreamGeom g, int l, const float* Z,
                                                     uint64_t seed, uint32_t tag, int okind,
                                                     float* part, double* sq_part, KrSpec kr) {
    contract_out_body<NB, MB, WK, CB, PR>(g, l, Z, seed, tag, okind, part, sq_part, kr,
                                          (int)blockIdx.x, (int)gridDim.x, (int)blockIdx.y);
}

// ---------------------------------------------------------------------------
// power_fused: partial Y = T_(n) (T_(n)^T Qt) in one pass over T.  Each tile
// (all I rows, I <= 64*MB) is held in LDS: first z = tile^T Qt (JT x LP),
// then Y += tile z.  The normalisation of Z in Algorithm 1's power iteration is an
// invertible upper-triangular right factor, which the QR of the next sketch
// absorbs, so it is not applied.

template <int NB, int MB, bool FUSED, bool CB, int PR>
__device__ __forceinline__ void power_fused_body(const StreamGeom& g, const float* Qt, float* part,
                                                 int lout, float* out, int accumulate, int bx,
                                                 int nbx) {
    constexpr int LPc = NB * 16;
    constexpr int IB = 64 * MB;
    extern __shared__ __align__(16) float smem[];
    float* Ts = smem;                       // IB x TS
    float* Qs = Ts + IB * TS;               // IB x LPc
    float* zp = Qs + IB * LPc;              // 4 x JT x LPc
    float* zs = zp + 4 * JT * LPc;          // JT x LPc

    const int I = (int)g.I;
    for (int e = threadIdx.x; e < IB * LPc; e += NTS) {
        const int r = e / LPc;
        Qs[e] = (r < I) ? Qt[e] : 0.0f;
    }

    f32x4 acc[MHalf<MB>::v][NB];
#pragma unroll
    for (int m = 0; m < MHalf<MB>::v; ++m)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[m][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

    TileRegs<MB> pf;
    int64_t t = bx;
    if (!CB && t < g.ntiles) tile_issue<MB>(g, tile_info(g, t), 0, I, pf);
    for (; t < g.ntiles; t += nbx) {
        const TileInfo ti = tile_info(g, t);
        __syncthreads();
        if (CB) load_tile(g, ti, 0, I, IB, Ts, false);
        else tile_commit<MB>(pf, Ts, false);
        const int64_t tn = t + nbx;
        if (!CB && tn < g.ntiles) tile_issue<MB>(g, tile_info(g, tn), 0, I, pf);
        __syncthreads();
        f32x4 zacc[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) zacc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
        tile_t_times_q<NB, PR>(Ts, Qs, LPc, IB, zacc);
        reduce_z<NB>(zacc, zp, zs);
        if (FUSED) {
            tile_times_w<NB, MB, PR>(Ts, zs, LPc, acc);
        } else {
            // mode product: write z^T into the (L, lout, Rr) output
            for (int e = threadIdx.x; e < lout * JT; e += NTS) {
                const int c = e / JT, jj = e % JT;
                if (jj < ti.width) {
                    int64_t a, b;
                    if (!g.caseB) { a = ti.a0; b = ti.b0 + jj; }
                    else { a = ti.a0 + jj / g.Rr; b = jj % g.Rr; }
                    float* o = out + (a * lout + c) * g.Rr + b;
                    *o = accumulate ? *o + zs[jj * LPc + c] : zs[jj * LPc + c];
                }
            }
        }
    }
    if (FUSED) store_partial<NB, MB>(acc, part + (int64_t)bx * g.I * LPc, g.I, 0);
}

template <int NB, int MB, bool FUSED, bool CB, int PR>
__global__ __launch_bounds__(NTS) void k_power_fused(StreamGeom g, const float* Qt, float* part,
                                                    int lout, float* out, int accumulate) {
    power_fused_body<NB, MB, FUSED, CB, PR>(g, Qt, part, lout, out, accumulate, (int)blockIdx.x,
                                            (int)gridDim.x);
}

// ---------------------------------------------------------------------------
// Grouped forms: blockIdx.z picks the problem.

template <int NB, int MB, int WK, bool CB, int PR>
__global__ __launch_bounds__(NTS) void k_contract_out_grp(const SketchDesc* d) {
    const SketchDesc& D = d[blockIdx.z];
    if ((int)blockIdx.x >= D.P || (int)blockIdx.y >= D.nIB) return;
    contract_out_body<NB, MB, WK, CB, PR>(D.g, D.l, D.Z, D.seed, D.tag, D.okind, D.part, D.sq_part,
                                          KrSpec{}, (int)blockIdx.x, D.P, (int)blockIdx.y);
}

template <int NB, int MB, bool FUSED, bool CB, int PR>
__global__ __launch_bounds__(NTS) void k_power_fused_grp(const PowerDesc* d) {
    const PowerDesc& D = d[blockIdx.z];
    if ((int)blockIdx.x >= D.P) return;
    power_fused_body<NB, MB, FUSED, CB, PR>(D.g, D.Qt, D.part, D.lout, D.out, D.accumulate,
                                            (int)blockIdx.x, D.P);
}

// ---------------------------------------------------------------------------
// contract_in: out[a, c, b] = sum_i Q[i, c] T[a, i, b] for c < lout
// (Algorithm 1's projection, T x_n Q^T; also Z = T_(n)^T Qt for the two-pass
// power iteration).  Rows are streamed in chunks of IC through LDS.

constexpr int IC = 128;

template <int NB, int PR>
__global__ __launch_bounds__(NTS) void k_contract_in(StreamGeom g, const float* Q, int lout,
                                                    float* out) {
    constexpr int LPc = NB * 16;
    extern __shared__ float smem[];
    float* Ts = smem;                       // IC x TS
    float* Qs = Ts + IC * TS;               // IC x LPc
    float* zp = Qs + IC * LPc;              // 4 x JT x LPc
    float* zs = zp + 4 * JT * LPc;          // JT x LPc

    for (int64_t t = blockIdx.x; t < g.ntiles; t += gridDim.x) {
        const TileInfo ti = tile_info(g, t);
        f32x4 zacc[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) zacc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int64_t i_lo = 0; i_lo < g.I; i_lo += IC) {
            const int64_t left = g.I - i_lo;
            const int nrows = (int)(left < IC ? left : IC);
            __syncthreads();
            load_tile(g, ti, i_lo, nrows, IC, Ts, false);
            for (int e = threadIdx.x; e < IC * LPc; e += NTS) {
                const int r = e / LPc;
                Qs[e] = (r < nrows) ? Q[(i_lo + r) * LPc + (e - r * LPc)] : 0.0f;
            }
            __syncthreads();
            tile_t_times_q<NB, PR>(Ts, Qs, LPc, IC, zacc);
        }
        reduce_z<NB>(zacc, zp, zs);
        // write z^T into the (L, lout, Rr) output
        for (int e = threadIdx.x; e < lout * JT; e += NTS) {
            const int c = e / JT, jj = e % JT;
            if (jj < ti.width) {
                int64_t a, b;
                if (!g.caseB) { a = ti.a0; b = ti.b0 + jj; }
                else { a = ti.a0 + jj / g.Rr; b = jj % g.Rr; }
                out[(a * lout + c) * g.Rr + b] = zs[jj * LPc + c];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// contract_in for tall modes (case A only): out[a, c, b] = sum_i Q[i, c]
// T[a, i, b] with every row i streamed.  A workgroup owns groups of CW
// consecutive columns (8 tiles, 1 KB runs per row) and walks their rows in
// chunks of RC through a double-buffered LDS pipeline: while the matrix cores
// consume chunk s, chunk s+1 is committed from registers into the other
// buffer and chunk s+2 is in flight from HBM; one barrier per chunk.  The
// (group, chunk) steps of a workgroup form one sequence, so the pipeline does
// not drain between groups.  Each group's z^T (LP x CW) stays in the
// accumulators and is written once: no partial outputs, no read-modify-write.
// Wavefront w owns column blocks 2w, 2w+1 and all LP/16 blocks of c.

constexpr int CW = 256;           // columns per group
constexpr int RC = 32;            // rows per chunk
constexpr int TSW = CW + 16;      // LDS row stride of a T chunk

template <int NB, int PR>
__global__ __launch_bounds__(NTS) void k_contract_in_tall(StreamGeom g, const float* Q, int lout,
                                                         float* out) {
    constexpr int LPc = NB * 16;
    constexpr int LQ = LPc + 16;            // LDS row stride of a Q chunk
    constexpr int TF4 = RC * CW / 4 / NTS;  // float4 of a T chunk per thread
    constexpr int QF4 = RC * LPc / 4;       // float4 of a Q chunk
    static_assert(RC * CW / 4 == TF4 * NTS, "T chunk split");
    static_assert(QF4 <= NTS, "Q chunk split");
    extern __shared__ __align__(16) float smem[];
    float* Tb = smem;                       // [2][RC][TSW]
    float* Qb = Tb + 2 * RC * TSW;          // [2][RC][LQ]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t gpa = (g.Rr + CW - 1) / CW;
    const int64_t ngroups = g.L * gpa;
    const int64_t I = g.I;
    const int nch = (int)((I + RC - 1) / RC);
    if ((int64_t)blockIdx.x >= ngroups) return;
    const int64_t my_groups = (ngroups - blockIdx.x + gridDim.x - 1) / gridDim.x;
    const int64_t nsteps = my_groups * nch;

    float4 tr[TF4];
    float4 qr = make_float4(0.f, 0.f, 0.f, 0.f);
    auto issue = [&](int64_t st) {
        const int64_t grp = blockIdx.x + (st / nch) * gridDim.x;
        const int64_t i0 = (st % nch) * RC;
        const int64_t a = grp / gpa;
        const int64_t b0 = (grp - a * gpa) * CW;
        const int64_t wl = g.Rr - b0;
        const int width = (int)(wl < CW ? wl : CW);
        const int64_t rl = I - i0;
        const int rows = (int)(rl < RC ? rl : RC);
        const float* base = g.T + ((a * g.Is + i0) * g.Rr + b0);
#pragma unroll
        for (int s2 = 0; s2 < TF4; ++s2) {
            const int f = tid + s2 * NTS;
            const int r = f / (CW / 4), c0 = (f % (CW / 4)) * 4;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < rows && c0 < width) {
                const float* p = base + (int64_t)r * g.Rr + c0;
                if (g.vec4 && c0 + 4 <= width) {
                    v = *reinterpret_cast<const float4*>(p);
                } else {
                    v.x = p[0];
                    if (c0 + 1 < width) v.y = p[1];
                    if (c0 + 2 < width) v.z = p[2];
                    if (c0 + 3 < width) v.w = p[3];
                }
            }
            tr[s2] = v;
        }
        if (tid < QF4) {
            const int r = tid / (LPc / 4), c0 = (tid % (LPc / 4)) * 4;
            qr = (i0 + r < I) ? *reinterpret_cast<const float4*>(Q + (i0 + r) * LPc + c0)
                              : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto commit = [&](int buf) {
        float* tb = Tb + buf * RC * TSW;
#pragma unroll
        for (int s2 = 0; s2 < TF4; ++s2) {
            const int f = tid + s2 * NTS;
            const int r = f / (CW / 4), c0 = (f % (CW / 4)) * 4;
            *reinterpret_cast<float4*>(tb + r * TSW + c0) = tr[s2];
        }
        if (tid < QF4) {
            const int r = tid / (LPc / 4), c0 = (tid % (LPc / 4)) * 4;
            *reinterpret_cast<float4*>(Qb + buf * RC * LQ + r * LQ + c0) = qr;
        }
    };

    f32x4 acc[2][NB];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[jb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

    issue(0);
    commit(0);
    if (nsteps > 1) issue(1);
    __syncthreads();
    for (int64_t st = 0; st < nsteps; ++st) {
        const int buf = (int)(st & 1);
        const float* tb = Tb + buf * RC * TSW + (2 * wave) * 16 + lr;
        const float* qb = Qb + buf * RC * LQ + lr;
        if constexpr (PR != kPrecFp32) {
#pragma unroll
            for (int k0 = 0; k0 < RC; k0 += 16) {
                const int kr = k0 + 4 * lk;
                s16x4 bt[2];
#pragma unroll
                for (int jb = 0; jb < 2; ++jb) {
                    const float* tp = tb + kr * TSW + jb * 16;
                    bt[jb] = to_lp<PR>(make_float4(tp[0], tp[TSW], tp[2 * TSW], tp[3 * TSW]));
                }
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const float* qp = qb + kr * LQ + nb * 16;
                    const s16x4 aq = to_lp<PR>(make_float4(qp[0], qp[LQ], qp[2 * LQ], qp[3 * LQ]));
#pragma unroll
                    for (int jb = 0; jb < 2; ++jb) acc[jb][nb] = mfma_lp<PR>(aq, bt[jb], acc[jb][nb]);
                }
            }
        } else {
#pragma unroll
            for (int k0 = 0; k0 < RC; k0 += 4) {
                const int kr = k0 + lk;
                const float b0v = tb[kr * TSW], b1v = tb[kr * TSW + 16];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const float aq = qb[kr * LQ + nb * 16];
                    acc[0][nb] = mfma16x16x4(aq, b0v, acc[0][nb]);
                    acc[1][nb] = mfma16x16x4(aq, b1v, acc[1][nb]);
                }
            }
        }
        if (st + 1 < nsteps) commit(buf ^ 1);
        if (st + 2 < nsteps) issue(st + 2);
        if ((int)(st % nch) == nch - 1) {
            // the group is complete: z^T[c, j] -> out[a, c, b0 + j]
            const int64_t grp = blockIdx.x + (st / nch) * gridDim.x;
            const int64_t a = grp / gpa;
            const int64_t b0 = (grp - a * gpa) * CW;
            const int64_t wl = g.Rr - b0;
            const int width = (int)(wl < CW ? wl : CW);
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) {
                const int j = (2 * wave + jb) * 16 + lr;
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int c = nb * 16 + 4 * lk + v;
                        if (c < lout && j < width) out[(a * lout + c) * g.Rr + b0 + j] = acc[jb][nb][v];
                    }
                    acc[jb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
            }
        }
        __syncthreads();
    }
}

inline size_t contract_in_tall_smem(int NB) {
    return (size_t)(2 * RC * TSW + 2 * RC * (NB * 16 + 16)) * sizeof(float);
}

inline int lp_blocks(int l) { return (l + 15) / 16; }

inline size_t contract_out_smem(int NB, int MB) {
    return (size_t)(64 * MB * TS + JT * NB * 16) * sizeof(float);
}

inline size_t power_fused_smem(int NB, int MB) {
    const int IB = 64 * MB, LPc = NB * 16;
    return (size_t)(IB * TS + IB * LPc + 4 * JT * LPc + JT * LPc) * sizeof(float);
}

inline size_t contract_in_smem(int NB) {
    const int LPc = NB * 16;
    return (size_t)(IC * TS + IC * LPc + 4 * JT * LPc + JT * LPc) * sizeof(float);
}

template <int NB, int MB, int WK, int PR>
static hipError_t launch_co(dim3 grid, size_t smem, hipStream_t s, const StreamGeom& g, int l,
                            const float* Z, uint64_t seed, uint32_t tag, int okind, float* part,
                            double* sq, const KrSpec& kr = KrSpec{}) {
    auto k = g.caseB ? k_contract_out<NB, MB, WK, true, PR> : k_contract_out<NB, MB, WK, false, PR>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, grid, dim3(NTS), smem, s, g, l, Z, seed, tag, okind, part, sq, kr);
    return hipGetLastError();
}

#define RCP_MB_SWITCH(MBV, ...)                                   \
    switch (MBV) {                                                \
        case 1: { constexpr int MB = 1; __VA_ARGS__; } break;     \
        case 2: { constexpr int MB = 2; __VA_ARGS__; } break;     \
        case 3: { constexpr int MB = 3; __VA_ARGS__; } break;     \
        case 4: { constexpr int MB = 4; __VA_ARGS__; } break;     \
        case 5: { constexpr int MB = 5; __VA_ARGS__; } break;     \
        case 6: { constexpr int MB = 6; __VA_ARGS__; } break;     \
        case 7: { constexpr int MB = 7; __VA_ARGS__; } break;     \
        default: { constexpr int MB = 8; __VA_ARGS__; } break;    \
    }

#define RCP_NB_SWITCH(NBV, ...)                                   \
    switch (NBV) {                                                \
        case 1: { constexpr int NB = 1; __VA_ARGS__; } break;     \
        case 2: { constexpr int NB = 2; __VA_ARGS__; } break;     \
        case 3: { constexpr int NB = 3; __VA_ARGS__; } break;     \
        default: { constexpr int NB = 4; __VA_ARGS__; } break;    \
    }

template <int PR>
hipError_t launch_contract_out_t(const StreamGeom& g, int l, const float* Z, uint64_t seed,
                                 uint32_t tag, int okind, float* part, int P, double* sq_part,
                                 hipStream_t s, int mb_cap) {
    const int NBv = lp_blocks(l);
    int MBv = (int)((g.I + 63) / 64);
    if (g.I <= 512 && MBv > mb_cap) MBv = mb_cap;    // the cap applies to short modes only
    if (g.I > 512) MBv = kTallMB;
    if (MBv < 1) MBv = 1;
    const int IB = 64 * MBv;
    const unsigned nIB = (unsigned)((g.I + IB - 1) / IB);
    const size_t smem = contract_out_smem(NBv, MBv);
    const dim3 grid((unsigned)P, nIB);
    hipError_t e = hipSuccess;
    if (Z == nullptr) {
        RCP_NB_SWITCH(NBv, RCP_MB_SWITCH(MBv, e = (launch_co<NB, MB, kWOmega, PR>(grid, smem, s, g, l, Z, seed, tag, okind, part, sq_part))));
    } else {
        RCP_NB_SWITCH(NBv, RCP_MB_SWITCH(MBv, e = (launch_co<NB, MB, kWStored, PR>(grid, smem, s, g, l, Z, seed, tag, okind, part, sq_part))));
    }
    return e;
}

template <int NB, int MB, bool FUSED, int PR>
static hipError_t launch_pf(int P, size_t smem, hipStream_t s, const StreamGeom& g,
                            const float* Qt, float* part, int lout, float* out,
                            int accumulate = 0) {
    auto k = g.caseB ? k_power_fused<NB, MB, FUSED, true, PR> : k_power_fused<NB, MB, FUSED, false, PR>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)P), dim3(NTS), smem, s, g, Qt, part, lout, out, accumulate);
    return hipGetLastError();
}

template <int PR>
hipError_t launch_power_fused_t(const StreamGeom& g, int l, const float* Qt, float* part, int P,
                                hipStream_t s) {
    const int NBv = lp_blocks(l);
    const int MBv = (int)((g.I + 63) / 64);
    const size_t smem = power_fused_smem(NBv, MBv);
    hipError_t e = hipSuccess;
    RCP_NB_SWITCH(NBv, RCP_MB_SWITCH(MBv, e = (launch_pf<NB, MB, true, PR>(P, smem, s, g, Qt, part, 0, nullptr))));
    return e;
}

template <int NB, int PR>
static hipError_t launch_ci(int P, size_t smem, hipStream_t s, const StreamGeom& g,
                            const float* Q, int lout, float* out) {
    auto k = k_contract_in<NB, PR>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)P), dim3(NTS), smem, s, g, Q, lout, out);
    return hipGetLastError();
}

// T x_n Q^T (or Z = T_(n)^T Q): the whole basis resident in LDS when the
// mode is short enough, else streamed in row chunks.
template <int PR>
hipError_t launch_contract_in_t(const StreamGeom& g, int l, const float* Qpadded, int lout,
                                float* out, int P, hipStream_t s) {
    const int NBv = lp_blocks(l);
    hipError_t e = hipSuccess;
    if (power_fused_fits(g.I, l, 160 * 1024)) {
        const int MBv = (int)((g.I + 63) / 64);
        const size_t smem = power_fused_smem(NBv, MBv);
        RCP_NB_SWITCH(NBv, RCP_MB_SWITCH(MBv, e = (launch_pf<NB, MB, false, PR>(P, smem, s, g, Qpadded, nullptr, lout, out))));
        return e;
    }
    // Taller modes with runs of at least one tile per row: every row streamed
    // through the double-buffered pipeline, the output written once.
    if (!g.caseB) {
        const int64_t ngroups = g.L * ((g.Rr + CW - 1) / CW);
        const int P2 = (int)(ngroups < P ? ngroups : P);
        const size_t smem = contract_in_tall_smem(NBv);
        RCP_NB_SWITCH(NBv, {
            auto k = k_contract_in_tall<NB, PR>;
            e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)smem);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k, dim3((unsigned)P2), dim3(NTS), smem, s, g, Qpadded, lout, out);
                e = hipGetLastError();
            }
        });
        return e;
    }
    // Otherwise (short a-slabs): slices of the rows whose basis rows fit in
    // LDS, each a resident-basis pass over its rows that adds its share of
    // T^T Q into the output (in slice order, so the sums are deterministic).
    int MBs = 8;
    while (MBs > 1 && power_fused_smem(NBv, MBs) > 160 * 1024) --MBs;
    if (power_fused_smem(NBv, MBs) <= 160 * 1024) {
        const int64_t Ir = 64 * MBs;
        for (int64_t i0 = 0; i0 < g.I; i0 += Ir) {
            StreamGeom g2 = g;
            g2.T = g.T + i0 * g.Rr;
            g2.I = (g.I - i0 < Ir) ? g.I - i0 : Ir;
            const int MBv = (int)((g2.I + 63) / 64);
            const size_t smem = power_fused_smem(NBv, MBv);
            const float* Qs = Qpadded + i0 * (int64_t)(16 * NBv);
            const int acc = i0 > 0 ? 1 : 0;
            RCP_NB_SWITCH(NBv, RCP_MB_SWITCH(MBv, e = (launch_pf<NB, MB, false, PR>(P, smem, s, g2, Qs, nullptr, lout, out, acc))));
            if (e != hipSuccess) return e;
        }
        return e;
    }
    const size_t smem = contract_in_smem(NBv);
    RCP_NB_SWITCH(NBv, e = (launch_ci<NB, PR>(P, smem, s, g, Qpadded, lout, out)));
    return e;
}


template <int PR>
hipError_t launch_sketch_group_t(const SketchDesc* d, int count, int gx, int gy, int NBv, int MBv,
                                 bool caseB, bool stored, hipStream_t s) {
    if (count < 1) return hipSuccess;
    const size_t smem = contract_out_smem(NBv, MBv);
    const dim3 grid((unsigned)gx, (unsigned)gy, (unsigned)count);
    hipError_t e = hipSuccess;
    RCP_NB_SWITCH(NBv, RCP_MB_SWITCH(MBv, {
        auto k = stored ? (caseB ? k_contract_out_grp<NB, MB, kWStored, true, PR>
                                 : k_contract_out_grp<NB, MB, kWStored, false, PR>)
                        : (caseB ? k_contract_out_grp<NB, MB, kWOmega, true, PR>
                                 : k_contract_out_grp<NB, MB, kWOmega, false, PR>);
        e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)smem);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k, grid, dim3(NTS), smem, s, d);
            e = hipGetLastError();
        }
    }));
    return e;
}

template <int PR>
hipError_t launch_power_group_t(const PowerDesc* d, int count, int gx, int NBv, int MBv,
                                bool fused, bool caseB, hipStream_t s) {
    if (count < 1) return hipSuccess;
    const size_t smem = power_fused_smem(NBv, MBv);
    const dim3 grid((unsigned)gx, 1, (unsigned)count);
    hipError_t e = hipSuccess;
    RCP_NB_SWITCH(NBv, RCP_MB_SWITCH(MBv, {
        auto k = fused ? (caseB ? k_power_fused_grp<NB, MB, true, true, PR>
                                : k_power_fused_grp<NB, MB, true, false, PR>)
                       : (caseB ? k_power_fused_grp<NB, MB, false, true, PR>
                                : k_power_fused_grp<NB, MB, false, false, PR>);
        e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)smem);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k, grid, dim3(NTS), smem, s, d);
            e = hipGetLastError();
        }
    }));
    return e;
}

}  // namespace rcp
