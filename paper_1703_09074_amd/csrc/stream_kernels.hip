// Streaming contractions: the float32 instantiations, the public launchers
// (which dispatch 16-bit operand precisions to stream_kernels_lp.hip) and
// the small kernels around them (partial-sum reduction, sum of squares,
// test-matrix dump, basis padding).

#include "stream_tiles.h"

namespace rcp {

// ---------------------------------------------------------------------------
// Deterministic reduction of the per-workgroup partials in one launch.  The
// partials are cut into ny = min(P, 16) consecutive groups; a workgroup
// takes 64 consecutive elements, wavefront y sums group y's partials of its
// element in partial order (float64, from 0), and the group sums are added
// in group order:  Y[e] = sum_y (sum_{p in group y} part[p, e]).
// Workgroup 0 of a reduction also sums the optional sum-of-squares partials.

constexpr int kRedSplit = 16;
constexpr int kRedCols = 64;                  // elements per workgroup
constexpr int kRedThreads = 64 * kRedSplit;   // one wavefront per group

__device__ __forceinline__ void reduce_body(const float* part, int P, int ny, int64_t count,
                                            int64_t blk, double* Y, const double* sq_part, int nsq,
                                            double* sq_out) {
    __shared__ double gs[kRedSplit][kRedCols];
    const int c = threadIdx.x & 63, y = threadIdx.x >> 6;
    const int64_t e = blk * kRedCols + c;
    double s = 0.0;
    if (y < ny && e < count) {
        const int p0 = (int)((int64_t)P * y / ny), p1 = (int)((int64_t)P * (y + 1) / ny);
        const float* src = part + e;
#pragma unroll 8
        for (int p = p0; p < p1; ++p) s += (double)src[(int64_t)p * count];
    }
    gs[y][c] = s;
    __syncthreads();
    if (y == 0 && e < count) {
        double t = 0.0;
        for (int g = 0; g < ny; ++g) t += gs[g][c];
        Y[e] = t;
    }
    if (sq_part != nullptr && blk == 0 && threadIdx.x == 0) {
        double t = 0.0;
        for (int p = 0; p < nsq; ++p) t += sq_part[p];
        *sq_out = t;
    }
}

__global__ __launch_bounds__(kRedThreads) void k_reduce(const float* part, int P, int64_t count,
                                                        double* Y, const double* sq_part, int nsq,
                                                        double* sq_out) {
    reduce_body(part, P, P < kRedSplit ? P : kRedSplit, count, blockIdx.x, Y, sq_part, nsq, sq_out);
}

// Grouped form: the problems' workgroups are numbered consecutively
// (d[i].blk0 is problem i's first), so the grid holds only real work; a
// workgroup finds its problem by binary search over blk0.
__global__ __launch_bounds__(kRedThreads) void k_reduce_grp(const ReduceDesc* d, int count) {
    const int bx = (int)blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].blk0 <= bx) lo = mid;
        else hi = mid - 1;
    }
    const ReduceDesc& D = d[lo];
    reduce_body(D.part, D.P, D.ny, D.count, bx - D.blk0, D.Y, D.sq_part, D.nsq, D.sq_out);
}

// Sum of squares of count floats: per-block float64 partials.
__global__ __launch_bounds__(NT) void k_sumsq(const float* x, int64_t count, double* part) {
    __shared__ double red[NT / 64];
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * NT) {
        const double v = x[e];
        s += v * v;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_sum_doubles(const double* part, int n, double* out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s;
    }
}

// Rows [row0, row0+nrows) of Omega (nrows x l).
__global__ __launch_bounds__(NT) void k_omega(uint64_t seed, uint32_t tag, int okind, int64_t row0,
                                              int64_t nrows, int l, float* out) {
    const int ng = (l + 3) / 4;
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= nrows * ng) return;
    const int64_t r = e / ng;
    const int gi = (int)(e - r * ng);
    float z[4];
    omega4k(okind, seed, tag, (uint64_t)(row0 + r), (uint32_t)gi, z);
    for (int v = 0; v < 4; ++v) {
        const int c = 4 * gi + v;
        if (c < l) out[r * l + c] = z[v];
    }
}

__global__ __launch_bounds__(NT) void k_philox_words(uint64_t seed, uint32_t tag, int64_t row0,
                                                     int64_t nrows, int ng, uint32_t* out) {
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= nrows * ng) return;
    const int64_t r = e / ng;
    const int gi = (int)(e - r * ng);
    const uint64_t j = (uint64_t)(row0 + r);
    U4 c;
    c.x = (uint32_t)j;
    c.y = (uint32_t)(j >> 32);
    c.z = (uint32_t)gi;
    c.w = tag;
    const U4 x = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    out[4 * e + 0] = x.x;
    out[4 * e + 1] = x.y;
    out[4 * e + 2] = x.z;
    out[4 * e + 3] = x.w;
}

// Q (I x l) -> Qpad (I x ldq), zero columns >= l.
__global__ __launch_bounds__(NT) void k_pad_q(const float* Q, int64_t I, int l, float* Qpad,
                                              int ldq) {
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= I * ldq) return;
    const int64_t i = e / ldq;
    const int c = (int)(e - i * ldq);
    Qpad[e] = (c < l) ? Q[i * l + c] : 0.0f;
}

__global__ __launch_bounds__(NT) void k_eye(float* Qpad, int64_t I, int ldq) {
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= I * ldq) return;
    const int64_t i = e / ldq;
    Qpad[e] = (e - i * ldq == i) ? 1.0f : 0.0f;
}

__global__ __launch_bounds__(NT) void k_fill_i32(int* p, int v, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e < n) p[e] = v;
}

// ---------------------------------------------------------------------------
// Host-side launchers.

hipError_t launch_fill_i32(int* p, int v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_eye(float* Qpad, int64_t I, int ldq, hipStream_t s) {
    const int64_t n = I * ldq;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eye, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, Qpad, I, ldq);
    return hipGetLastError();
}

// multiplier and shift for x / d with x < 2^32 (round-up method)
static void udiv_magic(uint32_t d, uint32_t* mul, uint32_t* shr) {
    uint32_t sh = 0;
    while (((uint64_t)1 << sh) < d) ++sh;
    *shr = sh;
    *mul = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << sh) - d)) / d + 1);
}

KrSpec kr_spec(int N, int n, const int* l, int R, const float* const* fac, const int* skip) {
    KrSpec k{};
    k.N = N;
    k.n = n;
    k.R = R;
    int off = 0;
    for (int m = 0; m < N; ++m) {
        k.l[m] = l[m];
        k.foff[m] = off;
        off += l[m] * R;
        udiv_magic((uint32_t)l[m], &k.mul[m], &k.shr[m]);
        k.fac[m] = fac[m];
    }
    k.ftotal = off;
    k.skip = skip;
    k.sweep = 0x7fffffff;
    return k;
}

hipError_t launch_mttkrp(const StreamGeom& g, const KrSpec& kr, float* part, int P, hipStream_t s) {
    if (g.I > 64 || kr.R < 1 || kr.R > RCP_MAX_RANK) return hipErrorInvalidValue;
    const int NBv = lp_blocks(kr.R);
    const size_t smem = contract_out_smem(NBv, 1) + (size_t)kr.ftotal * sizeof(float);
    if (smem > 160 * 1024) return hipErrorInvalidValue;
    const dim3 grid((unsigned)P, 1);
    hipError_t e = hipSuccess;
    RCP_NB_SWITCH(NBv, e = (launch_co<NB, 1, kWKr, kPrecFp32>(grid, smem, s, g, kr.R, nullptr, 0, 0,
                                                              0, part, nullptr, kr)));
    return e;
}

hipError_t launch_mttkrp_full(const StreamGeom& g, const KrSpec& kr, float* part, int P,
                              hipStream_t s) {
    if (kr.R < 1 || kr.R > RCP_MAX_RANK || g.L > 0xffffffffLL || g.Rr > 0xffffffffLL)
        return hipErrorInvalidValue;
    const int NBv = lp_blocks(kr.R);
    int MBv = (int)((g.I + 63) / 64);
    if (MBv > 8) MBv = 8;
    const int IB = 64 * MBv;
    const dim3 grid((unsigned)P, (unsigned)((g.I + IB - 1) / IB));
    const size_t smem = contract_out_smem(NBv, MBv);
    hipError_t e = hipSuccess;
    RCP_NB_SWITCH(NBv, RCP_MB_SWITCH(MBv, e = (launch_co<NB, MB, kWKrG, kPrecFp32>(
                                               grid, smem, s, g, kr.R, nullptr, 0, 0, 0, part,
                                               nullptr, kr))));
    return e;
}

StreamGeom make_geom(const float* T, const int64_t* dims, int ndim, int mode) {
    StreamGeom g;
    g.T = T;
    g.L = 1;
    g.Rr = 1;
    for (int m = 0; m < mode; ++m) g.L *= dims[m];
    for (int m = mode + 1; m < ndim; ++m) g.Rr *= dims[m];
    g.I = dims[mode];
    g.Is = g.I;
    g.vec4 = ((g.Rr % 4) == 0 && ((uintptr_t)T % 16) == 0) ? 1 : 0;
    if (g.Rr >= JT) {
        g.caseB = 0;
        g.TA = 1;
        g.tiles_per_a = (g.Rr + JT - 1) / JT;
        g.ntiles = g.L * g.tiles_per_a;
    } else {
        g.caseB = 1;
        g.TA = (int32_t)(JT / g.Rr);
        g.tiles_per_a = 0;
        g.ntiles = (g.L + g.TA - 1) / g.TA;
    }
    return g;
}

hipError_t launch_pad_q(const float* Q, int64_t I, int l, float* Qpad, int ldq, hipStream_t s) {
    const int64_t n = I * ldq;
    const unsigned blocks = (unsigned)((n + NT - 1) / NT);
    hipLaunchKernelGGL(k_pad_q, dim3(blocks), dim3(NT), 0, s, Q, I, l, Qpad, ldq);
    return hipGetLastError();
}

int contract_out_row_blocks(int64_t I, int mb_cap) {
    int MBv = (int)((I + 63) / 64);
    if (I <= 512 && MBv > mb_cap) MBv = mb_cap;
    if (I > 512) MBv = kTallMB;
    if (MBv < 1) MBv = 1;
    const int IB = 64 * MBv;
    return (int)((I + IB - 1) / IB);
}

bool power_fused_fits(int64_t I, int l, size_t smem_limit) {
    if (I > 512) return false;
    const int MBv = (int)((I + 63) / 64);
    return power_fused_smem(lp_blocks(l), MBv) <= smem_limit;
}

hipError_t launch_contract_out(const StreamGeom& g, int l, const float* Z, uint64_t seed,
                               uint32_t tag, int okind, float* part, int P, double* sq_part,
                               hipStream_t s, int precision, int mb_cap) {
    if (precision == kPrecFp32)
        return launch_contract_out_t<kPrecFp32>(g, l, Z, seed, tag, okind, part, P, sq_part, s, mb_cap);
    return launch_contract_out_lp(precision, g, l, Z, seed, tag, okind, part, P, sq_part, s, mb_cap);
}

hipError_t launch_power_fused(const StreamGeom& g, int l, const float* Qt, float* part, int P,
                              hipStream_t s, int precision) {
    if (precision == kPrecFp32) return launch_power_fused_t<kPrecFp32>(g, l, Qt, part, P, s);
    return launch_power_fused_lp(precision, g, l, Qt, part, P, s);
}

hipError_t launch_contract_in(const StreamGeom& g, int l, const float* Qpadded, int lout,
                              float* out, int P, hipStream_t s, int precision) {
    if (precision == kPrecFp32) return launch_contract_in_t<kPrecFp32>(g, l, Qpadded, lout, out, P, s);
    return launch_contract_in_lp(precision, g, l, Qpadded, lout, out, P, s);
}

int reduce_split(int P) { return P < kRedSplit ? P : kRedSplit; }

int64_t reduce_blocks(int64_t count) { return (count + kRedCols - 1) / kRedCols; }

hipError_t launch_reduce_partials(const float* part, int P, int64_t count, double* Y,
                                  const double* sq_part, int nsq, double* sq_out, hipStream_t s) {
    const int64_t blocks = reduce_blocks(count);
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(kRedThreads), 0, s,
                       part, P, count, Y, sq_part, nsq, sq_out);
    return hipGetLastError();
}

hipError_t launch_reduce_group(const ReduceDesc* d, int count, int64_t blocks, hipStream_t s) {
    if (count < 1 || blocks < 1) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_grp, dim3((unsigned)blocks), dim3(kRedThreads), 0, s, d, count);
    return hipGetLastError();
}

hipError_t launch_sketch_group(const SketchDesc* d, int count, int gx, int gy, int NB, int MB,
                               bool caseB, bool stored, int precision, hipStream_t s) {
    if (precision == kPrecFp32)
        return launch_sketch_group_t<kPrecFp32>(d, count, gx, gy, NB, MB, caseB, stored, s);
    return launch_sketch_group_lp(d, count, gx, gy, NB, MB, caseB, stored, precision, s);
}

hipError_t launch_power_group(const PowerDesc* d, int count, int gx, int NB, int MB, bool fused,
                              bool caseB, int precision, hipStream_t s) {
    if (precision == kPrecFp32)
        return launch_power_group_t<kPrecFp32>(d, count, gx, NB, MB, fused, caseB, s);
    return launch_power_group_lp(d, count, gx, NB, MB, fused, caseB, precision, s);
}

hipError_t launch_sumsq(const float* x, int64_t count, double* part, int nblocks, double* out,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_sumsq, dim3((unsigned)nblocks), dim3(NT), 0, s, x, count, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_doubles, dim3(1), dim3(64), 0, s, part, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_omega(uint64_t seed, uint32_t tag, int okind, int64_t row0, int64_t nrows,
                        int l, float* out, hipStream_t s) {
    const int ng = (l + 3) / 4;
    const int64_t n = nrows * ng;
    const unsigned blocks = (unsigned)((n + NT - 1) / NT);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_omega, dim3(blocks), dim3(NT), 0, s, seed, tag, okind, row0, nrows, l, out);
    return hipGetLastError();
}

// l distinct column indices out of J, sorted (the COLUMNS test matrix):
// Floyd's sampling without replacement on one thread, draw s from the
// Philox words of counter (s mod 2^32, s >> 32, 2^31, tag).
__global__ void k_select_columns(uint64_t seed, uint32_t tag, int64_t J, int l, int64_t* idx) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t sel[64];
    for (int s = 0; s < l; ++s) {
        const int64_t i = J - l + s;
        U4 c;
        c.x = (uint32_t)s;
        c.y = 0u;
        c.z = 0x80000000u;
        c.w = tag;
        const U4 x = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const uint64_t x64 = ((uint64_t)x.y << 32) | (uint64_t)x.x;
        const int64_t t = (int64_t)__umul64hi(x64, (uint64_t)(i + 1));
        bool seen = false;
        for (int u = 0; u < s; ++u) seen = seen || sel[u] == t;
        sel[s] = seen ? i : t;
    }
    for (int a = 1; a < l; ++a) {          // insertion sort
        const int64_t v = sel[a];
        int b = a - 1;
        while (b >= 0 && sel[b] > v) { sel[b + 1] = sel[b]; --b; }
        sel[b + 1] = v;
    }
    for (int s = 0; s < l; ++s) idx[s] = sel[s];
}

// Y (I x ldy, float64) <- the selected columns of the mode-n unfolding:
// column c of Y is unfolding column j = idx[c] = a Rr + b, zero for c >= l.
__global__ __launch_bounds__(NT) void k_gather_columns(StreamGeom g, int l, const int64_t* idx,
                                                       double* Y, int ldy) {
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= g.I * ldy) return;
    const int64_t i = e / ldy;
    const int c = (int)(e - i * ldy);
    double v = 0.0;
    if (c < l) {
        const int64_t j = idx[c];
        const int64_t a = j / g.Rr, b = j - a * g.Rr;
        v = (double)g.T[(a * g.Is + i) * g.Rr + b];
    }
    Y[e] = v;
}

hipError_t launch_select_columns(uint64_t seed, uint32_t tag, int64_t J, int l, int64_t* idx,
                                 hipStream_t s) {
    if (l < 1 || l > 64 || J < l) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_select_columns, dim3(1), dim3(64), 0, s, seed, tag, J, l, idx);
    return hipGetLastError();
}

hipError_t launch_gather_columns(const StreamGeom& g, int l, const int64_t* idx, double* Y, int ldy,
                                 hipStream_t s) {
    const int64_t n = g.I * ldy;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_columns, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, g, l,
                       idx, Y, ldy);
    return hipGetLastError();
}

hipError_t launch_philox_words(uint64_t seed, uint32_t tag, int64_t row0, int64_t nrows,
                               int ngroups, uint32_t* out, hipStream_t s) {
    const int64_t n = nrows * ngroups;
    const unsigned blocks = (unsigned)((n + NT - 1) / NT);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox_words, dim3(blocks), dim3(NT), 0, s, seed, tag, row0, nrows,
                       ngroups, out);
    return hipGetLastError();
}

}  // namespace rcp
