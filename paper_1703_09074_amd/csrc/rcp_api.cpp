// librcp host library: argument checking, workspace layout, launch
// sequencing.  Every entry point only enqueues work on the plan's stream.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/rcp.h"
#include "rcp_kernels.h"

using namespace rcp;

namespace {

constexpr int kPmax = 512;            // max workgroups of a streaming pass (partial buffers)
constexpr size_t kAlign = 256;
constexpr size_t kLdsBytes = 160 * 1024;   // LDS per workgroup on gfx950

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int lp_of(int l) { return (l + 15) / 16 * 16; }

struct Layout {
    int N, R;
    int64_t dims[RCP_MAX_NDIM];
    int l[RCP_MAX_NDIM];
    int LP[RCP_MAX_NDIM];
    int64_t Imax;
    int LPmax;
    // offsets (bytes)
    int ncompressed;       // modes Algorithm 1 compresses (the others keep Q_n = I)
    // deterministic CP-ALS (solver RCP_SOLVER_CP_ALS): float32 working
    // factors, sweep state, the subspace-iteration tensor of the start
    size_t cfac, cst, cpb;
    size_t part, red1, y64, qt, sq, norm, status, colidx, qb[RCP_MAX_NDIM], tb[2], zbuf, als, alsst,
        at[RCP_MAX_NDIM], lam, raw, estats, egram, total;
    int egram_stride;      // doubles per mode of egram
    size_t part_elems, tb_elems[2], zbuf_elems, als_doubles;
    int64_t core_dims[RCP_MAX_NDIM];
};

// Algorithm 1 variants (the remarks after Algorithm 1): which modes are
// compressed and their oversampling.
bool mode_compressed(const rcp_problem* p, int n) {
    return p->compress_mask == 0 || ((p->compress_mask >> n) & 1u) != 0;
}
int mode_oversampling(const rcp_problem* p, int n) { return p->per_mode_p ? p->mode_p[n] : p->p; }
// l_n for a (current) mode size I: the sketch width, or I for a mode left out
int64_t mode_width(const rcp_problem* p, int n, int64_t I) {
    return mode_compressed(p, n) ? std::min<int64_t>(p->k + mode_oversampling(p, n), I) : I;
}

bool valid_problem(const rcp_problem* p) {
    if (p == nullptr) return false;
    if (p->ndim < 2 || p->ndim > RCP_MAX_NDIM) return false;
    if (p->k < 1 || p->p < 0 || p->q < 0) return false;
    if (p->k > RCP_MAX_RANK || p->k + p->p > RCP_MAX_L) return false;
    if (p->max_iters < 1 || !(p->tol >= 0.0)) return false;
    if (p->scheme != RCP_SCHEME_SEQUENTIAL && p->scheme != RCP_SCHEME_INDEPENDENT) return false;
    if (p->precision != RCP_PREC_FP32 && p->precision != RCP_PREC_BF16 &&
        p->precision != RCP_PREC_FP16)
        return false;
    if (p->solver != RCP_SOLVER_ALS && p->solver != RCP_SOLVER_BCD && p->solver != RCP_SOLVER_CP_ALS)
        return false;
    if (p->test_matrix < RCP_TEST_GAUSSIAN || p->test_matrix > RCP_TEST_COLUMNS) return false;
    if ((p->compress_mask >> p->ndim) != 0) return false;
    if (p->per_mode_p != 0 && p->per_mode_p != 1) return false;
    for (int n = 0; n < p->ndim; ++n) {
        if (p->dims[n] < 1 || p->dims[n] > (int64_t)1 << 40) return false;
        if (mode_compressed(p, n)) {
            const int pn = mode_oversampling(p, n);
            if (pn < 0 || p->k + pn > RCP_MAX_L) return false;
        } else if (p->dims[n] > RCP_MAX_L) {
            return false;              // a mode kept whole must fit the core solvers
        }
        if (p->k > mode_width(p, n, p->dims[n])) return false;
    }
    if (p->test_matrix == RCP_TEST_COLUMNS) {
        // every compressed mode needs l_n <= J_n (the other current sizes)
        int64_t cur[RCP_MAX_NDIM];
        for (int n = 0; n < p->ndim; ++n) cur[n] = p->dims[n];
        for (int n = 0; n < p->ndim; ++n) {
            if (!mode_compressed(p, n)) continue;
            double J = 1.0;
            for (int m = 0; m < p->ndim; ++m)
                if (m != n) J *= (double)cur[m];
            if ((double)mode_width(p, n, cur[n]) > J) return false;
            if (p->scheme == RCP_SCHEME_SEQUENTIAL) cur[n] = mode_width(p, n, cur[n]);
        }
    }
    // total element count must stay well inside int64
    double S = 1.0;
    for (int n = 0; n < p->ndim; ++n) S *= (double)p->dims[n];
    if (S > 4.0e12) return false;
    return true;
}

// Workspace layout; identical for rcp_workspace_size and rcp_init.
Layout make_layout(const rcp_problem* p) {
    Layout L{};
    L.N = p->ndim;
    L.R = p->k;
    L.Imax = 1;
    L.LPmax = 16;
    for (int n = 0; n < L.N; ++n) {
        L.dims[n] = p->dims[n];
        L.l[n] = (int)mode_width(p, n, p->dims[n]);
        L.LP[n] = lp_of(L.l[n]);
        L.Imax = std::max(L.Imax, p->dims[n]);
        L.LPmax = std::max(L.LPmax, L.LP[n]);
    }
    // partials: any sketch on a tensor with dims <= the plan's dims
    size_t part = 0;
    for (int n = 0; n < L.N; ++n)
        part = std::max(part, (size_t)kPmax * (size_t)L.dims[n] * (size_t)L.LP[n]);
    L.part_elems = part;
    // compressed tensors: the c-th compressed mode writes buffer c % 2
    int64_t cur[RCP_MAX_NDIM];
    for (int n = 0; n < L.N; ++n) cur[n] = L.dims[n];
    L.tb_elems[0] = L.tb_elems[1] = 0;
    L.ncompressed = 0;
    for (int n = 0; n < L.N; ++n) {
        if (!mode_compressed(p, n)) continue;
        cur[n] = L.l[n];
        int64_t s = 1;
        for (int m = 0; m < L.N; ++m) s *= cur[m];
        const int buf = L.ncompressed % 2;
        L.tb_elems[buf] = std::max(L.tb_elems[buf], (size_t)s);
        ++L.ncompressed;
    }
    for (int n = 0; n < L.N; ++n) L.core_dims[n] = L.l[n];
    // stored Z for modes whose tile does not fit the fused power kernel
    L.zbuf_elems = 0;
    if (p->q > 0) {
        int64_t S = 1;
        for (int n = 0; n < L.N; ++n) S *= L.dims[n];
        for (int n = 0; n < L.N; ++n) {
            if (!power_fused_fits(L.dims[n], L.l[n], kLdsBytes))
                L.zbuf_elems = std::max(L.zbuf_elems, (size_t)(S / L.dims[n]) * (size_t)L.LP[n]);
        }
    }
    L.als_doubles = als_workspace_doubles(L.N, L.l, L.R);

    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes); return o; };
    L.part = take(L.part_elems * sizeof(float));
    L.red1 = take((size_t)16 * L.Imax * L.LPmax * sizeof(double));
    L.y64 = take((size_t)L.Imax * L.LPmax * sizeof(double));
    L.qt = take((size_t)L.Imax * L.LPmax * sizeof(float));
    int nib = 1;
    for (int n = 0; n < L.N; ++n) nib = std::max(nib, contract_out_row_blocks(L.dims[n], 1));
    L.sq = take((size_t)kPmax * nib * sizeof(double));
    L.norm = take(64 * sizeof(double));
    L.status = take(sizeof(int32_t));
    L.colidx = take(RCP_MAX_L * sizeof(int64_t));
    for (int n = 0; n < L.N; ++n) L.qb[n] = take((size_t)L.dims[n] * L.l[n] * sizeof(float));
    L.tb[0] = take(L.tb_elems[0] * sizeof(float));
    L.tb[1] = take(L.tb_elems[1] * sizeof(float));
    L.zbuf = take(L.zbuf_elems * sizeof(float));
    L.als = take(L.als_doubles * sizeof(double));
    L.alsst = take(als_state_doubles(L.N, L.R) * sizeof(double));
    for (int n = 0; n < L.N; ++n) L.at[n] = take((size_t)L.l[n] * L.R * sizeof(float));
    L.lam = take((size_t)L.R * sizeof(float));
    size_t raw = 0;
    for (int n = 0; n < L.N; ++n) raw += (size_t)L.dims[n] * L.R;
    L.raw = take(raw * sizeof(double));
    L.estats = take((size_t)(2 * L.N * L.R + L.R) * sizeof(double));
    // the eigenvector start of a core larger than LDS: the Grams of modes
    // 1..N-1 side by side
    L.egram_stride = 0;
    if (!als_core_in_lds(L.N, L.l, L.R) || p->solver == RCP_SOLVER_CP_ALS) {
        int lmax = 0;
        for (int n = 0; n < L.N; ++n) lmax = std::max(lmax, L.l[n]);
        L.egram_stride = lmax * lp_of(lmax);
        L.egram = take((size_t)(L.N - 1) * L.egram_stride * sizeof(double));
    }
    L.cfac = L.cst = L.cpb = 0;
    if (p->solver == RCP_SOLVER_CP_ALS) {
        L.cfac = take(raw * sizeof(float));
        L.cst = take(cp_state_doubles(L.N, L.R) * sizeof(double));
        int64_t S = 1;
        for (int n = 0; n < L.N; ++n) S *= L.dims[n];
        size_t bmax = 0;
        for (int n = 1; n < L.N; ++n) bmax = std::max(bmax, (size_t)(S / L.dims[n]) * L.l[n]);
        L.cpb = take(bmax * sizeof(float));
    }
    L.total = off;
    return L;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

}  // namespace

namespace {

constexpr int kMaxProfiled = 4096;

struct ProfRecord {
    int cls;
    double bytes, flops;
};

// Event pairs around every launch while profiling is on.
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> ev;            // 2 * kMaxProfiled
    std::vector<ProfRecord> rec;
    int64_t untimed[RCP_KERNEL_COUNT] = {};
    void clear() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        ev.clear();
        rec.clear();
        for (auto& u : untimed) u = 0;
        on = false;
    }
};

}  // namespace

struct rcp_plan_t {
    rcp_problem prob;
    Layout L;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    int P;                 // workgroups per streaming pass
    int mb_cap = 8;        // row-block height of the sketch passes, in 64-row units
    size_t smem_limit;
    Profiler prof;
    template <class T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
    int* status_word() const { return at<int>(L.status); }
};

namespace {

rcp_status hip_status(hipError_t e) { return e == hipSuccess ? RCP_OK : RCP_ERR_HIP; }

#define RCP_TRY(expr)                                       \
    do {                                                    \
        const hipError_t rcp_e_ = (expr);                   \
        if (rcp_e_ != hipSuccess) return RCP_ERR_HIP;       \
    } while (0)

// Runs `launch` (which enqueues one kernel) between two recorded events when
// profiling is on, with the launch's algorithmic bytes and flops.
template <class F>
hipError_t timed(rcp_plan_t* pl, int cls, double bytes, double flops, F&& launch) {
    Profiler& pr = pl->prof;
    if (!pr.on) return launch();
    const size_t idx = pr.rec.size();
    if (idx >= (size_t)kMaxProfiled) {
        ++pr.untimed[cls];
        return launch();
    }
    hipError_t e = hipEventRecord(pr.ev[2 * idx], pl->stream);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(pr.ev[2 * idx + 1], pl->stream);
    if (e != hipSuccess) return e;
    pr.rec.push_back(ProfRecord{cls, bytes, flops});
    return hipSuccess;
}

bool valid_cur_dims(const rcp_plan_t* pl, const int64_t* cur) {
    if (cur == nullptr) return false;
    for (int n = 0; n < pl->L.N; ++n)
        if (cur[n] < 1 || cur[n] > pl->L.dims[n]) return false;
    return true;
}

int64_t count_of(const int64_t* d, int N) {
    int64_t s = 1;
    for (int n = 0; n < N; ++n) s *= d[n];
    return s;
}

// Y (I x LP float64, in the workspace) <- partials
rcp_status reduce_y(rcp_plan_t* pl, int P, int64_t I, int LP, const double* sq, int nsq,
                    double* sq_out) {
    const double bytes = (double)P * I * LP * 4.0 + (double)I * LP * 8.0;
    RCP_TRY(timed(pl, RCP_KERNEL_REDUCE, bytes, (double)P * I * LP, [&] {
        return launch_reduce_partials(pl->at<float>(pl->L.part), P, I * LP, pl->at<double>(pl->L.y64),
                                      sq, nsq, sq_out, pl->stream);
    }));
    return RCP_OK;
}

// Algorithm 1's range finder for one mode.  On return the padded basis is in
// Qt (I x LP) and, if Q != null, the basis (I x l) is in Q.
rcp_status sketch_impl(rcp_plan_t* pl, const float* T, const int64_t* cur, int mode, float* Q,
                       double* norm_out) {
    const int N = pl->L.N;
    const int64_t I = cur[mode];
    const int l = (int)std::min<int64_t>(pl->prob.k + mode_oversampling(&pl->prob, mode), I);
    const int LP = lp_of(l);
    const StreamGeom g = make_geom(T, cur, N, mode);
    const int P = (int)std::max<int64_t>(1, std::min<int64_t>(pl->P, g.ntiles));
    float* part = pl->at<float>(pl->L.part);
    double* Y = pl->at<double>(pl->L.y64);
    float* Qt = pl->at<float>(pl->L.qt);
    double* sq = pl->at<double>(pl->L.sq);
    const uint32_t tag = omega_stream_tag(0, (uint32_t)mode);
    const int nIB = contract_out_row_blocks(I, pl->mb_cap);

    const double S = (double)count_of(cur, N);
    const double J = S / (double)I;
    // nominal QR work: per Cholesky QR pass a Gram (I l^2) and a triangular
    // product (I l^2) in float64; two passes, three for the returned basis
    const double qr_bytes = (double)I * l * 8.0 + (double)I * LP * 4.0;
    const double qr_flops = 2.0 * 2.0 * (double)I * l * l;
    rcp_status st = RCP_OK;
    if (pl->prob.test_matrix == RCP_TEST_COLUMNS) {
        // randomly selected columns in place of the product (the remark after
        // Algorithm 1): the sketch is a gather of l unfolding columns
        int64_t* idx = pl->at<int64_t>(pl->L.colidx);
        if ((double)l > J) return RCP_ERR_INVALID_ARG;
        RCP_TRY(launch_select_columns(pl->prob.seed, tag, (int64_t)J, l, idx, pl->stream));
        RCP_TRY(timed(pl, RCP_KERNEL_SKETCH, 4.0 * I * l + 8.0 * I * LP, 0.0,
                      [&] { return launch_gather_columns(g, l, idx, Y, LP, pl->stream); }));
        if (norm_out != nullptr) {
            const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kPmax, ((int64_t)S + 255) / 256));
            RCP_TRY(launch_sumsq(T, (int64_t)S, sq, nb, norm_out, pl->stream));
        }
    } else {
        RCP_TRY(timed(pl, RCP_KERNEL_SKETCH, 4.0 * S + 4.0 * I * l, 2.0 * S * l, [&] {
            return launch_contract_out(g, l, nullptr, pl->prob.seed, tag, pl->prob.test_matrix,
                                       part, P, norm_out ? sq : nullptr, pl->stream,
                                       pl->prob.precision, pl->mb_cap);
        }));
        st = reduce_y(pl, P, I, LP, norm_out ? sq : nullptr, P * nIB, norm_out);
        if (st != RCP_OK) return st;
    }
    const bool fused = power_fused_fits(I, l, pl->smem_limit);
    for (int it = 0; it < pl->prob.q; ++it) {
        RCP_TRY(timed(pl, RCP_KERNEL_QR, qr_bytes, 2.0 * qr_flops,
                      [&] { return launch_qr(Y, I, l, LP, Qt, LP, nullptr, false, pl->status_word(), pl->stream,
                                             pl->at<double>(pl->L.red1)); }));
        if (fused) {
            RCP_TRY(timed(pl, RCP_KERNEL_POWER, 4.0 * S + 4.0 * I * l, 4.0 * S * l,
                          [&] { return launch_power_fused(g, l, Qt, part, P, pl->stream, pl->prob.precision); }));
        } else {
            float* Z = pl->at<float>(pl->L.zbuf);
            RCP_TRY(timed(pl, RCP_KERNEL_CONTRACT_IN, 4.0 * S + 4.0 * J * LP, 2.0 * S * l,
                          [&] { return launch_contract_in(g, l, Qt, LP, Z, P, pl->stream, pl->prob.precision); }));
            RCP_TRY(timed(pl, RCP_KERNEL_CONTRACT_OUT, 4.0 * S + 4.0 * J * LP, 2.0 * S * l, [&] {
                return launch_contract_out(g, l, Z, 0, 0, 0, part, P, nullptr, pl->stream,
                                           pl->prob.precision, pl->mb_cap);
            }));
        }
        st = reduce_y(pl, P, I, LP, nullptr, 0, nullptr);
        if (st != RCP_OK) return st;
    }
    RCP_TRY(timed(pl, RCP_KERNEL_QR, qr_bytes, 3.0 * qr_flops,
                  [&] { return launch_qr(Y, I, l, LP, Qt, LP, Q, true, pl->status_word(), pl->stream,
                                         pl->at<double>(pl->L.red1)); }));
    return RCP_OK;
}

// T_out = T x_mode Q^T with the padded basis already in Qt.
rcp_status compress_impl(rcp_plan_t* pl, const float* T, const int64_t* cur, int mode,
                         float* T_out) {
    const int64_t I = cur[mode];
    const int l = (int)std::min<int64_t>(pl->prob.k + mode_oversampling(&pl->prob, mode), I);
    const StreamGeom g = make_geom(T, cur, pl->L.N, mode);
    const int P = (int)std::max<int64_t>(1, std::min<int64_t>(pl->P, g.ntiles));
    const double S = (double)count_of(cur, pl->L.N);
    RCP_TRY(timed(pl, RCP_KERNEL_CONTRACT_IN, 4.0 * S + 4.0 * (S / (double)I) * l,
                  2.0 * S * l, [&] {
                      // the compressed tensor is the core: float32 operands in every precision
                      return launch_contract_in(g, l, pl->at<float>(pl->L.qt), l, T_out, P,
                                                pl->stream, RCP_PREC_FP32);
                  }));
    return RCP_OK;
}

// CP-ALS for a core larger than LDS: per mode, the mode product over the
// whole GPU (Khatri-Rao kind of the streaming kernel), its float64
// reduction, and the one-workgroup solve; all max_iters sweeps are enqueued,
// and the device-side stop flag turns the launches after convergence into
// no-ops.  The factors live in At throughout.
hipError_t als_wide(rcp_plan_t* pl, AlsArgs a) {
    const Layout& L = pl->L;
    const int N = L.N, R = L.R;
    int64_t cd[RCP_MAX_NDIM];
    int64_t S = 1;
    for (int n = 0; n < N; ++n) { cd[n] = L.l[n]; S *= L.l[n]; }
    double* state = pl->at<double>(L.alsst);
    float* part = pl->at<float>(L.part);
    double* red1 = pl->at<double>(L.red1);
    double* Y = pl->at<double>(L.y64);
    a.Y = Y;
    a.state = state;
    if (a.normX2 == nullptr) {
        // ||core||^2 into a spare slot of the state (double 3)
        const int nb = (int)std::min<int64_t>(256, std::max<int64_t>(1, S / 4096));
        hipError_t e = launch_sumsq(a.B, S, red1, nb, state + 3, pl->stream);
        if (e != hipSuccess) return e;
        a.normX2 = state + 3;
    }
    if (a.warm) {
        // warm start: the Grams of the caller's factors, a fresh sweep state
        hipError_t e = launch_als_wide_warm(a, pl->stream);
        if (e != hipSuccess) return e;
    }
    if (!a.warm) {
        // Algorithm 2's initialisation: the Grams B_(n) B_(n)^T as Y = T (T^T I) over the
        // GPU, side by side, then every mode's eigenvectors at once
        double* eg = pl->at<double>(L.egram);
        for (int n = 1; n < N; ++n) {
            const StreamGeom g = make_geom(a.B, cd, N, n);
            const int P = (int)std::max<int64_t>(1, std::min<int64_t>(pl->P, g.ntiles));
            const int LPn = lp_of(L.l[n]);
            float* eye = pl->at<float>(L.qt);
            hipError_t e = launch_eye(eye, L.l[n], LPn, pl->stream);
            if (e == hipSuccess) e = launch_power_fused(g, L.l[n], eye, part, P, pl->stream, RCP_PREC_FP32);
            if (e == hipSuccess)
                e = launch_reduce_partials(part, P, (int64_t)L.l[n] * LPn,
                                           eg + (size_t)(n - 1) * L.egram_stride, nullptr, 0,
                                           nullptr, pl->stream);
            if (e != hipSuccess) return e;
        }
        hipError_t e = launch_fill_i32((int*)state, 0, 6, pl->stream);   // flags and rho
        AlsArgs ai = a;
        ai.Y = eg;
        if (e == hipSuccess) e = launch_als_wide_init(ai, L.egram_stride, pl->stream);
        if (e != hipSuccess) return e;
    }
    const float* facs[RCP_MAX_NDIM];
    for (int n = 0; n < N; ++n) facs[n] = a.At[n];
    const int LPR = lp_of(R);
    a.ldy = LPR;
    for (int it = 0; it < a.max_iters; ++it) {
        for (int n = 0; n < N; ++n) {
            const StreamGeom g = make_geom(a.B, cd, N, n);
            const int P = (int)std::max<int64_t>(1, std::min<int64_t>(pl->P, g.ntiles));
            const KrSpec kr = kr_spec(N, n, L.l, R, facs, (const int*)state);
            hipError_t e = launch_mttkrp(g, kr, part, P, pl->stream);
            if (e == hipSuccess)
                e = launch_reduce_partials(part, P, (int64_t)L.l[n] * LPR, Y, nullptr, 0,
                                           nullptr, pl->stream);
            if (e == hipSuccess) e = launch_als_wide_step(a, n, pl->stream);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

rcp_status als_impl(rcp_plan_t* pl, const float* core, float* const* At, float* lambda,
                    const double* normX2, rcp_als_info* info, int warm) {
    const Layout& L = pl->L;
    AlsArgs a{};
    a.B = core;
    a.N = L.N;
    for (int n = 0; n < L.N; ++n) { a.l[n] = L.l[n]; a.At[n] = At[n]; }
    a.R = L.R;
    a.max_iters = pl->prob.max_iters;
    a.warm = warm;
    a.tol = pl->prob.tol;
    a.normX2 = normX2;
    a.lambda = lambda;
    a.info = info;
    a.status_word = pl->status_word();
    int64_t S = 1;
    for (int n = 0; n < L.N; ++n) S *= L.l[n];
    const int R = L.R;
    a.Ebuf = pl->at<double>(L.als);
    // nominal algorithmic work: N mode products of the core with R columns per sweep
    const double sweeps = (double)pl->prob.max_iters;
    const bool in_lds = als_core_in_lds(L.N, L.l, R);
    RCP_TRY(timed(pl, RCP_KERNEL_ALS, sweeps * L.N * 4.0 * (double)S,
                  sweeps * L.N * 2.0 * (double)S * R, [&] {
                      return in_lds ? launch_als(a, pl->stream) : als_wide(pl, a);
                  }));
    return RCP_OK;
}

// Algorithm 3 on the core: one workgroup (the core in LDS when it fits);
// without ||X||^2 the fit is taken against ||core||^2 (second norm slot).
rcp_status bcd_impl(rcp_plan_t* pl, const float* core, float* const* At, float* lambda,
                    const double* normX2, rcp_als_info* info, int warm) {
    const Layout& L = pl->L;
    AlsArgs a{};
    a.B = core;
    a.N = L.N;
    for (int n = 0; n < L.N; ++n) { a.l[n] = L.l[n]; a.At[n] = At[n]; }
    a.R = L.R;
    a.max_iters = pl->prob.max_iters;
    a.warm = warm;
    a.tol = pl->prob.tol;
    a.lambda = lambda;
    a.info = info;
    a.status_word = pl->status_word();
    a.Ebuf = pl->at<double>(L.als);
    int64_t S = 1;
    for (int n = 0; n < L.N; ++n) S *= L.l[n];
    if (normX2 == nullptr) {
        double* slot = pl->at<double>(L.norm) + 1;
        const int nb = (int)std::min<int64_t>(256, std::max<int64_t>(1, S / 4096));
        RCP_TRY(launch_sumsq(core, S, pl->at<double>(L.red1), nb, slot, pl->stream));
        normX2 = slot;
    }
    a.normX2 = normX2;
    // nominal work: per sweep of each component, N products of the core with a vector
    const double sweeps = (double)pl->prob.max_iters * L.R;
    RCP_TRY(timed(pl, RCP_KERNEL_BCD, sweeps * L.N * 4.0 * (double)S, sweeps * L.N * 2.0 * (double)S,
                  [&] { return launch_bcd(a, pl->stream); }));
    return RCP_OK;
}

rcp_status expand_impl(rcp_plan_t* pl, const float* const* Q, const float* const* At,
                       const float* lam_in, float* const* A, float* lam_out) {
    const Layout& L = pl->L;
    ExpandArgs e{};
    e.N = L.N;
    e.R = L.R;
    for (int n = 0; n < L.N; ++n) {
        e.I[n] = L.dims[n];
        e.l[n] = L.l[n];
        e.Q[n] = Q[n];
        e.At[n] = At[n];
        e.A[n] = A[n];
    }
    e.lambda_in = lam_in;
    e.lambda_out = lam_out;
    e.raw = pl->at<double>(L.raw);
    e.stats = pl->at<double>(L.estats);
    double flops = 0.0, bytes = 0.0;
    for (int n = 0; n < L.N; ++n) {
        flops += 2.0 * (double)L.dims[n] * L.l[n] * L.R;
        bytes += 4.0 * ((double)L.dims[n] * L.l[n] + (double)L.dims[n] * L.R);
    }
    RCP_TRY(timed(pl, RCP_KERNEL_EXPAND, bytes, flops, [&] { return launch_expand(e, pl->stream); }));
    return RCP_OK;
}

}  // namespace

extern "C" {

const char* rcp_status_string(rcp_status s) {
    // a C caller may pass any int: read it as one (an rcp_status holding a
    // value outside the enumerators is not a valid C++ enum value)
    int v;
    static_assert(sizeof v == sizeof s, "rcp_status is int-sized");
    std::memcpy(&v, &s, sizeof v);
    switch (v) {
        case RCP_OK: return "RCP_OK: success";
        case RCP_ERR_INVALID_ARG: return "RCP_ERR_INVALID_ARG: invalid argument";
        case RCP_ERR_WORKSPACE: return "RCP_ERR_WORKSPACE: workspace missing or too small";
        case RCP_ERR_HIP: return "RCP_ERR_HIP: HIP runtime or launch failure";
        case RCP_ERR_NUMERIC: return "RCP_ERR_NUMERIC: numeric failure";
        case RCP_ERR_UNSUPPORTED: return "RCP_ERR_UNSUPPORTED: not supported by the library";
    }
    return "unknown rcp_status";
}

const char* rcp_version(void) { return "librcp 0.1 (gfx950)"; }

rcp_status rcp_workspace_size(const rcp_problem* prob, size_t* bytes) {
    if (bytes == nullptr || !valid_problem(prob)) return RCP_ERR_INVALID_ARG;
    *bytes = make_layout(prob).total;
    return RCP_OK;
}

}  // extern "C"

namespace {

// Checks the problem and the workspace and fills *pl (no allocation, no
// device work): shared by rcp_init and the allocation-free entry point.
rcp_status plan_setup(rcp_plan_t* pl, const rcp_problem* prob, void* workspace,
                      size_t workspace_bytes, void* hip_stream, int cus) {
    if (!valid_problem(prob)) return RCP_ERR_INVALID_ARG;
    const Layout L = make_layout(prob);
    if (!als_supported(L.N, L.l, L.R)) return RCP_ERR_UNSUPPORTED;
    if (prob->solver == RCP_SOLVER_BCD && !bcd_supported(L.N, L.l, L.R)) return RCP_ERR_UNSUPPORTED;
    if (workspace == nullptr || workspace_bytes < L.total || !aligned(workspace, kAlign))
        return RCP_ERR_WORKSPACE;
    pl->prob = *prob;
    pl->L = L;
    pl->stream = (hipStream_t)hip_stream;
    pl->ws = (char*)workspace;
    pl->ws_bytes = workspace_bytes;
    pl->P = std::max(1, std::min(kPmax, cus));
    pl->smem_limit = kLdsBytes;
    return RCP_OK;
}

// Compute units of the current device if it is a gfx950, else 0.
rcp_status device_cus(int* cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RCP_ERR_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return RCP_ERR_HIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return RCP_ERR_UNSUPPORTED;
    *cus = prop.multiProcessorCount;
    return RCP_OK;
}

}  // namespace

extern "C" {

rcp_status rcp_init(rcp_plan* plan, const rcp_problem* prob, void* workspace,
                    size_t workspace_bytes, void* hip_stream) {
    if (plan == nullptr) return RCP_ERR_INVALID_ARG;
    *plan = nullptr;
    rcp_plan_t probe;
    // argument errors before any device query
    rcp_status st = plan_setup(&probe, prob, workspace, workspace_bytes, hip_stream, 1);
    if (st != RCP_OK) return st;
    int cus = 0;
    st = device_cus(&cus);
    if (st != RCP_OK) return st;
    rcp_plan_t* pl = new (std::nothrow) rcp_plan_t;
    if (pl == nullptr) return RCP_ERR_HIP;
    st = plan_setup(pl, prob, workspace, workspace_bytes, hip_stream, cus);
    if (st != RCP_OK) { delete pl; return st; }
    if (hipMemsetAsync(pl->status_word(), 0, sizeof(int32_t), pl->stream) != hipSuccess) {
        delete pl;
        return RCP_ERR_HIP;
    }
    *plan = pl;
    return RCP_OK;
}

rcp_status rcp_read_status(rcp_plan plan, int32_t* status) {
    if (plan == nullptr || status == nullptr) return RCP_ERR_INVALID_ARG;
    int32_t v = 0;
    RCP_TRY(hipMemcpyAsync(&v, plan->status_word(), sizeof(int32_t), hipMemcpyDeviceToHost,
                           plan->stream));
    RCP_TRY(hipMemsetAsync(plan->status_word(), 0, sizeof(int32_t), plan->stream));
    RCP_TRY(hipStreamSynchronize(plan->stream));
    *status = v;
    return RCP_OK;
}

rcp_status rcp_destroy(rcp_plan plan) {
    if (plan == nullptr) return RCP_ERR_INVALID_ARG;
    plan->prof.clear();
    delete plan;
    return RCP_OK;
}

rcp_status rcp_profile(rcp_plan plan, int32_t enable) {
    if (plan == nullptr) return RCP_ERR_INVALID_ARG;
    Profiler& pr = plan->prof;
    pr.clear();
    if (!enable) return RCP_OK;
    pr.ev.resize(2 * kMaxProfiled);
    for (size_t i = 0; i < pr.ev.size(); ++i) {
        if (hipEventCreate(&pr.ev[i]) != hipSuccess) {
            pr.ev.resize(i);
            pr.clear();
            return RCP_ERR_HIP;
        }
    }
    pr.rec.reserve(kMaxProfiled);
    pr.on = true;
    return RCP_OK;
}

rcp_status rcp_profile_read(rcp_plan plan, int32_t kernel_class, int64_t* launches, double* ms,
                            double* bytes, double* flops) {
    if (plan == nullptr || kernel_class < 0 || kernel_class >= RCP_KERNEL_COUNT)
        return RCP_ERR_INVALID_ARG;
    const Profiler& pr = plan->prof;
    int64_t n = pr.untimed[kernel_class];
    double t = 0.0, b = 0.0, f = 0.0;
    for (size_t i = 0; i < pr.rec.size(); ++i) {
        if (pr.rec[i].cls != kernel_class) continue;
        if (hipEventSynchronize(pr.ev[2 * i + 1]) != hipSuccess) return RCP_ERR_HIP;
        float e = 0.0f;
        if (hipEventElapsedTime(&e, pr.ev[2 * i], pr.ev[2 * i + 1]) != hipSuccess) return RCP_ERR_HIP;
        t += e;
        b += pr.rec[i].bytes;
        f += pr.rec[i].flops;
        ++n;
    }
    if (launches) *launches = n;
    if (ms) *ms = t;
    if (bytes) *bytes = b;
    if (flops) *flops = f;
    return RCP_OK;
}

rcp_status rcp_sketch(rcp_plan plan, const float* T, const int64_t* cur_dims, int32_t mode,
                      float* Q) {
    if (plan == nullptr || T == nullptr || Q == nullptr) return RCP_ERR_INVALID_ARG;
    if (mode < 0 || mode >= plan->L.N || !valid_cur_dims(plan, cur_dims)) return RCP_ERR_INVALID_ARG;
    if (!aligned(T, 4) || !aligned(Q, 4)) return RCP_ERR_INVALID_ARG;
    return sketch_impl(plan, T, cur_dims, mode, Q, nullptr);
}

rcp_status rcp_compress(rcp_plan plan, const float* T, const int64_t* cur_dims, int32_t mode,
                        const float* Q, float* T_out) {
    if (plan == nullptr || T == nullptr || Q == nullptr || T_out == nullptr)
        return RCP_ERR_INVALID_ARG;
    if (mode < 0 || mode >= plan->L.N || !valid_cur_dims(plan, cur_dims)) return RCP_ERR_INVALID_ARG;
    if (!aligned(T, 4) || !aligned(Q, 4) || !aligned(T_out, 4)) return RCP_ERR_INVALID_ARG;
    const int N = plan->L.N;
    const int64_t I = cur_dims[mode];
    const int l = (int)std::min<int64_t>(plan->prob.k + mode_oversampling(&plan->prob, mode), I);
    const int64_t nin = count_of(cur_dims, N);
    const int64_t nout = nin / I * l;
    if (overlap(T, (size_t)nin * 4, T_out, (size_t)nout * 4)) return RCP_ERR_INVALID_ARG;
    RCP_TRY(launch_pad_q(Q, I, l, plan->at<float>(plan->L.qt), lp_of(l), plan->stream));
    return compress_impl(plan, T, cur_dims, mode, T_out);
}

rcp_status rcp_norm2(rcp_plan plan, const float* X, int64_t count, double* out) {
    if (plan == nullptr || X == nullptr || out == nullptr || count < 0) return RCP_ERR_INVALID_ARG;
    if (!aligned(X, 4) || !aligned(out, 8)) return RCP_ERR_INVALID_ARG;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kPmax, (count + 255) / 256));
    RCP_TRY(launch_sumsq(X, count, plan->at<double>(plan->L.sq), nb, out, plan->stream));
    return RCP_OK;
}

rcp_status rcp_als(rcp_plan plan, const float* core, float* const* At, float* lambda,
                   const double* normX2, rcp_als_info* info, int32_t use_given_init) {
    if (plan == nullptr || core == nullptr || At == nullptr || lambda == nullptr || info == nullptr)
        return RCP_ERR_INVALID_ARG;
    for (int n = 0; n < plan->L.N; ++n)
        if (At[n] == nullptr || !aligned(At[n], 4)) return RCP_ERR_INVALID_ARG;
    if (!aligned(core, 4) || !aligned(info, 8) || (normX2 && !aligned(normX2, 8)))
        return RCP_ERR_INVALID_ARG;
    return als_impl(plan, core, At, lambda, normX2, info, use_given_init != 0 ? 1 : 0);
}

rcp_status rcp_bcd(rcp_plan plan, const float* core, float* const* At, float* lambda,
                   const double* normX2, rcp_als_info* info, int32_t use_given_init) {
    if (plan == nullptr || core == nullptr || At == nullptr || lambda == nullptr || info == nullptr)
        return RCP_ERR_INVALID_ARG;
    for (int n = 0; n < plan->L.N; ++n)
        if (At[n] == nullptr || !aligned(At[n], 4)) return RCP_ERR_INVALID_ARG;
    if (!aligned(core, 4) || !aligned(info, 8) || (normX2 && !aligned(normX2, 8)))
        return RCP_ERR_INVALID_ARG;
    if (!bcd_supported(plan->L.N, plan->L.l, plan->L.R)) return RCP_ERR_UNSUPPORTED;
    return bcd_impl(plan, core, At, lambda, normX2, info, use_given_init != 0 ? 1 : 0);
}

rcp_status rcp_expand(rcp_plan plan, const float* const* Q, const float* const* At,
                      const float* lambda_in, float* const* A, float* lambda_out) {
    if (plan == nullptr || Q == nullptr || At == nullptr || A == nullptr || lambda_in == nullptr ||
        lambda_out == nullptr)
        return RCP_ERR_INVALID_ARG;
    for (int n = 0; n < plan->L.N; ++n)
        if (Q[n] == nullptr || At[n] == nullptr || A[n] == nullptr) return RCP_ERR_INVALID_ARG;
    return expand_impl(plan, Q, At, lambda_in, A, lambda_out);
}

namespace {

// Where the core ends up: the buffer of the last compressed mode.
float* core_location(rcp_plan_t* plan) {
    return plan->at<float>(plan->L.tb[(plan->L.ncompressed - 1) % 2]);
}

// Algorithm 1 over every mode: leaves the bases in the plan's qb buffers and
// the core in the buffer of the last compressed mode; *core_out points at it.
// A mode left out of rcp_problem.compress_mask gets Q_n = I and keeps its
// size; ||X||^2 comes from the first sketch pass when mode 0 takes a
// streamed sketch, else from a separate pass.
rcp_status compress_all(rcp_plan_t* plan, const float* X, const float** core_out) {
    const Layout& L = plan->L;
    const int N = L.N;
    const rcp_problem* pr = &plan->prob;
    double* normX2 = plan->at<double>(L.norm);
    float* Qb[RCP_MAX_NDIM];
    for (int n = 0; n < N; ++n) Qb[n] = plan->at<float>(L.qb[n]);
    int64_t cur[RCP_MAX_NDIM];
    for (int n = 0; n < N; ++n) cur[n] = L.dims[n];
    const bool norm_in_sketch = mode_compressed(pr, 0) && pr->test_matrix != RCP_TEST_COLUMNS;
    if (!norm_in_sketch) {
        const int64_t S = count_of(cur, N);
        const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kPmax, (S + 255) / 256));
        RCP_TRY(launch_sumsq(X, S, plan->at<double>(L.sq), nb, normX2, plan->stream));
    }
    for (int n = 0; n < N; ++n)
        if (!mode_compressed(pr, n)) RCP_TRY(launch_eye(Qb[n], L.dims[n], L.l[n], plan->stream));
    const float* T = X;
    int c = 0;
    rcp_status st;
    if (pr->scheme == RCP_SCHEME_SEQUENTIAL) {
        for (int n = 0; n < N; ++n) {
            if (!mode_compressed(pr, n)) continue;
            st = sketch_impl(plan, T, cur, n, Qb[n], (n == 0 && norm_in_sketch) ? normX2 : nullptr);
            if (st != RCP_OK) return st;
            float* out = plan->at<float>(L.tb[c % 2]);
            st = compress_impl(plan, T, cur, n, out);
            if (st != RCP_OK) return st;
            cur[n] = L.l[n];
            T = out;
            ++c;
        }
    } else {
        for (int n = 0; n < N; ++n) {
            if (!mode_compressed(pr, n)) continue;
            st = sketch_impl(plan, X, cur, n, Qb[n], (n == 0 && norm_in_sketch) ? normX2 : nullptr);
            if (st != RCP_OK) return st;
        }
        for (int n = 0; n < N; ++n) {
            if (!mode_compressed(pr, n)) continue;
            RCP_TRY(launch_pad_q(Qb[n], L.dims[n], L.l[n], plan->at<float>(L.qt), L.LP[n],
                                 plan->stream));
            float* out = plan->at<float>(L.tb[c % 2]);
            st = compress_impl(plan, T, cur, n, out);
            if (st != RCP_OK) return st;
            cur[n] = L.l[n];
            T = out;
            ++c;
        }
    }
    *core_out = T;
    return RCP_OK;
}

AlsArgs core_als_args(rcp_plan_t* plan, const float* core, rcp_als_info* info) {
    const Layout& L = plan->L;
    AlsArgs a{};
    a.B = core;
    a.N = L.N;
    for (int n = 0; n < L.N; ++n) { a.l[n] = L.l[n]; a.At[n] = plan->at<float>(L.at[n]); }
    a.R = L.R;
    a.max_iters = plan->prob.max_iters;
    a.tol = plan->prob.tol;
    a.normX2 = plan->at<double>(L.norm);
    a.lambda = plan->at<float>(L.lam);
    a.info = info;
    a.status_word = plan->status_word();
    a.Ebuf = plan->at<double>(L.als);
    return a;
}

ExpandArgs core_expand_args(rcp_plan_t* plan, float* const* A, float* lambda) {
    const Layout& L = plan->L;
    ExpandArgs e{};
    e.N = L.N;
    e.R = L.R;
    for (int n = 0; n < L.N; ++n) {
        e.I[n] = L.dims[n];
        e.l[n] = L.l[n];
        e.Q[n] = plan->at<float>(L.qb[n]);
        e.At[n] = plan->at<float>(L.at[n]);
        e.A[n] = A != nullptr ? A[n] : nullptr;
    }
    e.lambda_in = plan->at<float>(L.lam);
    e.lambda_out = lambda;
    e.raw = plan->at<double>(L.raw);
    e.stats = plan->at<double>(L.estats);
    return e;
}

}  // namespace

}  // extern "C"

namespace {

// Deterministic CP-ALS on X (Algorithm 2 with Q_n = I).  A_init: null (the
// eigenvector start by subspace iteration) or N device pointers (modes 1..N-1
// read).
rcp_status cp_als_impl(rcp_plan_t* pl, const float* X, const float* const* A_init,
                       float* const* A, float* lambda, rcp_als_info* info) {
    const Layout& L = pl->L;
    const int N = L.N, R = L.R;
    double* st = pl->at<double>(L.cst);
    double* raw = pl->at<double>(L.raw);
    float* facs = pl->at<float>(L.cfac);
    double* rawn[RCP_MAX_NDIM];
    float* facn[RCP_MAX_NDIM];
    int dims_i[RCP_MAX_NDIM];
    int64_t S = 1;
    {
        int64_t off = 0;
        for (int n = 0; n < N; ++n) {
            rawn[n] = raw + off;
            facn[n] = facs + off;
            off += L.dims[n] * R;
            dims_i[n] = (int)L.dims[n];
            S *= L.dims[n];
        }
    }
    for (int n = 0; n < N; ++n) {
        const double Lm = (double)S / (double)L.dims[n];
        int64_t Rr = 1;
        for (int m = n + 1; m < N; ++m) Rr *= L.dims[m];
        if (Lm / (double)Rr > 4294967295.0 || Rr > 4294967295LL) return RCP_ERR_UNSUPPORTED;
    }
    CpArgs c{};
    c.N = N;
    c.R = R;
    c.max_iters = pl->prob.max_iters;
    c.tol = pl->prob.tol;
    c.state = st;
    c.Y = pl->at<double>(L.y64);
    c.ldy = lp_of(R);
    c.lam_f = pl->at<float>(L.lam);
    c.info = info;
    c.status_word = pl->status_word();
    c.E = pl->at<double>(L.als);
    RCP_TRY(launch_fill_i32((int*)st, 0, 8, pl->stream));
    {
        const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kPmax, (S + 255) / 256));
        RCP_TRY(launch_sumsq(X, S, pl->at<double>(L.sq), nb, st + 3, pl->stream));
    }
    if (A_init == nullptr) {
        // Algorithm 2's initialisation: the leading eigenvectors of X_(n) X_(n)^T by
        // subspace iteration (Algorithm 1's power steps on an l_n-wide block)
        // and Rayleigh-Ritz on the Gram of X x_n Q_n^T
        double* eg = pl->at<double>(L.egram);
        float* B = pl->at<float>(L.cpb);
        float* part = pl->at<float>(L.part);
        for (int n = 1; n < N; ++n) {
            rcp_status r = sketch_impl(pl, X, L.dims, n, pl->at<float>(L.qb[n]), nullptr);
            if (r != RCP_OK) return r;
            r = compress_impl(pl, X, L.dims, n, B);
            if (r != RCP_OK) return r;
            int64_t cur[RCP_MAX_NDIM];
            for (int m = 0; m < N; ++m) cur[m] = L.dims[m];
            cur[n] = L.l[n];
            const StreamGeom g = make_geom(B, cur, N, n);
            const int P = (int)std::max<int64_t>(1, std::min<int64_t>(pl->P, g.ntiles));
            const int LPn = lp_of(L.l[n]);
            float* eye = pl->at<float>(L.qt);
            RCP_TRY(launch_eye(eye, L.l[n], LPn, pl->stream));
            RCP_TRY(launch_power_fused(g, L.l[n], eye, part, P, pl->stream, RCP_PREC_FP32));
            RCP_TRY(launch_reduce_partials(part, P, (int64_t)L.l[n] * LPn,
                                           eg + (size_t)(n - 1) * L.egram_stride, nullptr, 0,
                                           nullptr, pl->stream));
        }
        AlsArgs ai{};
        ai.N = N;
        ai.R = R;
        for (int n = 0; n < N; ++n) {
            ai.l[n] = L.l[n];
            ai.At[n] = pl->at<float>(L.at[n]);
        }
        ai.state = st;
        ai.Y = eg;
        RCP_TRY(launch_als_wide_init(ai, L.egram_stride, pl->stream));
        for (int n = 1; n < N; ++n)
            RCP_TRY(launch_cp_start(pl->at<float>(L.qb[n]), ai.At[n], L.dims[n], L.l[n], R, rawn[n],
                                    facn[n], pl->stream));
    } else {
        for (int n = 1; n < N; ++n)
            RCP_TRY(launch_cp_load(A_init[n], L.dims[n] * R, rawn[n], facn[n], pl->stream));
    }
    for (int n = 1; n < N; ++n) {
        CpArgs g = c;
        g.n = n;
        g.sweep = 0;
        g.I = L.dims[n];
        g.raw = rawn[n];
        g.fac = facn[n];
        RCP_TRY(launch_cp_gram(g, pl->stream));
    }
    const float* fac_c[RCP_MAX_NDIM];
    for (int n = 0; n < N; ++n) fac_c[n] = facn[n];
    float* part = pl->at<float>(L.part);
    const int LPR = lp_of(R);
    for (int it = 1; it <= pl->prob.max_iters; ++it) {
        for (int n = 0; n < N; ++n) {
            const StreamGeom g = make_geom(X, L.dims, N, n);
            const int P = (int)std::max<int64_t>(1, std::min<int64_t>(pl->P, g.ntiles));
            KrSpec kr = kr_spec(N, n, dims_i, R, fac_c, (const int*)st);
            kr.sweep = it;
            RCP_TRY(timed(pl, RCP_KERNEL_MTTKRP, 4.0 * (double)S, 2.0 * (double)S * R,
                          [&] { return launch_mttkrp_full(g, kr, part, P, pl->stream); }));
            RCP_TRY(timed(pl, RCP_KERNEL_REDUCE, (double)P * g.I * LPR * 4.0 + (double)g.I * LPR * 8.0,
                          (double)P * g.I * LPR, [&] {
                              return launch_reduce_partials(part, P, g.I * LPR, pl->at<double>(L.y64),
                                                            nullptr, 0, nullptr, pl->stream);
                          }));
            CpArgs u = c;
            u.n = n;
            u.sweep = it;
            u.I = L.dims[n];
            u.raw = rawn[n];
            u.fac = facn[n];
            RCP_TRY(timed(pl, RCP_KERNEL_CP_UPDATE, (double)g.I * LPR * 8.0 + (double)g.I * R * 12.0,
                          2.0 * (double)g.I * R * R * 2.0, [&] { return launch_cp_update(u, pl->stream); }));
        }
    }
    ExpandArgs e{};
    e.N = N;
    e.R = R;
    for (int n = 0; n < N; ++n) {
        e.I[n] = L.dims[n];
        e.l[n] = (int)L.dims[n];
        e.A[n] = A[n];
    }
    e.lambda_in = pl->at<float>(L.lam);
    e.lambda_out = lambda;
    e.raw = raw;
    e.stats = pl->at<double>(L.estats);
    RCP_TRY(timed(pl, RCP_KERNEL_EXPAND, 0.0, 0.0, [&] { return launch_expand_finish(e, pl->stream); }));
    return RCP_OK;
}

rcp_status decompose_impl(rcp_plan_t* plan, const float* X, float* const* A, float* lambda,
                          rcp_als_info* info) {
    const Layout& L = plan->L;
    const int N = L.N;
    if (plan->prob.solver == RCP_SOLVER_CP_ALS) return cp_als_impl(plan, X, nullptr, A, lambda, info);
    const float* core = nullptr;
    rcp_status st = compress_all(plan, X, &core);
    if (st != RCP_OK) return st;
    float* At[RCP_MAX_NDIM];
    for (int n = 0; n < N; ++n) At[n] = plan->at<float>(L.at[n]);
    float* lam = plan->at<float>(L.lam);
    st = plan->prob.solver == RCP_SOLVER_BCD
             ? bcd_impl(plan, core, At, lam, plan->at<double>(L.norm), info, 0)
             : als_impl(plan, core, At, lam, plan->at<double>(L.norm), info, 0);
    if (st != RCP_OK) return st;
    const float* Qc[RCP_MAX_NDIM];
    const float* Atc[RCP_MAX_NDIM];
    for (int n = 0; n < N; ++n) { Qc[n] = plan->at<float>(L.qb[n]); Atc[n] = At[n]; }
    return expand_impl(plan, Qc, Atc, lam, A, lambda);
}

bool valid_outputs(int N, const float* X, float* const* A, const float* lambda,
                   const rcp_als_info* info) {
    if (X == nullptr || A == nullptr || lambda == nullptr || info == nullptr) return false;
    for (int n = 0; n < N; ++n)
        if (A[n] == nullptr || !aligned(A[n], 4)) return false;
    return aligned(X, 4) && aligned(lambda, 4) && aligned(info, 8);
}

}  // namespace

extern "C" {

rcp_status rcp_decompose(rcp_plan plan, const float* X, float* const* A, float* lambda,
                         rcp_als_info* info) {
    if (plan == nullptr || !valid_outputs(plan->L.N, X, A, lambda, info)) return RCP_ERR_INVALID_ARG;
    return decompose_impl(plan, X, A, lambda, info);
}

rcp_status rcp_cp_als(rcp_plan plan, const float* X, const float* const* A_init, float* const* A,
                      float* lambda, rcp_als_info* info) {
    if (plan == nullptr || !valid_outputs(plan->L.N, X, A, lambda, info) ||
        plan->prob.solver != RCP_SOLVER_CP_ALS)
        return RCP_ERR_INVALID_ARG;
    if (A_init != nullptr)
        for (int n = 1; n < plan->L.N; ++n)
            if (A_init[n] == nullptr || !aligned(A_init[n], 4)) return RCP_ERR_INVALID_ARG;
    return cp_als_impl(plan, X, A_init, A, lambda, info);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free whole path.  Its workspace is this file-scope device array:
// every GPU the library runs on holds its own copy, at its own address, until
// the process ends.  In host code the array's name is only a host-side
// stand-in; the device address comes from hipGetSymbolAddress, taken once per
// device with that device current.
static __device__ __align__(256) unsigned char scratch[RCP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};
int g_scratch_cus[kMaxDevices] = {};

rcp_status scratch_of_current_device(char** ptr, int* cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RCP_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return RCP_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        int c = 0;
        const rcp_status st = device_cus(&c);
        if (st != RCP_OK) return st;
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
            return RCP_ERR_HIP;
        g_scratch[dev] = (char*)p;
        g_scratch_cus[dev] = c;
    }
    *ptr = g_scratch[dev];
    *cus = g_scratch_cus[dev];
    return RCP_OK;
}

}  // namespace

extern "C" {

rcp_status rcp_decompose_noalloc(const rcp_problem* prob, const float* X, float* const* A,
                                 float* lambda, rcp_als_info* info, void* hip_stream) {
    if (prob == nullptr || !valid_problem(prob)) return RCP_ERR_INVALID_ARG;
    if (!valid_outputs(prob->ndim, X, A, lambda, info)) return RCP_ERR_INVALID_ARG;
    const Layout L = make_layout(prob);
    if (!als_supported(L.N, L.l, L.R)) return RCP_ERR_UNSUPPORTED;
    if (L.total > (size_t)RCP_NOALLOC_SCRATCH_BYTES) return RCP_ERR_WORKSPACE;
    char* ws = nullptr;
    int cus = 0;
    rcp_status st = scratch_of_current_device(&ws, &cus);
    if (st != RCP_OK) return st;
    rcp_plan_t pl;
    st = plan_setup(&pl, prob, ws, (size_t)RCP_NOALLOC_SCRATCH_BYTES, hip_stream, cus);
    if (st != RCP_OK) return st;
    // the status word starts at zero (a fill kernel: no memset node under capture)
    RCP_TRY(launch_fill_i32(pl.status_word(), 0, 1, pl.stream));
    return decompose_impl(&pl, X, A, lambda, info);
}

// ---------------------------------------------------------------------------
// Batches of independent problems

constexpr int kBatchStreams = 16;       // branches the problems' compressions are spread over

// One launch of the grouped batched form.
struct GOp {
    enum Kind { SKETCH, REDUCE, QR, POWER } kind;
    int NB = 1, MB = 1, prec = 0;
    bool caseB = false, fused = true;
    size_t lds = 0;                       // QR: the group's largest dynamic LDS
    int count = 0;                        // descriptors
    size_t off = 0;                       // their byte offset in the tables
    int gx = 1, gy = 1;                   // grid maxima (reductions: gx = total workgroups)
};

struct rcp_batch_t {
    int count = 0;
    hipStream_t stream = nullptr;
    hipStream_t side[kBatchStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kBatchStreams] = {};
    std::vector<rcp_plan_t*> plans;
    std::vector<AlsArgs> h_als;           // per-problem arguments, outputs as last bound
    std::vector<int> als_order;           // device table order: estimated ALS work, largest first
    std::vector<ExpandArgs> h_exp;
    AlsArgs* pin_als = nullptr;           // pinned staging of the argument tables
    ExpandArgs* pin_exp = nullptr;
    AlsArgs* d_als = nullptr;             // device argument tables (in the workspace)
    ExpandArgs* d_exp = nullptr;
    bool bound = false;                   // output pointers uploaded at least once
    std::vector<const float*> X;          // inputs of the captured graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool use_graph = false;
    // launch shape (rcp_batch_autotune): side streams in use, workgroups per
    // streaming pass, row-block height of the sketch passes (64-row units)
    int streams = kBatchStreams;
    int workgroups = 0;
    int mb_cap = 8;
    // grouped form (every problem eligible): each step of the range finder is
    // one launch over all problems, reading descriptor tables
    bool grouped = false;
    unsigned char* d_grp = nullptr;       // descriptor tables (workspace)
    unsigned char* pin_grp = nullptr;     // pinned staging
    size_t grp_bytes = 0;
    std::vector<GOp> ops;                 // the launches, in order
    std::vector<const float*> grp_X;      // inputs the tables were built for
    int grp_workgroups = -1, grp_mb_cap = -1;
};

namespace {

struct BatchLayout {
    std::vector<size_t> off, size;
    size_t als = 0, exp = 0, grp = 0, grp_bytes = 0, total = 0;
};

// Whether a problem can take the grouped batched form: the sequential scheme,
// every mode compressed by a generated test matrix, every mode's power step
// in the fused kernel and every QR in its LDS form.  The others keep the
// per-problem chains.
bool grouped_eligible(const rcp_problem* p) {
    if (p->scheme != RCP_SCHEME_SEQUENTIAL || p->test_matrix == RCP_TEST_COLUMNS) return false;
    int64_t cur[RCP_MAX_NDIM];
    for (int n = 0; n < p->ndim; ++n) cur[n] = p->dims[n];
    for (int n = 0; n < p->ndim; ++n) {
        if (!mode_compressed(p, n)) return false;
        const int64_t I = cur[n];
        const int l = (int)mode_width(p, n, I);
        if (!power_fused_fits(I, l, kLdsBytes) || qr_group_lds(I, l) == 0) return false;
        cur[n] = l;
    }
    return true;
}

// bytes of descriptor tables one problem needs in the grouped form
size_t grouped_desc_bytes(const rcp_problem* p) {
    const size_t q = (size_t)p->q;
    return (size_t)p->ndim * (sizeof(SketchDesc) + (1 + q) * sizeof(ReduceDesc) +
                              (q + 1) * sizeof(QrDesc) + (q + 1) * sizeof(PowerDesc));
}

rcp_status batch_layout(const rcp_problem* probs, int32_t count, BatchLayout* out) {
    if (probs == nullptr || count < 1) return RCP_ERR_INVALID_ARG;
    BatchLayout B;
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        if (!valid_problem(&probs[i])) return RCP_ERR_INVALID_ARG;
        if (probs[i].solver != RCP_SOLVER_ALS) return RCP_ERR_UNSUPPORTED;
        const Layout L = make_layout(&probs[i]);
        if (!als_supported(L.N, L.l, L.R)) return RCP_ERR_UNSUPPORTED;
        B.off.push_back(off);
        B.size.push_back(L.total);
        off = align_up(off + L.total);
    }
    B.als = off;
    off = align_up(off + (size_t)count * sizeof(AlsArgs));
    B.exp = off;
    off = align_up(off + (size_t)count * sizeof(ExpandArgs));
    bool grouped = true;
    size_t gb = 0;
    for (int i = 0; i < count; ++i) {
        grouped = grouped && grouped_eligible(&probs[i]);
        gb += grouped_desc_bytes(&probs[i]);
    }
    B.grp = off;
    B.grp_bytes = grouped ? gb : 0;
    off = align_up(off + B.grp_bytes);
    B.total = off;
    *out = B;
    return RCP_OK;
}

// The compressions of the problems go round-robin to the side streams (forked
// from and joined back into the batch stream by events, so a recorded graph
// gets independent branches); CP-ALS and the back-projection of all problems
// then run as one launch each on the batch stream, reading their outputs from
// the device argument tables.
rcp_status batch_enqueue(rcp_batch_t* b, const float* const* X) {
    RCP_TRY(hipEventRecord(b->fork, b->stream));
    for (int s = 0; s < kBatchStreams; ++s) RCP_TRY(hipStreamWaitEvent(b->side[s], b->fork, 0));
    for (int i = 0; i < b->count; ++i) {
        const float* core = nullptr;
        rcp_status st = compress_all(b->plans[i], X[i], &core);
        if (st != RCP_OK) return st;
        if (core != b->h_als[i].B) return RCP_ERR_HIP;   // layout invariant
    }
    for (int s = 0; s < kBatchStreams; ++s) {
        RCP_TRY(hipEventRecord(b->join[s], b->side[s]));
        RCP_TRY(hipStreamWaitEvent(b->stream, b->join[s], 0));
    }
    RCP_TRY(launch_als_batch(b->d_als, b->h_als.data(), b->count, b->stream));
    RCP_TRY(launch_expand_batch(b->d_exp, b->h_exp.data(), b->count, b->stream));
    return RCP_OK;
}

// Binds every problem's plan to the batch's current launch shape.
void batch_apply_shape(rcp_batch_t* b) {
    for (int i = 0; i < b->count; ++i) {
        rcp_plan_t* pl = b->plans[i];
        pl->stream = b->side[i % b->streams];
        pl->P = b->workgroups;
        pl->mb_cap = b->mb_cap;
    }
}

void batch_drop_graph(rcp_batch_t* b) {
    if (b->exec != nullptr) hipGraphExecDestroy(b->exec);
    if (b->graph != nullptr) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

rcp_status batch_check_io(const rcp_batch_t* b, const float* const* X, float* const* const* A,
                          float* const* lambda, const rcp_als_info* info) {
    if (X == nullptr || A == nullptr || lambda == nullptr || info == nullptr || !aligned(info, 8))
        return RCP_ERR_INVALID_ARG;
    for (int i = 0; i < b->count; ++i) {
        if (X[i] == nullptr || !aligned(X[i], 4)) return RCP_ERR_INVALID_ARG;
        if (A[i] == nullptr || lambda[i] == nullptr || !aligned(lambda[i], 4)) return RCP_ERR_INVALID_ARG;
        for (int n = 0; n < b->h_exp[i].N; ++n)
            if (A[i][n] == nullptr || !aligned(A[i][n], 4)) return RCP_ERR_INVALID_ARG;
    }
    return RCP_OK;
}

// Points the argument tables at the given outputs.  Only when they differ
// from the last upload: the batch stream is drained first (an earlier launch
// may still read the tables), then the tables go up in stream order.
rcp_status batch_bind_outputs(rcp_batch_t* b, float* const* const* A, float* const* lambda,
                              rcp_als_info* info) {
    bool same = b->bound;
    for (int i = 0; same && i < b->count; ++i) {
        same = b->h_als[i].info == info + i && b->h_exp[i].lambda_out == lambda[i];
        for (int n = 0; same && n < b->h_exp[i].N; ++n) same = b->h_exp[i].A[n] == A[i][n];
    }
    if (same) return RCP_OK;
    RCP_TRY(hipStreamSynchronize(b->stream));
    for (int i = 0; i < b->count; ++i) {
        b->h_als[i].info = info + i;
        b->h_exp[i].lambda_out = lambda[i];
        for (int n = 0; n < b->h_exp[i].N; ++n) b->h_exp[i].A[n] = A[i][n];
    }
    for (int j = 0; j < b->count; ++j) b->pin_als[j] = b->h_als[b->als_order[j]];
    std::memcpy(b->pin_exp, b->h_exp.data(), b->count * sizeof(ExpandArgs));
    RCP_TRY(hipMemcpyAsync(b->d_als, b->pin_als, b->count * sizeof(AlsArgs), hipMemcpyHostToDevice,
                           b->stream));
    RCP_TRY(hipMemcpyAsync(b->d_exp, b->pin_exp, b->count * sizeof(ExpandArgs),
                           hipMemcpyHostToDevice, b->stream));
    b->bound = true;
    return RCP_OK;
}

// The grouped program: the steps of compress_all (sketch_impl and
// compress_impl) for every problem, round by round (mode n, then each power
// iteration), each round's descriptors split by kernel instantiation into
// one launch each.  Every problem gets the arguments and workgroup partition
// of its own single-problem launches, so its results are the same bits.
extern "C++" {
template <typename D>
struct GStep {
    struct Item { int NB, MB, prec; bool caseB, fused; size_t lds; D d; int gx, gy; double work = 0.0; };
    std::vector<Item> items;
};

template <typename D>
void gstep_emit(GStep<D>& st, GOp::Kind kind, std::vector<GOp>& ops, std::vector<unsigned char>& blob) {
    std::vector<bool> used(st.items.size(), false);
    for (size_t i = 0; i < st.items.size(); ++i) {
        if (used[i]) continue;
        const auto& a = st.items[i];
        GOp op;
        op.kind = kind;
        op.NB = a.NB; op.MB = a.MB; op.prec = a.prec; op.caseB = a.caseB; op.fused = a.fused;
        op.off = blob.size();
        // the launch's descriptors by work per workgroup, largest first:
        // workgroups dispatch in descriptor (blockIdx.z) order, so the
        // longest start first; each problem's arithmetic is unchanged
        std::vector<size_t> members;
        for (size_t j = i; j < st.items.size(); ++j) {
            const auto& c = st.items[j];
            if (used[j] || c.NB != a.NB || c.MB != a.MB || c.prec != a.prec || c.caseB != a.caseB ||
                c.fused != a.fused)
                continue;
            used[j] = true;
            members.push_back(j);
        }
        std::stable_sort(members.begin(), members.end(),
                         [&](size_t x, size_t y) { return st.items[x].work > st.items[y].work; });
        for (size_t j : members) {
            const auto& c = st.items[j];
            const unsigned char* src = (const unsigned char*)&c.d;
            blob.insert(blob.end(), src, src + sizeof(D));
            ++op.count;
            op.gx = std::max(op.gx, c.gx);
            op.gy = std::max(op.gy, c.gy);
            op.lds = std::max(op.lds, c.lds);
        }
        ops.push_back(op);
    }
    st.items.clear();
}
}  // extern "C++"

void batch_build_program(rcp_batch_t* b, const float* const* X, std::vector<unsigned char>& blob) {
    b->ops.clear();
    blob.clear();
    const int count = b->count;
    std::vector<const float*> T(count);
    std::vector<std::array<int64_t, RCP_MAX_NDIM>> cur(count);
    std::vector<int> comp(count, 0);
    int Nmax = 0, qmax = 0;
    for (int i = 0; i < count; ++i) {
        const rcp_plan_t* pl = b->plans[i];
        T[i] = X[i];
        for (int n = 0; n < pl->L.N; ++n) cur[i][n] = pl->L.dims[n];
        Nmax = std::max(Nmax, pl->L.N);
        qmax = std::max(qmax, pl->prob.q);
    }
    GStep<SketchDesc> sk;
    GStep<ReduceDesc> rd;
    GStep<QrDesc> qr;
    GStep<PowerDesc> pw;
    for (int n = 0; n < Nmax; ++n) {
        struct ModeGeo { StreamGeom g; int l, LP, NB, P; };
        std::vector<ModeGeo> mg(count);
        for (int i = 0; i < count; ++i) {
            rcp_plan_t* pl = b->plans[i];
            if (n >= pl->L.N) continue;
            const Layout& L = pl->L;
            const int64_t I = cur[i][n];
            ModeGeo& m = mg[i];
            m.l = (int)std::min<int64_t>(pl->prob.k + mode_oversampling(&pl->prob, n), I);
            m.LP = lp_of(m.l);
            m.NB = m.LP / 16;
            m.g = make_geom(T[i], cur[i].data(), L.N, n);
            m.P = (int)std::max<int64_t>(1, std::min<int64_t>(pl->P, m.g.ntiles));
            // sketch (Algorithm 1), as launch_contract_out with Z == null
            int MBv = (int)((I + 63) / 64);
            if (I <= 512 && MBv > pl->mb_cap) MBv = pl->mb_cap;
            MBv = std::max(1, std::min(8, MBv));
            const int nIB = (int)((I + 64 * MBv - 1) / (64 * MBv));
            SketchDesc d{};
            d.g = m.g;
            d.Z = nullptr;
            d.part = pl->at<float>(L.part);
            d.sq_part = (n == 0) ? pl->at<double>(L.sq) : nullptr;
            d.seed = pl->prob.seed;
            d.tag = omega_stream_tag(0, (uint32_t)n);
            d.okind = pl->prob.test_matrix;
            d.l = m.l;
            d.P = m.P;
            d.nIB = nIB;
            sk.items.push_back({m.NB, MBv, pl->prob.precision, m.g.caseB != 0, false, 0, d, m.P, nIB,
                                (double)((m.g.ntiles + m.P - 1) / m.P) * (double)(64 * MBv)});
            ReduceDesc r{};
            r.part = pl->at<float>(L.part);
            r.Y = pl->at<double>(L.y64);
            r.sq_part = d.sq_part;
            r.sq_out = (n == 0) ? pl->at<double>(L.norm) : nullptr;
            r.count = I * m.LP;
            r.P = m.P;
            r.ny = reduce_split(m.P);
            r.nsq = m.P * nIB;
            rd.items.push_back({0, 0, 0, false, false, 0, r, 1, 1});
        }
        gstep_emit(sk, GOp::SKETCH, b->ops, blob);
        gstep_emit(rd, GOp::REDUCE, b->ops, blob);
        auto add_qr = [&](int i, bool final_basis) {
            rcp_plan_t* pl = b->plans[i];
            const Layout& L = pl->L;
            const ModeGeo& m = mg[i];
            QrDesc d{};
            d.Y = pl->at<double>(L.y64);
            d.m = (int)cur[i][n];
            d.n = m.l;
            d.ldy = m.LP;
            d.Qpad = pl->at<float>(L.qt);
            d.ldq = m.LP;
            d.Qout = final_basis ? pl->at<float>(L.qb[n]) : nullptr;
            d.second_pass = final_basis ? 1 : 0;
            d.status = pl->status_word();
            qr.items.push_back({(m.l + 15) >> 4, 0, 0, false, false, qr_group_lds(d.m, d.n), d, 1, 1,
                                (double)d.m * d.n * d.n});
        };
        for (int it = 0; it < qmax; ++it) {
            for (int i = 0; i < count; ++i) {
                rcp_plan_t* pl = b->plans[i];
                if (n >= pl->L.N || it >= pl->prob.q) continue;
                add_qr(i, false);
                const ModeGeo& m = mg[i];
                PowerDesc d{};
                d.g = m.g;
                d.Qt = pl->at<float>(pl->L.qt);
                d.part = pl->at<float>(pl->L.part);
                d.out = nullptr;
                d.P = m.P;
                pw.items.push_back({m.NB, (int)((cur[i][n] + 63) / 64), pl->prob.precision,
                                    m.g.caseB != 0, true, 0, d, m.P, 1,
                                    (double)((m.g.ntiles + m.P - 1) / m.P) * (double)cur[i][n]});
                ReduceDesc r{};
                r.part = pl->at<float>(pl->L.part);
                r.Y = pl->at<double>(pl->L.y64);
                r.count = cur[i][n] * m.LP;
                r.P = m.P;
                r.ny = reduce_split(m.P);
                rd.items.push_back({0, 0, 0, false, false, 0, r, 1, 1});
            }
            gstep_emit(qr, GOp::QR, b->ops, blob);
            gstep_emit(pw, GOp::POWER, b->ops, blob);
            gstep_emit(rd, GOp::REDUCE, b->ops, blob);
        }
        for (int i = 0; i < count; ++i)
            if (n < b->plans[i]->L.N) add_qr(i, true);
        gstep_emit(qr, GOp::QR, b->ops, blob);
        // the mode product T x_n Q^T (Algorithm 1's projection), float32 operands,
        // as compress_impl's resident-basis kernel
        for (int i = 0; i < count; ++i) {
            rcp_plan_t* pl = b->plans[i];
            if (n >= pl->L.N) continue;
            const ModeGeo& m = mg[i];
            float* out = pl->at<float>(pl->L.tb[comp[i] % 2]);
            PowerDesc d{};
            d.g = m.g;
            d.Qt = pl->at<float>(pl->L.qt);
            d.part = nullptr;
            d.out = out;
            d.P = m.P;
            d.lout = m.l;
            pw.items.push_back({m.NB, (int)((cur[i][n] + 63) / 64), RCP_PREC_FP32, m.g.caseB != 0, false,
                                0, d, m.P, 1, (double)((m.g.ntiles + m.P - 1) / m.P) * (double)cur[i][n]});
            cur[i][n] = m.l;
            T[i] = out;
            ++comp[i];
        }
        gstep_emit(pw, GOp::POWER, b->ops, blob);
    }
    // the grouped reductions number their problems' workgroups consecutively
    for (GOp& op : b->ops) {
        if (op.kind != GOp::REDUCE) continue;
        int64_t blocks = 0;
        for (int i = 0; i < op.count; ++i) {
            unsigned char* at = blob.data() + op.off + (size_t)i * sizeof(ReduceDesc);
            ReduceDesc r;
            std::memcpy(&r, at, sizeof r);
            r.blk0 = (int)blocks;
            blocks += reduce_blocks(r.count);
            std::memcpy(at, &r, sizeof r);
        }
        op.gx = (int)blocks;
    }
}

rcp_status batch_enqueue_grouped(rcp_batch_t* b) {
    for (const GOp& op : b->ops) {
        const unsigned char* d = b->d_grp + op.off;
        switch (op.kind) {
            case GOp::SKETCH:
                RCP_TRY(launch_sketch_group((const SketchDesc*)d, op.count, op.gx, op.gy, op.NB, op.MB,
                                            op.caseB, false, op.prec, b->stream));
                break;
            case GOp::REDUCE:
                RCP_TRY(launch_reduce_group((const ReduceDesc*)d, op.count, op.gx,
                                            b->stream));
                break;
            case GOp::QR:
                RCP_TRY(launch_qr_group((const QrDesc*)d, op.count, op.NB, true, op.lds, b->stream));
                break;
            case GOp::POWER:
                RCP_TRY(launch_power_group((const PowerDesc*)d, op.count, op.gx, op.NB, op.MB, op.fused,
                                           op.caseB, op.prec, b->stream));
                break;
        }
    }
    RCP_TRY(launch_als_batch(b->d_als, b->h_als.data(), b->count, b->stream));
    RCP_TRY(launch_expand_batch(b->d_exp, b->h_exp.data(), b->count, b->stream));
    return RCP_OK;
}

// (Re)builds and uploads the grouped tables when the inputs or the launch
// shape changed; the batch stream is drained first (a launch in flight may
// still read them).
rcp_status batch_bind_grouped(rcp_batch_t* b, const float* const* X) {
    bool same = (int)b->grp_X.size() == b->count && b->grp_workgroups == b->workgroups &&
                b->grp_mb_cap == b->mb_cap;
    for (int i = 0; same && i < b->count; ++i) same = b->grp_X[i] == X[i];
    if (same) return RCP_OK;
    std::vector<unsigned char> blob;
    batch_build_program(b, X, blob);
    if (blob.size() > b->grp_bytes) return RCP_ERR_WORKSPACE;
    RCP_TRY(hipStreamSynchronize(b->stream));
    std::memcpy(b->pin_grp, blob.data(), blob.size());
    RCP_TRY(hipMemcpyAsync(b->d_grp, b->pin_grp, blob.size(), hipMemcpyHostToDevice, b->stream));
    RCP_TRY(hipStreamSynchronize(b->stream));
    b->grp_X.assign(X, X + b->count);
    b->grp_workgroups = b->workgroups;
    b->grp_mb_cap = b->mb_cap;
    return RCP_OK;
}

rcp_status batch_run(rcp_batch_t* batch, const float* const* X) {
    if (batch->grouped) {
        const rcp_status sb = batch_bind_grouped(batch, X);
        if (sb != RCP_OK) return sb;
    }
    auto enqueue = [&]() {
        return batch->grouped ? batch_enqueue_grouped(batch) : batch_enqueue(batch, X);
    };
    if (!batch->use_graph) return enqueue();
    bool same = batch->exec != nullptr && (int)batch->X.size() == batch->count;
    for (int i = 0; same && i < batch->count; ++i) same = batch->X[i] == X[i];
    if (!same) {
        batch_drop_graph(batch);
        if (hipStreamBeginCapture(batch->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
            batch->use_graph = false;
            return enqueue();
        }
        const rcp_status st = enqueue();
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(batch->stream, &g);
        if (st != RCP_OK) {
            if (g != nullptr) hipGraphDestroy(g);
            return st;
        }
        if (ec != hipSuccess || g == nullptr) return RCP_ERR_HIP;
        batch->graph = g;
        if (hipGraphInstantiate(&batch->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            batch_drop_graph(batch);
            return RCP_ERR_HIP;
        }
        batch->X.assign(X, X + batch->count);
    }
    RCP_TRY(hipGraphLaunch(batch->exec, batch->stream));
    return RCP_OK;
}

}  // namespace

rcp_status rcp_batch_workspace_size(const rcp_problem* probs, int32_t count, size_t* bytes) {
    if (bytes == nullptr) return RCP_ERR_INVALID_ARG;
    BatchLayout B;
    rcp_status st = batch_layout(probs, count, &B);
    if (st != RCP_OK) return st;
    *bytes = B.total;
    return RCP_OK;
}

rcp_status rcp_batch_init(rcp_batch* batch, const rcp_problem* probs, int32_t count,
                          void* workspace, size_t workspace_bytes, void* hip_stream) {
    if (batch == nullptr) return RCP_ERR_INVALID_ARG;
    *batch = nullptr;
    BatchLayout B;
    rcp_status st = batch_layout(probs, count, &B);
    if (st != RCP_OK) return st;
    if (workspace == nullptr || workspace_bytes < B.total || !aligned(workspace, kAlign))
        return RCP_ERR_WORKSPACE;
    rcp_batch_t* b = new (std::nothrow) rcp_batch_t;
    if (b == nullptr) return RCP_ERR_HIP;
    b->count = count;
    b->stream = (hipStream_t)hip_stream;
    bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
    for (int s = 0; ok && s < kBatchStreams; ++s)
        ok = hipStreamCreateWithFlags(&b->side[s], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&b->join[s], hipEventDisableTiming) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&b->pin_als, count * sizeof(AlsArgs), hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&b->pin_exp, count * sizeof(ExpandArgs), hipHostMallocDefault) == hipSuccess;
    if (!ok) { rcp_batch_destroy(b); return RCP_ERR_HIP; }
    char* ws = (char*)workspace;
    for (int i = 0; i < count; ++i) {
        rcp_plan pl = nullptr;
        st = rcp_init(&pl, &probs[i], ws + B.off[i], B.size[i], b->side[i % kBatchStreams]);
        if (st != RCP_OK) { rcp_batch_destroy(b); return st; }
        b->plans.push_back(pl);
        const float* core = core_location(pl);
        b->h_als.push_back(core_als_args(pl, core, nullptr));
        b->h_exp.push_back(core_expand_args(pl, nullptr, nullptr));
    }
    // The ALS launch runs one workgroup per problem, about two problems per
    // CU: the device table lists them by estimated work (core size x R x
    // sweeps), largest first, so the longest ones start in the first wave
    // (longest-processing-time order).  Each entry carries its own buffers.
    {
        std::vector<double> work(count);
        for (int i = 0; i < count; ++i) {
            const AlsArgs& a = b->h_als[i];
            double S = 1.0;
            for (int n = 0; n < a.N; ++n) S *= a.l[n];
            work[i] = S * a.R * a.max_iters;
        }
        b->als_order.resize(count);
        for (int i = 0; i < count; ++i) b->als_order[i] = i;
        std::stable_sort(b->als_order.begin(), b->als_order.end(),
                         [&](int x, int y) { return work[x] > work[y]; });
    }
    // the plans' status words are cleared on the side streams: the batch
    // stream waits for that before its first use of the workspace
    for (int s = 0; ok && s < kBatchStreams; ++s)
        ok = hipEventRecord(b->join[s], b->side[s]) == hipSuccess &&
             hipStreamWaitEvent(b->stream, b->join[s], 0) == hipSuccess;
    if (!ok) { rcp_batch_destroy(b); return RCP_ERR_HIP; }
    b->d_als = (AlsArgs*)(ws + B.als);
    b->d_exp = (ExpandArgs*)(ws + B.exp);
    if (B.grp_bytes > 0) {
        b->grouped = true;
        b->d_grp = (unsigned char*)(ws + B.grp);
        b->grp_bytes = B.grp_bytes;
        if (hipHostMalloc((void**)&b->pin_grp, B.grp_bytes, hipHostMallocDefault) != hipSuccess) {
            rcp_batch_destroy(b);
            return RCP_ERR_HIP;
        }
    }
    b->use_graph = hip_stream != nullptr;
    b->workgroups = b->plans[0]->P;
    *batch = b;
    return RCP_OK;
}

rcp_status rcp_batch_decompose(rcp_batch batch, const float* const* X, float* const* const* A,
                               float* const* lambda, rcp_als_info* info) {
    if (batch == nullptr) return RCP_ERR_INVALID_ARG;
    rcp_status st = batch_check_io(batch, X, A, lambda, info);
    if (st != RCP_OK) return st;
    st = batch_bind_outputs(batch, A, lambda, info);
    if (st != RCP_OK) return st;
    return batch_run(batch, X);
}

rcp_status rcp_batch_read_status(rcp_batch batch, int32_t index, int32_t* status) {
    if (batch == nullptr || index < 0 || index >= batch->count) return RCP_ERR_INVALID_ARG;
    RCP_TRY(hipStreamSynchronize(batch->stream));
    return rcp_read_status(batch->plans[index], status);
}

rcp_status rcp_batch_get_core(rcp_batch batch, int32_t index, float** core, int64_t* core_dims) {
    if (batch == nullptr || index < 0 || index >= batch->count) return RCP_ERR_INVALID_ARG;
    return rcp_get_core(batch->plans[index], core, core_dims);
}

constexpr double kAutotuneGain = 0.97;

// Coordinate search over the launch shape: each knob in turn takes every
// candidate value with the others at their best so far; each candidate is
// recorded (graph) once and timed over two replays.
rcp_status rcp_batch_autotune(rcp_batch batch, const float* const* X, float* const* const* A,
                              float* const* lambda, rcp_als_info* info, int32_t* shape,
                              double* best_ms) {
    if (batch == nullptr || shape == nullptr || best_ms == nullptr) return RCP_ERR_INVALID_ARG;
    rcp_status st = batch_check_io(batch, X, A, lambda, info);
    if (st != RCP_OK) return st;
    st = batch_bind_outputs(batch, A, lambda, info);
    if (st != RCP_OK) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0 != nullptr) (void)hipEventDestroy(e0);
        return RCP_ERR_HIP;
    }
    const int cus_default = batch->plans[0]->P;
    int best[3] = {batch->streams, batch->workgroups, batch->mb_cap};
    double best_t = -1.0;
    auto measure = [&](const int* c, double* ms) -> rcp_status {
        batch->streams = c[0];
        batch->workgroups = c[1];
        batch->mb_cap = c[2];
        batch_apply_shape(batch);
        batch_drop_graph(batch);
        rcp_status r = batch_run(batch, X);         // records the graph
        if (r != RCP_OK) return r;
        if (hipEventRecord(e0, batch->stream) != hipSuccess) return RCP_ERR_HIP;
        for (int rep = 0; rep < 2 && r == RCP_OK; ++rep) r = batch_run(batch, X);
        if (r != RCP_OK) return r;
        if (hipEventRecord(e1, batch->stream) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess)
            return RCP_ERR_HIP;
        float t = 0.0f;
        if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) return RCP_ERR_HIP;
        *ms = t / 2.0;
        return RCP_OK;
    };
    st = measure(best, &best_t);
    const int cand_s[] = {4, 8, kBatchStreams};
    const int cand_p[] = {16, 32, 64, 128, cus_default};
    const int cand_m[] = {1, 2, 4, 8};
    const int* cands[3] = {cand_s, cand_p, cand_m};
    const int ncand[3] = {3, 5, 4};
    // the grouped form runs on the batch stream alone: no stream knob
    for (int knob = batch->grouped ? 1 : 0; knob < 3 && st == RCP_OK; ++knob) {
        for (int c = 0; c < ncand[knob] && st == RCP_OK; ++c) {
            int trial[3] = {best[0], best[1], best[2]};
            if (trial[knob] == cands[knob][c]) continue;
            trial[knob] = cands[knob][c];
            double t = 0.0;
            st = measure(trial, &t);
            // two replays time a candidate to a few percent: only a clear gain moves the shape
            if (st == RCP_OK && t < kAutotuneGain * best_t) {
                best_t = t;
                for (int k = 0; k < 3; ++k) best[k] = trial[k];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    batch->streams = best[0];
    batch->workgroups = best[1];
    batch->mb_cap = best[2];
    batch_apply_shape(batch);
    batch_drop_graph(batch);
    if (st != RCP_OK) return st;
    for (int k = 0; k < 3; ++k) shape[k] = best[k];
    *best_ms = best_t;
    return RCP_OK;
}

rcp_status rcp_batch_destroy(rcp_batch batch) {
    if (batch == nullptr) return RCP_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(batch->stream);
    batch_drop_graph(batch);
    for (rcp_plan_t* p : batch->plans) rcp_destroy(p);
    for (int s = 0; s < kBatchStreams; ++s) {
        if (batch->side[s] != nullptr) hipStreamDestroy(batch->side[s]);
        if (batch->join[s] != nullptr) hipEventDestroy(batch->join[s]);
    }
    if (batch->fork != nullptr) hipEventDestroy(batch->fork);
    if (batch->pin_als != nullptr) hipHostFree(batch->pin_als);
    if (batch->pin_exp != nullptr) hipHostFree(batch->pin_exp);
    if (batch->pin_grp != nullptr) hipHostFree(batch->pin_grp);
    delete batch;
    return RCP_OK;
}

rcp_status rcp_get_bases(rcp_plan plan, float** Q) {
    if (plan == nullptr || Q == nullptr) return RCP_ERR_INVALID_ARG;
    if (plan->prob.solver == RCP_SOLVER_CP_ALS) return RCP_ERR_UNSUPPORTED;
    for (int n = 0; n < plan->L.N; ++n) Q[n] = plan->at<float>(plan->L.qb[n]);
    return RCP_OK;
}

rcp_status rcp_get_core(rcp_plan plan, float** core, int64_t* core_dims) {
    if (plan == nullptr || core == nullptr) return RCP_ERR_INVALID_ARG;
    if (plan->prob.solver == RCP_SOLVER_CP_ALS) return RCP_ERR_UNSUPPORTED;
    *core = core_location(plan);
    if (core_dims != nullptr)
        for (int n = 0; n < plan->L.N; ++n) core_dims[n] = plan->L.core_dims[n];
    return RCP_OK;
}

rcp_status rcp_debug_omega(rcp_plan plan, int32_t mode, int64_t row0, int64_t nrows, int32_t l,
                           float* omega) {
    if (plan == nullptr || omega == nullptr || mode < 0 || mode >= 256 || row0 < 0 || nrows < 0 ||
        l < 1 || l > RCP_MAX_L)
        return RCP_ERR_INVALID_ARG;
    if (!aligned(omega, 4) || plan->prob.test_matrix == RCP_TEST_COLUMNS) return RCP_ERR_INVALID_ARG;
    RCP_TRY(launch_omega(plan->prob.seed, omega_stream_tag(0, (uint32_t)mode), plan->prob.test_matrix,
                         row0, nrows, l, omega, plan->stream));
    return RCP_OK;
}

rcp_status rcp_debug_columns(rcp_plan plan, int32_t mode, int64_t J, int32_t l, int64_t* idx) {
    if (plan == nullptr || idx == nullptr || mode < 0 || mode >= 256 || l < 1 || l > RCP_MAX_L ||
        J < l || !aligned(idx, 8))
        return RCP_ERR_INVALID_ARG;
    RCP_TRY(launch_select_columns(plan->prob.seed, omega_stream_tag(0, (uint32_t)mode), J, l, idx,
                                  plan->stream));
    return RCP_OK;
}

rcp_status rcp_debug_philox(rcp_plan plan, int32_t mode, int64_t row0, int64_t nrows,
                            int32_t ngroups, uint32_t* words) {
    if (plan == nullptr || words == nullptr || mode < 0 || mode >= 256 || row0 < 0 || nrows < 0 ||
        ngroups < 1 || ngroups > RCP_MAX_L / 4)
        return RCP_ERR_INVALID_ARG;
    if (!aligned(words, 4)) return RCP_ERR_INVALID_ARG;
    RCP_TRY(launch_philox_words(plan->prob.seed, omega_stream_tag(0, (uint32_t)mode), row0, nrows,
                                ngroups, words, plan->stream));
    return RCP_OK;
}

}  // extern "C"
