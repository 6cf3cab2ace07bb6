// Internal launch interface between the host library and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rcp.h"

namespace rcp {

// Mode-n view (L, I, Rr) of a C-order tensor and its column tiling.
struct StreamGeom {
    const float* T;
    int64_t L, I, Rr;
    int32_t caseB;         // 0: tiles are b-runs inside one a; 1: tiles are TA whole a-slabs
    int32_t TA;
    int32_t vec4;          // case A rows can be read as aligned float4
    int32_t pad_;
    int64_t tiles_per_a;   // case A
    int64_t ntiles;
    int64_t Is;            // rows between consecutive a-slabs in memory (I unless a row slice)
};

StreamGeom make_geom(const float* T, const int64_t* dims, int ndim, int mode);

// Grouped launches: one launch runs the same step for many problems, each
// workgroup reading its problem's arguments from a device table (blockIdx.z
// for the streaming kernels and the reductions, blockIdx.x for the QR).
// Workgroups past a problem's own grid return at once, so every problem
// gets exactly the partition (P workgroups, nIB row blocks) that its
// single-problem launch would use.
struct SketchDesc {            // k_contract_out with a generated test matrix
    StreamGeom g;
    const float* Z;            // stored Z (two-pass power step) or null (sketch)
    float* part;
    double* sq_part;           // null: no sum of squares
    uint64_t seed;
    uint32_t tag;
    int okind, l, P, nIB;
};
struct PowerDesc {             // k_power_fused (fused power step or mode product)
    StreamGeom g;
    const float* Qt;
    float* part;
    float* out;
    int P, lout, accumulate, pad_;
};
struct ReduceDesc {            // k_reduce_grp
    const float* part;
    double* Y;
    const double* sq_part;
    double* sq_out;
    int64_t count;
    int P, ny, nsq;
    int blk0;                  // grouped launch: the problem's first workgroup
};
struct QrDesc {                // k_qr
    double* Y;
    float* Qpad;
    float* Qout;
    int* status;
    int m, n, ldy, ldq, second_pass, pad_;
};
// grid maxima of a group: gx workgroups along the tiles, gy row blocks (or
// reduction splits), count descriptors; key = the template instantiation
hipError_t launch_sketch_group(const SketchDesc* d, int count, int gx, int gy, int NB, int MB,
                               bool caseB, bool stored, int precision, hipStream_t s);
hipError_t launch_power_group(const PowerDesc* d, int count, int gx, int NB, int MB, bool fused,
                              bool caseB, int precision, hipStream_t s);
// blocks = the sum of reduce_blocks(d[i].count), d[i].blk0 the running sum
hipError_t launch_reduce_group(const ReduceDesc* d, int count, int64_t blocks, hipStream_t s);
hipError_t launch_qr_group(const QrDesc* d, int count, int NB, bool use_lds, size_t lds,
                           hipStream_t s);
size_t qr_group_lds(int64_t m, int n);
hipError_t launch_sketch_group_lp(const SketchDesc* d, int count, int gx, int gy, int NB, int MB,
                                  bool caseB, bool stored, int precision, hipStream_t s);
hipError_t launch_power_group_lp(const PowerDesc* d, int count, int gx, int NB, int MB, bool fused,
                                 bool caseB, int precision, hipStream_t s);

// streaming contractions (stream_kernels.hip)
// precision: matrix-core operand type of the contraction (RCP_PREC_*)
// mb_cap: at most 64 * mb_cap rows per row block for modes of at most 512
// rows (a tile shape the batched form's autotuner chooses; taller modes
// always take 512-row blocks)
// okind: the test matrix generated for a sketch (kOmega*, Z == null)
hipError_t launch_contract_out(const StreamGeom& g, int l, const float* Z, uint64_t seed,
                               uint32_t tag, int okind, float* part, int P, double* sq_part,
                               hipStream_t s, int precision, int mb_cap = 8);
int contract_out_row_blocks(int64_t I, int mb_cap = 8);
bool power_fused_fits(int64_t I, int l, size_t smem_limit);
hipError_t launch_power_fused(const StreamGeom& g, int l, const float* Qt, float* part, int P,
                              hipStream_t s, int precision);
hipError_t launch_contract_in(const StreamGeom& g, int l, const float* Qpadded, int lout,
                              float* out, int P, hipStream_t s, int precision);
// the 16-bit operand instantiations (stream_kernels_lp.hip)
hipError_t launch_contract_out_lp(int precision, const StreamGeom& g, int l, const float* Z,
                                  uint64_t seed, uint32_t tag, int okind, float* part, int P,
                                  double* sq_part, hipStream_t s, int mb_cap);
hipError_t launch_power_fused_lp(int precision, const StreamGeom& g, int l, const float* Qt,
                                 float* part, int P, hipStream_t s);
hipError_t launch_contract_in_lp(int precision, const StreamGeom& g, int l, const float* Qpadded,
                                 int lout, float* out, int P, hipStream_t s);
// Khatri-Rao operand of the mode-n product of the core: column j of the
// unfolding B_(n) is a mixed-radix number whose digits index the rows of the
// other modes' factors; entry (j, c) of the operand is the product of those
// rows' entries in column c (zero for c >= R).  Digits come out of j by
// division by invariant integers (multiply-high and shift, Granlund and
// Montgomery 1994), set up on the host by kr_spec().
struct KrSpec {
    int N, n, R, ftotal;                // ftotal: floats of all factors, packed
    int l[RCP_MAX_NDIM];
    int foff[RCP_MAX_NDIM];             // offset of factor m in the packed copy
    uint32_t mul[RCP_MAX_NDIM];
    uint32_t shr[RCP_MAX_NDIM];
    const float* fac[RCP_MAX_NDIM];     // l_m x R, row-major (device)
    const int* skip;                    // *skip != 0 and sweep > *skip: the launch does nothing
    int sweep;                          // the sweep this launch belongs to (INT_MAX: any stop)
};
KrSpec kr_spec(int N, int n, const int* l, int R, const float* const* fac, const int* skip);
// partial M = B_(n) KR (per workgroup, I x 16*ceil(R/16)) for the reduction
hipError_t launch_mttkrp(const StreamGeom& g, const KrSpec& kr, float* part, int P, hipStream_t s);
// the same for any mode size (row blocks of up to 512 rows, grid P x blocks),
// the factors read from global memory: partials P x I x 16*ceil(R/16)
hipError_t launch_mttkrp_full(const StreamGeom& g, const KrSpec& kr, float* part, int P,
                              hipStream_t s);
// p[0..n) <- v (a kernel, not a memset node, so that it can sit in a captured graph)
hipError_t launch_fill_i32(int* p, int v, int64_t n, hipStream_t s);
// Qpad (I x ldq) <- the identity padded with zero columns
hipError_t launch_eye(float* Qpad, int64_t I, int ldq, hipStream_t s);
int reduce_split(int P);
int64_t reduce_blocks(int64_t count);
// Y[e] = sum over the P partials (rows of count floats) in float64, in a fixed
// order; optionally *sq_out = the sum of the nsq sum-of-squares partials
hipError_t launch_reduce_partials(const float* part, int P, int64_t count, double* Y,
                                  const double* sq_part, int nsq, double* sq_out, hipStream_t s);
hipError_t launch_sumsq(const float* x, int64_t count, double* part, int nblocks, double* out,
                        hipStream_t s);
hipError_t launch_omega(uint64_t seed, uint32_t tag, int okind, int64_t row0, int64_t nrows,
                        int l, float* out, hipStream_t s);
// the COLUMNS test matrix: l <= 64 sorted distinct indices out of J, and the
// sketch made of those unfolding columns (I x ldy float64, zero past l)
hipError_t launch_select_columns(uint64_t seed, uint32_t tag, int64_t J, int l, int64_t* idx,
                                 hipStream_t s);
hipError_t launch_gather_columns(const StreamGeom& g, int l, const int64_t* idx, double* Y, int ldy,
                                 hipStream_t s);
// the raw Philox4x32-10 words behind rows [row0, row0 + nrows) of Omega:
// out[(r * ngroups + g) * 4 + i] is word i of column group g of row row0 + r
hipError_t launch_philox_words(uint64_t seed, uint32_t tag, int64_t row0, int64_t nrows,
                               int ngroups, uint32_t* out, hipStream_t s);
hipError_t launch_pad_q(const float* Q, int64_t I, int l, float* Qpad, int ldq, hipStream_t s);
constexpr uint32_t omega_stream_tag(uint32_t batch, uint32_t mode) { return (batch << 8) | (mode & 0xFFu); }

// small dense kernels (qr_kernel.hip)
// QR of the m x n float64 matrix Y (row stride ldy, overwritten): two
// Cholesky QR passes (the first shifted), a third for the returned basis
// (final_basis), Householder when a pivot vanishes.  Writes Q (diag(R) > 0) as
// float32 into Qpad (m x ldq, columns >= n zeroed) and, if non-null, into
// Qout (m x n).  status (device, may be null): RCP_INFO_QR_HOUSEHOLDER is
// or-ed in when the Householder fallback runs.
// work: device scratch of qr_tall_work_doubles(m, n) doubles for bases too
// tall for one workgroup's LDS (the row-block form); null: one workgroup
hipError_t launch_qr(double* Y, int64_t m, int n, int ldy, float* Qpad, int ldq, float* Qout,
                     bool final_basis, int* status, hipStream_t s, double* work = nullptr);
size_t qr_tall_work_doubles(int64_t m, int n);

// CP-ALS on the core (als_kernel.hip)
struct AlsArgs {
    const float* B;            // core, dims l[0..N-1]
    int N;
    int l[RCP_MAX_NDIM];
    int R;
    int max_iters;
    int warm;                  // nonzero: At[1..N-1] hold the starting factors (no eigenvector start)
    double tol;
    const double* normX2;      // may be null
    float* At[RCP_MAX_NDIM];   // l_n x R outputs
    float* lambda;             // R
    rcp_als_info* info;
    int* status_word;          // the plan's device status word (RCP_INFO_* or-ed in), may be null
    // workspace
    double* Ebuf;              // Jacobi scratch (2 x 64 x 64), then M_n (l_max x R)
    // grid-wide form (cores larger than LDS): reduced mode product or Gram
    // (l_n x ldy float64) and the sweep state (als_state_doubles)
    const double* Y;
    int ldy;
    double* state;
};
hipError_t launch_als(const AlsArgs& a, hipStream_t s);

// Deterministic CP-ALS on the full tensor (cpals_kernel.hip): one mode's
// update after its mode product M_n is in Y, or the Gram of a start.
struct CpArgs {
    int N, R, n, sweep;        // mode and sweep (1-based; 0 for the start) of the launch
    int64_t I;                 // rows of mode n
    int max_iters;
    double tol;
    double* state;             // sweep state (cp_state_doubles)
    const double* Y;           // M_n, I x ldy float64
    int ldy;
    double* raw;               // I x R float64 factor of mode n
    float* fac;                // I x R float32 copy (the mode products read it)
    float* lam_f;              // R: lambda as float (for the final ordering)
    rcp_als_info* info;
    int* status_word;
    double* E;                 // 2 x 64 x 64 Jacobi scratch (pseudo-inverse fallback)
};
size_t cp_state_doubles(int N, int R);
int cp_row_blocks(int64_t I);
// V^-1, raw = Y V^-1, norms, G_n (and for the last mode lambda, fit, stop), A_n
hipError_t launch_cp_update(const CpArgs& a, hipStream_t s);
// G_n of the start already in a.raw
hipError_t launch_cp_gram(const CpArgs& a, hipStream_t s);
// start of mode n from a subspace basis Q (I x l) and the Gram's leading
// eigenvectors W (l x R): unit, sign-fixed columns of Q W into raw and fac
hipError_t launch_cp_start(const float* Q, const float* W, int64_t I, int l, int R, double* raw,
                           float* fac, hipStream_t s);
// a caller's start (float32, cnt entries) into raw and fac
hipError_t launch_cp_load(const float* A, int64_t cnt, double* raw, float* fac, hipStream_t s);
// Block coordinate descent on the core (bcd_kernel.hip), one workgroup, the
// same arguments (a.normX2 must be set; At[1..N-1] read when a.warm)
bool bcd_supported(int N, const int* l, int R);
hipError_t launch_bcd(const AlsArgs& a, hipStream_t s);
// one launch for `count` problems: dargs on the device, hargs the same on the host
hipError_t launch_als_batch(const AlsArgs* dargs, const AlsArgs* hargs, int count, hipStream_t s);
size_t als_workspace_doubles(int N, const int* l, int R);
bool als_supported(int N, const int* l, int R);
// the core fits in one workgroup's LDS: the whole sweep loop in one launch
bool als_core_in_lds(int N, const int* l, int R);
// Grid-wide form for larger cores: per mode the product B_(n) KR runs over
// the whole GPU (launch_mttkrp), these one-workgroup kernels do the rest.
// The sweep state (iteration, stop flag, Grams, lambda) lives in a.state;
// the stop flag (an int at a.state) makes every later launch return at once.
size_t als_state_doubles(int N, int R);
// Algorithm 2's initialisation for every mode n >= 1 at once (one workgroup per
// mode) from the Grams B_(n) B_(n)^T at a.Y + (n - 1) ystride (row stride l_n
// rounded up to 16); the sweep state's first three doubles must be zero
hipError_t launch_als_wide_init(const AlsArgs& a, int ystride, hipStream_t s);
// warm start: the Grams of the given factors At[1..N-1] and a fresh state
hipError_t launch_als_wide_warm(const AlsArgs& a, hipStream_t s);

// Algorithm 2's update of mode n from its reduced mode product in a.Y; after the
// last mode, the fit and the stopping rule
hipError_t launch_als_wide_step(const AlsArgs& a, int n, hipStream_t s);

// back-projection (expand_kernel.hip)
struct ExpandArgs {
    int N;
    int64_t I[RCP_MAX_NDIM];
    int l[RCP_MAX_NDIM];
    int R;
    const float* Q[RCP_MAX_NDIM];
    const float* At[RCP_MAX_NDIM];
    const float* lambda_in;
    float* A[RCP_MAX_NDIM];
    float* lambda_out;
    double* raw;               // scratch: sum_n I_n x R
    double* stats;             // scratch: column norms, signs (N x R each), ranks (R)
};
hipError_t launch_expand(const ExpandArgs& a, hipStream_t s);
// the final step alone on factors already in a.raw (Q_n = I): renormalise,
// order by lambda, signs
hipError_t launch_expand_finish(const ExpandArgs& a, hipStream_t s);
hipError_t launch_expand_batch(const ExpandArgs* dargs, const ExpandArgs* hargs, int count,
                               hipStream_t s);

}  // namespace rcp
