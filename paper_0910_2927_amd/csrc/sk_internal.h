// Internal kernels and device state of libsignkrylov (not part of the C ABI).
#pragma once

#include "sk_common.h"

namespace sk {

constexpr int kMaxK = 256;       // longest Arnoldi cycle
constexpr int kMaxPoles = 64;    // most first-order poles
constexpr int kMaxDefl = 128;    // largest deflation space
constexpr int kTsThreads = 256;  // block size of the tall-skinny kernels
constexpr double kBreakdownTol = 1e-12;
constexpr double kDivergeFactor = 1e10;   // update growth that counts as divergence

// Scalars one restart cycle produces, in device memory.  The host reads the
// whole struct back once per cycle.
struct CycleState {
  double beta;        // ||r|| at the start of the cycle
  double xnorm2;      // ||x||^2 after the solution update
  double upd_norm;    // ||sum_i omega_i y_i||
  double leak;        // ||L^H r|| before the projection step
  double hnext;       // h_{k+1,k} of the cycle
  int kdone;          // Arnoldi steps completed (k unless breakdown)
  int breakdown;      // lucky breakdown happened in this cycle
  int singular;       // some H_k - sigma_i had a zero pivot
  int nonfinite;      // a NaN / Inf showed up
  double pad[2];
};

// Device bookkeeping of one Arnoldi cycle.
struct ArnoldiDev {
  double2* H;          // (k+1) x k, column-major, ld = k+1
  double* scale;       // s_j: v_j = s_j W_j  (k+2 entries)
  double* wnorm;       // ||A v_j|| before orthogonalisation (k entries)
  double2* coef;       // Gram-Schmidt coefficients of the current pass
  double2* partial;    // per-block partial sums
  unsigned* counter;   // last-block counters
  CycleState* st;
  int ldh;             // k + 1
};

// Tall-skinny reductions: which epilogue the last block runs.
enum TsEpilogue : int {
  EPI_NONE = 0,
  EPI_ARN_H1 = 1,     // first CGS pass:  H(:,j) = s.*h,  coef = s.*H(:,j), wnorm[j]
  EPI_ARN_H2 = 2,     // second CGS pass: H(:,j) += s.*h, coef = s.*h
  EPI_ARN_NORM = 3,   // h_{j+1,j}, s_{j+1}, breakdown / non-finite flags
  EPI_STORE = 4,      // out[i] = alpha * sums[i]   (alpha = *scale_in or 1)
  EPI_BETA = 5,       // beta = sqrt(sums[0]); scale[0] = 1/beta
  EPI_XNORM = 6,      // st->xnorm2 = sums[0]
  EPI_DEFL = 7,       // coef = alpha*sums (m); leak = ||coef||; coef2 = F coef
};

struct TsEpiArgs {
  int epi;
  int j;                   // Arnoldi step
  ArnoldiDev arn;
  double2* out;            // EPI_STORE / EPI_DEFL destination (coefficients)
  double2* out2;           // EPI_DEFL: F * coef
  const double2* F;        // EPI_DEFL: m x m column-major (nullable)
  const double* alpha;     // scale applied to the sums (nullable = 1)
  double* dst_scalar;      // EPI_BETA: where beta goes; EPI_XNORM
  double* dst_scale;       // EPI_BETA: where 1/beta goes
};

// Row blocking of the Gram-Schmidt dot kernels: rows per thread such that
// about 1024 blocks of kTsThreads threads cover a vector of n rows (enough
// waves in flight to cover memory latency), at most 8.
__host__ __device__ inline int gs_rpt(int64_t n) {
  int64_t r = (n + (int64_t)kTsThreads * 1024 - 1) / ((int64_t)kTsThreads * 1024);
  return (int)(r < 1 ? 1 : (r > 8 ? 8 : r));
}
// pack: consecutive rows a thread loads at once (2 for complex float: one
// 16-byte load); 1 gives the most row blocks, for sizing buffers.
__host__ __device__ inline int gs_row_blocks(int64_t n, int pack = 1) {
  const int64_t rb = (int64_t)kTsThreads * gs_rpt(n) * pack;
  return (int)((n + rb - 1) / rb);
}
// The single-system dot kernel runs blocks of kSdThreads threads with
// sd_rpt row packs per thread: as many as it takes for at most 32 row
// blocks to cover the vector (no folding kernel) if that is <= 8; for
// longer vectors enough for about 256 row blocks (then folded).
constexpr int kSdThreads = 1024;
__host__ __device__ inline int sd_rpt(int64_t n, int pack) {
  const int64_t few = (int64_t)kSdThreads * pack * 32;
  const int64_t r0 = (n + few - 1) / few;
  if (r0 <= 8) return (int)(r0 < 1 ? 1 : r0);
  const int64_t many = (int64_t)kSdThreads * pack * 256;
  const int64_t r = (n + many - 1) / many;
  return (int)(r < 1 ? 1 : (r > 8 ? 8 : r));
}
__host__ __device__ inline int sd_row_blocks(int64_t n, int pack = 1) {
  const int64_t rb = (int64_t)kSdThreads * sd_rpt(n, pack) * pack;
  return (int)((n + rb - 1) / rb);
}

// The dot kernel leaves one row of partial sums per row block.  Up to
// kGsDirect rows are summed by every update block itself; beyond that a
// small reduction kernel first folds them into kGsGroups rows (the update
// blocks would otherwise re-read all partials, a cost growing as n^2).
constexpr int kGsDirect = 32;
constexpr int kGsGroups = 8;
__host__ __device__ inline bool gs_reduced(int nrb) { return nrb > kGsDirect; }
// Entries of the partial-sum buffer for nrb row blocks and restart length k.
__host__ __device__ inline size_t gs_part_entries(int nrb, int k) {
  return (size_t)(nrb + kGsGroups) * (size_t)(2 * k + 2);
}

// Arnoldi step kernels with delayed reorthogonalisation (dcgs2.hip).
// Partials need gs_part_entries(sd_row_blocks(n), k) entries.
// t0, t1 (optional): events stamped at the start of the first and the end
// of the last kernel of the call (per-kernel timing).
// dc_dot: (t0, t1) stamp the dot kernel, (r0, r1) the folding kernel if any.
template <typename T>
hipError_t dc_dot(const T* W, int64_t ldq, int j, bool has_z, int64_t n, double2* part,
                  const int* skip, hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr,
                  hipEvent_t r0 = nullptr, hipEvent_t r1 = nullptr);
template <typename T>
hipError_t dc_update(T* W, int64_t ldq, int j, bool final_pass, int64_t n, const double2* part,
                     const ArnoldiDev& arn, const double2* s_prev, double2* s_cur, bool fresh,
                     const int* skip, hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);

// ------------------------------------------------------------ launchers
// Stencil: out = alpha * H_W(+-mu) in; alpha = *in_scale (nullable = 1).
template <typename TI, typename TL, typename TO>
hipError_t launch_wilson(const sk_operator* op, const TL* links, const TI* in, TO* out,
                         int adjoint, const double* in_scale, const int* skip_flag,
                         hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);

// Residual form: out = b - (H_W - sigma) in, in double; `in` of type TI.
// rpart (nullable): wilson_residual_partials(V) partial sums of ||out||^2.
template <typename TI>
hipError_t launch_wilson_residual(const sk_operator* op, const double2* links, const TI* in,
                                  const double2* b, double2 sigma, double2* out, double* rpart,
                                  hipStream_t s);
int wilson_residual_partials(int64_t V);
// rows[i] = sum of part[i * stride + 0 .. cnt_i), cnt_i = cnt for i < nrows - 1 and
// cnt_last for the last row; one block per row, fixed order.
hipError_t launch_fold_rows(const double* part, int64_t stride, int nrows, int cnt, int cnt_last,
                            double* rows, hipStream_t s);

// DOT: sums_i = sum_r conj(Q_i[r]) v[r] (i < p), plus ||v||^2 if with_norm.
template <typename TQ, typename TV>
hipError_t ts_dot(const TQ* Q, int64_t ldq, int p, const TV* v, int64_t n, bool with_norm,
                  const TsEpiArgs& epi, double2* partial, unsigned* counter,
                  const int* skip_flag, hipStream_t s);

// UPD: out = a * in - sum_i Q_i coef_i;  then RED = 0 none, 1 dots with Q, 2 ||out||^2.
template <typename TQ, typename TI, typename TO>
hipError_t ts_update(const TQ* Q, int64_t ldq, int p, const double2* coef, const double* a,
                     const TI* in, TO* out, int64_t n, int red, const TsEpiArgs& epi,
                     double2* partial, unsigned* counter, const int* skip_flag, hipStream_t s);

// GEMV: y = (accumulate ? y : 0) + sum_i Q_i coef_i; red = 2 gives ||y||^2.
// p is capped at *pdev when pdev is non-NULL (Arnoldi breakdown).
template <typename TQ>
hipError_t ts_gemv(const TQ* Q, int64_t ldq, int p, const double2* coef, double2* y,
                   int64_t n, bool accumulate, int red, const TsEpiArgs& epi,
                   double2* partial, unsigned* counter, const int* pdev, const int* skip,
                   hipStream_t s);

// Multi-output GEMV for per-shift solutions: X_i += sum_j Q_j C[i*ldc + j].
template <typename TQ>
hipError_t ts_multi_gemv(const TQ* Q, int64_t ldq, int p, const double2* C, int ldc, int nout,
                         double2* X, int64_t n, const int* pdev, hipStream_t s);

// Q_j *= scale[j] for j < min(p, *pdev + 1).
template <typename T>
hipError_t ts_scale_basis(T* Q, int64_t ldq, int p, const double* scale, const int* pdev,
                          int64_t n, hipStream_t s);

hipError_t launch_init_state(CycleState* st, double2* rho, int npoles, unsigned* counter,
                             int ncnt, hipStream_t s);

// Vector scale/convert: out = alpha * in (alpha = *alpha_dev or alpha_host).
template <typename TI, typename TO>
hipError_t ts_scale(const TI* in, TO* out, int64_t n, const double* alpha_dev, double alpha_host,
                    hipStream_t s);

// The small FP64 step of a restart cycle: shifted Hessenberg solves and
// the combined coefficients (one workgroup).
struct PoleSet {
  int n;
  double2 sigma[kMaxPoles];
  double2 omega[kMaxPoles];
};
hipError_t launch_fom_small(const ArnoldiDev& arn, int k, const PoleSet& poles,
                            double2* rho, double2* Y, double2* U, double2* ucoef,
                            double2* ycoef, hipStream_t s);

// End of a restart cycle without fences (cycle.hip): x += V_kk u and
// st->xnorm2 (xpart: cycle_xpart_entries(n) doubles), and the restart
// vector out = (I - R L^H) v (project) or v, with st->leak = ||L^H v||
// (dpart: cycle_dpart_rows(n) x m complex).
int cycle_xpart_entries(int64_t n);
int cycle_dpart_rows(int64_t n);
template <typename T>
hipError_t cycle_x_update(const T* W, int64_t n, const double2* ucoef, const int* kdone, double2* x,
                          double* xpart, CycleState* st, hipStream_t s);
template <typename T, typename TN>
hipError_t cycle_restart(const double2* R, const double2* L, int m, bool project, const T* v, TN* out,
                         int64_t n, double2* dpart, CycleState* st, const int* skip, hipStream_t s);

// Link and mu gradient of Re<eta, g(H) b> from per-shift solutions (backward.hip).
int grad_blocks(int64_t V);
hipError_t launch_grad(const sk_operator* op, const PoleSet& ps, const double2* X, const double2* Z,
                       double* grad, double* mu_part, hipStream_t s);

// deflate_project's argument checks and its launches on a given scratch area
// (driver.hip), shared by the workspace and the workspace-free entry points.
int deflate_project_check(int m, int64_t n, const double* R, const double* L, const double* F,
                          const double* in, const double* r_out, const double* xp_out, const double* coeff);
int deflate_project_run(int m, int64_t n, const double* R, const double* L, const double* F,
                        const double* in, double* r_out, double* xp_out, double* coeff, void* scratch,
                        hipStream_t s);

hipError_t launch_zero_counters(unsigned* counter, int n, hipStream_t s);
hipError_t launch_fill_zero(double* p, int64_t count, hipStream_t s);
hipError_t launch_fill_value(double* p, int64_t count, double v, hipStream_t s);

size_t ts_partial_entries(int64_t n, int pmax);
int ts_blocks(int64_t n);
// Counters one reducing kernel needs (group counters + one top counter);
// kernels that may be in flight together need disjoint counter slots.
int ts_counter_stride(int64_t n);
constexpr int kCounterSlots = 12;

}  // namespace sk
