// Arnoldi with classical Gram-Schmidt and delayed reorthogonalisation
// (Sect. 2, A V_k = V_k H_k + h_{k+1,k} v_{k+1} e_k^T).
//
// Every basis vector still gets two classical Gram-Schmidt passes, but the
// second pass of vector j is folded into step j+1, so one step needs one
// global reduction and two passes over the basis instead of three and four:
//
//   state before step j:  V_j = [v_0 .. v_{j-1}] final and orthonormal;
//                         u_j = A v_{j-1} - V_j s_{j-1}  (first pass done);
//                         s_{j-1} the first-pass coefficients of column j-1.
//   stencil   z = A u_j
//   dots      t = V_j^H u_j,  p = V_j^H z,  alpha = u_j^H u_j,  gamma = u_j^H z
//   update    beta = sqrt(alpha - |t|^2)            (second pass, Pythagoras)
//             v_j = (u_j - V_j t) / beta             column j-1 = s_{j-1} + t,
//                                                   h_{j,j-1} = beta
//             A v_j = (z - V_j H_j t - v_j beta t_{j-1}) / beta   (Arnoldi relation)
//             s_j = V_{j+1}^H A v_j from (t, p, gamma, H_j) alone
//             u_{j+1} = A v_j - V_{j+1} s_j = z/beta - (d/beta) u_j - V_j e
// with e, d small vectors; both v_j and u_{j+1} come from one pass over
// V_j.  The last vector gets its second pass in a final dots + update.
//
// Slots: W_j holds u_j and becomes v_j in place; the stencil writes z into
// W_{j+1}, which the update turns into u_{j+1} in place.  The first-pass
// coefficients live in two alternating buffers so that no block reads
// what another block of the same launch writes.  As in the other kernels,
// every reduction is finished by the next launch in a fixed order.
#include "dcgs2_dev.h"

#include <hip/hip_ext.h>

namespace sk {

namespace {

constexpr int kNT = kTsThreads;
constexpr int kVC = 8;

template <typename T>
__global__ __launch_bounds__(kSdThreads) void k_dc_dot(const T* __restrict__ W, int64_t ldq, int j,
                                                       int has_z, int64_t n, int rpt,
                                                       double2* __restrict__ part, const int* skip) {
  if (skip && *skip) return;
  dc_dot_body<T, kSdThreads>(W, ldq, j, has_z, n, rpt, part, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kNT) void k_dc_reduce(const double2* __restrict__ part, int nrb, int pr,
                                                   double2* __restrict__ out, const int* skip) {
  if (skip && *skip) return;
  dc_reduce_body(part, nrb, pr, out, blockIdx.x, blockIdx.y);
}

// Update blocks of kSuThreads threads: the per-block prologue (folding the
// partial sums, H_j t) is shared by more rows.  SPLIT lanes per row pack:
// 2 when one lane per pack would leave CUs idle (small n, latency-bound),
// else 1 (the basis pass is bandwidth-bound and the pair's repeated loads
// of u_j and z only cost).
constexpr int kSuThreads = 512;
constexpr int kCUs = 256;

template <typename T, bool FINAL, int SPLIT>
__global__ __launch_bounds__(kSuThreads, 4) void k_dc_update(T* __restrict__ W, int64_t ldq, int j, int64_t n,
                                                          const double2* __restrict__ part,
                                                          int nrb, ArnoldiDev arn,
                                                          const double2* __restrict__ s_prev,
                                                          double2* __restrict__ s_cur, int fresh,
                                                          const int* skip) {
  if (skip && *skip) return;
  dc_update_body<T, FINAL, kSuThreads, SPLIT>(
      W, ldq, j, n, part, nrb, arn, s_prev, s_cur, fresh,
      (int64_t)blockIdx.x * (kSuThreads / SPLIT) + threadIdx.x / SPLIT, 1, blockIdx.x == 0);
}

template <typename T, bool FINAL, int SPLIT>
hipError_t launch_update(T* W, int64_t ldq, int j, int64_t n, const double2* src, int nrows,
                         const ArnoldiDev& arn, const double2* s_prev, double2* s_cur, bool fresh,
                         const int* skip, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  const int64_t rows_per_block = (int64_t)(kSuThreads / SPLIT) * Pk<T>::P;   // one row pack per SPLIT lanes
  const dim3 grid((unsigned)((n + rows_per_block - 1) / rows_per_block));
  if (t0 || t1)
    hipExtLaunchKernelGGL((k_dc_update<T, FINAL, SPLIT>), grid, dim3(kSuThreads), 0, s, t0, t1, 0, W, ldq, j,
                          n, src, nrows, arn, s_prev, s_cur, fresh ? 1 : 0, skip);
  else
    hipLaunchKernelGGL((k_dc_update<T, FINAL, SPLIT>), grid, dim3(kSuThreads), 0, s, W, ldq, j, n, src, nrows,
                       arn, s_prev, s_cur, fresh ? 1 : 0, skip);
  return hipGetLastError();
}

}  // namespace

// Dots of step j; beyond kGsDirect row blocks the partials are folded into
// kGsGroups rows stored right after them (part + nrb * (2 j + 2)).
template <typename T>
hipError_t dc_dot(const T* W, int64_t ldq, int j, bool has_z, int64_t n, double2* part,
                  const int* skip, hipStream_t s, hipEvent_t t0, hipEvent_t t1, hipEvent_t r0,
                  hipEvent_t r1) {
  const int nrb = sd_row_blocks(n, Pk<T>::P);
  const int rpt = sd_rpt(n, Pk<T>::P);
  const bool red = gs_reduced(nrb);
  dim3 grid(nrb, j > 0 ? (j + kVC - 1) / kVC : 1);
  if (t0 || t1)
    hipExtLaunchKernelGGL((k_dc_dot<T>), grid, dim3(kSdThreads), 0, s, t0, t1, 0, W, ldq, j, has_z ? 1 : 0,
                          n, rpt, part, skip);
  else
    hipLaunchKernelGGL((k_dc_dot<T>), grid, dim3(kSdThreads), 0, s, W, ldq, j, has_z ? 1 : 0, n, rpt, part,
                       skip);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !red) return e;
  const int pr = 2 * j + 2;
  if (r0 || r1)
    hipExtLaunchKernelGGL(k_dc_reduce, dim3((pr + 63) / 64, kGsGroups), dim3(kNT), 0, s, r0, r1, 0, part,
                          nrb, pr, part + (size_t)nrb * pr, skip);
  else
    hipLaunchKernelGGL(k_dc_reduce, dim3((pr + 63) / 64, kGsGroups), dim3(kNT), 0, s, part, nrb, pr,
                       part + (size_t)nrb * pr, skip);
  return hipGetLastError();
}

template <typename T>
hipError_t dc_update(T* W, int64_t ldq, int j, bool final_pass, int64_t n, const double2* part,
                     const ArnoldiDev& arn, const double2* s_prev, double2* s_cur, bool fresh,
                     const int* skip, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  const int nrb = sd_row_blocks(n, Pk<T>::P);         // rows of partials (the dot kernel's grid)
  const int pr = 2 * j + 2;
  const double2* src = gs_reduced(nrb) ? part + (size_t)nrb * pr : part;
  const int nrows = gs_reduced(nrb) ? kGsGroups : nrb;
  const bool split = (n + (int64_t)kSuThreads * Pk<T>::P - 1) / ((int64_t)kSuThreads * Pk<T>::P) < kCUs;
  if (final_pass)
    return split ? launch_update<T, true, 2>(W, ldq, j, n, src, nrows, arn, s_prev, s_cur, fresh, skip, s, t0, t1)
                 : launch_update<T, true, 1>(W, ldq, j, n, src, nrows, arn, s_prev, s_cur, fresh, skip, s, t0, t1);
  return split ? launch_update<T, false, 2>(W, ldq, j, n, src, nrows, arn, s_prev, s_cur, fresh, skip, s, t0, t1)
               : launch_update<T, false, 1>(W, ldq, j, n, src, nrows, arn, s_prev, s_cur, fresh, skip, s, t0, t1);
}

template hipError_t dc_dot<double2>(const double2*, int64_t, int, bool, int64_t, double2*,
                                    const int*, hipStream_t, hipEvent_t, hipEvent_t, hipEvent_t,
                                    hipEvent_t);
template hipError_t dc_dot<float2>(const float2*, int64_t, int, bool, int64_t, double2*,
                                   const int*, hipStream_t, hipEvent_t, hipEvent_t, hipEvent_t,
                                   hipEvent_t);
template hipError_t dc_update<double2>(double2*, int64_t, int, bool, int64_t, const double2*,
                                       const ArnoldiDev&, const double2*, double2*, bool,
                                       const int*, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t dc_update<float2>(float2*, int64_t, int, bool, int64_t, const double2*,
                                      const ArnoldiDev&, const double2*, double2*, bool, const int*,
                                      hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace sk
