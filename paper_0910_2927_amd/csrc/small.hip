// The small FP64 step of one restart cycle (Algorithm 1, Sect. 3):
//   y_i = beta rho_i (H_k - sigma_i I)^{-1} e_1  for every pole i,
//   u = sum_i omega_i y_i,   rho_i <- -h_{k+1,k} e_k^T y_i,   ||u||.
// One wave per pole, 4 waves per workgroup (each wave has a SIMD to
// itself), then one workgroup for the combination.  Each solve is Gaussian
// elimination with partial pivoting specialised to the upper Hessenberg
// structure (one row to eliminate per column), followed by back
// substitution; a row of length k lives in registers across the 64 lanes
// (columns lane + 64 q).
#include "small_dev.h"

namespace sk {
namespace {

constexpr int kPoleWaves = 4;   // poles (waves) per workgroup

__global__ __launch_bounds__(kPoleWaves * 64) void k_fom_poles(ArnoldiDev arn, int kmax, PoleSet poles,
                                                               double2* rho, double2* Y, double2* Ubuf) {
  fom_poles_body(arn, kmax, poles, rho, Y, Ubuf);
}

__global__ __launch_bounds__(kWaves * 64) void k_fom_combine(ArnoldiDev arn, int kmax, PoleSet poles,
                                                             const double2* Y, double2* ucoef,
                                                             double2* ycoef) {
  const int kk = arn.st->kdone;
  if (kk < 1) {   // no Krylov vector (zero start): no update
    if (threadIdx.x == 0) {
      arn.st->upd_norm = 0.0;
      arn.st->hnext = 0.0;
    }
    return;
  }
  const double2 hnext = arn.H[(size_t)(kk - 1) * arn.ldh + kk];   // h_{k+1,k} (0 on breakdown)
  fom_combine(arn, kmax, kk, hnext, poles, Y, ucoef, ycoef);
}

}  // namespace

hipError_t launch_fom_small(const ArnoldiDev& arn, int k, const PoleSet& poles, double2* rho,
                            double2* Y, double2* U, double2* ucoef, double2* ycoef,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_fom_poles, dim3((poles.n + kPoleWaves - 1) / kPoleWaves), dim3(kPoleWaves * 64), 0, s,
                     arn, k, poles, rho, Y, U);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fom_combine, dim3(1), dim3(kWaves * 64), 0, s, arn, k, poles, Y, ucoef, ycoef);
  return hipGetLastError();
}

}  // namespace sk
