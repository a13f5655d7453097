// The small FP64 step of one restart cycle (Algorithm 1, Sect. 3):
//   y_i = beta rho_i (H_k - sigma_i I)^{-1} e_1  for every pole i,
//   u = sum_i omega_i y_i,   rho_i <- -h_{k+1,k} e_k^T y_i,   ||u||.
// One workgroup of 16 waves; wave w takes poles w, w+16, ...  Each solve is
// Gaussian elimination with partial pivoting specialised to the upper
// Hessenberg structure (one row to eliminate per column), followed by back
// substitution; a row of length k lives in registers across the 64 lanes
// (columns lane + 64 q).
#include "small_dev.h"

namespace sk {
namespace {

__global__ __launch_bounds__(kWaves * 64) void k_fom_small(ArnoldiDev arn, int kmax, PoleSet poles,
                                                           double2* rho, double2* Y, double2* Ubuf,
                                                           double2* ucoef, double2* ycoef) {
  fom_small_body(arn, kmax, poles, rho, Y, Ubuf, ucoef, ycoef);
}

}  // namespace

hipError_t launch_fom_small(const ArnoldiDev& arn, int k, const PoleSet& poles, double2* rho,
                            double2* Y, double2* U, double2* ucoef, double2* ycoef,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_fom_small, dim3(1), dim3(kWaves * 64), 0, s, arn, k, poles, rho, Y, U,
                     ucoef, ycoef);
  return hipGetLastError();
}

}  // namespace sk
