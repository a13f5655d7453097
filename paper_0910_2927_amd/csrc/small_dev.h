// Device body of the per-cycle shifted Hessenberg solves (one workgroup
// of kFomWaves waves per system), shared by small.hip and batched.hip.
#pragma once

#include "sk_internal.h"

namespace sk {
namespace {

constexpr int kWaves = 16;   // waves of the solving workgroup
constexpr int kQ = kMaxK / 64;   // columns per lane

__device__ inline double2 bcast(double2 v, int src) {
  return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

__device__ inline void fom_small_body(const ArnoldiDev& arn, int kmax, const PoleSet& poles,
                                      double2* rho, double2* Y, double2* Ubuf, double2* ucoef,
                                      double2* ycoef) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int kk = arn.st->kdone;
  if (kk < 1) {   // no Krylov vector (zero start): no update
    if (threadIdx.x == 0) {
      arn.st->upd_norm = 0.0;
      arn.st->hnext = 0.0;
    }
    for (int i = threadIdx.x; i < poles.n; i += blockDim.x) rho[i] = make_double2(0.0, 0.0);
    return;
  }
  const int ld = arn.ldh;
  const double beta = arn.st->beta;
  const double2* H = arn.H;
  const double2 hnext = H[(size_t)(kk - 1) * ld + kk];   // h_{k+1,k} (0 on breakdown)
  for (int i = wv; i < poles.n; i += kWaves) {
    const double2 sig = poles.sigma[i];
    double2* U = Ubuf + (size_t)i * kmax * kmax;   // row-major kk x kk (upper part used)
    double2* Ub = Y + (size_t)i * kmax;             // rhs after elimination, then y
    double2 cur[kQ], nxt[kQ];
    // row 0 of H - sigma I
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int c = lane + 64 * q;
      cur[q] = (c < kk) ? H[(size_t)c * ld + 0] : make_double2(0.0, 0.0);
      if (c == 0) cur[q] = csub(cur[q], sig);
    }
    double2 rhs_cur = cscale(rho[i], beta);
    int singular = 0;
    for (int j = 0; j + 1 < kk; ++j) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int c = lane + 64 * q;
        nxt[q] = (c < kk && c >= j) ? H[(size_t)c * ld + (j + 1)] : make_double2(0.0, 0.0);
        if (c == j + 1) nxt[q] = csub(nxt[q], sig);
      }
      double2 rhs_nxt = make_double2(0.0, 0.0);
      const int qj = j >> 6, lj = j & 63;
      double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < kQ; ++q)
        if (q == qj) {
          a = bcast(cur[q], lj);
          b = bcast(nxt[q], lj);
        }
      if (cabs2(b) > cabs2(a)) {   // partial pivoting: swap the two rows
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          double2 tmp = cur[q];
          cur[q] = nxt[q];
          nxt[q] = tmp;
        }
        double2 tr = rhs_cur;
        rhs_cur = rhs_nxt;
        rhs_nxt = tr;
        double2 ta = a;
        a = b;
        b = ta;
      }
      if (cabs2(a) == 0.0) singular = 1;
      const double2 l = singular ? make_double2(0.0, 0.0) : cdiv(b, a);
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int c = lane + 64 * q;
        if (c < kk && c >= j) U[(size_t)j * kmax + c] = cur[q];
        nxt[q] = (c > j) ? csub(nxt[q], cmul(l, cur[q])) : make_double2(0.0, 0.0);
        cur[q] = nxt[q];
      }
      if (lane == 0) Ub[j] = rhs_cur;
      rhs_cur = csub(rhs_nxt, cmul(l, rhs_cur));
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int c = lane + 64 * q;
      if (c == kk - 1) U[(size_t)(kk - 1) * kmax + c] = cur[q];
    }
    if (lane == 0) Ub[kk - 1] = rhs_cur;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // back substitution, y kept across lanes
    double2 y[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) y[q] = make_double2(0.0, 0.0);
    for (int r = kk - 1; r >= 0; --r) {
      double pr = 0.0, pi = 0.0;
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int c = lane + 64 * q;
        if (c > r && c < kk) {
          double2 t = cmul(U[(size_t)r * kmax + c], y[q]);
          pr += t.x;
          pi += t.y;
        }
      }
      pr = wave_sum(pr);
      pi = wave_sum(pi);
      const double2 d = U[(size_t)r * kmax + r];
      if (cabs2(d) == 0.0) singular = 1;
      const double2 yr = singular ? make_double2(0.0, 0.0) : cdiv(csub(Ub[r], make_double2(pr, pi)), d);
      const int qr = r >> 6, lr = r & 63;
#pragma unroll
      for (int q = 0; q < kQ; ++q)
        if (q == qr && lane == lr) y[q] = yr;
    }
    bool bad = false;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int c = lane + 64 * q;
      if (c < kk) {
        Y[(size_t)i * kmax + c] = y[q];
        if (!isfinite(y[q].x) || !isfinite(y[q].y)) bad = true;
      }
    }
    // new collinearity factor from the last entry of y
    const int ql = (kk - 1) >> 6, ll = (kk - 1) & 63;
    double2 ylast = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < kQ; ++q)
      if (q == ql) ylast = bcast(y[q], ll);
    if (lane == 0) {
      rho[i] = make_double2(-(hnext.x * ylast.x - hnext.y * ylast.y),
                            -(hnext.x * ylast.y + hnext.y * ylast.x));
      if (singular) arn.st->singular = 1;
    }
    if (bad) arn.st->nonfinite = 1;
  }
  __syncthreads();
  // combined coefficients u = sum_i omega_i y_i and per-shift coefficients
  __shared__ double red[kWaves];
  double un2 = 0.0;
  for (int c = threadIdx.x; c < kk; c += kWaves * 64) {
    double2 u = make_double2(0.0, 0.0);
    for (int i = 0; i < poles.n; ++i) u = cadd(u, cmul(poles.omega[i], Y[(size_t)i * kmax + c]));
    un2 += cabs2(u);
    const double s = arn.scale[c];
    ucoef[c] = cscale(u, s);
    if (ycoef)
      for (int i = 0; i < poles.n; ++i) ycoef[(size_t)i * kmax + c] = cscale(Y[(size_t)i * kmax + c], s);
  }
  un2 = wave_sum(un2);
  if (lane == 0) red[wv] = un2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < kWaves; ++w) tot += red[w];
    arn.st->upd_norm = sqrt(tot);
    arn.st->hnext = sqrt(cabs2(hnext));
    if (!isfinite(tot)) arn.st->nonfinite = 1;
  }
}

}  // namespace
}  // namespace sk
