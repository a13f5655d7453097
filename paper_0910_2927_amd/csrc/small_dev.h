// Device body of the per-cycle shifted Hessenberg solves (one workgroup
// of kFomWaves waves per system), shared by small.hip and batched.hip.
#pragma once

#include "sk_internal.h"

namespace sk {
namespace {

constexpr int kWaves = 16;   // waves of the solving workgroup

__device__ inline double2 bcast(double2 v, int src) {
  return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

// Value of lane `src` (the same for the whole wave) in every lane.
__device__ inline double2 readlane2(double2 v, int src) {
  const int a = __builtin_amdgcn_readlane(__double2loint(v.x), src);
  const int b = __builtin_amdgcn_readlane(__double2hiint(v.x), src);
  const int c = __builtin_amdgcn_readlane(__double2loint(v.y), src);
  const int d = __builtin_amdgcn_readlane(__double2hiint(v.y), src);
  return make_double2(__hiloint2double(b, a), __hiloint2double(d, c));
}

// kQ: columns per lane, ceil(kmax / 64) (registers scale with it).
// hl: LDS staging area of kLdsH complex entries for H (used when H fits).
constexpr int kLdsH = 4096;
template <int kQ>
__device__ inline void fom_small_body_q(const ArnoldiDev& arn, int kmax, const PoleSet& poles,
                                        double2* rho, double2* Y, double2* Ubuf, double2* ucoef,
                                        double2* ycoef, double2* hl) {
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
  // H is read row by row by every pole's wave: stage it in LDS when it fits
  const bool staged = (int64_t)kk * ld <= kLdsH;   // uniform over the block
  if (staged) {
    for (int e = threadIdx.x; e < kk * ld; e += blockDim.x) hl[e] = arn.H[e];
    __syncthreads();
  }
  const double2* H = staged ? hl : arn.H;
  const double2 hnext = H[(size_t)(kk - 1) * ld + kk];   // h_{k+1,k} (0 on breakdown)
  for (int i = wv; i < poles.n; i += kWaves) {
    const double2 sig = poles.sigma[i];
    double2* U = Ubuf + (size_t)i * kmax * kmax;   // row-major kk x kk (upper part used)
    double2* Ub = Y + (size_t)i * kmax;             // rhs after elimination, then y
    double2 cur[kQ], nxt[kQ], pre[kQ];
    // row 0 of H - sigma I; row 1 of H loaded ahead
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int c = lane + 64 * q;
      cur[q] = (c < kk) ? H[(size_t)c * ld + 0] : make_double2(0.0, 0.0);
      if (c == 0) cur[q] = csub(cur[q], sig);
      pre[q] = (kk > 1 && c < kk) ? H[(size_t)c * ld + 1] : make_double2(0.0, 0.0);
    }
    double2 rhs_cur = cscale(rho[i], beta);
    int singular = 0;
    for (int j = 0; j + 1 < kk; ++j) {
      // row j + 1 of H - sigma I (loaded one step ahead), then row j + 2 ahead
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int c = lane + 64 * q;
        nxt[q] = (c >= j) ? pre[q] : make_double2(0.0, 0.0);
        if (c == j + 1) nxt[q] = csub(nxt[q], sig);
      }
      if (j + 2 < kk)
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          const int c = lane + 64 * q;
          pre[q] = (c < kk && c >= j + 1) ? H[(size_t)c * ld + (j + 2)] : make_double2(0.0, 0.0);
        }
      double2 rhs_nxt = make_double2(0.0, 0.0);
      const int qj = j >> 6, lj = j & 63;
      double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < kQ; ++q)
        if (q == qj) {
          a = readlane2(cur[q], lj);
          b = readlane2(nxt[q], lj);
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
    // back substitution by columns: y_r = b_r / U_rr, then b_c -= U_cr y_r
    // for c < r; the next column is loaded while the current one is used
    // (columns are loaded three steps ahead)
    double2 y[kQ], bb[kQ], c1[kQ], c2[kQ], c3[kQ];
    auto load_col = [&](double2 (&dst)[kQ], int r) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int c = lane + 64 * q;
        dst[q] = (r >= 0 && c <= r) ? U[(size_t)c * kmax + r] : make_double2(0.0, 0.0);
      }
    };
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int c = lane + 64 * q;
      y[q] = make_double2(0.0, 0.0);
      bb[q] = (c < kk) ? Ub[c] : make_double2(0.0, 0.0);
    }
    load_col(c1, kk - 1);
    load_col(c2, kk - 2);
    load_col(c3, kk - 3);
    for (int r = kk - 1; r >= 0; --r) {
      double2 cc[kQ];
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        cc[q] = c1[q];
        c1[q] = c2[q];
        c2[q] = c3[q];
      }
      load_col(c3, r - 3);
      const int qr = r >> 6, lr = r & 63;
      double2 d = make_double2(0.0, 0.0), br = make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < kQ; ++q)
        if (q == qr) {
          d = readlane2(cc[q], lr);
          br = readlane2(bb[q], lr);
        }
      if (cabs2(d) == 0.0) singular = 1;
      const double2 yr = singular ? make_double2(0.0, 0.0) : cdiv(br, d);
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int c = lane + 64 * q;
        if (c < r) bb[q] = csub(bb[q], cmul(cc[q], yr));
        if (c == r) y[q] = yr;
      }
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

__device__ inline void fom_small_body(const ArnoldiDev& arn, int kmax, const PoleSet& poles,
                                      double2* rho, double2* Y, double2* Ubuf, double2* ucoef,
                                      double2* ycoef) {
  static_assert(kMaxK <= 256, "row registers cover at most 4 x 64 columns");
  __shared__ double2 hl[kLdsH];
  if (kmax <= 64) fom_small_body_q<1>(arn, kmax, poles, rho, Y, Ubuf, ucoef, ycoef, hl);
  else if (kmax <= 128) fom_small_body_q<2>(arn, kmax, poles, rho, Y, Ubuf, ucoef, ycoef, hl);
  else if (kmax <= 192) fom_small_body_q<3>(arn, kmax, poles, rho, Y, Ubuf, ucoef, ycoef, hl);
  else fom_small_body_q<4>(arn, kmax, poles, rho, Y, Ubuf, ucoef, ycoef, hl);
}

}  // namespace
}  // namespace sk
