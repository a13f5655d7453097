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

// H (kk columns of ld entries) staged in LDS by the whole block when it
// fits (the decision is uniform over the block); returns the copy to read.
__device__ inline const double2* stage_h(const ArnoldiDev& arn, int kk, double2* hl) {
  const int ne = kk * arn.ldh;
  if (ne > kLdsH) return arn.H;
  constexpr int kU = 8;   // loads in flight per thread
  for (int e0 = threadIdx.x; e0 < ne; e0 += kU * blockDim.x) {
    double2 v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + u * blockDim.x;
      v[u] = e < ne ? arn.H[e] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + u * blockDim.x;
      if (e < ne) hl[e] = v[u];
    }
  }
  __syncthreads();
  return hl;
}

// Pole i, one wave: y_i = beta rho_i (H_kk - sigma_i I)^{-1} e_1 into Y and
// rho_i <- -h_{k+1,k} e_k^T y_i.  U: this pole's kmax x kmax scratch.
template <int kQ>
__device__ inline void fom_pole_q(int i, int kk, int kmax, int ld, const double2* H, double2 hnext,
                                  double beta, const PoleSet& poles, double2* rho, double2* Y,
                                  double2* Ubuf, CycleState* st) {
  const int lane = threadIdx.x & 63;
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
    if (singular) st->singular = 1;
  }
  if (bad) st->nonfinite = 1;
}

// u = sum_i omega_i y_i (times the basis scales) into ucoef, the per-shift
// coefficients into ycoef (if set), ||u|| and |h_{k+1,k}| into the state.
// Whole block, after every y_i is in Y.
__device__ inline void fom_combine(const ArnoldiDev& arn, int kmax, int kk, double2 hnext,
                                   const PoleSet& poles, const double2* Y, double2* ucoef,
                                   double2* ycoef) {
  __shared__ double red[kWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double un2 = 0.0;
  for (int c = threadIdx.x; c < kk; c += blockDim.x) {
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
    for (int w = 0; w < nw; ++w) tot += red[w];
    arn.st->upd_norm = sqrt(tot);
    arn.st->hnext = sqrt(cabs2(hnext));
    if (!isfinite(tot)) arn.st->nonfinite = 1;
  }
}

// All poles and the combination in one workgroup of kWaves waves (wave w
// takes poles w, w + kWaves, ...).
template <int kQ>
__device__ inline void fom_small_body_q(const ArnoldiDev& arn, int kmax, const PoleSet& poles,
                                        double2* rho, double2* Y, double2* Ubuf, double2* ucoef,
                                        double2* ycoef, double2* hl) {
  const int wv = threadIdx.x >> 6;
  const int kk = arn.st->kdone;
  if (kk < 1) {   // no Krylov vector (zero start): no update
    if (threadIdx.x == 0) {
      arn.st->upd_norm = 0.0;
      arn.st->hnext = 0.0;
    }
    for (int i = threadIdx.x; i < poles.n; i += blockDim.x) rho[i] = make_double2(0.0, 0.0);
    return;
  }
  const double beta = arn.st->beta;
  const double2* H = stage_h(arn, kk, hl);
  const double2 hnext = H[(size_t)(kk - 1) * arn.ldh + kk];   // h_{k+1,k} (0 on breakdown)
  for (int i = wv; i < poles.n; i += kWaves)
    fom_pole_q<kQ>(i, kk, kmax, arn.ldh, H, hnext, beta, poles, rho, Y, Ubuf, arn.st);
  __syncthreads();
  fom_combine(arn, kmax, kk, hnext, poles, Y, ucoef, ycoef);
}

// Poles only, spread over blocks: wave w of block b takes pole
// b * (waves per block) + w, so that every wave has a SIMD to itself
// (the elimination and substitution chains are vector-ALU bound when
// several share one).  fom_combine runs in the next kernel.
template <int kQ>
__device__ inline void fom_poles_body_q(const ArnoldiDev& arn, int kmax, const PoleSet& poles,
                                        double2* rho, double2* Y, double2* Ubuf, double2* hl) {
  const int kk = arn.st->kdone;
  const int i = blockIdx.x * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
  if (kk < 1) {
    if ((threadIdx.x & 63) == 0 && i < poles.n) rho[i] = make_double2(0.0, 0.0);
    return;
  }
  const double beta = arn.st->beta;
  const double2* H = stage_h(arn, kk, hl);   // every wave of the block takes part
  if (i >= poles.n) return;
  const double2 hnext = H[(size_t)(kk - 1) * arn.ldh + kk];
  fom_pole_q<kQ>(i, kk, kmax, arn.ldh, H, hnext, beta, poles, rho, Y, Ubuf, arn.st);
}

__device__ inline void fom_poles_body(const ArnoldiDev& arn, int kmax, const PoleSet& poles,
                                      double2* rho, double2* Y, double2* Ubuf) {
  __shared__ double2 hl[kLdsH];
  if (kmax <= 64) fom_poles_body_q<1>(arn, kmax, poles, rho, Y, Ubuf, hl);
  else if (kmax <= 128) fom_poles_body_q<2>(arn, kmax, poles, rho, Y, Ubuf, hl);
  else if (kmax <= 192) fom_poles_body_q<3>(arn, kmax, poles, rho, Y, Ubuf, hl);
  else fom_poles_body_q<4>(arn, kmax, poles, rho, Y, Ubuf, hl);
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
