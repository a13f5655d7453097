// The end of a restart cycle of Algorithm 1 (Sect. 5) for one system:
// the solution update x += V_k u with ||x||^2, and the restart vector
// r = (I - R L^H) v_{k+1} (projection step, Sect. 4).  Reductions are
// finished by the next kernel in a fixed order (no fences, deterministic);
// the deflation dots cover 8 rows per thread so that every projection
// block can fold all their partial sums itself.
#include "dcgs2_dev.h"

namespace sk {
namespace {

constexpr int kCT = kTsThreads;
constexpr int kCW = kCT / 64;
constexpr int kDefRpt = 8;   // rows per thread of the deflation dots

// x += V_kk u (kk = *kdone: fewer vectors after a breakdown); partial ||x||^2.
template <typename T>
__global__ __launch_bounds__(kCT) void k_cx_update(const T* __restrict__ W, int64_t n,
                                                   const double2* __restrict__ ucoef,
                                                   const int* __restrict__ kdone, double2* __restrict__ x,
                                                   double* __restrict__ xpart) {
  __shared__ double2 c[kMaxK + 2];
  __shared__ double red[kCW];
  const int kk = *kdone;
  for (int i = threadIdx.x; i < kk; i += kCT) c[i] = ucoef[i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * kCT + threadIdx.x;
  double nrm = 0.0;
  if (r < n) {
    double2 acc = x[r];
    constexpr int B = 8;   // loads in flight per thread
    for (int i = 0; i < kk; i += B) {
      T raw[B];
#pragma unroll
      for (int b = 0; b < B; ++b) raw[b] = W[(int64_t)min(i + b, kk - 1) * n + r];
#pragma unroll
      for (int b = 0; b < B; ++b)
        if (i + b < kk) acc = cadd(acc, cmul(cvt(raw[b]), c[i + b]));
    }
    x[r] = acc;
    nrm = cabs2(acc);
  }
  nrm = wave_sum(nrm);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int w = 0; w < kCW; ++w) a += red[w];
    xpart[blockIdx.x] = a;
  }
}

__global__ __launch_bounds__(kCT) void k_cx_norm(const double* __restrict__ xpart, int nb,
                                                 CycleState* st) {
  __shared__ double red[kCW];
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += kCT) a += xpart[b];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kCW; ++w) t += red[w];
    st->xnorm2 = t;
    if (!isfinite(t)) st->nonfinite = 1;
  }
}

// Partial L^H v over row blocks of kDefRpt * kCT rows, 8 vectors of L per
// block row (grid.y): dpart[rb * m + i].
template <typename T>
__global__ __launch_bounds__(kCT) void k_cp_dot(const double2* __restrict__ L, int m,
                                                const T* __restrict__ v, int64_t n,
                                                double2* __restrict__ dpart, const int* skip) {
  if (skip && *skip) return;
  const int i0 = blockIdx.y * 8;
  const int cnt = min(8, m - i0);
  double2 acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = z2();
  const int64_t base = (int64_t)blockIdx.x * kCT * kDefRpt + threadIdx.x;
  for (int q = 0; q < kDefRpt; ++q) {
    const int64_t r = base + (int64_t)q * kCT;
    if (r >= n) break;
    const double2 vv = cvt(v[r]);
    double2 lv[8];   // all loads in flight before any is used
#pragma unroll
    for (int c = 0; c < 8; ++c) lv[c] = L[(int64_t)(i0 + min(c, cnt - 1)) * n + r];
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (c < cnt) acc[c] = cadd(acc[c], cconjmul(lv[c], vv));
  }
  __shared__ double2 red[kCW][8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    acc[c].x = wave_sum(acc[c].x);
    acc[c].y = wave_sum(acc[c].y);
  }
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int c = 0; c < 8; ++c) red[threadIdx.x >> 6][c] = acc[c];
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    double2 s = red[0][threadIdx.x];
    for (int w = 1; w < kCW; ++w) s = cadd(s, red[w][threadIdx.x]);
    dpart[(size_t)blockIdx.x * m + i0 + threadIdx.x] = s;
  }
}

// out = v - R c with c = L^H v (folded from dpart by every block), first
// mp columns of R (mp = m: projection, 0: copy); block 0 records ||c|| as
// the leak.  Precision conversion T -> TN on the way.
template <typename T, typename TN>
__global__ __launch_bounds__(kCT) void k_cp_apply(const double2* __restrict__ R, int m, int mp,
                                                  const double2* __restrict__ dpart, int nrb,
                                                  const T* __restrict__ v, TN* __restrict__ out,
                                                  int64_t n, CycleState* cs, const int* skip) {
  if (skip && *skip) return;
  __shared__ double2 c[kMaxDefl];
  __shared__ double2 scratch[kCT];
  if (m > 0) {
    reduce_cols(dpart, nrb, m, c, scratch);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      double l2 = 0.0;
      for (int i = 0; i < m; ++i) l2 += cabs2(c[i]);
      cs->leak = sqrt(l2);
    }
    __syncthreads();
  }
  const int64_t r = (int64_t)blockIdx.x * kCT + threadIdx.x;
  if (r >= n) return;
  double2 w = cvt(v[r]);
  constexpr int B = 8;
  for (int i = 0; i < mp; i += B) {
    double2 rv[B];
#pragma unroll
    for (int b = 0; b < B; ++b) rv[b] = R[(int64_t)min(i + b, mp - 1) * n + r];
#pragma unroll
    for (int b = 0; b < B; ++b)
      if (i + b < mp) w = csub(w, cmul(rv[b], c[i + b]));
  }
  st(out + r, w);
}

}  // namespace

int cycle_xpart_entries(int64_t n) { return (int)((n + kCT - 1) / kCT); }
int cycle_dpart_rows(int64_t n) { return (int)((n + (int64_t)kCT * kDefRpt - 1) / ((int64_t)kCT * kDefRpt)); }

template <typename T>
hipError_t cycle_x_update(const T* W, int64_t n, const double2* ucoef, const int* kdone, double2* x,
                          double* xpart, CycleState* st, hipStream_t s) {
  const int nb = cycle_xpart_entries(n);
  hipLaunchKernelGGL((k_cx_update<T>), dim3(nb), dim3(kCT), 0, s, W, n, ucoef, kdone, x, xpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cx_norm, dim3(1), dim3(kCT), 0, s, xpart, nb, st);
  return hipGetLastError();
}

template <typename T, typename TN>
hipError_t cycle_restart(const double2* R, const double2* L, int m, bool project, const T* v, TN* out,
                         int64_t n, double2* dpart, CycleState* st, const int* skip, hipStream_t s) {
  const int nrb = cycle_dpart_rows(n);
  if (m > 0) {
    hipLaunchKernelGGL((k_cp_dot<T>), dim3(nrb, (m + 7) / 8), dim3(kCT), 0, s, L, m, v, n, dpart, skip);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_cp_apply<T, TN>), dim3(cycle_xpart_entries(n)), dim3(kCT), 0, s, R, m,
                     project ? m : 0, dpart, nrb, v, out, n, st, skip);
  return hipGetLastError();
}

template hipError_t cycle_x_update<double2>(const double2*, int64_t, const double2*, const int*, double2*,
                                            double*, CycleState*, hipStream_t);
template hipError_t cycle_x_update<float2>(const float2*, int64_t, const double2*, const int*, double2*,
                                           double*, CycleState*, hipStream_t);
template hipError_t cycle_restart<double2, double2>(const double2*, const double2*, int, bool,
                                                    const double2*, double2*, int64_t, double2*,
                                                    CycleState*, const int*, hipStream_t);
template hipError_t cycle_restart<double2, float2>(const double2*, const double2*, int, bool,
                                                   const double2*, float2*, int64_t, double2*,
                                                   CycleState*, const int*, hipStream_t);
template hipError_t cycle_restart<float2, float2>(const double2*, const double2*, int, bool,
                                                  const float2*, float2*, int64_t, double2*,
                                                  CycleState*, const int*, hipStream_t);

}  // namespace sk
