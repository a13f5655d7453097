// Classical Gram-Schmidt with one reorthogonalisation (CGS2) for the
// Arnoldi process of Sect. 2 (A V_k = V_k H_k + h_{k+1,k} v_{k+1} e_k^T).
//
// One Arnoldi step j is five launches, each a plain stream over rows:
//   stencil      w = s_j A W_j          (wilson.hip; reduces the previous norm)
//   gs_dot       partial dots  W_i^H w, i <= j, and ||w||^2       [2-D grid]
//   gs_update    h1 = sum of partials; w -= sum_i W_i s_i h1_i    [1-D grid]
//   gs_dot       partial dots  W_i^H w                            [2-D grid]
//   gs_update    h2; w -= sum_i W_i s_i h2_i; partial ||w||^2
// The basis is stored unnormalised, v_i = s_i W_i, so normalising a vector
// never costs a pass over it.
//
// No kernel communicates with another block of the same launch: every
// reduction is finished by the next launch, which sums the per-block
// partials in a fixed order (deterministic results, and no device-scope
// fences, which on a multi-XCD part write back or invalidate whole L2s).
#include "sk_internal.h"

namespace sk {

int gs_rpt(int64_t n) {
  // rows per thread such that about 96 row blocks cover the vector
  int64_t r = (n + (int64_t)kTsThreads * 96 - 1) / ((int64_t)kTsThreads * 96);
  return (int)std::max<int64_t>(1, std::min<int64_t>(8, r));
}
int gs_row_blocks(int64_t n) {
  const int64_t rb = (int64_t)kTsThreads * gs_rpt(n);
  return (int)((n + rb - 1) / rb);
}

namespace {

constexpr int NT = kTsThreads;
constexpr int NW = NT / 64;
constexpr int VC = 8;         // vectors per dot block

__device__ inline double2 z2() { return make_double2(0.0, 0.0); }

// Sum rows [0, nrows) of src (row stride pr) for columns [0, pr) into
// LDS `sums`, in a fixed order, with all threads of the block.
__device__ inline void reduce_cols(const double2* __restrict__ src, int nrows, int pr, double2* sums,
                                   double2* scratch /* NT */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i0 = 0; i0 < pr; i0 += 64) {
    const int i = i0 + lane;
    double2 acc = z2();
    if (i < pr)
      for (int b = wid; b < nrows; b += NW) acc = cadd(acc, src[(size_t)b * pr + i]);
    scratch[threadIdx.x] = acc;
    __syncthreads();
    if (wid == 0 && i < pr) {
      double2 s = scratch[lane];
#pragma unroll
      for (int w = 1; w < NW; ++w) s = cadd(s, scratch[w * 64 + lane]);
      sums[i] = s;
    }
    __syncthreads();
  }
}

// Partial dots: block (rb, ch) sums conj(W_i[r]) w[r] over its rows for
// the VC vectors of chunk ch; chunk 0 also sums |w[r]|^2 (column p).
template <typename T>
__global__ __launch_bounds__(NT) void k_gs_dot(const T* __restrict__ W, int64_t ldq, int p,
                                               const T* __restrict__ w, int64_t n, int rpt,
                                               int with_norm, double2* __restrict__ part,
                                               const int* skip) {
  if (skip && *skip) return;
  __shared__ double2 red[NW][VC + 1];
  const int rb = blockIdx.x, ch = blockIdx.y;
  const int i0 = ch * VC;
  const int cnt = min(VC, p - i0);
  double2 acc[VC + 1];
#pragma unroll
  for (int u = 0; u <= VC; ++u) acc[u] = z2();
  const int64_t base = (int64_t)rb * NT * rpt + threadIdx.x;
  for (int q = 0; q < rpt; ++q) {
    const int64_t r = base + (int64_t)q * NT;
    if (r < n) {
      const double2 wv = ld(w + r);
#pragma unroll
      for (int u = 0; u < VC; ++u)
        if (u < cnt) acc[u] = cadd(acc[u], cconjmul(ld(W + (int64_t)(i0 + u) * ldq + r), wv));
      if (with_norm && ch == 0) acc[VC].x += cabs2(wv);
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int u = 0; u <= VC; ++u) {
    acc[u].x = wave_sum(acc[u].x);
    acc[u].y = wave_sum(acc[u].y);
  }
  if (lane == 0) {
#pragma unroll
    for (int u = 0; u <= VC; ++u) red[wid][u] = acc[u];
  }
  __syncthreads();
  const int pr = p + 1;
  if (threadIdx.x < cnt) {
    double2 s = red[0][threadIdx.x];
#pragma unroll
    for (int ww = 1; ww < NW; ++ww) s = cadd(s, red[ww][threadIdx.x]);
    part[(size_t)rb * pr + i0 + threadIdx.x] = s;
  }
  if (with_norm && ch == 0 && threadIdx.x == 0) {
    double2 s = red[0][VC];
#pragma unroll
    for (int ww = 1; ww < NW; ++ww) s = cadd(s, red[ww][VC]);
    part[(size_t)rb * pr + p] = s;
  }
}

// w <- w - sum_i W_i c_i, with c from the reduced partial dots of the
// previous gs_dot launch.  pass 1: H(:,j) = s.*h, wnorm[j] = ||w||;
// pass 2: H(:,j) += s.*h and the partial ||w||^2 of the result.
template <typename T, int PASS>
__global__ __launch_bounds__(NT) void k_gs_update(T* __restrict__ W, int64_t ldq, int j,
                                                  T* __restrict__ w, int64_t n, int rpt,
                                                  const double2* __restrict__ part, int nrb,
                                                  ArnoldiDev arn, double* __restrict__ norm_part,
                                                  const int* skip) {
  if (skip && *skip) return;
  __shared__ double2 sums[kMaxK + 4];
  __shared__ double2 coef[kMaxK + 4];
  __shared__ double2 scratch[NT];
  __shared__ double nred[NW];
  const int p = j + 1;
  const int pr = p + 1;
  reduce_cols(part, nrb, pr, sums, scratch);
  for (int i = threadIdx.x; i < p; i += NT) {
    const double s = arn.scale[i];
    const double2 h = cscale(sums[i], s);
    coef[i] = cscale(h, s);
    if (blockIdx.x == 0) {
      const size_t idx = (size_t)j * arn.ldh + i;
      arn.H[idx] = (PASS == 1) ? h : cadd(arn.H[idx], h);
    }
  }
  if (PASS == 1 && blockIdx.x == 0 && threadIdx.x == 0) arn.wnorm[j] = sqrt(sums[p].x);
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * NT * rpt + threadIdx.x;
  double nrm = 0.0;
  for (int q = 0; q < rpt; ++q) {
    const int64_t r = base + (int64_t)q * NT;
    if (r >= n) break;
    double2 v = ld(w + r);
    int i = 0;
    for (; i + 4 <= p; i += 4) {
      const double2 q0 = ld(W + (int64_t)(i + 0) * ldq + r);
      const double2 q1 = ld(W + (int64_t)(i + 1) * ldq + r);
      const double2 q2 = ld(W + (int64_t)(i + 2) * ldq + r);
      const double2 q3 = ld(W + (int64_t)(i + 3) * ldq + r);
      v = csub(v, cmul(q0, coef[i + 0]));
      v = csub(v, cmul(q1, coef[i + 1]));
      v = csub(v, cmul(q2, coef[i + 2]));
      v = csub(v, cmul(q3, coef[i + 3]));
    }
    for (; i < p; ++i) v = csub(v, cmul(ld(W + (int64_t)i * ldq + r), coef[i]));
    st(w + r, v);
    if (PASS == 2) nrm += cabs2(ld(w + r));   // norm of the stored value
  }
  if (PASS == 2) {
    nrm = wave_sum(nrm);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) nred[wid] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = nred[0];
#pragma unroll
      for (int ww = 1; ww < NW; ++ww) s += nred[ww];
      norm_part[blockIdx.x] = s;
    }
  }
}

}  // namespace

namespace {
__global__ __launch_bounds__(NT) void k_gs_finish(const double* norm_part, int nrb, int j,
                                                  ArnoldiDev arn, const int* skip) {
  if (skip && *skip) return;
  gs_finish_norm(norm_part, nrb, j, arn, true);
}
}  // namespace

template <typename T>
hipError_t gs_dot(const T* W, int64_t ldq, int p, const T* w, int64_t n, bool with_norm,
                  double2* part, const int* skip, hipStream_t s) {
  const int rpt = gs_rpt(n);
  dim3 grid(gs_row_blocks(n), (p + VC - 1) / VC);
  hipLaunchKernelGGL((k_gs_dot<T>), grid, dim3(NT), 0, s, W, ldq, p, w, n, rpt, with_norm ? 1 : 0,
                     part, skip);
  return hipGetLastError();
}

template <typename T>
hipError_t gs_update(T* W, int64_t ldq, int j, T* w, int64_t n, int pass, const double2* part,
                     const ArnoldiDev& arn, double* norm_part, const int* skip, hipStream_t s) {
  const int rpt = gs_rpt(n);
  const int nrb = gs_row_blocks(n);
  if (pass == 1)
    hipLaunchKernelGGL((k_gs_update<T, 1>), dim3(nrb), dim3(NT), 0, s, W, ldq, j, w, n, rpt, part, nrb,
                       arn, norm_part, skip);
  else
    hipLaunchKernelGGL((k_gs_update<T, 2>), dim3(nrb), dim3(NT), 0, s, W, ldq, j, w, n, rpt, part, nrb,
                       arn, norm_part, skip);
  return hipGetLastError();
}

hipError_t gs_finish(const double* norm_part, int64_t n, int j, const ArnoldiDev& arn,
                     const int* skip, hipStream_t s) {
  hipLaunchKernelGGL(k_gs_finish, dim3(1), dim3(NT), 0, s, norm_part, gs_row_blocks(n), j, arn, skip);
  return hipGetLastError();
}

template hipError_t gs_dot<double2>(const double2*, int64_t, int, const double2*, int64_t, bool,
                                    double2*, const int*, hipStream_t);
template hipError_t gs_dot<float2>(const float2*, int64_t, int, const float2*, int64_t, bool,
                                   double2*, const int*, hipStream_t);
template hipError_t gs_update<double2>(double2*, int64_t, int, double2*, int64_t, int,
                                       const double2*, const ArnoldiDev&, double*, const int*,
                                       hipStream_t);
template hipError_t gs_update<float2>(float2*, int64_t, int, float2*, int64_t, int, const double2*,
                                      const ArnoldiDev&, double*, const int*, hipStream_t);

}  // namespace sk
