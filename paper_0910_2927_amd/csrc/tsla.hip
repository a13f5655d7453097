// Tall-skinny kernels: the Gram-Schmidt sweeps of the Arnoldi process
// (Sect. 2, Arnoldi relation), the solution update x += V_k u (Algorithm 1)
// and the deflation projections (Sect. 4).  All are bandwidth-bound
// streams over n-row vectors; every reduction accumulates in double and is
// finished deterministically by the last block to arrive (fixed order).
#include "sk_internal.h"

namespace sk {

int ts_blocks(int64_t n) { return (int)((n + kTsThreads - 1) / kTsThreads); }
int ts_counter_stride(int64_t n) { return 1 + (ts_blocks(n) + 15) / 16; }
size_t ts_partial_entries(int64_t n, int pmax) {
  const size_t nb = (size_t)ts_blocks(n);
  return (nb + (nb + 15) / 16) * (size_t)(pmax + 2);
}

namespace {

constexpr int NT = kTsThreads;   // threads per block
constexpr int NW = NT / 64;      // waves per block
constexpr int CH = 8;            // vectors per reduction round

__device__ inline double2 zero2() { return make_double2(0.0, 0.0); }

// Reduce `cnt` (<= CH) complex values over the block; thread i < cnt writes
// the block total of value i to dst[i].
__device__ inline void block_reduce_store(double2 (&v)[CH], int cnt, double2* lds, double2* dst) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int u = 0; u < CH; ++u) {
    if (u < cnt) {
      v[u].x = wave_sum(v[u].x);
      v[u].y = wave_sum(v[u].y);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (u < cnt) lds[wid * CH + u] = v[u];
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    double2 s = lds[threadIdx.x];
#pragma unroll
    for (int w = 1; w < NW; ++w) s = cadd(s, lds[w * CH + threadIdx.x]);
    dst[threadIdx.x] = s;
  }
  __syncthreads();
}

__device__ inline double block_sum1(double v, double* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double s = lds[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) s += lds[w];
  __syncthreads();
  return s;
}

// The work the last block does with the reduced sums.
__device__ void run_epilogue(const TsEpiArgs& e, const double2* sums, int p) {
  const int t = threadIdx.x;
  const ArnoldiDev& a = e.arn;
  switch (e.epi) {
    case EPI_ARN_H1: {
      const int j = e.j;
      for (int i = t; i <= j; i += NT) {
        double s = a.scale[i];
        double2 h = cscale(sums[i], s);
        a.H[(size_t)j * a.ldh + i] = h;
        a.coef[i] = cscale(h, s);
      }
      if (t == 0) a.wnorm[j] = sqrt(sums[p].x);
      break;
    }
    case EPI_ARN_H2: {
      const int j = e.j;
      for (int i = t; i <= j; i += NT) {
        double s = a.scale[i];
        double2 h = cscale(sums[i], s);
        size_t idx = (size_t)j * a.ldh + i;
        a.H[idx] = cadd(a.H[idx], h);
        a.coef[i] = cscale(h, s);
      }
      break;
    }
    case EPI_ARN_NORM: {
      if (t == 0) {
        const int j = e.j;
        double nrm = sqrt(sums[0].x);
        double ref = a.wnorm[j];
        size_t idx = (size_t)j * a.ldh + j + 1;
        if (!isfinite(nrm) || !isfinite(ref)) {
          a.st->nonfinite = 1;
          a.st->breakdown = 1;
          a.st->kdone = j + 1;
          a.H[idx] = zero2();
          a.scale[j + 1] = 0.0;
        } else if (nrm <= kBreakdownTol * ref) {
          a.st->breakdown = 1;
          a.st->kdone = j + 1;
          a.H[idx] = zero2();
          a.scale[j + 1] = 0.0;
        } else {
          a.H[idx] = make_double2(nrm, 0.0);
          a.scale[j + 1] = 1.0 / nrm;
          a.st->kdone = j + 1;
        }
      }
      break;
    }
    case EPI_STORE: {
      double al = e.alpha ? *e.alpha : 1.0;
      for (int i = t; i < p; i += NT) e.out[i] = cscale(sums[i], al);
      break;
    }
    case EPI_BETA: {
      if (t == 0) {
        double beta = sqrt(sums[0].x);
        *e.dst_scalar = beta;
        *e.dst_scale = (beta > 0.0 && isfinite(beta)) ? 1.0 / beta : 0.0;
        if (!isfinite(beta)) a.st->nonfinite = 1;
      }
      break;
    }
    case EPI_XNORM: {
      if (t == 0) {
        *e.dst_scalar = sums[0].x;
        if (!isfinite(sums[0].x)) a.st->nonfinite = 1;
      }
      break;
    }
    case EPI_DEFL: {
      __shared__ double red[NW];
      double al = e.alpha ? *e.alpha : 1.0;
      double l2 = 0.0;
      for (int i = t; i < p; i += NT) {
        double2 c = cscale(sums[i], al);
        e.out[i] = c;
        l2 += cabs2(c);
      }
      __syncthreads();
      double tot = block_sum1(l2, red);
      if (t == 0 && e.dst_scalar) *e.dst_scalar = sqrt(tot);
      if (e.F && e.out2) {
        __syncthreads();
        for (int i = t; i < p; i += NT) {
          double2 acc = zero2();
          for (int l = 0; l < p; ++l) acc = cadd(acc, cmul(e.F[(size_t)l * p + i], cscale(sums[l], al)));
          e.out2[i] = acc;
        }
      }
      break;
    }
    default:
      break;
  }
}

// Two-level deterministic reduction of the per-block partial sums
// partial[b*pr + i]: blocks form groups of kGroup; the last block of a group
// to finish sums the group's partials (fixed order) into gpart[g*pr + i];
// the last group to finish sums the group totals and runs the epilogue.
// Counters: counter[0] counts finished groups, counter[1 + g] blocks of group g;
// each is reset by the block that consumed it.
constexpr int kGroup = 16;

__device__ inline void sum_rows(const double2* src, int rows, int pr, double2* dst, bool to_lds) {
  __shared__ double2 lds[NT];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i0 = 0; i0 < pr; i0 += 64) {
    const int i = i0 + lane;
    double2 acc = zero2();
    if (i < pr) {
#pragma unroll 4
      for (int b = wid; b < rows; b += NW) acc = cadd(acc, src[(size_t)b * pr + i]);
    }
    lds[threadIdx.x] = acc;
    __syncthreads();
    if (wid == 0 && i < pr) {
      double2 s = lds[lane];
#pragma unroll
      for (int w = 1; w < NW; ++w) s = cadd(s, lds[w * 64 + lane]);
      dst[i] = s;
    }
    __syncthreads();
  }
  (void)to_lds;
}

__device__ inline void finish(const TsEpiArgs& e, double2* partial, int pr, int p,
                              unsigned* counter) {
  __shared__ int flag;
  __shared__ double2 sums[kMaxK + 4];
  const int nb = gridDim.x;
  const int ngroups = (nb + kGroup - 1) / kGroup;
  const int g = blockIdx.x / kGroup;
  const int gsize = min(kGroup, nb - g * kGroup);
  double2* gpart = partial + (size_t)nb * pr;   // group totals follow the block partials
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) flag = (atomicAdd(&counter[1 + g], 1u) == (unsigned)gsize - 1);
  __syncthreads();
  if (!flag) return;
  __threadfence();
  sum_rows(partial + (size_t)g * kGroup * pr, gsize, pr, gpart + (size_t)g * pr, false);
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    counter[1 + g] = 0u;
    flag = (atomicAdd(&counter[0], 1u) == (unsigned)ngroups - 1);
  }
  __syncthreads();
  if (!flag) return;
  __threadfence();
  sum_rows(gpart, ngroups, pr, sums, true);
  run_epilogue(e, sums, p);
  __syncthreads();
  if (threadIdx.x == 0) counter[0] = 0u;
}

// ------------------------------------------------------------------ kernels
template <typename TQ, typename TV>
__global__ __launch_bounds__(NT) void k_ts_dot(const TQ* __restrict__ Q, int64_t ldq, int p,
                                               const TV* __restrict__ v, int64_t n, int with_norm,
                                               TsEpiArgs epi, double2* partial, unsigned* counter,
                                               const int* skip) {
  if (skip && *skip) return;
  __shared__ double2 lds[NW * CH];
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  const bool act = r < n;
  const double2 w = act ? ld(v + r) : zero2();
  const int pr = p + with_norm;
  double2* part = partial + (size_t)blockIdx.x * pr;
  const int64_t rr = act ? r : 0;   // inactive lanes load a valid row and discard it
  for (int i0 = 0; i0 < p; i0 += CH) {
    double2 acc[CH];
    const int cnt = min(CH, p - i0);
    TQ raw[CH];   // all loads of the chunk in flight before any is used
#pragma unroll
    for (int u = 0; u < CH; ++u) raw[u] = Q[(int64_t)(i0 + min(u, cnt - 1)) * ldq + rr];
#pragma unroll
    for (int u = 0; u < CH; ++u) acc[u] = (act && u < cnt) ? cconjmul(cvt(raw[u]), w) : zero2();
    block_reduce_store(acc, cnt, lds, part + i0);
  }
  if (with_norm) {
    double2 acc[CH];
    acc[0] = make_double2(cabs2(w), 0.0);
    block_reduce_store(acc, 1, lds, part + p);
  }
  finish(epi, partial, pr, p, counter);
}

template <typename TQ, typename TI, typename TO>
__global__ __launch_bounds__(NT) void k_ts_update(const TQ* __restrict__ Q, int64_t ldq, int p,
                                                  const double2* __restrict__ coef,
                                                  const double* a, const TI* in, TO* out,
                                                  int64_t n, int red, TsEpiArgs epi,
                                                  double2* partial, unsigned* counter,
                                                  const int* skip) {
  if (skip && *skip) return;
  __shared__ double2 c[kMaxK + 4];
  __shared__ double2 lds[NW * CH];
  for (int i = threadIdx.x; i < p; i += NT) c[i] = coef[i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  const bool act = r < n;
  double2 w = zero2();
  if (act) {
    const double al = a ? *a : 1.0;
    w = cscale(ld(in + r), al);
    constexpr int B = 8;   // loads in flight per thread
    for (int i = 0; i < p; i += B) {
      TQ raw[B];
#pragma unroll
      for (int u = 0; u < B; ++u) raw[u] = Q[(int64_t)min(i + u, p - 1) * ldq + r];
#pragma unroll
      for (int u = 0; u < B; ++u)
        if (i + u < p) w = csub(w, cmul(cvt(raw[u]), c[i + u]));
    }
    st(out + r, w);
    // the stored (possibly rounded) value is what later passes see
    w = ld(out + r);
  }
  if (red == 0) return;
  int pr = 1;
  double2* part;
  if (red == 1) {
    pr = p;
    part = partial + (size_t)blockIdx.x * pr;
    const int64_t rr = act ? r : 0;
    for (int i0 = 0; i0 < p; i0 += CH) {
      double2 acc[CH];
      const int cnt = min(CH, p - i0);
      TQ raw[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) raw[u] = Q[(int64_t)(i0 + min(u, cnt - 1)) * ldq + rr];
#pragma unroll
      for (int u = 0; u < CH; ++u) acc[u] = (act && u < cnt) ? cconjmul(cvt(raw[u]), w) : zero2();
      block_reduce_store(acc, cnt, lds, part + i0);
    }
  } else {
    part = partial + blockIdx.x;
    double2 acc[CH];
    acc[0] = make_double2(cabs2(w), 0.0);
    block_reduce_store(acc, 1, lds, part);
  }
  finish(epi, partial, pr, red == 1 ? p : 1, counter);
}

template <typename TQ>
__global__ __launch_bounds__(NT) void k_ts_gemv(const TQ* __restrict__ Q, int64_t ldq, int p,
                                                const double2* __restrict__ coef, double2* y,
                                                int64_t n, int accumulate, int red, TsEpiArgs epi,
                                                double2* partial, unsigned* counter,
                                                const int* pdev, const int* skip) {
  if (skip && *skip) return;
  if (pdev) p = min(p, *pdev);
  __shared__ double2 c[kMaxK + 4];
  __shared__ double2 lds[NW * CH];
  for (int i = threadIdx.x; i < p; i += NT) c[i] = coef[i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  const bool act = r < n;
  double2 acc0 = zero2();
  if (act) {
    double2 s = accumulate ? y[r] : zero2();
    constexpr int B = 8;   // loads in flight per thread
    for (int i = 0; i < p; i += B) {
      TQ raw[B];
#pragma unroll
      for (int u = 0; u < B; ++u) raw[u] = Q[(int64_t)min(i + u, p - 1) * ldq + r];
#pragma unroll
      for (int u = 0; u < B; ++u)
        if (i + u < p) s = cadd(s, cmul(cvt(raw[u]), c[i + u]));
    }
    y[r] = s;
    acc0 = make_double2(cabs2(s), 0.0);
  }
  if (red != 2) return;
  double2 acc[CH];
  acc[0] = acc0;
  block_reduce_store(acc, 1, lds, partial + blockIdx.x);
  finish(epi, partial, 1, 1, counter);
}

// X_i += sum_j Q_j C[i*ldc + j] for the outputs i of this block row
// (grid.y picks kMgOut consecutive outputs).  Each thread takes kMgRows rows
// (r and r + NT) with kMgOut accumulators each, so that every coefficient,
// read from LDS (the same entry for all lanes), feeds kMgRows complex
// multiply-adds; 8 basis loads per row in flight.
constexpr int kMgOut = 8;
constexpr int kMgRows = 2;
template <typename TQ>
__global__ __launch_bounds__(NT) void k_ts_multi_gemv(const TQ* __restrict__ Q, int64_t ldq, int p,
                                                      const double2* __restrict__ C, int ldc,
                                                      int nout, double2* X, int64_t n,
                                                      const int* pdev) {
  if (pdev) p = min(p, *pdev);
  const int64_t r0 = (int64_t)blockIdx.x * (NT * kMgRows) + threadIdx.x;
  const int o0 = blockIdx.y * kMgOut;
  extern __shared__ double2 cl[];   // kMgOut x p
  for (int e = threadIdx.x; e < kMgOut * p; e += NT) {
    const int u = e / p, jj = e % p;
    cl[e] = (o0 + u < nout) ? C[(size_t)(o0 + u) * ldc + jj] : zero2();
  }
  __syncthreads();
  if (r0 >= n) return;
  int64_t rr[kMgRows];
#pragma unroll
  for (int w = 0; w < kMgRows; ++w) rr[w] = min(r0 + (int64_t)w * NT, n - 1);   // clamped rows are not stored
  double2 acc[kMgRows][kMgOut];
#pragma unroll
  for (int w = 0; w < kMgRows; ++w)
#pragma unroll
    for (int u = 0; u < kMgOut; ++u) acc[w][u] = zero2();
  constexpr int B = 8;   // basis loads in flight per row
  for (int j = 0; j < p; j += B) {
    TQ raw[kMgRows][B];
#pragma unroll
    for (int w = 0; w < kMgRows; ++w)
#pragma unroll
      for (int b = 0; b < B; ++b) raw[w][b] = Q[(int64_t)min(j + b, p - 1) * ldq + rr[w]];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (j + b >= p) break;
      double2 q[kMgRows];
#pragma unroll
      for (int w = 0; w < kMgRows; ++w) q[w] = cvt(raw[w][b]);
#pragma unroll
      for (int u = 0; u < kMgOut; ++u) {
        const double2 cf = cl[u * p + j + b];
#pragma unroll
        for (int w = 0; w < kMgRows; ++w) acc[w][u] = cadd(acc[w][u], cmul(q[w], cf));
      }
    }
  }
#pragma unroll
  for (int w = 0; w < kMgRows; ++w) {
    const int64_t r = r0 + (int64_t)w * NT;
    if (r >= n) break;
#pragma unroll
    for (int u = 0; u < kMgOut; ++u)
      if (o0 + u < nout) {
        double2* px = X + (int64_t)(o0 + u) * n + r;
        *px = cadd(*px, acc[w][u]);
      }
  }
}

template <typename TI, typename TO>
__global__ __launch_bounds__(NT) void k_ts_scale(const TI* in, TO* out, int64_t n,
                                                 const double* adev, double ahost) {
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (r >= n) return;
  const double a = adev ? *adev : ahost;
  st(out + r, cscale(ld(in + r), a));
}

template <typename T>
__global__ __launch_bounds__(NT) void k_scale_basis(T* Q, int64_t ldq, int p, const double* scale,
                                                    const int* pdev, int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= n) return;
  const int pe = pdev ? min(p, *pdev + 1) : p;
  if (j >= pe) return;
  T* q = Q + (int64_t)j * ldq + r;
  st(q, cscale(ld(q), scale[j]));
}

__global__ __launch_bounds__(NT) void k_fold_rows(const double* __restrict__ part, int64_t stride, int nrows,
                                                  int cnt, int cnt_last, double* __restrict__ rows) {
  __shared__ double red[NW];
  const int i = blockIdx.x;
  const int c = (i == nrows - 1) ? cnt_last : cnt;
  double a = 0.0;
  for (int e = threadIdx.x; e < c; e += NT) a += part[(size_t)i * stride + e];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += red[w];
    rows[i] = t;
  }
}

__global__ void k_init_state(CycleState* st, double2* rho, int npoles, unsigned* counter, int ncnt) {
  const int t = threadIdx.x;
  if (t == 0) {
    st->beta = 0.0; st->xnorm2 = 0.0; st->upd_norm = 0.0; st->leak = 0.0; st->hnext = 0.0;
    st->kdone = 0; st->breakdown = 0; st->singular = 0; st->nonfinite = 0;
  }
  for (int i = t; i < npoles; i += blockDim.x) rho[i] = make_double2(1.0, 0.0);
  for (int i = t; i < ncnt; i += blockDim.x) counter[i] = 0u;
}

__global__ void k_zero_u(unsigned* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}
__global__ void k_zero_d(double* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

}  // namespace

// ------------------------------------------------------------------ launchers
template <typename TQ, typename TV>
hipError_t ts_dot(const TQ* Q, int64_t ldq, int p, const TV* v, int64_t n, bool with_norm,
                  const TsEpiArgs& epi, double2* partial, unsigned* counter, const int* skip,
                  hipStream_t s) {
  hipLaunchKernelGGL((k_ts_dot<TQ, TV>), dim3(ts_blocks(n)), dim3(NT), 0, s, Q, ldq, p, v, n,
                     with_norm ? 1 : 0, epi, partial, counter, skip);
  return hipGetLastError();
}

template <typename TQ, typename TI, typename TO>
hipError_t ts_update(const TQ* Q, int64_t ldq, int p, const double2* coef, const double* a,
                     const TI* in, TO* out, int64_t n, int red, const TsEpiArgs& epi,
                     double2* partial, unsigned* counter, const int* skip, hipStream_t s) {
  hipLaunchKernelGGL((k_ts_update<TQ, TI, TO>), dim3(ts_blocks(n)), dim3(NT), 0, s, Q, ldq, p,
                     coef, a, in, out, n, red, epi, partial, counter, skip);
  return hipGetLastError();
}

template <typename TQ>
hipError_t ts_gemv(const TQ* Q, int64_t ldq, int p, const double2* coef, double2* y, int64_t n,
                   bool accumulate, int red, const TsEpiArgs& epi, double2* partial,
                   unsigned* counter, const int* pdev, const int* skip, hipStream_t s) {
  hipLaunchKernelGGL((k_ts_gemv<TQ>), dim3(ts_blocks(n)), dim3(NT), 0, s, Q, ldq, p, coef, y, n,
                     accumulate ? 1 : 0, red, epi, partial, counter, pdev, skip);
  return hipGetLastError();
}

template <typename TQ>
hipError_t ts_multi_gemv(const TQ* Q, int64_t ldq, int p, const double2* C, int ldc, int nout,
                         double2* X, int64_t n, const int* pdev, hipStream_t s) {
  const unsigned nbx = (unsigned)((n + (int64_t)NT * kMgRows - 1) / ((int64_t)NT * kMgRows));
  hipLaunchKernelGGL((k_ts_multi_gemv<TQ>), dim3(nbx, (nout + kMgOut - 1) / kMgOut), dim3(NT),
                     (size_t)kMgOut * (p > 0 ? p : 1) * sizeof(double2), s, Q, ldq, p, C, ldc, nout, X, n, pdev);
  return hipGetLastError();
}

template <typename TI, typename TO>
hipError_t ts_scale(const TI* in, TO* out, int64_t n, const double* adev, double ahost,
                    hipStream_t s) {
  hipLaunchKernelGGL((k_ts_scale<TI, TO>), dim3(ts_blocks(n)), dim3(NT), 0, s, in, out, n, adev,
                     ahost);
  return hipGetLastError();
}

template <typename T>
hipError_t ts_scale_basis(T* Q, int64_t ldq, int p, const double* scale, const int* pdev, int64_t n,
                          hipStream_t s) {
  hipLaunchKernelGGL((k_scale_basis<T>), dim3(ts_blocks(n), p), dim3(NT), 0, s, Q, ldq, p, scale,
                     pdev, n);
  return hipGetLastError();
}
template hipError_t ts_scale_basis<double2>(double2*, int64_t, int, const double*, const int*,
                                            int64_t, hipStream_t);
template hipError_t ts_scale_basis<float2>(float2*, int64_t, int, const double*, const int*,
                                           int64_t, hipStream_t);

hipError_t launch_init_state(CycleState* st, double2* rho, int npoles, unsigned* counter, int ncnt,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(256), 0, s, st, rho, npoles, counter, ncnt);
  return hipGetLastError();
}

hipError_t launch_fold_rows(const double* part, int64_t stride, int nrows, int cnt, int cnt_last,
                            double* rows, hipStream_t s) {
  hipLaunchKernelGGL(k_fold_rows, dim3(nrows), dim3(NT), 0, s, part, stride, nrows, cnt, cnt_last, rows);
  return hipGetLastError();
}

hipError_t launch_zero_counters(unsigned* counter, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u, dim3((n + 255) / 256), dim3(256), 0, s, counter, n);
  return hipGetLastError();
}

__global__ void k_fill_value(double* p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_value(double* p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_value, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_d, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

// explicit instantiations
#define SK_INST_DOT(TQ, TV)                                                                  \
  template hipError_t ts_dot<TQ, TV>(const TQ*, int64_t, int, const TV*, int64_t, bool,     \
                                     const TsEpiArgs&, double2*, unsigned*, const int*,     \
                                     hipStream_t);
SK_INST_DOT(double2, double2)
SK_INST_DOT(float2, float2)
SK_INST_DOT(double2, float2)
SK_INST_DOT(float2, double2)

#define SK_INST_UPD(TQ, TI, TO)                                                             \
  template hipError_t ts_update<TQ, TI, TO>(const TQ*, int64_t, int, const double2*,       \
                                            const double*, const TI*, TO*, int64_t, int,   \
                                            const TsEpiArgs&, double2*, unsigned*,         \
                                            const int*, hipStream_t);
SK_INST_UPD(double2, double2, double2)
SK_INST_UPD(float2, float2, float2)
SK_INST_UPD(double2, float2, float2)
SK_INST_UPD(double2, double2, float2)
SK_INST_UPD(double2, float2, double2)

template hipError_t ts_gemv<double2>(const double2*, int64_t, int, const double2*, double2*,
                                     int64_t, bool, int, const TsEpiArgs&, double2*, unsigned*,
                                     const int*, const int*, hipStream_t);
template hipError_t ts_gemv<float2>(const float2*, int64_t, int, const double2*, double2*,
                                    int64_t, bool, int, const TsEpiArgs&, double2*, unsigned*,
                                    const int*, const int*, hipStream_t);
template hipError_t ts_multi_gemv<double2>(const double2*, int64_t, int, const double2*, int,
                                           int, double2*, int64_t, const int*, hipStream_t);
template hipError_t ts_multi_gemv<float2>(const float2*, int64_t, int, const double2*, int, int,
                                          double2*, int64_t, const int*, hipStream_t);
template hipError_t ts_scale<double2, double2>(const double2*, double2*, int64_t, const double*,
                                               double, hipStream_t);
template hipError_t ts_scale<float2, float2>(const float2*, float2*, int64_t, const double*,
                                             double, hipStream_t);
template hipError_t ts_scale<double2, float2>(const double2*, float2*, int64_t, const double*,
                                              double, hipStream_t);
template hipError_t ts_scale<float2, double2>(const float2*, double2*, int64_t, const double*,
                                              double, hipStream_t);

}  // namespace sk
