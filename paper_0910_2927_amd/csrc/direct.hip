// The direct projection methods that Sect. 6 compares restarted FOM-LR
// with: one long Krylov run and the exact sign of the projected matrix,
//
//   x_k = x_P + ||(I - P) b|| V_k sign(M_k) e_1                  (eq. (direct))
//
// with M_k = H_k from k Arnoldi steps (CGS2, the kernels of the restarted
// solver) or M_k = T_k, the tridiagonal matrix of k two-sided Lanczos
// steps (the "2sL" method of Fig. 1).  sign(M_k) comes from Roberts'
// method, the Newton iteration X <- (X + X^{-1}) / 2 (Sect. 6), run in FP64
// by one workgroup on the device with Gauss-Jordan inversions.
#include "krylov_ws.h"

#include <chrono>
#include <cstring>
#include <vector>

namespace sk {
namespace {

constexpr int kNewtonThreads = 1024;
constexpr int kNewtonMaxK = kMaxK;

struct NewtonState {
  int iters;
  int singular;
  int converged;
  int pad;
  double change;      // relative Frobenius change of the last iteration
};

__device__ inline double2 cinv(double2 a) { return cdiv(make_double2(1.0, 0.0), a); }

// Block-wide sum of two doubles (fixed order).
__device__ inline void block_sum2(double& a, double& b, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) {
    red[2 * w] = a;
    red[2 * w + 1] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
  for (int i = 0; i < kNewtonThreads / 64; ++i) {
    sa += red[2 * i];
    sb += red[2 * i + 1];
  }
  a = sa;
  b = sb;
  __syncthreads();
}

// sign(M) for the leading kk x kk block of M (column-major, leading
// dimension ldm), by the Newton iteration with determinantal scaling
// X <- (mu X + (mu X)^{-1}) / 2, mu = |det X|^{-1/kk}, while the change is
// large (Higham's scaled Newton), unscaled afterwards.  X: kk x kk result
// (ld kk); Y: scratch of the same size.  On exit coef[i] = beta * X[i, 0]
// (the coefficients of V_k sign(M_k) e_1 beta).  One workgroup.
__global__ __launch_bounds__(kNewtonThreads) void k_newton_sign(const double2* __restrict__ M, int ldm,
                                                                const int* kk_dev, int kk_host,
                                                                double2* __restrict__ X,
                                                                double2* __restrict__ Y, int* piv,
                                                                const double* beta, double2* coef,
                                                                NewtonState* ns, int maxit) {
  __shared__ double2 colp[kNewtonMaxK];
  __shared__ double2 rowp[kNewtonMaxK];
  __shared__ double redv[kNewtonThreads / 64 * 2];
  __shared__ int redi[kNewtonThreads / 64];
  __shared__ double s_logdet;
  __shared__ int s_sing;
  const int k = kk_dev ? min(*kk_dev, kk_host) : kk_host;
  const int t = threadIdx.x, nt = kNewtonThreads;
  const int kk2 = k * k;
  for (int e = t; e < kk2; e += nt) X[e] = M[(e % k) + (size_t)(e / k) * ldm];
  if (t == 0) {
    s_sing = 0;
    ns->singular = 0;
    ns->converged = 0;
  }
  __syncthreads();
  double d_prev = 1e300;
  int it = 0;
  double change = 0.0;
  for (; it < maxit; ++it) {
    for (int e = t; e < kk2; e += nt) Y[e] = X[e];
    if (t == 0) s_logdet = 0.0;
    __syncthreads();
    // ---- Gauss-Jordan inversion of Y in place, row pivoting
    for (int p = 0; p < k; ++p) {
      double best = -1.0;
      int bi = k;
      for (int i = p + t; i < k; i += nt) {
        const double a = cabs2(Y[i + (size_t)p * k]);
        if (a > best) {
          best = a;
          bi = i;
        }
      }
      // argmax over the block, ties to the smaller row
      const int lane = t & 63, w = t >> 6;
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_down(best, off, 64);
        const int oi = __shfl_down(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == 0) {
        redv[w] = best;
        redi[w] = bi;
      }
      __syncthreads();
      if (t == 0) {
        double bb = redv[0];
        int ii = redi[0];
        for (int q = 1; q < nt / 64; ++q)
          if (redv[q] > bb || (redv[q] == bb && redi[q] < ii)) {
            bb = redv[q];
            ii = redi[q];
          }
        if (!(bb > 0.0) || ii >= k) {
          s_sing = 1;
          ii = p;
        }
        piv[p] = ii;
      }
      __syncthreads();
      if (s_sing) break;
      const int r = piv[p];
      if (r != p)
        for (int j = t; j < k; j += nt) {
          const double2 a = Y[p + (size_t)j * k];
          Y[p + (size_t)j * k] = Y[r + (size_t)j * k];
          Y[r + (size_t)j * k] = a;
        }
      __syncthreads();
      const double2 pv = Y[p + (size_t)p * k];
      const double2 ip = cinv(pv);
      for (int i = t; i < k; i += nt) colp[i] = (i == p) ? make_double2(0.0, 0.0) : Y[i + (size_t)p * k];
      for (int j = t; j < k; j += nt) rowp[j] = (j == p) ? ip : cmul(Y[p + (size_t)j * k], ip);
      if (t == 0) s_logdet += 0.5 * log(cabs2(pv));
      __syncthreads();
      for (int j = t; j < k; j += nt) Y[p + (size_t)j * k] = rowp[j];
      for (int e = t; e < kk2; e += nt) {
        const int i = e % k, j = e / k;
        if (i == p) continue;
        const double2 base = (j == p) ? make_double2(0.0, 0.0) : Y[e];
        Y[e] = csub(base, cmul(colp[i], rowp[j]));
      }
      __syncthreads();
    }
    if (s_sing) break;
    // undo the row interchanges as column interchanges, last first
    for (int p = k - 1; p >= 0; --p) {
      const int r = piv[p];
      if (r != p)
        for (int i = t; i < k; i += nt) {
          const double2 a = Y[i + (size_t)p * k];
          Y[i + (size_t)p * k] = Y[i + (size_t)r * k];
          Y[i + (size_t)r * k] = a;
        }
      __syncthreads();
    }
    // ---- X <- (mu X + Y / mu) / 2
    const double mu = (d_prev > 1e-2) ? exp(-s_logdet / k) : 1.0;
    double dn = 0.0, xn = 0.0;
    for (int e = t; e < kk2; e += nt) {
      const double2 x = X[e];
      const double2 xnew = make_double2(0.5 * (mu * x.x + Y[e].x / mu), 0.5 * (mu * x.y + Y[e].y / mu));
      dn += cabs2(csub(xnew, x));
      xn += cabs2(xnew);
      X[e] = xnew;
    }
    block_sum2(dn, xn, redv);
    change = sqrt(dn / xn);
    if (!isfinite(change)) {
      if (t == 0) s_sing = 1;
      __syncthreads();
      break;
    }
    // quadratic convergence levels off at rounding: stop at the tolerance or
    // once a small change no longer halves
    const bool stop = change < 1e-14 || (change < 1e-10 && change > 0.5 * d_prev);
    d_prev = change;
    if (stop) {
      ++it;
      if (t == 0) ns->converged = 1;
      break;
    }
  }
  __syncthreads();
  if (t == 0) {
    ns->iters = it;
    ns->singular = s_sing;
    ns->change = change;
  }
  const double b = beta ? *beta : 1.0;
  for (int i = t; i < k; i += nt) coef[i] = cscale(X[i], b);
}

// ---- two-sided Lanczos pieces (complex double).  Scalars of step j live
// in the (k+1) x k tridiagonal T: alpha_j = T[j, j], delta_j = T[j+1, j]
// (subdiagonal), beta_j = T[j, j+1] (superdiagonal).
struct LanczosState {
  int kdone;        // steps completed
  int stop;         // 1: no further steps (invariant subspace or breakdown)
  int serious;      // 1: w^H v = 0 with both vectors nonzero
  int pad;
};

constexpr int kLzThreads = 256;

// vh = z - alpha v_j - beta_{j-1} v_{j-1},  wh = y - conj(alpha) w_j - conj(delta_{j-1}) w_{j-1}
// in place (z, y in slots j+1), with per-block partial sums of
// [wh^H vh, ||vh||^2, ||wh||^2, ||z||^2].
__global__ __launch_bounds__(kLzThreads) void k_lz_update(double2* __restrict__ Vb, double2* __restrict__ Wb,
                                                          int64_t n, int j, const double2* __restrict__ T,
                                                          int ldt, const double2* __restrict__ alpha,
                                                          double2* __restrict__ part, const LanczosState* st) {
  if (st->stop) return;
  const double2 al = *alpha;
  const double2 bprev = j > 0 ? T[(j - 1) + (size_t)j * ldt] : make_double2(0.0, 0.0);
  const double2 dprev = j > 0 ? T[j + (size_t)(j - 1) * ldt] : make_double2(0.0, 0.0);
  const double2 alc = make_double2(al.x, -al.y), dpc = make_double2(dprev.x, -dprev.y);
  double s_re = 0.0, s_im = 0.0, vv = 0.0, ww = 0.0, zz = 0.0;
  const int64_t r = (int64_t)blockIdx.x * kLzThreads + threadIdx.x;
  if (r < n) {
    double2* v1 = Vb + (size_t)(j + 1) * n;
    double2* w1 = Wb + (size_t)(j + 1) * n;
    const double2 z = v1[r], y = w1[r];
    double2 vh = csub(z, cmul(al, Vb[(size_t)j * n + r]));
    double2 wh = csub(y, cmul(alc, Wb[(size_t)j * n + r]));
    if (j > 0) {
      vh = csub(vh, cmul(bprev, Vb[(size_t)(j - 1) * n + r]));
      wh = csub(wh, cmul(dpc, Wb[(size_t)(j - 1) * n + r]));
    }
    v1[r] = vh;
    w1[r] = wh;
    const double2 c = cconjmul(wh, vh);
    s_re = c.x;
    s_im = c.y;
    vv = cabs2(vh);
    ww = cabs2(wh);
    zz = cabs2(z);
  }
  __shared__ double red[5][kLzThreads / 64];
  s_re = wave_sum(s_re);
  s_im = wave_sum(s_im);
  vv = wave_sum(vv);
  ww = wave_sum(ww);
  zz = wave_sum(zz);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = s_re;
    red[1][w] = s_im;
    red[2][w] = vv;
    red[3][w] = ww;
    red[4][w] = zz;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double a = 0.0;
    for (int q = 0; q < kLzThreads / 64; ++q) a += red[threadIdx.x][q];
    reinterpret_cast<double*>(part + (size_t)blockIdx.x * 3)[threadIdx.x] = a;
  }
}

// One block: fold the partials (fixed order), set delta_j, beta_j, alpha_j
// in T and the stop flags.
__global__ __launch_bounds__(kLzThreads) void k_lz_scalars(const double2* __restrict__ part, int nb, int j,
                                                           int k, double2* T, int ldt,
                                                           const double2* __restrict__ alpha,
                                                           LanczosState* st, double tol) {
  if (st->stop) return;
  __shared__ double red[5][kLzThreads / 64];
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += kLzThreads) {
    const double* pp = reinterpret_cast<const double*>(part + (size_t)b * 3);
#pragma unroll
    for (int q = 0; q < 5; ++q) acc[q] += pp[q];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    acc[q] = wave_sum(acc[q]);
    if (lane == 0) red[q][w] = acc[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot[5];
    for (int q = 0; q < 5; ++q) {
      tot[q] = 0.0;
      for (int i = 0; i < kLzThreads / 64; ++i) tot[q] += red[q][i];
    }
    T[j + (size_t)j * ldt] = *alpha;
    const double2 s = make_double2(tot[0], tot[1]);
    const double vn = sqrt(tot[2]), wn = sqrt(tot[3]), zn = sqrt(tot[4]);
    st->kdone = j + 1;
    if (!isfinite(vn) || !isfinite(wn) || !isfinite(s.x) || !isfinite(s.y)) {
      st->stop = 1;
      st->serious = 1;
    } else if (vn <= tol * zn) {
      st->stop = 1;   // the right Krylov space is invariant: the projection is exact
      T[(j + 1) + (size_t)j * ldt] = make_double2(0.0, 0.0);
    } else {
      const double as = sqrt(cabs2(s));
      if (as <= tol * vn * wn) {
        st->stop = 1;
        st->serious = 1;
      } else {
        const double delta = sqrt(as);
        T[(j + 1) + (size_t)j * ldt] = make_double2(delta, 0.0);
        if (j + 1 < k) T[j + (size_t)(j + 1) * ldt] = cscale(s, 1.0 / delta);
      }
    }
  }
}

// v_{j+1} = vh / delta_j,  w_{j+1} = wh / conj(beta_j)
__global__ __launch_bounds__(kLzThreads) void k_lz_scale(double2* __restrict__ Vb, double2* __restrict__ Wb,
                                                         int64_t n, int j, const double2* __restrict__ T,
                                                         int ldt, const LanczosState* st) {
  if (st->stop) return;
  const double2 delta = T[(j + 1) + (size_t)j * ldt];
  // beta_j = s / delta; for the last step (no superdiagonal slot) recompute it
  // from delta alone is not possible, so the left vector keeps 1/delta there
  // (it is never used again).
  const double2 bj = (j + 1 < ldt - 1) ? T[j + (size_t)(j + 1) * ldt] : delta;
  const double2 ib = cinv(make_double2(bj.x, -bj.y));
  const double id = 1.0 / delta.x;
  const int64_t r = (int64_t)blockIdx.x * kLzThreads + threadIdx.x;
  if (r < n) {
    double2* v1 = Vb + (size_t)(j + 1) * n;
    double2* w1 = Wb + (size_t)(j + 1) * n;
    v1[r] = cscale(v1[r], id);
    w1[r] = cmul(w1[r], ib);
  }
}

__global__ void k_lz_init(LanczosState* st) {
  st->kdone = 0;
  st->stop = 0;
  st->serious = 0;
}

struct DirectWs {
  KrylovWs<double2> w;   // Arnoldi basis (slots 0..k) and scratch; V of Lanczos
  double2* Wl;           // Lanczos left basis (k+1 slots)
  double2* X;            // k x k sign
  double2* Y;            // k x k inverse scratch
  int* piv;
  NewtonState* ns;
  LanczosState* ls;
  double2* scal;         // Lanczos alpha (one per step)
  double2* lpart;        // Lanczos partials (3 complex per block)
  double* beta;
  double2* tmp;          // (I - L R^H) v_1 coefficients / scratch vector
};

size_t carve_direct(Carver& c, DirectWs& d, int64_t n, int k, int m, int method) {
  carve_krylov(c, d.w, n, k, 0, m, false);
  d.Wl = method == 1 ? c.take<double2>((size_t)(k + 1) * n) : nullptr;
  d.X = c.take<double2>((size_t)k * k);
  d.Y = c.take<double2>((size_t)k * k);
  d.piv = c.take<int>(k);
  d.ns = c.take<NewtonState>(1);
  d.ls = c.take<LanczosState>(1);
  d.scal = c.take<double2>(k + 1);
  d.lpart = c.take<double2>((size_t)3 * ts_blocks(n));
  d.beta = c.take<double>(2);
  return c.off;
}

}  // namespace
}  // namespace sk

using namespace sk;

extern "C" {

size_t direct_sign_workspace_bytes(const sk_operator* op, int method, int k, int m) {
  if (!op || volume_of(op) <= 0 || k < 1 || k > kMaxK || m < 0 || m > kMaxDefl ||
      (method != 0 && method != 1))
    return 0;
  Carver c;
  DirectWs d;
  return carve_direct(c, d, 12 * volume_of(op), k, m, method);
}

int direct_sign_apply(const sk_operator* op, int method, int k, int m, const double* R, const double* L,
                      const double* F, const double* b, double* x, double* S, sk_direct_stats* stats,
                      void* ws, size_t ws_bytes, hipStream_t s) {
  const auto t_start = std::chrono::steady_clock::now();
  SK_TRY(check_operator(op, SK_C128));
  SK_CHECK(method == 0 || method == 1, "method %d is neither 0 (Arnoldi) nor 1 (two-sided Lanczos)", method);
  SK_CHECK(k >= 1 && k <= kMaxK, "k = %d outside [1, %d]", k, kMaxK);
  SK_CHECK(m >= 0 && m <= kMaxDefl, "m = %d outside [0, %d]", m, kMaxDefl);
  SK_CHECK(m == 0 || (R && L && F), "m > 0 needs R, L and F");
  SK_CHECK(b && x && ws, "b, x and ws must be non-NULL");
  const int64_t n = 12 * volume_of(op);
  SK_CHECK(!overlap(b, n * 16, x, n * 16), "b and x overlap");
  const size_t need = direct_sign_workspace_bytes(op, method, k, m);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return SK_ERR_WORKSPACE;
  }
  SK_CHECK(!overlap(ws, need, x, n * 16) && !overlap(ws, need, b, n * 16), "workspace overlaps b or x");
  Carver c;
  c.base = (char*)ws;
  DirectWs d;
  carve_direct(c, d, n, k, m, method);
  KrylovWs<double2>& w = d.w;
  const ArnoldiDev a = arn_of(w, k);
  const int cs = ts_counter_stride(n);
  const double2* Rd = (const double2*)R;
  const double2* Ld = (const double2*)L;
  SK_LAUNCH(launch_init_state(w.st, w.rho, 0, w.counter, kCounterSlots * cs, s));
  SK_LAUNCH(launch_fill_zero((double*)w.H, (int64_t)(k + 1) * k * 2, s));
  SK_LAUNCH(launch_fill_value(w.scale, k + 2, 1.0, s));
  // x = x_P = R F L^H b ;  W_0 = r = (I - P) b, beta = ||r||
  const TsEpiArgs e0 = epi_of(EPI_NONE, a);
  if (m > 0) {
    TsEpiArgs ed = epi_of(EPI_DEFL, a);
    ed.out = w.dc;
    ed.out2 = w.dc2;
    ed.F = (const double2*)F;
    ed.dst_scalar = &w.st->leak;
    SK_LAUNCH((ts_dot<double2, double2>(Ld, n, m, (const double2*)b, n, false, ed, w.partial,
                                        w.counter + 4 * cs, nullptr, s)));
    SK_LAUNCH((ts_gemv<double2>(Rd, n, m, w.dc2, (double2*)x, n, false, 0, e0, nullptr, nullptr, nullptr,
                                nullptr, s)));
  } else {
    SK_LAUNCH(launch_fill_zero(x, n * 2, s));
  }
  TsEpiArgs eb = epi_of(EPI_BETA, a);
  eb.dst_scalar = d.beta;
  eb.dst_scale = d.beta + 1;
  SK_LAUNCH((ts_update<double2, double2, double2>(m > 0 ? Rd : nullptr, n, m, w.dc, nullptr,
                                                  (const double2*)b, w.W, n, 2, eb, w.partial,
                                                  w.counter + 5 * cs, nullptr, s)));
  double bh[2];
  SK_HIP(hipMemcpyAsync(bh, d.beta, sizeof(bh), hipMemcpyDeviceToHost, s));
  SK_HIP(hipStreamSynchronize(s));
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!std::isfinite(bh[0])) {
    set_error("source contains non-finite values");
    return SK_ERR_NAN;
  }
  if (bh[0] == 0.0) {   // (I - P) b = 0: x = x_P exactly
    if (stats) stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return SK_OK;
  }
  int kk = k;
  const double2* M = w.H;
  if (method == 0) {
    // k Arnoldi steps from r / beta (the first Gram-Schmidt step normalises W_0)
    SK_TRY(enqueue_arnoldi<double2>(op, w, n, k, 0, s));
    CycleState hs;
    SK_HIP(hipMemcpyAsync(&hs, w.st, sizeof(hs), hipMemcpyDeviceToHost, s));
    SK_HIP(hipStreamSynchronize(s));
    if (hs.nonfinite) {
      set_error("non-finite value in the Arnoldi process");
      return SK_ERR_NAN;
    }
    kk = hs.kdone;
    if (stats) stats->breakdown = hs.breakdown;
  } else {
    // two-sided Lanczos: v_1 = r / beta, w_1 = (I - L R^H) v_1 (w_1^H v_1 = 1
    // since L^H v_1 = 0)
    double2* Vb = w.W;
    double2* Wb = d.Wl;
    SK_LAUNCH((ts_scale<double2, double2>(Vb, Vb, n, d.beta + 1, 0.0, s)));
    if (m > 0) {
      TsEpiArgs es = epi_of(EPI_STORE, a);
      es.out = w.dc2;
      SK_LAUNCH((ts_dot<double2, double2>(Rd, n, m, Vb, n, false, es, w.partial, w.counter + 4 * cs,
                                          nullptr, s)));
      SK_LAUNCH((ts_update<double2, double2, double2>(Ld, n, m, w.dc2, nullptr, Vb, Wb, n, 0, e0,
                                                      w.partial, w.counter + 5 * cs, nullptr, s)));
    } else {
      SK_LAUNCH((ts_scale<double2, double2>(Vb, Wb, n, nullptr, 1.0, s)));
    }
    hipLaunchKernelGGL(k_lz_init, dim3(1), dim3(1), 0, s, d.ls);
    SK_LAUNCH(hipGetLastError());
    const int nb = ts_blocks(n);
    const int* stop = &d.ls->stop;
    for (int j = 0; j < k; ++j) {
      double2* vj = Vb + (size_t)j * n;
      double2* wj = Wb + (size_t)j * n;
      SK_LAUNCH((launch_wilson<double2, double2, double2>(op, (const double2*)op->links, vj,
                                                          Vb + (size_t)(j + 1) * n, 0, nullptr, stop, s)));
      SK_LAUNCH((launch_wilson<double2, double2, double2>(op, (const double2*)op->links, wj,
                                                          Wb + (size_t)(j + 1) * n, 1, nullptr, stop, s)));
      TsEpiArgs ea = epi_of(EPI_STORE, a);
      ea.out = d.scal + j;
      SK_LAUNCH((ts_dot<double2, double2>(wj, n, 1, Vb + (size_t)(j + 1) * n, n, false, ea, w.partial,
                                          w.counter + 4 * cs, stop, s)));
      hipLaunchKernelGGL(k_lz_update, dim3(nb), dim3(kLzThreads), 0, s, Vb, Wb, n, j, w.H, k + 1,
                         d.scal + j, d.lpart, d.ls);
      SK_LAUNCH(hipGetLastError());
      hipLaunchKernelGGL(k_lz_scalars, dim3(1), dim3(kLzThreads), 0, s, d.lpart, nb, j, k, w.H, k + 1,
                         d.scal + j, d.ls, kBreakdownTol);
      SK_LAUNCH(hipGetLastError());
      hipLaunchKernelGGL(k_lz_scale, dim3(nb), dim3(kLzThreads), 0, s, Vb, Wb, n, j, w.H, k + 1, d.ls);
      SK_LAUNCH(hipGetLastError());
    }
    LanczosState ls;
    SK_HIP(hipMemcpyAsync(&ls, d.ls, sizeof(ls), hipMemcpyDeviceToHost, s));
    SK_HIP(hipStreamSynchronize(s));
    if (ls.serious) {
      set_error("two-sided Lanczos broke down at step %d (w^H v = 0 or non-finite)", ls.kdone);
      if (stats) stats->k_done = ls.kdone;
      return SK_ERR_SINGULAR;
    }
    kk = ls.kdone;
    if (stats) stats->breakdown = ls.stop;
  }
  // sign(M_kk) by Newton, coefficients beta sign(M_kk) e_1, x += V_kk coef
  hipLaunchKernelGGL(k_newton_sign, dim3(1), dim3(kNewtonThreads), 0, s, M, k + 1, (const int*)nullptr, kk,
                     d.X, d.Y, d.piv, (const double*)d.beta, w.coef, d.ns, 100);
  SK_LAUNCH(hipGetLastError());
  SK_LAUNCH((ts_gemv<double2>(w.W, n, kk, w.coef, (double2*)x, n, true, 0, e0, nullptr, nullptr, nullptr,
                              nullptr, s)));
  if (S) SK_HIP(hipMemcpyAsync(S, d.X, (size_t)kk * kk * 16, hipMemcpyDeviceToDevice, s));
  NewtonState ns;
  SK_HIP(hipMemcpyAsync(&ns, d.ns, sizeof(ns), hipMemcpyDeviceToHost, s));
  SK_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->k_done = kk;
    stats->newton_iters = ns.iters;
    stats->newton_change = ns.change;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  }
  if (ns.singular) {
    set_error("sign of the projected %d x %d matrix: singular Newton iterate", kk, kk);
    return SK_ERR_SINGULAR;
  }
  if (!ns.converged) {
    set_error("Newton iteration for sign of the projected matrix did not converge (change %.3e)", ns.change);
    return SK_ERR_NOCONV;
  }
  return SK_OK;
}

}  // extern "C"
