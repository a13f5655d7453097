// The overlap Dirac operator at nonzero chemical potential (Sect. 1: its
// inversion by iterative methods, each step applying sign(H_W) to a
// vector, is the main numerical effort that the paper's methods serve):
//
//   D(m) = (1 - m/2) (1 + gamma5 sign(H_W)) + m,
//
// massless at m = 0, with sign(H_W) b computed by sign_apply (Algorithm 1,
// restarted FOM-LR).  overlap_solve inverts D(m) by restarted GMRES with
// classical Gram-Schmidt applied twice; the small least-squares problem of
// each outer cycle (Givens rotations, at most 256 columns) runs on the host.
#include "krylov_ws.h"

#include <chrono>
#include <complex>
#include <cstring>
#include <vector>

namespace sk {
namespace {

constexpr int kOvThreads = 256;
constexpr int kMaxOuterK = 256;

// y = (1 + m/2) b + (1 - m/2) gamma5 s ; gamma5 = diag(1,1,-1,-1) in spin,
// i.e. the components 6..11 of the component-major field change sign.
__global__ __launch_bounds__(kOvThreads) void k_ov_combine(const double2* __restrict__ b,
                                                           const double2* __restrict__ s, double2* __restrict__ y,
                                                           int64_t n, int64_t V, double mass) {
  const int64_t r = (int64_t)blockIdx.x * kOvThreads + threadIdx.x;
  if (r >= n) return;
  const double cb = 1.0 + 0.5 * mass;
  const double cs = (r >= 6 * V ? -1.0 : 1.0) * (1.0 - 0.5 * mass);
  const double2 bv = b[r], sv = s[r];
  y[r] = make_double2(cb * bv.x + cs * sv.x, cb * bv.y + cs * sv.y);
}

// out = b - v
__global__ __launch_bounds__(kOvThreads) void k_ov_sub(const double2* __restrict__ b, const double2* __restrict__ v,
                                                       double2* __restrict__ out, int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * kOvThreads + threadIdx.x;
  if (r < n) out[r] = csub(b[r], v[r]);
}

struct OvWs {
  void* sign_ws;
  size_t sign_bytes;
  double2* sb;        // sign(H_W) v
  double2* r;         // residual / operator output
  double2* Vo;        // outer basis, (k+1) slots
  double2* h;         // Gram-Schmidt coefficients (two passes)
  double2* h2;
  double2* coef;      // x += V y
  double* nrm;        // norms
  double2* partial;
  unsigned* counter;
  CycleState* st;
};

size_t carve_ov(Carver& c, OvWs& o, const sk_operator* op, const sk_sign_params* p, int kout) {
  const int64_t n = 12 * volume_of(op);
  o.sign_bytes = sign_apply_workspace_bytes(op, p);
  o.sign_ws = c.take<char>(o.sign_bytes);
  o.sb = c.take<double2>(n);
  o.r = c.take<double2>(n);
  o.Vo = kout > 0 ? c.take<double2>((size_t)(kout + 1) * n) : nullptr;
  o.h = c.take<double2>(kMaxOuterK + 2);
  o.h2 = c.take<double2>(kMaxOuterK + 2);
  o.coef = c.take<double2>(kMaxOuterK + 2);
  o.nrm = c.take<double>(4);
  o.partial = c.take<double2>(ts_partial_entries(n, kMaxOuterK + 1));
  o.counter = c.take<unsigned>((size_t)4 * ts_counter_stride(n));
  o.st = c.take<CycleState>(1);
  return c.off;
}

// out = D(m) v, with one sign_apply; inner statistics added to *mv.
int apply_d(const sk_operator* op, const sk_sign_params* p, double mass, const double2* v, double2* out,
            OvWs& o, int64_t n, int64_t* mv, int64_t* calls, hipStream_t s) {
  sk_stats st;
  std::memset(&st, 0, sizeof(st));
  const int rc = sign_apply(op, p, (const double*)v, (double*)o.sb, &st, o.sign_ws, o.sign_bytes, s);
  if (mv) *mv += st.matvecs;
  if (calls) *calls += 1;
  if (rc != SK_OK) return rc;   // the message of the inner solve stays in place
  hipLaunchKernelGGL(k_ov_combine, dim3((unsigned)((n + kOvThreads - 1) / kOvThreads)), dim3(kOvThreads), 0, s,
                     v, o.sb, out, n, n / 12, mass);
  SK_LAUNCH(hipGetLastError());
  return SK_OK;
}

// ||v||^2 into nrm[slot] (fixed-order reduction), read back.
int norm_of(const double2* v, int64_t n, OvWs& o, int slot, double& out, hipStream_t s) {
  ArnoldiDev a;
  std::memset(&a, 0, sizeof(a));
  a.st = o.st;
  TsEpiArgs e = epi_of(EPI_XNORM, a);
  e.dst_scalar = o.nrm + slot;
  SK_LAUNCH((ts_dot<double2, double2>(nullptr, n, 0, v, n, true, e, o.partial, o.counter, nullptr, s)));
  double h;
  SK_HIP(hipMemcpyAsync(&h, o.nrm + slot, sizeof(double), hipMemcpyDeviceToHost, s));
  SK_HIP(hipStreamSynchronize(s));
  out = std::sqrt(h);
  return SK_OK;
}

}  // namespace
}  // namespace sk

using namespace sk;

extern "C" {

size_t overlap_workspace_bytes(const sk_operator* op, const sk_sign_params* p, int k_outer) {
  if (!op || !p || volume_of(op) <= 0 || k_outer < 0 || k_outer > kMaxOuterK || p->X_shift) return 0;
  if (sign_apply_workspace_bytes(op, p) == 0) return 0;
  Carver c;
  OvWs o;
  return carve_ov(c, o, op, p, k_outer);
}

int overlap_apply(const sk_operator* op, const sk_sign_params* p, double mass, const double* b, double* y,
                  sk_stats* stats, void* ws, size_t ws_bytes, hipStream_t s) {
  SK_TRY(check_operator(op, SK_C128));
  SK_CHECK(std::isfinite(mass), "mass must be finite");
  SK_CHECK(b && y && ws, "b, y and ws must be non-NULL");
  const int64_t n = 12 * volume_of(op);
  SK_CHECK(!overlap(b, n * 16, y, n * 16), "b and y overlap");
  const size_t need = overlap_workspace_bytes(op, p, 0);
  if (need == 0) {
    set_error("invalid sign parameters for the overlap operator");
    return SK_ERR_ARG;
  }
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return SK_ERR_WORKSPACE;
  }
  SK_CHECK(!overlap(ws, need, b, n * 16) && !overlap(ws, need, y, n * 16), "workspace overlaps b or y");
  Carver c;
  c.base = (char*)ws;
  OvWs o;
  carve_ov(c, o, op, p, 0);
  const int rc = sign_apply(op, p, b, (double*)o.sb, stats, o.sign_ws, o.sign_bytes, s);
  if (rc != SK_OK) return rc;
  hipLaunchKernelGGL(k_ov_combine, dim3((unsigned)((n + kOvThreads - 1) / kOvThreads)), dim3(kOvThreads), 0, s,
                     (const double2*)b, o.sb, (double2*)y, n, n / 12, mass);
  SK_LAUNCH(hipGetLastError());
  return SK_OK;
}

int overlap_solve(const sk_operator* op, const sk_sign_params* p, double mass, int k_outer, int max_outer,
                  double tol_outer, const double* b, double* x, sk_overlap_stats* stats, void* ws,
                  size_t ws_bytes, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  SK_TRY(check_operator(op, SK_C128));
  SK_CHECK(std::isfinite(mass), "mass must be finite");
  SK_CHECK(k_outer >= 1 && k_outer <= kMaxOuterK, "k_outer = %d outside [1, %d]", k_outer, kMaxOuterK);
  SK_CHECK(max_outer >= 1, "max_outer must be >= 1");
  SK_CHECK(tol_outer > 0.0 && std::isfinite(tol_outer), "tol_outer must be positive");
  SK_CHECK(b && x && ws, "b, x and ws must be non-NULL");
  const int64_t n = 12 * volume_of(op);
  SK_CHECK(!overlap(b, n * 16, x, n * 16), "b and x overlap");
  const size_t need = overlap_workspace_bytes(op, p, k_outer);
  if (need == 0) {
    set_error("invalid sign parameters for the overlap operator");
    return SK_ERR_ARG;
  }
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return SK_ERR_WORKSPACE;
  }
  SK_CHECK(!overlap(ws, need, b, n * 16) && !overlap(ws, need, x, n * 16), "workspace overlaps b or x");
  Carver c;
  c.base = (char*)ws;
  OvWs o;
  carve_ov(c, o, op, p, k_outer);
  if (stats) std::memset(stats, 0, sizeof(*stats));
  int64_t mv = 0, calls = 0;
  ArnoldiDev a;
  std::memset(&a, 0, sizeof(a));
  a.st = o.st;
  const TsEpiArgs e0 = epi_of(EPI_NONE, a);
  const int cs = ts_counter_stride(n);
  SK_LAUNCH(launch_init_state(o.st, nullptr, 0, o.counter, 4 * cs, s));
  SK_LAUNCH(launch_fill_zero(x, n * 2, s));
  double bnorm = 0.0;
  SK_TRY(norm_of((const double2*)b, n, o, 0, bnorm, s));
  if (!std::isfinite(bnorm)) {
    set_error("source contains non-finite values");
    return SK_ERR_NAN;
  }
  using cd = std::complex<double>;
  const int ld = k_outer + 1;
  std::vector<cd> H((size_t)ld * k_outer), g(ld), cs_(k_outer), sn(k_outer), y(k_outer);
  int status = SK_ERR_NOCONV;
  int outer = 0, restarts = 0;
  double relres = bnorm > 0.0 ? 1.0 : 0.0;
  if (bnorm == 0.0) status = SK_OK;
  while (status != SK_OK && outer < max_outer) {
    // r = b - D x (x = 0 at the first cycle: r = b)
    if (outer == 0) {
      SK_LAUNCH((ts_scale<double2, double2>((const double2*)b, o.Vo, n, nullptr, 1.0, s)));
    } else {
      SK_TRY(apply_d(op, p, mass, (const double2*)x, o.r, o, n, &mv, &calls, s));
      hipLaunchKernelGGL(k_ov_sub, dim3((unsigned)((n + kOvThreads - 1) / kOvThreads)), dim3(kOvThreads), 0, s,
                         (const double2*)b, o.r, o.Vo, n);
      SK_LAUNCH(hipGetLastError());
    }
    double beta = 0.0;
    SK_TRY(norm_of(o.Vo, n, o, 1, beta, s));
    relres = beta / bnorm;
    if (relres <= tol_outer) {
      status = SK_OK;
      break;
    }
    SK_LAUNCH((ts_scale<double2, double2>(o.Vo, o.Vo, n, nullptr, 1.0 / beta, s)));
    std::fill(g.begin(), g.end(), cd(0.0));
    g[0] = beta;
    int j = 0;
    for (; j < k_outer && outer < max_outer; ++j, ++outer) {
      double2* vj1 = o.Vo + (size_t)(j + 1) * n;
      SK_TRY(apply_d(op, p, mass, o.Vo + (size_t)j * n, vj1, o, n, &mv, &calls, s));
      // two classical Gram-Schmidt passes against v_0..v_j
      TsEpiArgs eh = epi_of(EPI_STORE, a);
      eh.out = o.h;
      SK_LAUNCH((ts_dot<double2, double2>(o.Vo, n, j + 1, vj1, n, false, eh, o.partial, o.counter, nullptr, s)));
      SK_LAUNCH((ts_update<double2, double2, double2>(o.Vo, n, j + 1, o.h, nullptr, vj1, vj1, n, 0, e0, o.partial,
                                                      o.counter + cs, nullptr, s)));
      TsEpiArgs eh2 = epi_of(EPI_STORE, a);
      eh2.out = o.h2;
      SK_LAUNCH((ts_dot<double2, double2>(o.Vo, n, j + 1, vj1, n, false, eh2, o.partial, o.counter + 2 * cs,
                                          nullptr, s)));
      TsEpiArgs en = epi_of(EPI_XNORM, a);
      en.dst_scalar = o.nrm + 2;
      SK_LAUNCH((ts_update<double2, double2, double2>(o.Vo, n, j + 1, o.h2, nullptr, vj1, vj1, n, 2, en,
                                                      o.partial, o.counter + 3 * cs, nullptr, s)));
      std::vector<double2> hh(j + 1), hh2(j + 1);
      double hn2 = 0.0;
      SK_HIP(hipMemcpyAsync(hh.data(), o.h, (j + 1) * sizeof(double2), hipMemcpyDeviceToHost, s));
      SK_HIP(hipMemcpyAsync(hh2.data(), o.h2, (j + 1) * sizeof(double2), hipMemcpyDeviceToHost, s));
      SK_HIP(hipMemcpyAsync(&hn2, o.nrm + 2, sizeof(double), hipMemcpyDeviceToHost, s));
      SK_HIP(hipStreamSynchronize(s));
      const double hn = std::sqrt(hn2);
      if (!std::isfinite(hn)) {
        set_error("non-finite value in the outer GMRES");
        return SK_ERR_NAN;
      }
      for (int i = 0; i <= j; ++i) H[i + (size_t)j * ld] = cd(hh[i].x + hh2[i].x, hh[i].y + hh2[i].y);
      H[j + 1 + (size_t)j * ld] = hn;
      // previous rotations, then a new one zeroing H[j+1, j]
      for (int i = 0; i < j; ++i) {
        const cd t = cs_[i] * H[i + (size_t)j * ld] + sn[i] * H[i + 1 + (size_t)j * ld];
        H[i + 1 + (size_t)j * ld] = -std::conj(sn[i]) * H[i + (size_t)j * ld] + cs_[i] * H[i + 1 + (size_t)j * ld];
        H[i + (size_t)j * ld] = t;
      }
      const cd hjj = H[j + (size_t)j * ld];
      const double den = std::sqrt(std::norm(hjj) + hn * hn);
      if (den == 0.0) {
        set_error("outer GMRES: zero column (operator maps a basis vector to 0)");
        return SK_ERR_SINGULAR;
      }
      cs_[j] = std::abs(hjj) / den;
      const cd ph = std::abs(hjj) > 0.0 ? hjj / std::abs(hjj) : cd(1.0);
      sn[j] = ph * hn / den;
      H[j + (size_t)j * ld] = ph * den;
      H[j + 1 + (size_t)j * ld] = 0.0;
      g[j + 1] = -std::conj(sn[j]) * g[j];
      g[j] = cs_[j] * g[j];
      relres = std::abs(g[j + 1]) / bnorm;
      if (relres <= tol_outer || hn <= 1e-14 * std::abs(H[j + (size_t)j * ld])) {
        ++j;
        ++outer;
        break;
      }
      SK_LAUNCH((ts_scale<double2, double2>(vj1, vj1, n, nullptr, 1.0 / hn, s)));
    }
    // y = R^{-1} g, x += V_j y
    for (int i = j - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int q = i + 1; q < j; ++q) acc -= H[i + (size_t)q * ld] * y[q];
      y[i] = acc / H[i + (size_t)i * ld];
    }
    std::vector<double2> yd(j);
    for (int i = 0; i < j; ++i) yd[i] = make_double2(y[i].real(), y[i].imag());
    SK_HIP(hipMemcpyAsync(o.coef, yd.data(), j * sizeof(double2), hipMemcpyHostToDevice, s));
    SK_LAUNCH((ts_gemv<double2>(o.Vo, n, j, o.coef, (double2*)x, n, true, 0, e0, nullptr, nullptr, nullptr,
                                nullptr, s)));
    SK_HIP(hipStreamSynchronize(s));   // yd leaves scope
    ++restarts;
    if (relres <= tol_outer) {
      // confirm with the true residual
      SK_TRY(apply_d(op, p, mass, (const double2*)x, o.r, o, n, &mv, &calls, s));
      hipLaunchKernelGGL(k_ov_sub, dim3((unsigned)((n + kOvThreads - 1) / kOvThreads)), dim3(kOvThreads), 0, s,
                         (const double2*)b, o.r, o.r, n);
      SK_LAUNCH(hipGetLastError());
      double rn = 0.0;
      SK_TRY(norm_of(o.r, n, o, 3, rn, s));
      relres = rn / bnorm;
      if (relres <= 10.0 * tol_outer) status = SK_OK;
    }
  }
  if (stats) {
    stats->outer_iters = outer;
    stats->restarts = restarts;
    stats->sign_calls = calls;
    stats->inner_matvecs = mv;
    stats->rel_residual = relres;
    stats->converged = status == SK_OK;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (status != SK_OK) set_error("overlap_solve: relative residual %.3e after %d outer iterations", relres, outer);
  return status;
}

}  // extern "C"
