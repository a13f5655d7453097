// Host side of libsignkrylov: argument checks, workspace layout, and the
// restart loop of Algorithm 1 (restarted FOM-LR(m,k)) built from the
// kernels in wilson.hip, tsla.hip and small.hip.
#include "krylov_ws.h"
#include "dense_host.h"

#include <chrono>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

namespace sk {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int check_operator(const sk_operator* op, sk_dtype dtype) {
  SK_CHECK(op != nullptr, "operator is NULL");
  for (int i = 0; i < 4; ++i) SK_CHECK(op->dims[i] >= 1, "dims[%d] = %d must be >= 1", i, op->dims[i]);
  const int64_t V = volume_of(op);
  SK_CHECK(V * 12 < (int64_t(1) << 31), "lattice too large (V = %lld)", (long long)V);
  SK_CHECK(std::isfinite(op->kappa) && std::isfinite(op->mu), "kappa and mu must be finite");
  SK_CHECK(dtype == SK_C128 || dtype == SK_C64, "unknown dtype %d", (int)dtype);
  if (dtype == SK_C128) SK_CHECK(op->links != nullptr, "links (complex double) are NULL");
  else SK_CHECK(op->links_c64 != nullptr, "links_c64 are NULL but a complex-float call was made");
  return SK_OK;
}

namespace {

std::mutex g_mu;

}  // namespace
}  // namespace sk

using namespace sk;

extern "C" {

const char* sk_last_error(void) { return sk::g_err; }

int kl_poles(int s, double c, double* sigma, double* omega) {
  SK_CHECK(s >= 1 && 2 * s <= kMaxPoles, "s = %d outside [1, %d]", s, kMaxPoles / 2);
  SK_CHECK(c > 0.0 && std::isfinite(c), "scale c must be positive");
  SK_CHECK(sigma && omega, "sigma/omega are NULL");
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < s; ++i) {
    const double th = pi / (2.0 * s) * (i + 0.5);
    const double tau = std::tan(th), cs = std::cos(th);
    const double w = 1.0 / (s * cs * cs);
    sigma[4 * i + 0] = 0.0;
    sigma[4 * i + 1] = tau / c;
    sigma[4 * i + 2] = 0.0;
    sigma[4 * i + 3] = -tau / c;
    omega[4 * i + 0] = w / (2.0 * c);
    omega[4 * i + 1] = 0.0;
    omega[4 * i + 2] = w / (2.0 * c);
    omega[4 * i + 3] = 0.0;
  }
  return SK_OK;
}

int64_t sk_volume(const sk_operator* op) { return volume_of(op); }

int wilson_apply(const sk_operator* op, sk_dtype dtype, const void* in, void* out, int adjoint,
                 hipStream_t stream) {
  SK_TRY(check_operator(op, dtype));
  const int64_t n = 12 * volume_of(op);
  SK_CHECK(in && out, "in/out must be non-NULL");
  SK_CHECK(!overlap(in, n * cbytes(dtype), out, n * cbytes(dtype)), "in and out overlap");
  if (dtype == SK_C128)
    SK_LAUNCH((launch_wilson<double2, double2, double2>(op, (const double2*)op->links, (const double2*)in,
                                                        (double2*)out, adjoint, nullptr, nullptr, stream)));
  else
    SK_LAUNCH((launch_wilson<float2, float2, float2>(op, (const float2*)op->links_c64, (const float2*)in,
                                                     (float2*)out, adjoint, nullptr, nullptr, stream)));
  return SK_OK;
}

// ------------------------------------------------------------------ arnoldi_cycle
}  // extern "C"

namespace sk {
// Scratch of arnoldi_cycle: everything but the basis and H, which the caller owns.
template <typename T>
static size_t carve_arnoldi(Carver& c, KrylovWs<T>& w, int64_t n, int k) {
  std::memset(&w, 0, sizeof(w));
  w.scale = c.template take<double>(k + 2);
  w.wnorm = c.template take<double>(k + 1);
  w.coef = c.template take<double2>(kMaxK + 4);
  w.partial = c.template take<double2>(ts_partial_entries(n, k));
  w.counter = c.template take<unsigned>((size_t)kCounterSlots * ts_counter_stride(n));
  w.st = c.template take<CycleState>(1);
  w.rho = c.template take<double2>(1);
  carve_gs(c, w, n, k);
  return c.off;
}

}  // namespace sk

extern "C" {

size_t arnoldi_cycle_workspace_bytes(const sk_operator* op, int k) {
  if (!op || k < 1 || k > kMaxK || volume_of(op) <= 0) return 0;
  Carver c;
  KrylovWs<double2> w;
  return carve_arnoldi(c, w, 12 * volume_of(op), k);
}

}  // extern "C"

namespace sk {
template <typename T>
static int arnoldi_impl(const sk_operator* op, T* V, double2* H, int k, int* k_done, void* ws,
                        hipStream_t s) {
  const int64_t n = 12 * volume_of(op);
  Carver c;
  c.base = (char*)ws;
  KrylovWs<T> w;
  carve_arnoldi(c, w, n, k);
  w.W = V;
  w.H = H;
  const ArnoldiDev a = arn_of(w, k);
  const int cs = ts_counter_stride(n);
  SK_LAUNCH(launch_init_state(w.st, w.rho, 0, w.counter, kCounterSlots * cs, s));
  SK_LAUNCH(launch_fill_zero((double*)H, (int64_t)(k + 1) * k * 2, s));
  (void)a;
  SK_TRY(enqueue_arnoldi<T>(op, w, n, k, 0, s));
  CycleState hs;
  SK_HIP(hipMemcpyAsync(&hs, w.st, sizeof(hs), hipMemcpyDeviceToHost, s));
  SK_HIP(hipStreamSynchronize(s));
  if (!(hs.beta > 0.0) || !std::isfinite(hs.beta)) {
    set_error("start vector is zero or not finite");
    return hs.beta > 0.0 ? SK_ERR_NAN : SK_ERR_ARG;
  }
  if (hs.nonfinite) {
    set_error("non-finite value in the Arnoldi process");
    return SK_ERR_NAN;
  }
  if (k_done) *k_done = hs.kdone;
  return SK_OK;
}

}  // namespace sk

extern "C" {

int arnoldi_cycle(const sk_operator* op, sk_dtype dtype, void* V, double* H, int k, int* k_done,
                  void* ws, size_t ws_bytes, hipStream_t stream) {
  SK_TRY(check_operator(op, dtype));
  SK_CHECK(k >= 1 && k <= kMaxK, "k = %d outside [1, %d]", k, kMaxK);
  SK_CHECK(V && H && ws, "V, H and ws must be non-NULL");
  const int64_t n = 12 * volume_of(op);
  const size_t need = arnoldi_cycle_workspace_bytes(op, k);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return SK_ERR_WORKSPACE;
  }
  SK_CHECK(!overlap(V, (size_t)(k + 1) * n * cbytes(dtype), H, (size_t)(k + 1) * k * 16),
           "V and H overlap");
  if (dtype == SK_C128) return arnoldi_impl<double2>(op, (double2*)V, (double2*)H, k, k_done, ws, stream);
  return arnoldi_impl<float2>(op, (float2*)V, (double2*)H, k, k_done, ws, stream);
}

// ------------------------------------------------------------------ multishift_fom_restart
size_t multishift_fom_restart_workspace_bytes(int k, int npoles) {
  if (k < 1 || k > kMaxK || npoles < 1 || npoles > kMaxPoles) return 0;
  Carver c;
  c.take<double>(k + 2);                      // scale (ones)
  c.take<CycleState>(1);
  c.take<double2>((size_t)npoles * k);        // Y
  c.take<double2>((size_t)npoles * k * k);    // U
  c.take<double2>(k + 1);                     // ucoef
  c.take<double2>((size_t)npoles * k);        // ycoef
  c.take<double2>(ts_partial_entries(1, 1));
  c.take<unsigned>(kCounterSlots * ts_counter_stride(1));
  return c.off;
}

}  // extern "C"

namespace sk {
__global__ void k_prep_small(double* scale, int k, CycleState* st, const double* beta) {
  int t = threadIdx.x;
  for (int i = t; i < k + 2; i += blockDim.x) scale[i] = 1.0;
  if (t == 0) {
    st->beta = *beta;
    st->kdone = k;
    st->breakdown = 0;
    st->singular = 0;
    st->nonfinite = 0;
  }
}

template <typename T>
static int msfom_impl(int k, int64_t n, const double2* H, const PoleSet& ps, const double* beta,
                      double2* rho, const T* V, double2* x, double2* X, double* upd, void* ws,
                      hipStream_t s) {
  Carver c;
  c.base = (char*)ws;
  double* scale = c.take<double>(k + 2);
  CycleState* st = c.take<CycleState>(1);
  double2* Y = c.take<double2>((size_t)ps.n * k);
  double2* U = c.take<double2>((size_t)ps.n * k * k);
  double2* ucoef = c.take<double2>(k + 1);
  double2* ycoef = c.take<double2>((size_t)ps.n * k);
  double2* partial = c.take<double2>(ts_partial_entries(1, 1));
  unsigned* counter = c.take<unsigned>(kCounterSlots * ts_counter_stride(1));
  ArnoldiDev a;
  std::memset(&a, 0, sizeof(a));
  a.H = const_cast<double2*>(H);
  a.scale = scale;
  a.st = st;
  a.ldh = k + 1;
  a.partial = partial;
  a.counter = counter;
  hipLaunchKernelGGL(k_prep_small, dim3(1), dim3(256), 0, s, scale, k, st, beta);
  SK_LAUNCH(hipGetLastError());
  SK_LAUNCH(launch_fom_small(a, k, ps, rho, Y, U, ucoef, X ? ycoef : nullptr, s));
  TsEpiArgs e = epi_of(EPI_NONE, a);
  SK_LAUNCH((ts_gemv<T>(V, n, k, ucoef, x, n, true, 0, e, nullptr, nullptr, nullptr, nullptr, s)));
  if (X) SK_LAUNCH((ts_multi_gemv<T>(V, n, k, ycoef, k, ps.n, X, n, nullptr, s)));
  CycleState hs;
  SK_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
  SK_HIP(hipStreamSynchronize(s));
  if (upd) *upd = hs.upd_norm;
  if (hs.singular) {
    set_error("H_k - sigma_i is singular for some pole");
    return SK_ERR_SINGULAR;
  }
  if (hs.nonfinite) {
    set_error("non-finite FOM iterate");
    return SK_ERR_NAN;
  }
  return SK_OK;
}

}  // namespace sk

extern "C" {

}  // extern "C"

namespace sk {
static int fill_poles(PoleSet& ps, int npoles, const double* sigma, const double* omega) {
  SK_CHECK(npoles >= 1 && npoles <= kMaxPoles, "npoles = %d outside [1, %d]", npoles, kMaxPoles);
  SK_CHECK(sigma && omega, "sigma/omega are NULL");
  ps.n = npoles;
  for (int i = 0; i < npoles; ++i) {
    ps.sigma[i] = make_double2(sigma[2 * i], sigma[2 * i + 1]);
    ps.omega[i] = make_double2(omega[2 * i], omega[2 * i + 1]);
    SK_CHECK(std::isfinite(sigma[2 * i]) && std::isfinite(sigma[2 * i + 1]) &&
                 std::isfinite(omega[2 * i]) && std::isfinite(omega[2 * i + 1]),
             "pole %d is not finite", i);
  }
  return SK_OK;
}

}  // namespace sk

extern "C" {

int multishift_fom_restart(int k, int64_t n, sk_dtype dtype, const double* H, int npoles,
                           const double* sigma, const double* omega, const double* beta,
                           double* rho, const void* V, double* x, double* X_shift,
                           double* upd_norm, void* ws, size_t ws_bytes, hipStream_t stream) {
  SK_CHECK(k >= 1 && k <= kMaxK, "k = %d outside [1, %d]", k, kMaxK);
  SK_CHECK(n >= 1, "n must be positive");
  SK_CHECK(dtype == SK_C128 || dtype == SK_C64, "unknown dtype");
  SK_CHECK(H && beta && rho && V && x && ws, "NULL argument");
  PoleSet ps;
  SK_TRY(fill_poles(ps, npoles, sigma, omega));
  const size_t need = multishift_fom_restart_workspace_bytes(k, npoles);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return SK_ERR_WORKSPACE;
  }
  if (dtype == SK_C128)
    return msfom_impl<double2>(k, n, (const double2*)H, ps, beta, (double2*)rho, (const double2*)V,
                               (double2*)x, (double2*)X_shift, upd_norm, ws, stream);
  return msfom_impl<float2>(k, n, (const double2*)H, ps, beta, (double2*)rho, (const float2*)V,
                            (double2*)x, (double2*)X_shift, upd_norm, ws, stream);
}

}  // extern "C"

namespace sk {
int deflate_project_check(int m, int64_t n, const double* R, const double* L, const double* F,
                          const double* in, const double* r_out, const double* xp_out, const double* coeff) {
  SK_CHECK(m >= 1 && m <= kMaxDefl, "m = %d outside [1, %d]", m, kMaxDefl);
  SK_CHECK(n >= 1, "n must be positive");
  SK_CHECK(R && L && in && r_out && coeff, "NULL argument");
  SK_CHECK(r_out == in || !overlap(in, n * 16, r_out, n * 16), "r_out partially overlaps in");
  if (xp_out) {
    SK_CHECK(F != nullptr, "xp_out requested without F");
    SK_CHECK(!overlap(xp_out, n * 16, in, n * 16) && !overlap(xp_out, n * 16, r_out, n * 16),
             "xp_out overlaps in/r_out");
  }
  return SK_OK;
}

// The projection kernels with their scratch (partial sums, counters, F c,
// state) carved from `scratch`, at least deflate_project_workspace_bytes(m, n).
// The counters are cleared by a kernel at the start of every call.
int deflate_project_run(int m, int64_t n, const double* R, const double* L, const double* F,
                        const double* in, double* r_out, double* xp_out, double* coeff, void* scratch,
                        hipStream_t s) {
  Carver c;
  c.base = (char*)scratch;
  double2* partial = c.take<double2>(ts_partial_entries(n, m));
  const int cs = ts_counter_stride(n);
  unsigned* counter = c.take<unsigned>(2 * cs);
  double2* fc = c.take<double2>(m);
  CycleState* st = c.take<CycleState>(1);
  ArnoldiDev a;
  std::memset(&a, 0, sizeof(a));
  a.st = st;
  SK_LAUNCH(launch_init_state(st, nullptr, 0, counter, 2 * cs, s));
  TsEpiArgs e = epi_of(EPI_DEFL, a);
  e.out = (double2*)coeff;
  e.out2 = xp_out ? fc : nullptr;
  e.F = xp_out ? (const double2*)F : nullptr;
  SK_LAUNCH((ts_dot<double2, double2>((const double2*)L, n, m, (const double2*)in, n, false, e,
                                      partial, counter, nullptr, s)));
  if (xp_out) {
    TsEpiArgs e0 = epi_of(EPI_NONE, a);
    SK_LAUNCH((ts_gemv<double2>((const double2*)R, n, m, fc, (double2*)xp_out, n, false, 0, e0,
                                nullptr, nullptr, nullptr, nullptr, s)));
  }
  TsEpiArgs e1 = epi_of(EPI_NONE, a);
  SK_LAUNCH((ts_update<double2, double2, double2>((const double2*)R, n, m, (const double2*)coeff,
                                                  nullptr, (const double2*)in, (double2*)r_out, n, 0,
                                                  e1, partial, counter + cs, nullptr, s)));
  return SK_OK;
}
}  // namespace sk

extern "C" {

// ------------------------------------------------------------------ deflate_project
size_t deflate_project_workspace_bytes(int m, int64_t n) {
  if (m < 1 || m > kMaxDefl || n < 1) return 0;
  Carver c;
  c.take<double2>(ts_partial_entries(n, m));
  c.take<unsigned>(2 * ts_counter_stride(n));
  c.take<double2>(m);
  c.take<CycleState>(1);
  return c.off;
}

int deflate_project(int m, int64_t n, const double* R, const double* L, const double* F,
                    const double* in, double* r_out, double* xp_out, double* coeff, void* ws,
                    size_t ws_bytes, hipStream_t s) {
  SK_TRY(deflate_project_check(m, n, R, L, F, in, r_out, xp_out, coeff));
  SK_CHECK(ws != nullptr, "NULL argument");
  const size_t need = deflate_project_workspace_bytes(m, n);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return SK_ERR_WORKSPACE;
  }
  return deflate_project_run(m, n, R, L, F, in, r_out, xp_out, coeff, ws, s);
}

}  // extern "C"

// ------------------------------------------------------------------ sign_apply
namespace sk {
namespace {

bool params_ok(const sk_sign_params* p, char* msg, size_t len) {
  if (!p) return snprintf(msg, len, "params are NULL"), false;
  if (p->npoles < 1 || p->npoles > kMaxPoles) return snprintf(msg, len, "npoles = %d outside [1, %d]", p->npoles, kMaxPoles), false;
  if (!p->sigma || !p->omega) return snprintf(msg, len, "sigma/omega are NULL"), false;
  if (p->k < 1 || p->k > kMaxK) return snprintf(msg, len, "k = %d outside [1, %d]", p->k, kMaxK), false;
  if (p->max_cycles < 1) return snprintf(msg, len, "max_cycles must be >= 1"), false;
  if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return snprintf(msg, len, "tol must be positive"), false;
  if (p->m < 0 || p->m > kMaxDefl) return snprintf(msg, len, "m = %d outside [0, %d]", p->m, kMaxDefl), false;
  if (p->m > 0 && (!p->R || !p->L || !p->F)) return snprintf(msg, len, "m > 0 needs R, L and F"), false;
  if (p->precision != SK_PREC_FP64 && p->precision != SK_PREC_MIXED) return snprintf(msg, len, "unknown precision %d", p->precision), false;
  if (p->method != SK_METHOD_FOM && p->method != SK_METHOD_GMRES) return snprintf(msg, len, "unknown method %d", p->method), false;
  if (p->method == SK_METHOD_GMRES && p->precision != SK_PREC_FP64) return snprintf(msg, len, "GMRES-LR runs in complex double only"), false;
  if (p->method == SK_METHOD_GMRES && (p->seed < -1 || p->seed >= p->npoles)) return snprintf(msg, len, "seed %d outside [-1, %d)", p->seed, p->npoles), false;
  if (!(p->mixed_switch >= 0.0)) return snprintf(msg, len, "mixed_switch must be >= 0"), false;
  return true;
}

// Two views of one workspace: the complex-double basis and, for the mixed
// path, a complex-float basis; every other array is shared.
struct SignWs {
  KrylovWs<double2> w64;
  KrylovWs<float2> w32;
  bool mixed;
  // per-shift solutions kept in the workspace (mixed precision without a
  // caller X_shift), and the buffers of the FP64 true-residual check
  double2* Xint;
  double2* rhs;       // (I - P) b
  double2* tmp;       // one shifted residual
  double* resid2;     // npoles squared residual norms, then ||rhs||^2
  double* rpart;      // per-pole partial sums of the squared residual norms
  double2* rnext;     // GMRES-LR: the next restart vector V_{k+1} z
  double2* zdev;      // GMRES-LR: z (k+1 entries)
};

size_t carve_sign(Carver& c, SignWs& sw, int64_t n, const sk_sign_params* p) {
  sw.mixed = p->precision == SK_PREC_MIXED;
  const bool keep = p->X_shift != nullptr || sw.mixed;
  carve_krylov(c, sw.w64, n, p->k, p->npoles, p->m, keep);
  std::memcpy(&sw.w32, &sw.w64, sizeof(sw.w32));   // same small arrays
  sw.w32.W = sw.mixed ? c.take<float2>((size_t)(p->k + 1) * n) : nullptr;
  sw.Xint = (sw.mixed && !p->X_shift) ? c.take<double2>((size_t)p->npoles * n) : nullptr;
  sw.rhs = keep ? c.take<double2>(n) : nullptr;
  sw.tmp = keep ? c.take<double2>(n) : nullptr;
  sw.resid2 = keep ? c.take<double>(p->npoles + 2) : nullptr;
  sw.rpart = keep ? c.take<double>((size_t)p->npoles * wilson_residual_partials(n / 12)) : nullptr;
  sw.rnext = p->method == SK_METHOD_GMRES ? c.take<double2>(n) : nullptr;
  sw.zdev = p->method == SK_METHOD_GMRES ? c.take<double2>((size_t)p->k + 1) : nullptr;
  return c.off;
}

// FP64 true residuals of the shifted systems, ||(I-P)b - (A - sigma_i) X_i||,
// relative to ||(I-P)b||, from N complex-double stencil applications
// (residual form of the Wilson kernel) and fixed-order norm reductions.
int true_residuals(const sk_operator* op, const sk_sign_params* p, const PoleSet& ps,
                   const double2* b, const double2* X, SignWs& sw, int64_t n,
                   std::vector<double>& rel, double& rhs_norm, hipStream_t s) {
  KrylovWs<double2>& w = sw.w64;
  const ArnoldiDev a = arn_of(w, p->k);
  const int cs = ts_counter_stride(n);
  const int N = ps.n;
  // rhs = (I - R L^H) b with the start's coefficients L^H b (still in dc)
  TsEpiArgs er = epi_of(EPI_XNORM, a);
  er.dst_scalar = sw.resid2 + N;
  SK_LAUNCH((ts_update<double2, double2, double2>(p->m > 0 ? (const double2*)p->R : nullptr, n, p->m,
                                                  w.dc, nullptr, b, sw.rhs, n, 2, er, w.partial,
                                                  w.counter + 5 * cs, nullptr, s)));
  // the residual stencil leaves per-wave partial norms; one fold per pole
  const int P = wilson_residual_partials(n / 12);
  for (int i = 0; i < N; ++i)
    SK_LAUNCH((launch_wilson_residual<double2>(op, (const double2*)op->links, X + (size_t)i * n,
                                               sw.rhs, ps.sigma[i], sw.tmp, sw.rpart + (size_t)i * P, s)));
  SK_LAUNCH(launch_fold_rows(sw.rpart, P, N, P, P, sw.resid2, s));
  std::vector<double> r2(N + 1);
  SK_HIP(hipMemcpyAsync(r2.data(), sw.resid2, (N + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
  SK_HIP(hipStreamSynchronize(s));
  rhs_norm = std::sqrt(r2[N]);
  rel.assign(N, 0.0);
  for (int i = 0; i < N; ++i) rel[i] = rhs_norm > 0.0 ? std::sqrt(r2[i]) / rhs_norm : std::sqrt(r2[i]);
  return SK_OK;
}

template <typename T> KrylovWs<T>& view(SignWs& sw);
template <> KrylovWs<double2>& view<double2>(SignWs& sw) { return sw.w64; }
template <> KrylovWs<float2>& view<float2>(SignWs& sw) { return sw.w32; }

struct CycleArgs {
  const sk_operator* op;
  const sk_sign_params* p;
  int64_t n;
  const PoleSet* ps;
  double2* x;
  double2* X;
  KTimer* tm;
  hipStream_t s;
};

// One restart cycle of Algorithm 1 with the basis in precision T; the
// restart vector goes to W_0 of the next cycle's precision TN.
template <typename T, typename TN>
int enqueue_cycle(const CycleArgs& ca, SignWs& sw) {
  KrylovWs<T>& w = view<T>(sw);
  KrylovWs<TN>& wn = view<TN>(sw);
  const int64_t n = ca.n;
  const int k = ca.p->k, m = ca.p->m, N = ca.ps->n;
  const ArnoldiDev a = arn_of(w, k);
  const int* skip = &w.st->breakdown;
  KTimer& tm = *ca.tm;
  const double cb = (double)sizeof(T), nn = (double)n;
  const double2* R = (const double2*)ca.p->R;
  const double2* Lv = (const double2*)ca.p->L;
  SK_TRY(enqueue_arnoldi<T>(ca.op, w, n, k, 0, ca.s, &tm));
  tm.begin(SK_K_SMALL, 0.0);
  SK_LAUNCH(launch_fom_small(a, k, *ca.ps, w.rho, w.Y, w.U, w.ucoef, ca.X ? w.ycoef : nullptr, ca.s));
  tm.end();
  tm.begin(SK_K_SOL_UPDATE, k * nn * cb + 2.0 * nn * 16.0);
  SK_LAUNCH((cycle_x_update<T>(w.W, n, w.ucoef, &w.st->kdone, ca.x, (double*)w.partial, w.st, ca.s)));
  tm.end();
  if (ca.X) {
    tm.begin(SK_K_SOL_UPDATE, k * nn * cb + 2.0 * N * nn * 16.0);
    SK_LAUNCH((ts_multi_gemv<T>(w.W, n, k, w.ycoef, k, N, ca.X, n, &w.st->kdone, ca.s)));
    tm.end();
  }
  // r = v_{k+1};  r = (I - P) r  (projection step); ||r|| is taken by the
  // next cycle's first Gram-Schmidt step
  const T* Wk = w.W + (size_t)k * n;
  const bool proj = m > 0 && ca.p->project_each_cycle;
  tm.begin(SK_K_PROJECT, (m > 0 ? m * nn * 16.0 + nn * cb : 0.0) + (proj ? m * nn * 16.0 : 0.0) + nn * cb +
                             nn * (double)sizeof(TN));
  SK_LAUNCH((cycle_restart<T, TN>(R, Lv, m, proj, Wk, wn.W, n, w.partial, w.st, skip, ca.s)));
  tm.end();
  return SK_OK;
}

// A stream that belongs to the library, used only to capture restart cycles
// into HIP graphs (the caller's stream may be the legacy null stream, which
// cannot be captured).  Default priority.
hipStream_t capture_stream() {
  static hipStream_t cs = nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!cs) {
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) cs = nullptr;
  }
  return cs;
}

// The three kinds of restart cycle (basis precision now -> next), each
// captured once per solve and replayed every cycle.
struct CycleGraphs {
  hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
  ~CycleGraphs() {
    for (auto& e : exec)
      if (e) hipGraphExecDestroy(e);
  }
};

// Instantiated cycle graphs outlive the call: a later call whose captured
// arguments are the same (operator, poles and parameters, x, X and the
// workspace -- every address a cycle's kernels use derives from these)
// replays them without capturing again.  Least recently used first out;
// the cache is never torn down at process exit (the HIP runtime may be gone).
constexpr size_t kGraphCacheSize = 8;

struct GraphCache {
  std::mutex mu;
  std::list<std::pair<std::string, std::shared_ptr<CycleGraphs>>> lru;
};

GraphCache& graph_cache() {
  static GraphCache* c = new GraphCache();
  return *c;
}

template <typename T> void put_bytes(std::string& k, const T& v) {
  k.append(reinterpret_cast<const char*>(&v), sizeof(T));
}

std::string graph_key(const sk_operator* op, const sk_sign_params* p, const void* x, const void* X,
                      const void* ws) {
  std::string k;
  for (int i = 0; i < 4; ++i) put_bytes(k, op->dims[i]);
  put_bytes(k, op->t_antiperiodic);
  put_bytes(k, op->kappa);
  put_bytes(k, op->mu);
  put_bytes(k, op->links);
  put_bytes(k, op->links_c64);
  put_bytes(k, p->npoles);
  k.append(reinterpret_cast<const char*>(p->sigma), 16 * (size_t)p->npoles);
  k.append(reinterpret_cast<const char*>(p->omega), 16 * (size_t)p->npoles);
  put_bytes(k, p->k);
  put_bytes(k, p->m);
  put_bytes(k, p->R);
  put_bytes(k, p->L);
  put_bytes(k, p->F);
  put_bytes(k, p->project_each_cycle);
  put_bytes(k, p->precision);
  put_bytes(k, p->X_shift);
  put_bytes(k, x);
  put_bytes(k, X);
  put_bytes(k, ws);
  return k;
}

std::shared_ptr<CycleGraphs> graphs_for(const std::string& key) {
  GraphCache& c = graph_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (auto it = c.lru.begin(); it != c.lru.end(); ++it)
    if (it->first == key) {
      c.lru.splice(c.lru.begin(), c.lru, it);
      return c.lru.front().second;
    }
  c.lru.emplace_front(key, std::make_shared<CycleGraphs>());
  while (c.lru.size() > kGraphCacheSize) c.lru.pop_back();
  return c.lru.front().second;
}

int enqueue_cycle_kind(int kind, const CycleArgs& ca, SignWs& sw) {
  if (kind == 0) return enqueue_cycle<double2, double2>(ca, sw);
  if (kind == 1) return enqueue_cycle<double2, float2>(ca, sw);
  return enqueue_cycle<float2, float2>(ca, sw);
}

int run_cycle(int kind, const CycleArgs& ca, SignWs& sw, CycleGraphs& g, bool use_graph) {
  if (!use_graph) return enqueue_cycle_kind(kind, ca, sw);
  if (!g.exec[kind]) {
    hipStream_t cs = capture_stream();
    if (!cs) return enqueue_cycle_kind(kind, ca, sw);
    CycleArgs cc = ca;
    cc.s = cs;
    SK_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int st = enqueue_cycle_kind(kind, cc, sw);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &graph);
    if (st != SK_OK) {
      if (graph) hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) {
      set_error("graph capture failed: %s", hipGetErrorString(e));
      return SK_ERR_HIP;
    }
    e = hipGraphInstantiate(&g.exec[kind], graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g.exec[kind] = nullptr;
      set_error("graph instantiation failed: %s", hipGetErrorString(e));
      return SK_ERR_HIP;
    }
  }
  SK_HIP(hipGraphLaunch(g.exec[kind], ca.s));
  return SK_OK;
}

int sign_impl(const sk_operator* op, const sk_sign_params* p, const double2* b, double2* x,
              sk_stats* stats, void* ws, hipStream_t s) {
  const int64_t n = 12 * volume_of(op);
  const int k = p->k, m = p->m, N = p->npoles;
  const double2* R = (const double2*)p->R;
  const double2* Lv = (const double2*)p->L;
  Carver c;
  c.base = (char*)ws;
  SignWs sw;
  carve_sign(c, sw, n, p);
  double2* X = p->X_shift ? (double2*)p->X_shift : sw.Xint;
  KrylovWs<double2>& w = sw.w64;
  PoleSet ps;
  SK_TRY(fill_poles(ps, N, p->sigma, p->omega));
  const ArnoldiDev a = arn_of(w, k);
  const int cs = ts_counter_stride(n);
  const double theta = !sw.mixed ? 0.0 : (p->mixed_switch > 0.0 ? p->mixed_switch : 1e-3);
  bool low = sw.mixed && theta >= 1.0;   // precision of the current cycle

  SK_LAUNCH(launch_init_state(w.st, w.rho, N, w.counter, kCounterSlots * cs, s));
  SK_LAUNCH(launch_fill_zero((double*)w.H, (int64_t)(k + 1) * k * 2, s));
  SK_LAUNCH(launch_fill_value(w.scale, k + 2, 1.0, s));   // the basis is stored normalised
  if (X) SK_LAUNCH(launch_fill_zero((double*)X, (int64_t)N * n * 2, s));
  TsEpiArgs eb = epi_of(EPI_BETA, a);
  eb.dst_scalar = &w.st->beta;
  eb.dst_scale = w.scale + k + 1;   // unused slot: every stored v_j has unit norm
  const TsEpiArgs e0 = epi_of(EPI_NONE, a);
  // x = x_P = R f(Lambda) L^H b ;  r = (I - P) b  (Algorithm 1, first two lines)
  if (m > 0) {
    TsEpiArgs ed = epi_of(EPI_DEFL, a);
    ed.out = w.dc;
    ed.out2 = w.dc2;
    ed.F = (const double2*)p->F;
    ed.dst_scalar = &w.st->leak;
    SK_LAUNCH((ts_dot<double2, double2>(Lv, n, m, b, n, false, ed, w.partial, w.counter + 4 * cs,
                                        nullptr, s)));
    SK_LAUNCH((ts_gemv<double2>(R, n, m, w.dc2, x, n, false, 0, e0, nullptr, nullptr, nullptr,
                                nullptr, s)));
  } else {
    SK_LAUNCH(launch_fill_zero((double*)x, n * 2, s));
  }
  if (low)
    SK_LAUNCH((ts_update<double2, double2, float2>(m > 0 ? R : nullptr, n, m, w.dc, nullptr, b,
                                                   sw.w32.W, n, 2, eb, w.partial, w.counter + 5 * cs,
                                                   nullptr, s)));
  else
    SK_LAUNCH((ts_update<double2, double2, double2>(m > 0 ? R : nullptr, n, m, w.dc, nullptr, b, w.W,
                                                    n, 2, eb, w.partial, w.counter + 5 * cs, nullptr,
                                                    s)));
  CycleState hs;
  SK_HIP(hipMemcpyAsync(&hs, w.st, sizeof(hs), hipMemcpyDeviceToHost, s));
  SK_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->cycles = 0;
    stats->cycles_c64 = 0;
    stats->matvecs = 0;
    stats->converged = 0;
    stats->breakdown = 0;
    stats->final_update_norm = 0.0;
    stats->x_norm = 0.0;
    stats->resid_checked = 0;
    stats->resid_ok = 0;
  }
  if (hs.nonfinite || !std::isfinite(hs.beta)) {
    set_error("source contains non-finite values");
    return SK_ERR_NAN;
  }
  if (hs.beta == 0.0) {   // (I - P) b = 0: x = x_P exactly
    if (stats) stats->converged = 1;
    return SK_OK;
  }
  KTimer tm;
  if (stats && stats->times) {
    tm.out = stats->times;
    tm.s = s;
  }
  CycleArgs ca{op, p, n, &ps, x, X, &tm, s};
  const bool use_graph = !tm.on();   // per-kernel timing needs plain launches
  std::shared_ptr<CycleGraphs> gptr = use_graph ? graphs_for(graph_key(op, p, x, X, ws))
                                                : std::make_shared<CycleGraphs>();
  CycleGraphs& graphs = *gptr;
  int small = 0, status = SK_ERR_NOCONV;
  double first_upd = 0.0;
  bool diverged = false;
  std::vector<double2> rho_h(N);
  const bool want_rho = stats && stats->hist_rho;
  for (int cyc = 0; cyc < p->max_cycles; ++cyc) {
    // the next cycle's precision is decided before this one is enqueued:
    // once low, it stays low
    const bool low_next = low || (sw.mixed && cyc > 0 && hs.upd_norm <= theta * std::sqrt(hs.xnorm2));
    const bool cur = low;
    SK_TRY(run_cycle(!cur ? (low_next ? 1 : 0) : 2, ca, sw, graphs, use_graph));
    low = low_next;
    SK_HIP(hipMemcpyAsync(&hs, w.st, sizeof(hs), hipMemcpyDeviceToHost, s));
    if (want_rho && cyc < stats->hist_cap)
      SK_HIP(hipMemcpyAsync(rho_h.data(), w.rho, N * sizeof(double2), hipMemcpyDeviceToHost, s));
    SK_HIP(hipStreamSynchronize(s));
    tm.flush();
    if (want_rho && cyc < stats->hist_cap)
      for (int i = 0; i < N; ++i)
        stats->hist_rho[(size_t)cyc * N + i] = std::sqrt(cabs2(rho_h[i]));
    if (stats) {
      stats->cycles = cyc + 1;
      stats->cycles_c64 += cur ? 1 : 0;
      stats->matvecs += hs.kdone;
      stats->final_update_norm = hs.upd_norm;
      stats->x_norm = std::sqrt(hs.xnorm2);
      if (cyc < stats->hist_cap) {
        if (stats->hist_update) stats->hist_update[cyc] = hs.upd_norm;
        if (stats->hist_beta) stats->hist_beta[cyc] = hs.beta;   // ||r|| at the cycle's start
        if (stats->hist_leak) stats->hist_leak[cyc] = hs.leak;
      }
    }
    if (hs.nonfinite) {
      set_error("non-finite value in cycle %d (restarted FOM diverged or bad input)", cyc + 1);
      status = SK_ERR_NAN;
      break;
    }
    if (hs.singular) {
      set_error("H_k - sigma_i singular in cycle %d", cyc + 1);
      status = SK_ERR_SINGULAR;
      break;
    }
    if (hs.breakdown) {
      if (stats) stats->breakdown = 1;
      status = SK_OK;
      break;
    }
    small = (hs.upd_norm <= p->tol * std::sqrt(hs.xnorm2)) ? small + 1 : 0;
    if (small >= 2) {
      status = SK_OK;
      break;
    }
    // restarted FOM is not monotone; an update 1e10 times the first one
    // means the restarted iteration diverges for this k
    if (cyc == 0) first_upd = hs.upd_norm;
    else if (hs.upd_norm > kDivergeFactor * first_upd) {
      set_error("restarted FOM diverged (cycle %d, update %.3e): try another restart length",
                cyc + 1, hs.upd_norm);
      diverged = true;
      break;
    }
  }
  if (stats) stats->converged = (status == SK_OK);
  if (status == SK_ERR_NOCONV && !diverged) set_error("not converged after %d cycles", p->max_cycles);
  // FP64 check of the per-shift solutions: always in mixed precision (the
  // complex-float cycles must not have moved the iterate off the residuals
  // the iteration carries), on request otherwise
  const bool want_resid = stats && (stats->shift_resid || stats->shift_resid_implicit);
  if (X && (status == SK_OK || want_resid) && (sw.mixed || want_resid)) {
    std::vector<double> rel;
    double rn = 0.0;
    SK_TRY(true_residuals(op, p, ps, b, X, sw, n, rel, rn, s));
    SK_HIP(hipMemcpyAsync(rho_h.data(), w.rho, N * sizeof(double2), hipMemcpyDeviceToHost, s));
    SK_HIP(hipStreamSynchronize(s));
    const double rtol = p->resid_tol > 0.0 ? p->resid_tol : 100.0 * p->tol;
    bool ok = true;
    int worst = 0;
    for (int i = 0; i < N; ++i) {
      const double imp = rn > 0.0 ? std::sqrt(cabs2(rho_h[i])) / rn : 0.0;
      if (stats && stats->shift_resid) stats->shift_resid[i] = rel[i];
      if (stats && stats->shift_resid_implicit) stats->shift_resid_implicit[i] = imp;
      if (!(rel[i] <= 10.0 * imp + rtol)) {
        if (ok || rel[i] > rel[worst]) worst = i;
        ok = false;
      }
    }
    if (stats) {
      stats->resid_checked = 1;
      stats->resid_ok = ok ? 1 : 0;
    }
    if (sw.mixed && status == SK_OK && !ok) {
      set_error("FP64 check failed: true residual of shift %d is %.3e of ||(I-P)b|| (the iteration "
                "carries %.3e)", worst, rel[worst], std::sqrt(cabs2(rho_h[worst])) / rn);
      status = SK_ERR_NOCONV;
      if (stats) stats->converged = 0;
    }
  }
  return status;
}

// GMRES-LR: the restart loop of sign_impl with the GMRES small problems
// (seed least squares, collinear residuals for the other poles) solved on
// the host from H read back once per cycle.
int gmres_small(int kk, const std::vector<dense::cd>& H, int ld, double beta, std::vector<dense::cd>& rho,
                const PoleSet& ps, int seed, bool breakdown, std::vector<dense::cd>& Y, std::vector<dense::cd>& z) {
  using cd = dense::cd;
  const int N = ps.n;
  Y.assign((size_t)N * kk, cd(0.0));
  z.assign(kk + 1, cd(0.0));
  auto h = [&](int i, int j) { return H[i + (size_t)j * ld]; };
  auto sig = [&](int i) { return cd(ps.sigma[i].x, ps.sigma[i].y); };
  if (breakdown) {   // invariant space: every system exactly, from the square H_kk
    for (int i = 0; i < N; ++i) {
      std::vector<cd> A((size_t)kk * kk), rhs(kk, cd(0.0));
      for (int c = 0; c < kk; ++c)
        for (int r = 0; r < kk; ++r) A[r + (size_t)c * kk] = h(r, c) - (r == c ? sig(i) : cd(0.0));
      rhs[0] = beta * rho[i];
      if (!dense::lu_solve(kk, A, rhs, 1)) return SK_ERR_SINGULAR;
      for (int r = 0; r < kk; ++r) Y[(size_t)i * kk + r] = rhs[r];
      rho[i] = 0.0;
    }
    return SK_OK;
  }
  // seed: least squares on the (kk+1) x kk Hessenberg by Givens rotations
  std::vector<cd> Hs((size_t)(kk + 1) * kk), g(kk + 1, cd(0.0));
  for (int c = 0; c < kk; ++c)
    for (int r = 0; r <= kk; ++r) Hs[r + (size_t)c * (kk + 1)] = h(r, c) - (r == c ? sig(seed) : cd(0.0));
  g[0] = beta * rho[seed];
  std::vector<cd> G(g);
  std::vector<double> gc(kk);
  std::vector<cd> gs(kk);
  for (int j = 0; j < kk; ++j) {
    const cd a = Hs[j + (size_t)j * (kk + 1)], b = Hs[j + 1 + (size_t)j * (kk + 1)];
    const double den = std::sqrt(std::norm(a) + std::norm(b));
    if (den == 0.0) return SK_ERR_SINGULAR;
    const cd ph = std::abs(a) > 0.0 ? a / std::abs(a) : cd(1.0);
    gc[j] = std::abs(a) / den;
    gs[j] = ph * std::conj(b) / den;
    for (int c = j; c < kk; ++c) {
      const cd t = Hs[j + (size_t)c * (kk + 1)], u = Hs[j + 1 + (size_t)c * (kk + 1)];
      Hs[j + (size_t)c * (kk + 1)] = gc[j] * t + gs[j] * u;
      Hs[j + 1 + (size_t)c * (kk + 1)] = -std::conj(gs[j]) * t + gc[j] * u;
    }
    const cd t = G[j], u = G[j + 1];
    G[j] = gc[j] * t + gs[j] * u;
    G[j + 1] = -std::conj(gs[j]) * t + gc[j] * u;
  }
  std::vector<cd> ys(kk);
  for (int i = kk - 1; i >= 0; --i) {
    cd acc = G[i];
    for (int q = i + 1; q < kk; ++q) acc -= Hs[i + (size_t)q * (kk + 1)] * ys[q];
    const cd d = Hs[i + (size_t)i * (kk + 1)];
    if (std::abs(d) == 0.0) return SK_ERR_SINGULAR;
    ys[i] = acc / d;
  }
  // z = beta rho_s e_1 - (Hbar - sigma_s I~) y_s, from the original matrix
  for (int r = 0; r <= kk; ++r) {
    cd acc = (r == 0) ? g[0] : cd(0.0);
    for (int c = 0; c < kk; ++c) acc -= (h(r, c) - (r == c ? sig(seed) : cd(0.0))) * ys[c];
    z[r] = acc;
  }
  for (int r = 0; r < kk; ++r) Y[(size_t)seed * kk + r] = ys[r];
  std::vector<cd> rho_new(N, cd(0.0));
  rho_new[seed] = 1.0;
  for (int i = 0; i < N; ++i) {
    if (i == seed) continue;
    const int m1 = kk + 1;
    std::vector<cd> A((size_t)m1 * m1), rhs(m1, cd(0.0));
    for (int c = 0; c < kk; ++c)
      for (int r = 0; r <= kk; ++r) A[r + (size_t)c * m1] = h(r, c) - (r == c ? sig(i) : cd(0.0));
    for (int r = 0; r <= kk; ++r) A[r + (size_t)kk * m1] = z[r];
    rhs[0] = beta * rho[i];
    if (!dense::lu_solve(m1, A, rhs, 1)) return SK_ERR_SINGULAR;
    for (int r = 0; r < kk; ++r) Y[(size_t)i * kk + r] = rhs[r];
    rho_new[i] = rhs[kk];
  }
  rho = rho_new;
  return SK_OK;
}

int gmres_impl(const sk_operator* op, const sk_sign_params* p, const double2* b, double2* x, sk_stats* stats,
               void* ws, hipStream_t s) {
  using cd = dense::cd;
  const int64_t n = 12 * volume_of(op);
  const int k = p->k, m = p->m, N = p->npoles;
  const double2* R = (const double2*)p->R;
  const double2* Lv = (const double2*)p->L;
  Carver c;
  c.base = (char*)ws;
  SignWs sw;
  carve_sign(c, sw, n, p);
  KrylovWs<double2>& w = sw.w64;
  double2* X = (double2*)p->X_shift;
  PoleSet ps;
  SK_TRY(fill_poles(ps, N, p->sigma, p->omega));
  int seed = p->seed;
  if (seed < 0) {
    seed = 0;
    for (int i = 1; i < N; ++i)
      if (cabs2(ps.sigma[i]) < cabs2(ps.sigma[seed])) seed = i;
  }
  const ArnoldiDev a = arn_of(w, k);
  const int cs = ts_counter_stride(n);
  SK_LAUNCH(launch_init_state(w.st, w.rho, N, w.counter, kCounterSlots * cs, s));
  SK_LAUNCH(launch_fill_zero((double*)w.H, (int64_t)(k + 1) * k * 2, s));
  SK_LAUNCH(launch_fill_value(w.scale, k + 2, 1.0, s));
  if (X) SK_LAUNCH(launch_fill_zero((double*)X, (int64_t)N * n * 2, s));
  const TsEpiArgs e0 = epi_of(EPI_NONE, a);
  TsEpiArgs eb = epi_of(EPI_BETA, a);
  eb.dst_scalar = &w.st->beta;
  eb.dst_scale = w.scale + k + 1;
  if (m > 0) {
    TsEpiArgs ed = epi_of(EPI_DEFL, a);
    ed.out = w.dc;
    ed.out2 = w.dc2;
    ed.F = (const double2*)p->F;
    ed.dst_scalar = &w.st->leak;
    SK_LAUNCH((ts_dot<double2, double2>(Lv, n, m, b, n, false, ed, w.partial, w.counter + 4 * cs, nullptr, s)));
    SK_LAUNCH((ts_gemv<double2>(R, n, m, w.dc2, x, n, false, 0, e0, nullptr, nullptr, nullptr, nullptr, s)));
  } else {
    SK_LAUNCH(launch_fill_zero((double*)x, n * 2, s));
  }
  SK_LAUNCH((ts_update<double2, double2, double2>(m > 0 ? R : nullptr, n, m, w.dc, nullptr, b, w.W, n, 2, eb,
                                                  w.partial, w.counter + 5 * cs, nullptr, s)));
  CycleState hs;
  SK_HIP(hipMemcpyAsync(&hs, w.st, sizeof(hs), hipMemcpyDeviceToHost, s));
  SK_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->cycles = stats->cycles_c64 = stats->matvecs = stats->converged = stats->breakdown = 0;
    stats->final_update_norm = stats->x_norm = 0.0;
    stats->resid_checked = stats->resid_ok = 0;
  }
  if (hs.nonfinite || !std::isfinite(hs.beta)) {
    set_error("source contains non-finite values");
    return SK_ERR_NAN;
  }
  if (hs.beta == 0.0) {
    if (stats) stats->converged = 1;
    return SK_OK;
  }
  std::vector<cd> rho(N, cd(1.0)), Hh, Y, z;
  std::vector<double2> hbuf((size_t)(k + 1) * k), ubuf(k + 1), ybuf((size_t)N * k), zbuf(k + 1);
  int small = 0, status = SK_ERR_NOCONV;
  double first = 0.0;
  for (int cyc = 0; cyc < p->max_cycles; ++cyc) {
    SK_TRY(enqueue_arnoldi<double2>(op, w, n, k, 0, s));
    SK_HIP(hipMemcpyAsync(&hs, w.st, sizeof(hs), hipMemcpyDeviceToHost, s));
    SK_HIP(hipMemcpyAsync(hbuf.data(), w.H, hbuf.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
    SK_HIP(hipStreamSynchronize(s));
    if (hs.nonfinite) {
      set_error("non-finite value in cycle %d", cyc + 1);
      status = SK_ERR_NAN;
      break;
    }
    const int kk = hs.kdone;
    Hh.assign(hbuf.size(), cd(0.0));
    for (size_t e = 0; e < hbuf.size(); ++e) Hh[e] = cd(hbuf[e].x, hbuf[e].y);
    const int rc = gmres_small(kk, Hh, k + 1, hs.beta, rho, ps, seed, hs.breakdown != 0, Y, z);
    if (rc != SK_OK) {
      set_error("GMRES-LR: singular small system in cycle %d", cyc + 1);
      status = rc;
      break;
    }
    double un2 = 0.0;
    for (int r = 0; r < kk; ++r) {
      cd u = 0.0;
      for (int i = 0; i < N; ++i) u += cd(ps.omega[i].x, ps.omega[i].y) * Y[(size_t)i * kk + r];
      ubuf[r] = make_double2(u.real(), u.imag());
      un2 += std::norm(u);
    }
    const double un = std::sqrt(un2);
    for (int i = 0; i < N; ++i)
      for (int r = 0; r < kk; ++r) ybuf[(size_t)i * k + r] = make_double2(Y[(size_t)i * kk + r].real(), Y[(size_t)i * kk + r].imag());
    for (int r = 0; r <= kk; ++r) zbuf[r] = make_double2(z[r].real(), z[r].imag());
    SK_HIP(hipMemcpyAsync(w.ucoef, ubuf.data(), kk * sizeof(double2), hipMemcpyHostToDevice, s));
    if (X) SK_HIP(hipMemcpyAsync(w.ycoef, ybuf.data(), (size_t)N * k * sizeof(double2), hipMemcpyHostToDevice, s));
    SK_HIP(hipMemcpyAsync(sw.zdev, zbuf.data(), (kk + 1) * sizeof(double2), hipMemcpyHostToDevice, s));
    // x += V_kk u (and X_i += V_kk y_i), ||x||^2
    TsEpiArgs ex = epi_of(EPI_XNORM, a);
    ex.dst_scalar = &w.st->xnorm2;
    SK_LAUNCH((ts_gemv<double2>(w.W, n, kk, w.ucoef, x, n, true, 2, ex, w.partial, w.counter + 6 * cs, nullptr,
                                nullptr, s)));
    if (X) SK_LAUNCH((ts_multi_gemv<double2>(w.W, n, kk, w.ycoef, k, N, X, n, nullptr, s)));
    const bool done_exact = hs.breakdown != 0;
    if (!done_exact) {
      // r = (I - P) V_{kk+1} z, the next cycle's start vector (normalised by its first step)
      SK_LAUNCH((ts_gemv<double2>(w.W, n, kk + 1, sw.zdev, sw.rnext, n, false, 0, e0, nullptr, nullptr, nullptr,
                                  nullptr, s)));
      if (m > 0 && p->project_each_cycle) {
        TsEpiArgs el = epi_of(EPI_DEFL, a);
        el.out = w.dc2;
        el.dst_scalar = &w.st->leak;
        SK_LAUNCH((ts_dot<double2, double2>(Lv, n, m, sw.rnext, n, false, el, w.partial, w.counter + 4 * cs,
                                            nullptr, s)));
        SK_LAUNCH((ts_update<double2, double2, double2>(R, n, m, w.dc2, nullptr, sw.rnext, w.W, n, 0, e0,
                                                        w.partial, w.counter + 5 * cs, nullptr, s)));
      } else {
        SK_LAUNCH((ts_scale<double2, double2>(sw.rnext, w.W, n, nullptr, 1.0, s)));
      }
    }
    SK_HIP(hipMemcpyAsync(&hs, w.st, sizeof(hs), hipMemcpyDeviceToHost, s));
    SK_HIP(hipStreamSynchronize(s));
    if (stats) {
      stats->cycles = cyc + 1;
      stats->matvecs += kk;
      stats->final_update_norm = un;
      stats->x_norm = std::sqrt(hs.xnorm2);
      if (cyc < stats->hist_cap) {
        if (stats->hist_update) stats->hist_update[cyc] = un;
        if (stats->hist_beta) stats->hist_beta[cyc] = hs.beta;
        if (stats->hist_leak) stats->hist_leak[cyc] = hs.leak;
        if (stats->hist_rho)
          for (int i = 0; i < N; ++i) stats->hist_rho[(size_t)cyc * N + i] = std::abs(rho[i]);
      }
    }
    if (done_exact) {
      if (stats) stats->breakdown = 1;
      status = SK_OK;
      break;
    }
    if (!std::isfinite(un) || hs.nonfinite) {
      set_error("non-finite value in cycle %d (restarted GMRES diverged)", cyc + 1);
      status = SK_ERR_NAN;
      break;
    }
    small = (un <= p->tol * std::sqrt(hs.xnorm2)) ? small + 1 : 0;
    if (small >= 2) {
      status = SK_OK;
      break;
    }
    if (cyc == 0) first = un;
    else if (un > kDivergeFactor * first) {
      set_error("restarted GMRES diverged (cycle %d, update %.3e): try another restart length", cyc + 1, un);
      if (stats) stats->converged = 0;
      return SK_ERR_NOCONV;
    }
    // rho lives on the host; the device copy is only for the statistics of FOM
  }
  if (stats) stats->converged = (status == SK_OK);
  if (status == SK_ERR_NOCONV) set_error("not converged after %d cycles", p->max_cycles);
  return status;
}

}  // namespace
}  // namespace sk

extern "C" {

size_t sign_apply_workspace_bytes(const sk_operator* op, const sk_sign_params* p) {
  if (!op || !p || volume_of(op) <= 0) return 0;
  char msg[256];
  if (!params_ok(p, msg, sizeof msg)) return 0;
  Carver c;
  SignWs sw;
  return carve_sign(c, sw, 12 * volume_of(op), p);
}

int sign_apply(const sk_operator* op, const sk_sign_params* p, const double* b, double* x,
               sk_stats* stats, void* ws, size_t ws_bytes, hipStream_t stream) {
  SK_TRY(check_operator(op, SK_C128));
  if (p && p->precision == SK_PREC_MIXED) SK_TRY(check_operator(op, SK_C64));
  const int64_t n = 12 * volume_of(op);
  char msg[256];
  SK_CHECK(params_ok(p, msg, sizeof msg), "%s", msg);
  SK_CHECK(b && x && ws, "b, x and ws must be non-NULL");
  SK_CHECK(!overlap(b, n * 16, x, n * 16), "b and x overlap");
  if (p->X_shift)
    SK_CHECK(!overlap(p->X_shift, (size_t)p->npoles * n * 16, x, n * 16) &&
                 !overlap(p->X_shift, (size_t)p->npoles * n * 16, b, n * 16),
             "X_shift overlaps b or x");
  const size_t need = sign_apply_workspace_bytes(op, p);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return SK_ERR_WORKSPACE;
  }
  SK_CHECK(!overlap(ws, need, x, n * 16) && !overlap(ws, need, b, n * 16), "workspace overlaps b or x");
  const auto t0 = std::chrono::steady_clock::now();
  const int st = p->method == SK_METHOD_GMRES
                     ? gmres_impl(op, p, (const double2*)b, (double2*)x, stats, ws, stream)
                     : sign_impl(op, p, (const double2*)b, (double2*)x, stats, ws, stream);
  if (stats) stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

size_t sign_apply_backward_workspace_bytes(const sk_operator* op, const sk_sign_params* p) {
  if (!op || !p || volume_of(op) <= 0 || p->m != 0 || p->precision != SK_PREC_FP64 ||
      p->method != SK_METHOD_FOM)
    return 0;
  char msg[256];
  if (!params_ok(p, msg, sizeof msg)) return 0;
  const int64_t n = 12 * volume_of(op);
  sk_sign_params q = *p;
  q.X_shift = (double*)16;   // sized with per-shift solutions
  Carver c;
  SignWs sw;
  carve_sign(c, sw, n, &q);
  c.take<double2>((size_t)2 * p->npoles * n);     // X, Z
  c.take<double2>(n);                              // scratch for the adjoint result
  c.take<double>(grad_blocks(volume_of(op)));      // mu partials
  return c.off;
}

int sign_apply_backward(const sk_operator* op, const sk_sign_params* p, const double* b,
                        const double* eta, double* x_out, double* grad_theta, double* grad_mu,
                        sk_stats* stats, void* ws, size_t ws_bytes, hipStream_t stream) {
  SK_TRY(check_operator(op, SK_C128));
  char msg[256];
  SK_CHECK(params_ok(p, msg, sizeof msg), "%s", msg);
  SK_CHECK(p->m == 0, "the gradient is defined without deflation (m must be 0)");
  SK_CHECK(p->precision == SK_PREC_FP64, "the gradient runs in complex double");
  SK_CHECK(p->method == SK_METHOD_FOM, "the gradient uses the FOM per-shift solutions");
  SK_CHECK(b && eta && grad_theta && grad_mu && ws, "NULL argument");
  const int64_t n = 12 * volume_of(op), V = volume_of(op);
  const size_t need = sign_apply_backward_workspace_bytes(op, p);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return SK_ERR_WORKSPACE;
  }
  SK_CHECK(!overlap(grad_theta, 32 * V * 8, ws, need), "grad_theta overlaps the workspace");
  const int N = p->npoles;
  sk_sign_params q = *p;
  q.X_shift = (double*)16;
  Carver c;
  c.base = (char*)ws;
  SignWs sw;
  carve_sign(c, sw, n, &q);
  const size_t solver_bytes = c.off;
  double2* X = c.take<double2>((size_t)N * n);
  double2* Z = c.take<double2>((size_t)N * n);
  double2* xa = c.take<double2>(n);
  double* mu_part = c.take<double>(grad_blocks(V));
  // forward: x_j = (H - sigma_j)^{-1} b
  q.X_shift = (double*)X;
  double2* xf = x_out ? (double2*)x_out : xa;
  SK_TRY(sign_impl(op, &q, (const double2*)b, xf, stats ? &stats[0] : nullptr, ws, stream));
  // adjoint: z_j = (H(-mu) - conj sigma_j)^{-1} eta
  sk_operator opa = *op;
  opa.mu = -op->mu;
  std::vector<double> sg(2 * N), om(2 * N);
  for (int i = 0; i < N; ++i) {
    sg[2 * i] = p->sigma[2 * i];
    sg[2 * i + 1] = -p->sigma[2 * i + 1];
    om[2 * i] = p->omega[2 * i];
    om[2 * i + 1] = -p->omega[2 * i + 1];
  }
  q.sigma = sg.data();
  q.omega = om.data();
  q.X_shift = (double*)Z;
  SK_TRY(sign_impl(&opa, &q, (const double2*)eta, xa, stats ? &stats[1] : nullptr, ws, stream));
  (void)solver_bytes;
  PoleSet ps;
  SK_TRY(fill_poles(ps, N, p->sigma, p->omega));
  SK_LAUNCH(launch_grad(op, ps, X, Z, grad_theta, mu_part, stream));
  std::vector<double> mp(grad_blocks(V));
  SK_HIP(hipMemcpyAsync(mp.data(), mu_part, mp.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
  SK_HIP(hipStreamSynchronize(stream));
  double acc = 0.0;
  for (double v : mp) acc += v;
  *grad_mu = acc;
  return SK_OK;
}

int sk_links_to_c64(const double* links, float* links_c64, int64_t V, hipStream_t stream) {
  SK_CHECK(links && links_c64 && V >= 1, "bad arguments");
  SK_CHECK(!overlap(links, 36 * V * 16, links_c64, 36 * V * 8), "buffers overlap");
  SK_LAUNCH((ts_scale<double2, float2>((const double2*)links, (float2*)links_c64, 36 * V, nullptr, 1.0,
                                       stream)));
  return SK_OK;
}

}  // extern "C"
