// Deflation eigensolver: the m eigenpairs of H_W nearest zero, right and
// left, as an oblique projector in an orthonormal Schur basis (Sect. 4 uses
// R_m, L_m, Lambda_m; the paper treats them as inputs and gives no method).
//
// Krylov-Schur (thick-restart Arnoldi) on B = A^2 for the eigenvalues of
// smallest real part: for lambda near zero, lambda^2 sits at the left edge
// of the spectrum of B, where Arnoldi converges like for an extreme
// eigenvalue.  The B-invariant subspace of those eigenvalues is A-invariant
// (A and B commute), so the Rayleigh quotient M = X^H A X gives the
// eigenvalues of A and a Schur basis for the selected ones.  The device
// does the Arnoldi extensions (the CGS2 kernels of the solver, with the
// stencil applied twice per step) and the basis recombinations; the small
// Schur problems run on the host in FP64.
#include "krylov_ws.h"
#include "dense_host.h"

#include <algorithm>
#include <complex>
#include <vector>

namespace sk {
namespace {

using cd = std::complex<double>;

// Deterministic start vector: a counter-based generator (splitmix64 of the
// index) mapped to [-1, 1) for both parts.
__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__global__ void k_start_vector(double2* v, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t a = splitmix64(seed ^ (2 * (uint64_t)i)), b = splitmix64(seed ^ (2 * (uint64_t)i + 1));
  v[i] = make_double2((double)(a >> 11) * 0x1.0p-52 - 1.0, (double)(b >> 11) * 0x1.0p-52 - 1.0);
}

struct EigCtx {
  const sk_operator* op;
  int64_t n;
  int ncv;
  KrylovWs<double2> w;
  double2* tmp;      // one vector
  double2* Vnew;     // ncv vectors
  double2* C;        // ncv x ncv coefficients
  double2* Mdev;     // ncv x ncv
  hipStream_t s;
  int64_t matvecs = 0;
};

int to_dev(double2* dst, const std::vector<cd>& src, hipStream_t s) {
  SK_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(cd), hipMemcpyHostToDevice, s));
  return SK_OK;
}

// X_i = sum_j Q_j coeff(j, i) for i < nout, coeff column-major (ld = ldc),
// into dst (zeroed first).
int combine(EigCtx& e, const double2* Q, int p, const std::vector<cd>& coeff, int ldc, int nout,
            double2* dst) {
  SK_TRY(to_dev(e.C, coeff, e.s));
  SK_LAUNCH(launch_fill_zero((double*)dst, (int64_t)nout * e.n * 2, e.s));
  SK_LAUNCH((ts_multi_gemv<double2>(Q, e.n, p, e.C, ldc, nout, dst, e.n, nullptr, e.s)));
  return SK_OK;
}

// M = X^H op(A) X for the first p vectors X of `X` (column-major p x p, host).
int rayleigh(EigCtx& e, const double2* X, int p, int adjoint, std::vector<cd>& M) {
  const ArnoldiDev a = arn_of(e.w, e.ncv);
  const int cs = ts_counter_stride(e.n);
  for (int i = 0; i < p; ++i) {
    SK_LAUNCH((launch_wilson<double2, double2, double2>(e.op, (const double2*)e.op->links,
                                                        X + (size_t)i * e.n, e.tmp, adjoint,
                                                        nullptr, nullptr, e.s)));
    TsEpiArgs es = epi_of(EPI_STORE, a);
    es.out = e.Mdev + (size_t)i * p;
    SK_LAUNCH((ts_dot<double2, double2>(X, e.n, p, e.tmp, e.n, false, es, e.w.partial,
                                        e.w.counter + 9 * cs, nullptr, e.s)));
  }
  e.matvecs += p;
  M.resize((size_t)p * p);
  SK_HIP(hipMemcpyAsync(M.data(), e.Mdev, M.size() * sizeof(cd), hipMemcpyDeviceToHost, e.s));
  SK_HIP(hipStreamSynchronize(e.s));
  return SK_OK;
}

// Krylov-Schur on op(A)^2 for the nev eigenvalues of smallest real part.
// On success the first nev basis vectors of e.w.W are orthonormal and span
// the invariant subspace; T (nev x nev) is the Schur form of op(A)^2 there.
int krylov_schur(EigCtx& e, int adjoint, int nev, int keep_req, double tol, int max_restarts,
                 uint64_t seed, std::vector<cd>& Tout, int& restarts, double& resid_out) {
  const int ncv = e.ncv;
  const int64_t n = e.n;
  KrylovWs<double2>& w = e.w;
  const int cs = ts_counter_stride(n);
  const ArnoldiDev a = arn_of(w, ncv);
  hipStream_t s = e.s;
  // start vector, scale[0] = 1/||v||
  hipLaunchKernelGGL(k_start_vector, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w.W, n, seed);
  SK_LAUNCH(hipGetLastError());
  SK_LAUNCH(launch_init_state(w.st, w.rho, 0, w.counter, kCounterSlots * cs, s));
  (void)a;
  int kk = 0;
  std::vector<cd> Tkk, bkk, Hd((size_t)(ncv + 1) * ncv), K, Q;
  CycleState hs;
  for (restarts = 0; restarts < max_restarts; ++restarts) {
    SK_LAUNCH(launch_init_state(w.st, w.rho, 0, w.counter, kCounterSlots * cs, s));
    // H starts as the restarted Rayleigh quotient [T_kk; b^T] in columns < kk
    std::fill(Hd.begin(), Hd.end(), cd(0.0));
    for (int j = 0; j < kk; ++j) {
      for (int i = 0; i <= j; ++i) Hd[i + (size_t)j * (ncv + 1)] = Tkk[i + (size_t)j * kk];
      Hd[kk + (size_t)j * (ncv + 1)] = bkk[j];
    }
    SK_TRY(to_dev(w.H, Hd, s));
    SK_TRY(enqueue_arnoldi<double2>(e.op, w, n, ncv, adjoint, s, nullptr, kk, 2, e.tmp));
    SK_HIP(hipMemcpyAsync(Hd.data(), w.H, Hd.size() * sizeof(cd), hipMemcpyDeviceToHost, s));
    SK_HIP(hipMemcpyAsync(&hs, w.st, sizeof(hs), hipMemcpyDeviceToHost, s));
    SK_HIP(hipStreamSynchronize(s));
    e.matvecs += 2 * (ncv - kk);
    if (hs.nonfinite) {
      set_error("non-finite value in the eigensolver");
      return SK_ERR_NAN;
    }
    if (hs.breakdown) {
      set_error("Krylov-Schur basis hit an invariant subspace of dimension %d < ncv", hs.kdone);
      return SK_ERR_NOCONV;
    }
    // Rayleigh-quotient matrix of the Krylov decomposition
    K.assign((size_t)ncv * ncv, cd(0.0));
    for (int j = 0; j < kk; ++j) {
      for (int i = 0; i <= j; ++i) K[i + (size_t)j * ncv] = Tkk[i + (size_t)j * kk];
      K[kk + (size_t)j * ncv] = bkk[j];
    }
    for (int j = kk; j < ncv; ++j)
      for (int i = 0; i < ncv; ++i) K[i + (size_t)j * ncv] = Hd[i + (size_t)j * (ncv + 1)];
    const cd beta = Hd[ncv + (size_t)(ncv - 1) * (ncv + 1)];
    if (!dense::schur(ncv, K, Q)) {
      set_error("QR iteration for the Krylov-Schur Rayleigh quotient did not converge");
      return SK_ERR_NOCONV;
    }
    dense::reorder_schur(ncv, K, Q, [](cd z) { return z.real(); }, ncv);
    std::vector<cd> b(ncv);
    for (int i = 0; i < ncv; ++i) b[i] = beta * Q[(ncv - 1) + (size_t)i * ncv];
    int nconv = 0;
    double resid = 0.0;
    for (int i = 0; i < nev; ++i) {
      const double r = std::abs(b[i]) / std::max(std::abs(K[i + (size_t)i * ncv]), 1e-300);
      resid = std::max(resid, r);
      if (r <= tol && nconv == i) ++nconv;
    }
    resid_out = resid;
    const bool done = nconv >= nev;
    const int keep = done ? nev : (keep_req > 0 ? keep_req : std::min(ncv - 8, nev + (ncv - nev) / 2));
    // thick restart: W[0..keep) = W Q(:, :keep), W[keep] = W[ncv]
    SK_TRY(combine(e, w.W, ncv, Q, ncv, keep, e.Vnew));
    SK_HIP(hipMemcpyAsync(w.W, e.Vnew, (size_t)keep * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
    if (done) {
      Tout.assign((size_t)nev * nev, cd(0.0));
      for (int j = 0; j < nev; ++j)
        for (int i = 0; i <= j; ++i) Tout[i + (size_t)j * nev] = K[i + (size_t)j * ncv];
      SK_HIP(hipStreamSynchronize(s));
      ++restarts;
      return SK_OK;
    }
    SK_HIP(hipMemcpyAsync(w.W + (size_t)keep * n, w.W + (size_t)ncv * n, n * sizeof(double2),
                          hipMemcpyDeviceToDevice, s));
    Tkk.assign((size_t)keep * keep, cd(0.0));
    for (int j = 0; j < keep; ++j)
      for (int i = 0; i <= j; ++i) Tkk[i + (size_t)j * keep] = K[i + (size_t)j * ncv];
    bkk.assign(b.begin(), b.begin() + keep);
    kk = keep;
  }
  set_error("Krylov-Schur eigensolver did not converge in %d restarts", max_restarts);
  return SK_ERR_NOCONV;
}

struct Carved {
  EigCtx e;
  size_t bytes;
};

size_t carve_eig(Carver& c, EigCtx& e, int64_t n, int ncv) {
  carve_krylov(c, e.w, n, ncv, 1, 0, false);
  e.tmp = c.take<double2>(n);
  e.Vnew = c.take<double2>((size_t)ncv * n);
  e.C = c.take<double2>((size_t)ncv * ncv);
  e.Mdev = c.take<double2>((size_t)ncv * ncv);
  return c.off;
}

int auto_ncv(const sk_eig_params* p) {
  const int nev = p->m + p->nev_extra;
  int ncv = p->ncv > 0 ? p->ncv : std::max(2 * nev + 20, nev + 32);
  return std::min(ncv, kMaxK);
}

}  // namespace
}  // namespace sk

using namespace sk;

extern "C" {

size_t deflation_eigensolve_workspace_bytes(const sk_operator* op, const sk_eig_params* p) {
  if (!op || !p || volume_of(op) <= 0 || p->m < 1 || p->m > kMaxDefl || p->nev_extra < 0) return 0;
  const int ncv = auto_ncv(p);
  if (ncv < p->m + p->nev_extra + 8) return 0;
  Carver c;
  EigCtx e;
  return carve_eig(c, e, 12 * volume_of(op), ncv);
}

int deflation_eigensolve(const sk_operator* op, const sk_eig_params* p, double* R, double* L,
                         double* F, double* lambda, sk_eig_stats* stats, void* ws, size_t ws_bytes,
                         hipStream_t stream) {
  SK_TRY(check_operator(op, SK_C128));
  SK_CHECK(p != nullptr, "params are NULL");
  SK_CHECK(p->m >= 1 && p->m <= kMaxDefl, "m = %d outside [1, %d]", p->m, kMaxDefl);
  SK_CHECK(p->nev_extra >= 1, "nev_extra must be >= 1 (needed to certify the selection)");
  SK_CHECK(p->key == 0 || p->key == 1, "key must be 0 (|lambda|) or 1 (|Re lambda|)");
  SK_CHECK(p->tol > 0.0 && p->max_restarts >= 1, "tol and max_restarts must be positive");
  SK_CHECK(R && L && F && lambda && ws, "NULL argument");
  const int m = p->m, nev = p->m + p->nev_extra, ncv = auto_ncv(p);
  SK_CHECK(ncv >= nev + 8 && ncv <= kMaxK, "ncv = %d must be in [m + nev_extra + 8, %d]", ncv, kMaxK);
  SK_CHECK(p->keep == 0 || (p->keep >= nev && p->keep <= ncv - 8),
           "keep = %d must be 0 or in [m + nev_extra, ncv - 8] = [%d, %d]", p->keep, nev, ncv - 8);
  const int64_t n = 12 * volume_of(op);
  SK_CHECK((int64_t)ncv + 1 <= n, "lattice too small for ncv = %d", ncv);
  const size_t need = deflation_eigensolve_workspace_bytes(op, p);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return SK_ERR_WORKSPACE;
  }
  Carver c;
  c.base = (char*)ws;
  EigCtx e;
  carve_eig(c, e, n, ncv);
  e.op = op;
  e.n = n;
  e.ncv = ncv;
  e.s = stream;
  auto keyf = [&](cd z) { return p->key == 0 ? std::abs(z) : std::abs(z.real()); };
  if (stats) std::memset(stats, 0, sizeof(*stats));

  // ---- right invariant subspace
  std::vector<cd> TB, M, Z;
  int rr = 0;
  double resr = 0.0;
  SK_TRY(krylov_schur(e, 0, nev, p->keep, p->tol, p->max_restarts, 0x5eed0001ull, TB, rr, resr));
  double window = -1e300;
  for (int i = 0; i < nev; ++i) window = std::max(window, TB[i + (size_t)i * nev].real());
  SK_TRY(rayleigh(e, e.w.W, nev, 0, M));
  if (!dense::schur(nev, M, Z)) {
    set_error("Schur form of the Rayleigh quotient did not converge");
    return SK_ERR_NOCONV;
  }
  dense::reorder_schur(nev, M, Z, keyf, nev);
  std::vector<cd> lam(nev);
  for (int i = 0; i < nev; ++i) lam[i] = M[i + (size_t)i * nev];
  const double gap = keyf(lam[m]) - keyf(lam[m - 1]);
  if (stats) {
    stats->restarts[0] = rr;
    stats->resid[0] = resr;
    stats->gap = gap;
    stats->key_window = window;
  }
  // every eigenvalue with |lambda| (or |Re lambda|) up to the m-th selected
  // has Re(lambda^2) below key^2, so it is among those computed iff the
  // largest computed Re(lambda^2) is at least key^2
  if (window < keyf(lam[m - 1]) * keyf(lam[m - 1])) {
    set_error("selection not certified: raise nev_extra (window %.4g < %.4g)", window,
              keyf(lam[m - 1]) * keyf(lam[m - 1]));
    return SK_ERR_NOCONV;
  }
  if (gap < 1e-6) {
    set_error("no selection gap after %d eigenvalues (gap %.3g): choose another m", m, gap);
    return SK_ERR_ARG;
  }
  // R = X Z(:, :m): orthonormal Schur basis of the selected eigenvalues
  SK_TRY(combine(e, e.w.W, nev, Z, nev, m, (double2*)R));
  std::vector<cd> Tm((size_t)m * m);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) Tm[i + (size_t)j * m] = M[i + (size_t)j * nev];

  // ---- left invariant subspace (A^H = H_W(-mu)), matched to conj(lambda)
  std::vector<cd> TBl, Ml, Zl;
  int rl = 0;
  double resl = 0.0;
  SK_TRY(krylov_schur(e, 1, nev, p->keep, p->tol, p->max_restarts, 0x5eed0002ull, TBl, rl, resl));
  SK_TRY(rayleigh(e, e.w.W, nev, 1, Ml));
  if (!dense::schur(nev, Ml, Zl)) {
    set_error("Schur form of the left Rayleigh quotient did not converge");
    return SK_ERR_NOCONV;
  }
  std::vector<cd> sel(lam.begin(), lam.begin() + m);
  auto lkey = [&](cd z) {
    for (int i = 0; i < m; ++i)
      if (std::abs(std::conj(z) - sel[i]) <= 1e-8 * std::max(1.0, std::abs(sel[i]))) return (double)i;
    return 1e300;
  };
  dense::reorder_schur(nev, Ml, Zl, lkey, m);
  for (int i = 0; i < m; ++i)
    if (lkey(Ml[i + (size_t)i * nev]) >= 1e299) {
      set_error("left and right eigenvalue sets do not match");
      return SK_ERR_NOCONV;
    }
  SK_TRY(combine(e, e.w.W, nev, Zl, nev, m, e.Vnew));   // W~ (m vectors)
  // G = W~^H R,  L = W~ G^{-H}  so that L^H R = I
  std::vector<cd> G;
  {
    const ArnoldiDev a = arn_of(e.w, ncv);
    const int cs = ts_counter_stride(n);
    for (int i = 0; i < m; ++i) {
      TsEpiArgs es = epi_of(EPI_STORE, a);
      es.out = e.Mdev + (size_t)i * m;
      SK_LAUNCH((ts_dot<double2, double2>(e.Vnew, n, m, (const double2*)R + (size_t)i * n, n, false,
                                          es, e.w.partial, e.w.counter + 9 * cs, nullptr, stream)));
    }
    G.resize((size_t)m * m);
    SK_HIP(hipMemcpyAsync(G.data(), e.Mdev, G.size() * sizeof(cd), hipMemcpyDeviceToHost, stream));
    SK_HIP(hipStreamSynchronize(stream));
  }
  std::vector<cd> GH((size_t)m * m), E;
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) GH[i + (size_t)j * m] = std::conj(G[j + (size_t)i * m]);
  if (!dense::inverse(m, GH, E)) {
    set_error("left/right bases are not biorthogonalisable (singular W^H R)");
    return SK_ERR_SINGULAR;
  }
  SK_TRY(combine(e, e.Vnew, m, E, m, m, (double2*)L));
  // F = sign(T_m) by Newton's iteration
  std::vector<cd> S;
  if (!dense::newton_sign(m, Tm, S, 1e-14, 100)) {
    set_error("Newton iteration for sign(T_m) did not converge");
    return SK_ERR_NOCONV;
  }
  SK_TRY(to_dev((double2*)F, S, stream));
  SK_HIP(hipStreamSynchronize(stream));
  for (int i = 0; i < m; ++i) {
    lambda[2 * i] = lam[i].real();
    lambda[2 * i + 1] = lam[i].imag();
  }
  if (stats) {
    stats->restarts[1] = rl;
    stats->resid[1] = resl;
    stats->matvecs = e.matvecs;
    stats->converged = 1;
  }
  return SK_OK;
}

// ---- host helpers around the dense routines
int sk_dense_schur(int n, const double* A, double* T, double* Q, int key, int count) {
  SK_CHECK(n >= 1 && n <= 4096 && A && T && Q, "bad arguments");
  SK_CHECK(key >= 0 && key <= 2, "key must be 0, 1 or 2");
  std::vector<cd> a((size_t)n * n), q;
  for (size_t i = 0; i < a.size(); ++i) a[i] = cd(A[2 * i], A[2 * i + 1]);
  if (!dense::schur(n, a, q)) {
    set_error("QR iteration did not converge");
    return SK_ERR_NOCONV;
  }
  auto kf = [key](cd z) { return key == 0 ? z.real() : (key == 1 ? std::abs(z) : std::abs(z.real())); };
  if (count > 0) dense::reorder_schur(n, a, q, kf, std::min(count, n));
  for (size_t i = 0; i < a.size(); ++i) {
    T[2 * i] = a[i].real();
    T[2 * i + 1] = a[i].imag();
    Q[2 * i] = q[i].real();
    Q[2 * i + 1] = q[i].imag();
  }
  return SK_OK;
}

int sk_dense_sign(int n, const double* A, double* S) {
  SK_CHECK(n >= 1 && n <= 4096 && A && S, "bad arguments");
  std::vector<cd> a((size_t)n * n), s;
  for (size_t i = 0; i < a.size(); ++i) a[i] = cd(A[2 * i], A[2 * i + 1]);
  if (!dense::newton_sign(n, a, s, 1e-14, 100)) {
    set_error("Newton sign iteration did not converge (singular or eigenvalue on the imaginary axis)");
    return SK_ERR_NOCONV;
  }
  for (size_t i = 0; i < s.size(); ++i) {
    S[2 * i] = s[i].real();
    S[2 * i + 1] = s[i].imag();
  }
  return SK_OK;
}

}  // extern "C"
