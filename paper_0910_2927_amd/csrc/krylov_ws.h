// Workspace layout, timing and the Arnoldi enqueue shared by the drivers
// (driver.hip, eigs.hip).  Internal to libsignkrylov.
#pragma once

#include "sk_internal.h"

#include <cstring>
#include <vector>

namespace sk {
namespace {

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

// Carves the caller's workspace into aligned pieces.
struct Carver {
  size_t off = 0;
  char* base = nullptr;
  template <typename T> T* take(size_t count) {
    size_t o = off;
    off = align256(off + count * sizeof(T));
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

// Device scratch used by an Arnoldi-based driver.
template <typename T>
struct KrylovWs {
  T* W;                // (k+1) basis slots, unnormalised: v_j = scale[j] W_j
  double2* H;
  double* scale;
  double* wnorm;
  double2* coef;
  double2* partial;
  unsigned* counter;
  CycleState* st;
  double2* rho;
  double2* Y;
  double2* U;
  double2* ucoef;
  double2* ycoef;
  double2* dc;
  double2* dc2;
  double2* gpart;      // Gram-Schmidt partial dots, gs_part_entries(sd_row_blocks(n), k)
  double2* sbuf;       // first-pass coefficients, 2 x (k+2) (alternating)
  size_t gpart_cap;    // entries of gpart
  int sbuf_k;          // k the first-pass buffers were sized for
};

// The Gram-Schmidt scratch of an Arnoldi run of length k (shared by every
// workspace layout that runs enqueue_arnoldi).
template <typename T>
void carve_gs(Carver& c, KrylovWs<T>& w, int64_t n, int k) {
  w.gpart_cap = gs_part_entries(sd_row_blocks(n), k);
  w.gpart = c.template take<double2>(w.gpart_cap);
  w.sbuf = c.template take<double2>((size_t)2 * (k + 2));
  w.sbuf_k = k;
}

template <typename T>
size_t carve_krylov(Carver& c, KrylovWs<T>& w, int64_t n, int k, int npoles, int m, bool keep) {
  const int pmax = k > m ? k : m;
  w.W = c.template take<T>((size_t)(k + 1) * n);
  w.H = c.template take<double2>((size_t)(k + 1) * k);
  w.scale = c.template take<double>(k + 2);
  w.wnorm = c.template take<double>(k + 1);
  w.coef = c.template take<double2>(kMaxK + 4);
  w.partial = c.template take<double2>(ts_partial_entries(n, pmax));
  w.counter = c.template take<unsigned>((size_t)kCounterSlots * ts_counter_stride(n));
  w.st = c.template take<CycleState>(1);
  w.rho = c.template take<double2>(npoles > 0 ? npoles : 1);
  w.Y = c.template take<double2>((size_t)(npoles > 0 ? npoles : 1) * k);
  w.U = c.template take<double2>((size_t)(npoles > 0 ? npoles : 1) * k * k);
  w.ucoef = c.template take<double2>(k + 1);
  w.ycoef = keep ? c.template take<double2>((size_t)npoles * k) : nullptr;
  w.dc = c.template take<double2>(m > 0 ? m : 1);
  w.dc2 = c.template take<double2>(m > 0 ? m : 1);
  carve_gs(c, w, n, k);
  return c.off;
}

template <typename T>
ArnoldiDev arn_of(const KrylovWs<T>& w, int k) {
  ArnoldiDev a;
  a.H = w.H;
  a.scale = w.scale;
  a.wnorm = w.wnorm;
  a.coef = w.coef;
  a.partial = w.partial;
  a.counter = w.counter;
  a.st = w.st;
  a.ldh = k + 1;
  return a;
}

TsEpiArgs epi_of(int kind, const ArnoldiDev& a, int j = 0) {
  TsEpiArgs e;
  std::memset(&e, 0, sizeof(e));
  e.epi = kind;
  e.j = j;
  e.arn = a;
  return e;
}

// Optional per-kernel timing: HIP events around every launch of a solve,
// summed per kernel class after each cycle's host synchronisation.
struct KTimer {
  sk_kernel_times* out = nullptr;
  hipStream_t s = nullptr;
  std::vector<hipEvent_t> pool;
  struct Rec { int cls; double bytes; int e0, e1; };
  std::vector<Rec> recs;
  size_t used = 0;
  int cur_cls = 0, cur_e0 = 0;
  double cur_bytes = 0.0;
  bool on() const { return out != nullptr; }
  int record() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      pool.push_back(e);
    }
    hipEventRecord(pool[used], s);
    return (int)used++;
  }
  void begin(int cls, double bytes) {
    if (!on()) return;
    cur_cls = cls;
    cur_bytes = bytes;
    cur_e0 = record();
  }
  void end() {
    if (!on()) return;
    int e1 = record();
    if (cur_e0 >= 0 && e1 >= 0) recs.push_back({cur_cls, cur_bytes, cur_e0, e1});
  }
  // Kernel-stamped timing: two events that the launches themselves record
  // at the start of the first and the end of the last kernel of the class
  // (no event packets between kernels, so the interval is kernel time only,
  // as a kernel trace reports it).  Both null when timing is off.
  struct Ext {
    hipEvent_t t0 = nullptr, t1 = nullptr;
  };
  int reserve() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      pool.push_back(e);
    }
    return (int)used++;
  }
  Ext begin_ext(int cls, double bytes) {
    if (!on()) return {};
    const int a = reserve(), b = reserve();
    if (a < 0 || b < 0) return {};
    recs.push_back({cls, bytes, a, b});
    return {pool[a], pool[b]};
  }
  // call after the stream has been synchronised
  void flush() {
    if (!on()) return;
    for (const Rec& r : recs) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pool[r.e0], pool[r.e1]) == hipSuccess) {
        out->ms[r.cls] += ms;
        out->bytes[r.cls] += r.bytes;
        out->launches[r.cls] += 1;
      }
    }
    recs.clear();
    used = 0;
  }
  ~KTimer() {
    for (hipEvent_t e : pool) hipEventDestroy(e);
  }
};

template <typename T> const T* links_as(const sk_operator* op);
template <> const double2* links_as<double2>(const sk_operator* op) { return (const double2*)op->links; }
template <> const float2* links_as<float2>(const sk_operator* op) { return (const float2*)op->links_c64; }

#define SK_LAUNCH(call)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      ::sk::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), __FILE__, \
                      __LINE__);                                                          \
      return SK_ERR_HIP;                                                                  \
    }                                                                                     \
  } while (0)

// k Arnoldi steps on the unnormalised basis in w.W; W_0 and scale[0] must be
// set.  Kernels after a breakdown return at once (skip flag).
// Arnoldi steps j = j0 .. k-1 on the basis in w.W, then the final second
// pass of vector k (delayed reorthogonalisation, dcgs2.hip).  W_{j0} holds
// the start vector (any norm when j0 = 0).  power = 2 applies the operator
// twice per step (A^2, through `tmp`), as the deflation eigensolver needs;
// j0 > 0 continues a thick-restarted decomposition whose columns < j0 are
// already in H.  After a breakdown every later kernel returns at once.
template <typename T>
int enqueue_arnoldi(const sk_operator* op, const KrylovWs<T>& w, int64_t n, int k, int adjoint,
                    hipStream_t s, KTimer* tm = nullptr, int j0 = 0, int power = 1,
                    T* tmp = nullptr) {
  const ArnoldiDev a = arn_of(w, k);
  const T* U = links_as<T>(op);
  const int* skip = &w.st->breakdown;
  // every buffer the step kernels index must be there and large enough
  if (!w.W || !w.H || !w.st || !w.sbuf || !w.gpart || w.sbuf_k < k ||
      w.gpart_cap < gs_part_entries(sd_row_blocks(n), k) || (power == 2 && !tmp)) {
    set_error("internal: Arnoldi workspace is missing a buffer or is too small");
    return SK_ERR_WORKSPACE;
  }
  KTimer dummy;
  KTimer& t = tm ? *tm : dummy;
  const double c = (double)sizeof(T), nn = (double)n;
  auto sb = [&](int j) { return w.sbuf + (size_t)(j & 1) * (k + 2); };
  for (int j = j0; j < k; ++j) {
    T* wj = w.W + (size_t)j * n;
    T* wj1 = w.W + (size_t)(j + 1) * n;
    // stencil: 12 in + 36 link + 12 out complex per site = 5 n complex
    const auto es = t.begin_ext(SK_K_STENCIL, 5.0 * nn * c * power);
    if (power == 2) {
      SK_LAUNCH((launch_wilson<T, T, T>(op, U, wj, tmp, adjoint, nullptr, skip, s, es.t0, nullptr)));
      SK_LAUNCH((launch_wilson<T, T, T>(op, U, tmp, wj1, adjoint, nullptr, skip, s, nullptr, es.t1)));
    } else {
      SK_LAUNCH((launch_wilson<T, T, T>(op, U, wj, wj1, adjoint, nullptr, skip, s, es.t0, es.t1)));
    }
    // V_j^H [u, z]: j basis vectors + u + z read once
    const auto ed = t.begin_ext(SK_K_GS_DOT, (j + 2) * nn * c);
    const int nrb = sd_row_blocks(n, sizeof(T) == 8 ? 2 : 1);
    const auto er = gs_reduced(nrb) ? t.begin_ext(SK_K_GS_REDUCE, (nrb + kGsGroups) * (2.0 * j + 2) * 16.0)
                                    : KTimer::Ext{};
    SK_LAUNCH((dc_dot<T>(w.W, n, j, true, n, w.gpart, skip, s, ed.t0, ed.t1, er.t0, er.t1)));
    // v_j and u_{j+1} from one pass over V_j (+ read u, z; write v_j, u_{j+1})
    const auto eu = t.begin_ext(SK_K_GS_UPD_DOT, (j + 4) * nn * c);
    SK_LAUNCH((dc_update<T>(w.W, n, j, false, n, w.gpart, a, sb(j - 1), sb(j), j == j0 && j0 > 0,
                            skip, s, eu.t0, eu.t1)));
  }
  const auto ef = t.begin_ext(SK_K_GS_UPD_NORM, (2 * k + 3) * nn * c);
  SK_LAUNCH((dc_dot<T>(w.W, n, k, false, n, w.gpart, skip, s, ef.t0, nullptr)));
  SK_LAUNCH((dc_update<T>(w.W, n, k, true, n, w.gpart, a, sb(k - 1), sb(k), k == j0 && j0 > 0, skip,
                          s, nullptr, ef.t1)));
  return SK_OK;
}

}  // namespace
}  // namespace sk
