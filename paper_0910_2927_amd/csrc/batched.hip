// Many sign(H_W) b solves at once: Algorithm 1 for a batch of independent
// systems (sources, possibly on lattices of different sizes), stepped in
// lockstep so that every kernel of a restart cycle is one launch for the
// whole batch (system index in blockIdx.z; blocks past a smaller system's
// extent return at once).  Systems on the same gauge field form a group:
// the stencil keeps each hop's link in registers and applies it to every
// right-hand side of the group in turn.  Converged systems drop out via a
// device activity mask, so a cycle's launch sequence never changes and is
// replayed from a captured HIP graph.
#include "krylov_ws.h"
#include "stencil_dev.h"
#include "dcgs2_dev.h"
#include "small_dev.h"

#include <map>
#include <mutex>
#include <vector>

namespace sk {
namespace {

constexpr int kBNT = kTsThreads;
constexpr int kMaxGroupRhs = 64;
constexpr int kSites = 64;            // sites per stencil block
constexpr int kBStencilThreads = 512; // one wave per hop

// One system of the batch.
struct BSys {
  int64_t n;
  int group;
  double2* W64;        // complex-double basis, (k+1) x n
  float2* W32;         // complex-float basis (mixed precision), or null
  ArnoldiDev arn;      // H (ld k+1), scale (ones), st
  double2* gpart;      // Gram-Schmidt partial dots, gs_row_blocks(n) x (2k+2)
  double2* sbuf;       // first-pass coefficients, 2 x (k+2)
  double2* rho;        // N
  double2* Y;          // N x k
  double2* U;          // N x k x k
  double2* ucoef;      // k + 1
  double2* x;          // solution (caller)
  const double2* b;    // source (caller)
  double* xpart;       // partial ||x||^2 per row block of kBNT rows
  const double2* R;    // deflation (caller), m x n, or null
  const double2* L;
  const double2* F;    // m x m column-major
  int m;
  int proj;            // project every restart vector (else only measure the leak)
  double2* dpart;      // partial L^H v, gs_row_blocks(n) x m
};

struct BGroup {
  StencilGeom g;
  const double2* links64;
  const float2* links32;
  int nsys;
  int sys[kMaxGroupRhs];
};

template <typename T> __device__ inline T* basis(const BSys& S);
template <> __device__ inline double2* basis<double2>(const BSys& S) { return S.W64; }
template <> __device__ inline float2* basis<float2>(const BSys& S) { return S.W32; }
template <typename T> __device__ inline const T* group_links(const BGroup& G);
template <> __device__ inline const double2* group_links<double2>(const BGroup& G) { return G.links64; }
template <> __device__ inline const float2* group_links<float2>(const BGroup& G) { return G.links32; }

__device__ inline bool live(const BSys& S, const int* act, int z) {
  return act[z] != 0 && S.arn.st->breakdown == 0;
}

// ---- stencil: z = A u_j for every live system of a group
template <int H, typename T>
__device__ inline void bhop(double2 (*hs)[64], const T* in, const double2 (&u)[3][3], int V, int nb,
                            double fac, int lane) {
  double2 u0[3], u1[3];
  half_with_link<(H >> 1), (H & 1) ? 1 : -1>(u0, u1, in, V, nb, u, fac);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    hs[a][lane] = u0[a];
    hs[3 + a][lane] = u1[a];
  }
}

template <int H, typename T>
__device__ inline void load_hop_link(double2 (&u)[3][3], const T* U, int V, int ulink) {
  load_link<(H >> 1), (H & 1) == 1>(u, U, V, ulink);
}

template <typename T>
__global__ __launch_bounds__(kBStencilThreads) void k_bstencil(const BGroup* __restrict__ groups,
                                                               const BSys* __restrict__ sys,
                                                               const int* __restrict__ act, int j) {
  const BGroup& G = groups[blockIdx.z];
  const StencilGeom& g = G.g;
  const int lane = threadIdx.x & 63, h = threadIdx.x >> 6;
  const int s = blockIdx.x * kSites + lane;
  if (blockIdx.x * kSites >= g.V) return;
  const bool act_site = s < g.V;
  __shared__ double2 hs[8][6][64];
  // neighbour, hop factor and this wave's link, once for all right-hand sides
  int nb = 0, ulink = 0;
  double fac = 0.0;
  double2 u[3][3];
  if (act_site) {
    int r = s;
    const int x = r % g.Lx; r /= g.Lx;
    const int y = r % g.Ly; r /= g.Ly;
    const int zc = r % g.Lz;
    const int t = r / g.Lz;
    const int coord[4] = {x, y, zc, t};
    const int ext[4] = {g.Lx, g.Ly, g.Lz, g.Lt};
    const int stride[4] = {1, g.Lx, g.Lx * g.Ly, g.Lx * g.Ly * g.Lz};
    const int nu = h >> 1;
    neighbour(h, g, s, coord[nu], ext[nu], stride[nu], nb, ulink, fac);
    const T* U = group_links<T>(G);
    switch (h) {
      case 0: load_hop_link<0>(u, U, g.V, ulink); break;
      case 1: load_hop_link<1>(u, U, g.V, ulink); break;
      case 2: load_hop_link<2>(u, U, g.V, ulink); break;
      case 3: load_hop_link<3>(u, U, g.V, ulink); break;
      case 4: load_hop_link<4>(u, U, g.V, ulink); break;
      case 5: load_hop_link<5>(u, U, g.V, ulink); break;
      case 6: load_hop_link<6>(u, U, g.V, ulink); break;
      default: load_hop_link<7>(u, U, g.V, ulink); break;
    }
  }
  for (int rr = 0; rr < G.nsys; ++rr) {
    const int z = G.sys[rr];
    const BSys& S = sys[z];
    if (!live(S, act, z)) continue;   // uniform over the block
    const T* in = basis<T>(S) + (int64_t)j * S.n;
    T* out = basis<T>(S) + (int64_t)(j + 1) * S.n;
    if (act_site) {
      switch (h) {
        case 0: bhop<0>(hs[0], in, u, g.V, nb, fac, lane); break;
        case 1: bhop<1>(hs[1], in, u, g.V, nb, fac, lane); break;
        case 2: bhop<2>(hs[2], in, u, g.V, nb, fac, lane); break;
        case 3: bhop<3>(hs[3], in, u, g.V, nb, fac, lane); break;
        case 4: bhop<4>(hs[4], in, u, g.V, nb, fac, lane); break;
        case 5: bhop<5>(hs[5], in, u, g.V, nb, fac, lane); break;
        case 6: bhop<6>(hs[6], in, u, g.V, nb, fac, lane); break;
        default: bhop<7>(hs[7], in, u, g.V, nb, fac, lane); break;
      }
    }
    __syncthreads();
    if (h < 3 && act_site) {
      const int a = h;
      double2 acc[4];
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) acc[sp] = make_double2(0.0, 0.0);
      add_hop<0>(acc, hs[0], a, lane);
      add_hop<1>(acc, hs[1], a, lane);
      add_hop<2>(acc, hs[2], a, lane);
      add_hop<3>(acc, hs[3], a, lane);
      add_hop<4>(acc, hs[4], a, lane);
      add_hop<5>(acc, hs[5], a, lane);
      add_hop<6>(acc, hs[6], a, lane);
      add_hop<7>(acc, hs[7], a, lane);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        const int c = sp * 3 + a;
        double2 v = cadd(ld(in + c * g.V + s), acc[sp]);
        if (sp >= 2) v = make_double2(-v.x, -v.y);   // gamma5
        st(out + c * g.V + s, v);
      }
    }
    __syncthreads();
  }
}

// ---- Gram-Schmidt (delayed reorthogonalisation) for every live system
template <typename T>
__global__ __launch_bounds__(kBNT) void k_bdot(const BSys* __restrict__ sys, const int* __restrict__ act,
                                               int j, int has_z) {
  const int z = blockIdx.z;
  const BSys& S = sys[z];
  if (!live(S, act, z)) return;
  if ((int)blockIdx.x >= gs_row_blocks(S.n)) return;
  dc_dot_body<T>(basis<T>(S), S.n, j, has_z, S.n, gs_rpt(S.n), S.gpart, blockIdx.x, blockIdx.y);
}

template <typename T, bool FINAL>
__global__ __launch_bounds__(kBNT) void k_bupdate(const BSys* __restrict__ sys,
                                                  const int* __restrict__ act, int j, int k) {
  const int z = blockIdx.z;
  const BSys& S = sys[z];
  if (!live(S, act, z)) return;
  if ((int64_t)blockIdx.x * kBNT >= S.n) return;
  dc_update_body<T, FINAL>(basis<T>(S), S.n, j, S.n, S.gpart, gs_row_blocks(S.n), S.arn,
                           S.sbuf + (size_t)((j - 1) & 1) * (k + 2), S.sbuf + (size_t)(j & 1) * (k + 2),
                           0, (int64_t)blockIdx.x * kBNT + threadIdx.x, blockIdx.x == 0);
}

// ---- shifted Hessenberg solves: one workgroup per live system
__global__ __launch_bounds__(1024) void k_bsmall(const BSys* __restrict__ sys, const int* __restrict__ act,
                                                 int k, PoleSet poles) {
  const int z = blockIdx.x;
  const BSys& S = sys[z];
  if (act[z] == 0) return;
  fom_small_body(S.arn, k, poles, S.rho, S.Y, S.U, S.ucoef, nullptr);
}

// ---- x += V_k u and partial ||x||^2
template <typename T>
__global__ __launch_bounds__(kBNT) void k_bxupdate(const BSys* __restrict__ sys, const int* __restrict__ act) {
  const int z = blockIdx.z;
  const BSys& S = sys[z];
  if (act[z] == 0) return;
  if ((int64_t)blockIdx.x * kBNT >= S.n) return;
  const int kk = S.arn.st->kdone;
  const T* W = basis<T>(S);
  const int64_t r = (int64_t)blockIdx.x * kBNT + threadIdx.x;
  double nrm = 0.0;
  if (r < S.n) {
    double2 acc = S.x[r];
    int c = 0;
    for (; c + 8 <= kk; c += 8) {
      double2 v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = ld(W + (int64_t)(c + q) * S.n + r);
#pragma unroll
      for (int q = 0; q < 8; ++q) acc = cadd(acc, cmul(v[q], S.ucoef[c + q]));
    }
    for (; c < kk; ++c) acc = cadd(acc, cmul(ld(W + (int64_t)c * S.n + r), S.ucoef[c]));
    S.x[r] = acc;
    nrm = cabs2(acc);
  }
  __shared__ double red[kBNT / 64];
  nrm = wave_sum(nrm);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int w = 0; w < kBNT / 64; ++w) a += red[w];
    S.xpart[blockIdx.x] = a;
  }
}

__global__ __launch_bounds__(kBNT) void k_bxnorm(const BSys* __restrict__ sys, const int* __restrict__ act) {
  const int z = blockIdx.x;
  const BSys& S = sys[z];
  if (act[z] == 0) return;
  const int nb = (int)((S.n + kBNT - 1) / kBNT);
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBNT) a += S.xpart[b];
  __shared__ double red[kBNT / 64];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBNT / 64; ++w) t += red[w];
    S.arn.st->xnorm2 = t;
    if (!isfinite(t)) S.arn.st->nonfinite = 1;
  }
}

// ---- deflation: partial L^H v over row blocks (v = basis slot `slot`, or b)
template <typename T>
__global__ __launch_bounds__(kBNT) void k_bpdot(const BSys* __restrict__ sys, const int* __restrict__ act,
                                                int slot, int from_b) {
  const int z = blockIdx.z;
  const BSys& S = sys[z];
  if (act[z] == 0 || S.m == 0) return;
  if (!from_b && S.arn.st->breakdown) return;
  const int nrb = gs_row_blocks(S.n);
  if ((int)blockIdx.x >= nrb) return;
  const int i0 = blockIdx.y * 8;
  if (i0 >= S.m) return;
  const int cnt = min(8, S.m - i0);
  const int rpt = gs_rpt(S.n);
  double2 acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = make_double2(0.0, 0.0);
  const int64_t base = (int64_t)blockIdx.x * kBNT * rpt + threadIdx.x;
  for (int q = 0; q < rpt; ++q) {
    const int64_t r = base + (int64_t)q * kBNT;
    if (r >= S.n) break;
    const double2 v = from_b ? S.b[r] : ld(basis<T>(S) + (int64_t)slot * S.n + r);
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (c < cnt) acc[c] = cadd(acc[c], cconjmul(S.L[(int64_t)(i0 + c) * S.n + r], v));
  }
  __shared__ double2 red[kBNT / 64][8];
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
    for (int w = 1; w < kBNT / 64; ++w) s = cadd(s, red[w][threadIdx.x]);
    S.dpart[(size_t)blockIdx.x * S.m + i0 + threadIdx.x] = s;
  }
}

// r = v - R (L^H v) into basis slot 0 of precision TN (v = slot k of T, or b);
// with init: also x = R F (L^H b).  Without deflation: r = v, x = 0 (init).
template <typename T, typename TN, bool INIT>
__global__ __launch_bounds__(kBNT) void k_bproject(const BSys* __restrict__ sys, const int* __restrict__ act,
                                                   int slot) {
  const int z = blockIdx.z;
  const BSys& S = sys[z];
  if (act[z] == 0) return;
  if (!INIT && S.arn.st->breakdown) return;
  if ((int64_t)blockIdx.x * kBNT >= S.n) return;
  __shared__ double2 c[kMaxDefl];
  __shared__ double2 fc[kMaxDefl];
  __shared__ double2 scratch[kBNT];
  const int m = S.m;
  const int mp = (INIT || S.proj) ? m : 0;   // columns of R applied
  if (m > 0) {
    reduce_cols(S.dpart, gs_row_blocks(S.n), m, c, scratch);
    if (INIT) {
      for (int i = threadIdx.x; i < m; i += kBNT) {
        double2 a = make_double2(0.0, 0.0);
        for (int l = 0; l < m; ++l) a = cadd(a, cmul(S.F[(size_t)l * m + i], c[l]));
        fc[i] = a;
      }
    } else if (blockIdx.x == 0 && threadIdx.x == 0) {
      double l2 = 0.0;
      for (int i = 0; i < m; ++i) l2 += cabs2(c[i]);
      S.arn.st->leak = sqrt(l2);
    }
    __syncthreads();
  }
  const int64_t r = (int64_t)blockIdx.x * kBNT + threadIdx.x;
  if (r >= S.n) return;
  double2 v = INIT ? S.b[r] : ld(basis<T>(S) + (int64_t)slot * S.n + r);
  double2 xp = make_double2(0.0, 0.0);
  for (int i = 0; i < mp; ++i) {
    const double2 Ri = S.R[(int64_t)i * S.n + r];
    v = csub(v, cmul(Ri, c[i]));
    if (INIT) xp = cadd(xp, cmul(Ri, fc[i]));
  }
  st(basis<TN>(S) + r, v);
  if (INIT) S.x[r] = xp;
}

__global__ void k_binit(const BSys* __restrict__ sys, int nsys, int npoles, int k) {
  const int z = blockIdx.x;
  if (z >= nsys) return;
  const BSys& S = sys[z];
  for (int i = threadIdx.x; i < (k + 1) * k; i += blockDim.x) S.arn.H[i] = make_double2(0.0, 0.0);
  for (int i = threadIdx.x; i < k + 2; i += blockDim.x) S.arn.scale[i] = 1.0;
  for (int i = threadIdx.x; i < npoles; i += blockDim.x) S.rho[i] = make_double2(1.0, 0.0);
  if (threadIdx.x == 0) {
    CycleState* st = S.arn.st;
    st->beta = st->xnorm2 = st->upd_norm = st->leak = st->hnext = 0.0;
    st->kdone = st->breakdown = st->singular = st->nonfinite = 0;
  }
}

// ---- host side
struct BatchPlan {
  int nsys, ngroups, k, N, mmax;
  int64_t nmax;
  bool mixed;
  BSys* dsys;        // device descriptors
  BGroup* dgroups;
  int* act;          // device activity mask
  CycleState* st;    // device, nsys contiguous
};

size_t carve_batch(Carver& c, int nsys, const sk_operator* ops, const int* mlist,
                   const sk_sign_params* p, std::vector<BSys>* hs, int* ngroups_out,
                   std::vector<BGroup>* hg, BatchPlan* plan) {
  const int k = p->k, N = p->npoles;
  const bool mixed = p->precision == SK_PREC_MIXED;
  // groups: systems sharing links, geometry and mu
  std::vector<BGroup> groups;
  std::vector<int> gid(nsys);
  for (int z = 0; z < nsys; ++z) {
    const sk_operator* o = &ops[z];
    int found = -1;
    for (size_t q = 0; q < groups.size(); ++q) {
      const sk_operator* r = &ops[groups[q].sys[0]];
      if (r->links == o->links && r->links_c64 == o->links_c64 && r->mu == o->mu &&
          r->kappa == o->kappa && r->t_antiperiodic == o->t_antiperiodic &&
          std::memcmp(r->dims, o->dims, sizeof(r->dims)) == 0 && groups[q].nsys < kMaxGroupRhs) {
        found = (int)q;
        break;
      }
    }
    if (found < 0) {
      BGroup G;
      std::memset(&G, 0, sizeof(G));
      G.g = make_stencil_geom(o, 0);
      G.links64 = (const double2*)o->links;
      G.links32 = (const float2*)o->links_c64;
      groups.push_back(G);
      found = (int)groups.size() - 1;
    }
    groups[found].sys[groups[found].nsys++] = z;
    gid[z] = found;
  }
  if (hg) *hg = groups;
  if (ngroups_out) *ngroups_out = (int)groups.size();
  BatchPlan pl;
  std::memset(&pl, 0, sizeof(pl));
  pl.nsys = nsys;
  pl.ngroups = (int)groups.size();
  pl.k = k;
  pl.N = N;
  pl.mixed = mixed;
  pl.dsys = c.take<BSys>(nsys);
  pl.dgroups = c.take<BGroup>(groups.size());
  pl.act = c.take<int>(nsys);
  pl.st = c.take<CycleState>(nsys);
  if (hs) hs->resize(nsys);
  for (int z = 0; z < nsys; ++z) {
    const int64_t n = 12 * volume_of(&ops[z]);
    pl.nmax = std::max(pl.nmax, n);
    pl.mmax = std::max(pl.mmax, mlist ? mlist[z] : 0);
    BSys S;
    std::memset(&S, 0, sizeof(S));
    S.n = n;
    S.group = gid[z];
    S.W64 = c.take<double2>((size_t)(k + 1) * n);
    S.W32 = mixed ? c.take<float2>((size_t)(k + 1) * n) : nullptr;
    S.arn.H = c.take<double2>((size_t)(k + 1) * k);
    S.arn.scale = c.take<double>(k + 2);
    S.arn.ldh = k + 1;
    S.arn.st = pl.st ? pl.st + z : nullptr;
    S.gpart = c.take<double2>((size_t)gs_row_blocks(n) * (2 * k + 2));
    S.sbuf = c.take<double2>((size_t)2 * (k + 2));
    S.rho = c.take<double2>(N);
    S.Y = c.take<double2>((size_t)N * k);
    S.U = c.take<double2>((size_t)N * k * k);
    S.ucoef = c.take<double2>(k + 1);
    S.xpart = c.take<double>((n + kBNT - 1) / kBNT);
    S.m = mlist ? mlist[z] : 0;
    S.proj = p->project_each_cycle ? 1 : 0;
    S.dpart = c.take<double2>((size_t)gs_row_blocks(n) * (S.m > 0 ? S.m : 1));
    if (hs) (*hs)[z] = S;
  }
  if (plan) *plan = pl;
  return c.off;
}

std::mutex g_bmu;
hipStream_t batch_capture_stream() {
  static hipStream_t cs = nullptr;
  std::lock_guard<std::mutex> lk(g_bmu);
  if (!cs && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) cs = nullptr;
  return cs;
}

template <typename T, typename TN>
int enqueue_bcycle(const BatchPlan& P, const PoleSet& ps, hipStream_t s) {
  const int k = P.k;
  const int maxtiles = (int)((P.nmax / 12 + kSites - 1) / kSites);
  const int maxrb = gs_row_blocks(P.nmax);
  const unsigned maxrows = (unsigned)((P.nmax + kBNT - 1) / kBNT);
  for (int j = 0; j <= k; ++j) {
    if (j < k) {
      hipLaunchKernelGGL((k_bstencil<T>), dim3(maxtiles, 1, P.ngroups), dim3(kBStencilThreads), 0, s,
                         P.dgroups, P.dsys, P.act, j);
      SK_LAUNCH(hipGetLastError());
    }
    const bool last = (j == k);
    hipLaunchKernelGGL((k_bdot<T>), dim3(maxrb, j > 0 ? (j + 7) / 8 : 1, P.nsys), dim3(kBNT), 0, s,
                       P.dsys, P.act, j, last ? 0 : 1);
    SK_LAUNCH(hipGetLastError());
    if (last)
      hipLaunchKernelGGL((k_bupdate<T, true>), dim3(maxrows, 1, P.nsys), dim3(kBNT), 0, s, P.dsys, P.act, j, k);
    else
      hipLaunchKernelGGL((k_bupdate<T, false>), dim3(maxrows, 1, P.nsys), dim3(kBNT), 0, s, P.dsys, P.act, j, k);
    SK_LAUNCH(hipGetLastError());
  }
  hipLaunchKernelGGL(k_bsmall, dim3(P.nsys), dim3(1024), 0, s, P.dsys, P.act, k, ps);
  SK_LAUNCH(hipGetLastError());
  hipLaunchKernelGGL((k_bxupdate<T>), dim3(maxrows, 1, P.nsys), dim3(kBNT), 0, s, P.dsys, P.act);
  SK_LAUNCH(hipGetLastError());
  hipLaunchKernelGGL(k_bxnorm, dim3(P.nsys), dim3(kBNT), 0, s, P.dsys, P.act);
  SK_LAUNCH(hipGetLastError());
  if (P.mmax > 0) {
    hipLaunchKernelGGL((k_bpdot<T>), dim3(maxrb, (P.mmax + 7) / 8, P.nsys), dim3(kBNT), 0, s, P.dsys,
                       P.act, k, 0);
    SK_LAUNCH(hipGetLastError());
  }
  hipLaunchKernelGGL((k_bproject<T, TN, false>), dim3(maxrows, 1, P.nsys), dim3(kBNT), 0, s, P.dsys,
                     P.act, k);
  SK_LAUNCH(hipGetLastError());
  return SK_OK;
}

int enqueue_bcycle_kind(int kind, const BatchPlan& P, const PoleSet& ps, hipStream_t s) {
  if (kind == 0) return enqueue_bcycle<double2, double2>(P, ps, s);
  if (kind == 1) return enqueue_bcycle<double2, float2>(P, ps, s);
  return enqueue_bcycle<float2, float2>(P, ps, s);
}

}  // namespace
}  // namespace sk

using namespace sk;

extern "C" {

size_t sign_apply_batched_workspace_bytes(int nsys, const sk_operator* ops, const int* m,
                                          const sk_sign_params* p) {
  if (nsys < 1 || !ops || !p || p->k < 1 || p->k > kMaxK || p->npoles < 1 || p->npoles > kMaxPoles)
    return 0;
  for (int z = 0; z < nsys; ++z)
    if (volume_of(&ops[z]) <= 0 || (m && (m[z] < 0 || m[z] > kMaxDefl))) return 0;
  Carver c;
  return carve_batch(c, nsys, ops, m, p, nullptr, nullptr, nullptr, nullptr);
}

int sign_apply_batched(int nsys, const sk_operator* ops, const double* const* b, double* const* x,
                       const int* m, const double* const* R, const double* const* L,
                       const double* const* F, const sk_sign_params* p, sk_stats* stats, void* ws,
                       size_t ws_bytes, hipStream_t stream) {
  SK_CHECK(nsys >= 1 && ops && b && x && p && ws, "NULL argument or nsys < 1");
  SK_CHECK(p->k >= 1 && p->k <= kMaxK, "k = %d outside [1, %d]", p->k, kMaxK);
  SK_CHECK(p->npoles >= 1 && p->npoles <= kMaxPoles, "npoles outside [1, %d]", kMaxPoles);
  SK_CHECK(p->max_cycles >= 1 && p->tol > 0.0, "max_cycles and tol must be positive");
  SK_CHECK(p->precision == SK_PREC_FP64 || p->precision == SK_PREC_MIXED, "unknown precision");
  SK_CHECK(p->X_shift == nullptr, "per-shift solutions are not available in the batched solver");
  SK_CHECK(!(p->mixed_switch < 0.0), "mixed_switch must be >= 0");
  const bool mixed = p->precision == SK_PREC_MIXED;
  for (int z = 0; z < nsys; ++z) {
    SK_TRY(check_operator(&ops[z], SK_C128));
    if (mixed) SK_TRY(check_operator(&ops[z], SK_C64));
    SK_CHECK(b[z] && x[z], "b[%d] / x[%d] is NULL", z, z);
    const size_t nb = (size_t)12 * volume_of(&ops[z]) * 16;
    SK_CHECK(!overlap(b[z], nb, x[z], nb), "system %d: b and x overlap", z);
    for (int y = 0; y < z; ++y) {
      const size_t ny = (size_t)12 * volume_of(&ops[y]) * 16;
      SK_CHECK(!overlap(x[y], ny, x[z], nb) && !overlap(b[y], ny, x[z], nb) && !overlap(x[y], ny, b[z], nb),
               "systems %d and %d share solution memory", y, z);
    }
    const int mz = m ? m[z] : 0;
    SK_CHECK(mz >= 0 && mz <= kMaxDefl, "m[%d] = %d outside [0, %d]", z, mz, kMaxDefl);
    if (mz > 0) SK_CHECK(R && L && F && R[z] && L[z] && F[z], "system %d: m > 0 needs R, L, F", z);
  }
  const size_t need = sign_apply_batched_workspace_bytes(nsys, ops, m, p);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return SK_ERR_WORKSPACE;
  }
  for (int z = 0; z < nsys; ++z) {
    const size_t nb = (size_t)12 * volume_of(&ops[z]) * 16;
    SK_CHECK(!overlap(ws, need, x[z], nb) && !overlap(ws, need, b[z], nb),
             "workspace overlaps b or x of system %d", z);
  }
  PoleSet ps;
  SK_CHECK(p->sigma && p->omega, "sigma/omega are NULL");
  ps.n = p->npoles;
  for (int i = 0; i < ps.n; ++i) {
    ps.sigma[i] = make_double2(p->sigma[2 * i], p->sigma[2 * i + 1]);
    ps.omega[i] = make_double2(p->omega[2 * i], p->omega[2 * i + 1]);
  }
  Carver c;
  c.base = (char*)ws;
  std::vector<BSys> hs;
  std::vector<BGroup> hg;
  BatchPlan P;
  int ng = 0;
  carve_batch(c, nsys, ops, m, p, &hs, &ng, &hg, &P);
  for (int z = 0; z < nsys; ++z) {
    hs[z].x = (double2*)x[z];
    hs[z].b = (const double2*)b[z];
    if (hs[z].m > 0) {
      hs[z].R = (const double2*)R[z];
      hs[z].L = (const double2*)L[z];
      hs[z].F = (const double2*)F[z];
    }
  }
  hipStream_t s = stream;
  SK_HIP(hipMemcpyAsync(P.dsys, hs.data(), nsys * sizeof(BSys), hipMemcpyHostToDevice, s));
  SK_HIP(hipMemcpyAsync(P.dgroups, hg.data(), ng * sizeof(BGroup), hipMemcpyHostToDevice, s));
  std::vector<int> act(nsys, 1);
  SK_HIP(hipMemcpyAsync(P.act, act.data(), nsys * sizeof(int), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_binit, dim3(nsys), dim3(256), 0, s, P.dsys, nsys, ps.n, P.k);
  SK_LAUNCH(hipGetLastError());
  const double theta = !mixed ? 0.0 : (p->mixed_switch > 0.0 ? p->mixed_switch : 1e-3);
  bool low = mixed && theta >= 1.0;
  // x = x_P, W_0 = (I - P) b
  const int maxrb = gs_row_blocks(P.nmax);
  const unsigned maxrows = (unsigned)((P.nmax + kBNT - 1) / kBNT);
  if (P.mmax > 0) {
    hipLaunchKernelGGL((k_bpdot<double2>), dim3(maxrb, (P.mmax + 7) / 8, nsys), dim3(kBNT), 0, s, P.dsys,
                       P.act, 0, 1);
    SK_LAUNCH(hipGetLastError());
  }
  if (low)
    hipLaunchKernelGGL((k_bproject<double2, float2, true>), dim3(maxrows, 1, nsys), dim3(kBNT), 0, s,
                       P.dsys, P.act, 0);
  else
    hipLaunchKernelGGL((k_bproject<double2, double2, true>), dim3(maxrows, 1, nsys), dim3(kBNT), 0, s,
                       P.dsys, P.act, 0);
  SK_LAUNCH(hipGetLastError());
  std::vector<CycleState> st(nsys);
  std::vector<int> small(nsys, 0), status(nsys, SK_ERR_NOCONV);
  std::vector<double> first(nsys, 0.0);
  if (stats)
    for (int z = 0; z < nsys; ++z) {
      stats[z].cycles = stats[z].cycles_c64 = stats[z].matvecs = stats[z].converged = 0;
      stats[z].breakdown = 0;
      stats[z].final_update_norm = stats[z].x_norm = 0.0;
    }
  hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
  struct GraphGuard {
    hipGraphExec_t* e;
    ~GraphGuard() {
      for (int i = 0; i < 3; ++i)
        if (e[i]) hipGraphExecDestroy(e[i]);
    }
  } guard{exec};
  int nact = nsys;
  for (int cyc = 0; cyc < p->max_cycles && nact > 0; ++cyc) {
    bool all_small = true;
    for (int z = 0; z < nsys; ++z)
      if (act[z] && !(cyc > 0 && st[z].upd_norm <= theta * std::sqrt(st[z].xnorm2))) all_small = false;
    const bool low_next = low || (mixed && cyc > 0 && all_small);
    const int kind = !low ? (low_next ? 1 : 0) : 2;
    if (!exec[kind]) {
      hipStream_t cs = batch_capture_stream();
      SK_CHECK(cs != nullptr, "could not create the capture stream");
      SK_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      const int rc = enqueue_bcycle_kind(kind, P, ps, cs);
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(cs, &graph);
      if (rc != SK_OK) {
        if (graph) hipGraphDestroy(graph);
        return rc;
      }
      if (e != hipSuccess) {
        set_error("graph capture failed: %s", hipGetErrorString(e));
        return SK_ERR_HIP;
      }
      const hipError_t ei = hipGraphInstantiate(&exec[kind], graph, nullptr, nullptr, 0);
      hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        exec[kind] = nullptr;
        set_error("graph instantiation failed: %s", hipGetErrorString(ei));
        return SK_ERR_HIP;
      }
    }
    SK_HIP(hipGraphLaunch(exec[kind], s));
    SK_HIP(hipMemcpyAsync(st.data(), P.st, nsys * sizeof(CycleState), hipMemcpyDeviceToHost, s));
    SK_HIP(hipStreamSynchronize(s));
    const bool cur_low = low;
    low = low_next;
    bool changed = false;
    for (int z = 0; z < nsys; ++z) {
      if (!act[z]) continue;
      const CycleState& q = st[z];
      if (stats) {
        stats[z].cycles = cyc + 1;
        stats[z].cycles_c64 += cur_low ? 1 : 0;
        stats[z].matvecs += q.kdone;
        stats[z].final_update_norm = q.upd_norm;
        stats[z].x_norm = std::sqrt(q.xnorm2);
        if (cyc < stats[z].hist_cap) {
          if (stats[z].hist_update) stats[z].hist_update[cyc] = q.upd_norm;
          if (stats[z].hist_beta) stats[z].hist_beta[cyc] = q.beta;
          if (stats[z].hist_leak) stats[z].hist_leak[cyc] = q.leak;
        }
      }
      int done = 0;
      if (q.nonfinite) {
        status[z] = SK_ERR_NAN;
        done = 1;
      } else if (q.singular) {
        status[z] = SK_ERR_SINGULAR;
        done = 1;
      } else if (q.breakdown) {
        status[z] = SK_OK;
        if (stats) stats[z].breakdown = 1;
        done = 1;
      } else {
        small[z] = (q.upd_norm <= p->tol * std::sqrt(q.xnorm2)) ? small[z] + 1 : 0;
        if (small[z] >= 2) {
          status[z] = SK_OK;
          done = 1;
        } else if (cyc == 0) {
          first[z] = q.upd_norm;
        } else if (q.upd_norm > kDivergeFactor * first[z]) {
          status[z] = SK_ERR_NOCONV;
          done = 1;
        }
      }
      if (done) {
        act[z] = 0;
        --nact;
        changed = true;
        if (stats) stats[z].converged = status[z] == SK_OK;
      }
    }
    if (changed) SK_HIP(hipMemcpyAsync(P.act, act.data(), nsys * sizeof(int), hipMemcpyHostToDevice, s));
  }
  SK_HIP(hipStreamSynchronize(s));
  int worst = SK_OK;
  for (int z = 0; z < nsys; ++z)
    if (status[z] != SK_OK) worst = status[z];
  if (worst != SK_OK) set_error("some systems did not converge (first failing status %d)", worst);
  return worst;
}

}  // extern "C"
