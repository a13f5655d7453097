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

#include <hip/hip_ext.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

namespace sk {
namespace {

constexpr int kBNT = kTsThreads;
constexpr int kMaxGroupRhs = 64;
constexpr int kSites = 64;            // sites per stencil block
constexpr int kBStencilThreads = 512; // one wave per hop

// Launch shapes chosen by the tuner: rows per thread of the Gram-Schmidt
// dot kernel (hence row blocks of partial sums) and of the update kernel
// (both in row packs), and right-hand sides per stencil block (the links of
// a block's sites are loaded once for all of them).
struct BTile {
  int rpt;
  int urt;
  int rhs;
};

// One system of the batch.
struct BSys {
  int64_t n;
  int k;               // this system's restart length
  int group;
  double2* W64;        // complex-double basis, (k+1) x n
  float2* W32;         // complex-float basis (mixed precision), or null
  ArnoldiDev arn;      // H (ld k+1), scale (ones), st
  double2* gpart;      // Gram-Schmidt partial dots, row blocks x (2k+2)
  double2* sbuf;       // first-pass coefficients, 2 x (k+2)
  double2* rho;        // N
  double2* Y;          // N x k
  double2* U;          // N x k x k
  double2* ucoef;      // k + 1
  const double2* sigma;   // this system's poles and weights (npoles each)
  const double2* omega;
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
// Hop H of one site from the neighbour's 12 components already in registers:
// project to the half spinor, multiply by the link (in registers), scale.
template <int H, typename T>
__device__ inline void bhop(double2 (*hs)[64], const T (&raw)[12], const double2 (&u)[3][3], double fac,
                            int lane) {
  using PJ = Proj<(H >> 1), (H & 1) ? 1 : -1>;
  double2 h0[3], h1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h0[c] = cadd(cvt(raw[c]), ph<PJ::P0>(cvt(raw[PJ::A0 * 3 + c])));
    h1[c] = cadd(cvt(raw[3 + c]), ph<PJ::P1>(cvt(raw[PJ::A1 * 3 + c])));
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double2 s0 = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      s0 = cadd(s0, cmul(u[a][b], h0[b]));
      s1 = cadd(s1, cmul(u[a][b], h1[b]));
    }
    hs[a][lane] = cscale(s0, fac);
    hs[3 + a][lane] = cscale(s1, fac);
  }
}

template <int H, typename T>
__device__ inline void load_hop_link(double2 (&u)[3][3], const T* U, int V, int ulink) {
  load_link<(H >> 1), (H & 1) == 1>(u, U, V, ulink);
}

template <typename T>
__global__ __launch_bounds__(kBStencilThreads) void k_bstencil(const BGroup* __restrict__ groups,
                                                               const BSys* __restrict__ sys,
                                                               const int* __restrict__ act, int j,
                                                               int rhs) {
  const BGroup& G = groups[blockIdx.z];
  const StencilGeom& g = G.g;
  const int lane = threadIdx.x & 63, h = threadIdx.x >> 6;
  const int s = blockIdx.x * kSites + lane;
  if (blockIdx.x * kSites >= g.V || (int)blockIdx.y * rhs >= G.nsys) return;
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
  // Right-hand sides of this block in turn; the neighbour components (hop
  // waves) and the diagonal (combining waves) of the next one are loaded
  // while the current one is combined.
  const int rbeg = blockIdx.y * rhs;
  const int rend = min(G.nsys, rbeg + rhs);
  T rc[12], rn[12], dc[4], dn[4];
  auto prefetch = [&](int r, T (&raw)[12], T (&dia)[4]) {
    // slot j exists for this system (its basis has k + 1 slots)
    if (!act_site || r >= rend || j >= sys[G.sys[r]].k) return;
    const T* in = basis<T>(sys[G.sys[r]]) + (int64_t)j * sys[G.sys[r]].n;
#pragma unroll
    for (int c = 0; c < 12; ++c) raw[c] = in[c * g.V + nb];
    if (h < 3)
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) dia[sp] = in[(sp * 3 + h) * g.V + s];
  };
  prefetch(rbeg, rc, dc);
  for (int rr = rbeg; rr < rend; ++rr) {
    const int z = G.sys[rr];
    const BSys& S = sys[z];
    const bool on = j < S.k && live(S, act, z);   // uniform over the block
    prefetch(rr + 1, rn, dn);
    if (on) {
      T* out = basis<T>(S) + (int64_t)(j + 1) * S.n;
      if (act_site) {
        switch (h) {
          case 0: bhop<0>(hs[0], rc, u, fac, lane); break;
          case 1: bhop<1>(hs[1], rc, u, fac, lane); break;
          case 2: bhop<2>(hs[2], rc, u, fac, lane); break;
          case 3: bhop<3>(hs[3], rc, u, fac, lane); break;
          case 4: bhop<4>(hs[4], rc, u, fac, lane); break;
          case 5: bhop<5>(hs[5], rc, u, fac, lane); break;
          case 6: bhop<6>(hs[6], rc, u, fac, lane); break;
          default: bhop<7>(hs[7], rc, u, fac, lane); break;
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
          double2 v = cadd(cvt(dc[sp]), acc[sp]);
          if (sp >= 2) v = make_double2(-v.x, -v.y);   // gamma5
          st(out + c * g.V + s, v);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) rc[c] = rn[c];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) dc[sp] = dn[sp];
  }
}

// ---- Gram-Schmidt (delayed reorthogonalisation) for every live system
// row blocks of rpt row packs of `pack` rows per thread
__host__ __device__ inline int brow_blocks(int64_t n, int rpt, int pack = 1) {
  const int64_t rb = (int64_t)kBNT * rpt * pack;
  return (int)((n + rb - 1) / rb);
}

// Step j of every live system with j <= k (z = A u_j is there for j < k;
// j = k is the final second pass of the last vector).
template <typename T>
__global__ __launch_bounds__(kBNT) void k_bdot(const BSys* __restrict__ sys, const int* __restrict__ act,
                                               int j, BTile tile) {
  const int z = blockIdx.z;
  const BSys& S = sys[z];
  if (j > S.k || !live(S, act, z)) return;
  if ((int)blockIdx.x >= brow_blocks(S.n, tile.rpt, Pk<T>::P)) return;
  dc_dot_body<T>(basis<T>(S), S.n, j, j < S.k ? 1 : 0, S.n, tile.rpt, S.gpart, blockIdx.x, blockIdx.y);
}

// Fold the dot partials of systems with many row blocks into kGsGroups rows
// (stored after them), so that update blocks read a few rows only.
template <typename T>
__global__ __launch_bounds__(kBNT) void k_breduce(const BSys* __restrict__ sys, const int* __restrict__ act,
                                                  int j, BTile tile) {
  const int z = blockIdx.z;
  const BSys& S = sys[z];
  if (j > S.k || !live(S, act, z)) return;
  const int nrb = brow_blocks(S.n, tile.rpt, Pk<T>::P);
  if (!gs_reduced(nrb)) return;
  const int pr = 2 * j + 2;
  dc_reduce_body(S.gpart, nrb, pr, S.gpart + (size_t)nrb * pr, blockIdx.x, blockIdx.y);
}

// FINAL: systems whose k is j; otherwise systems with j < k.
template <typename T, bool FINAL>
__global__ __launch_bounds__(kBNT) void k_bupdate(const BSys* __restrict__ sys,
                                                  const int* __restrict__ act, int j, BTile tile) {
  const int z = blockIdx.z;
  const BSys& S = sys[z];
  if ((FINAL ? j != S.k : j >= S.k) || !live(S, act, z)) return;
  const int64_t r0 = (int64_t)blockIdx.x * kBNT * tile.urt;   // in row packs
  if (r0 * Pk<T>::P >= S.n) return;
  const int k = S.k;
  const int nrb = brow_blocks(S.n, tile.rpt, Pk<T>::P);
  const double2* src = gs_reduced(nrb) ? S.gpart + (size_t)nrb * (2 * j + 2) : S.gpart;
  dc_update_body<T, FINAL>(basis<T>(S), S.n, j, S.n, src, gs_reduced(nrb) ? kGsGroups : nrb, S.arn,
                           S.sbuf + (size_t)((j - 1) & 1) * (k + 2), S.sbuf + (size_t)(j & 1) * (k + 2),
                           0, r0 + threadIdx.x, tile.urt, blockIdx.x == 0);
}

// Tuning data: slot i (i <= j) is the indicator of rows r = i mod (j + 2)
// (mutually orthogonal, so the step runs its full course without a
// breakdown) and slot j + 1 is all ones.  Timing does not depend on values.
template <typename T>
__global__ __launch_bounds__(kBNT) void k_btune_fill(const BSys* __restrict__ sys, int j) {
  const BSys& S = sys[blockIdx.z];
  const int64_t r = (int64_t)blockIdx.x * kBNT + threadIdx.x;
  if (r >= S.n) return;
  T* W = basis<T>(S);
  const int64_t mod = r % (j + 2);
  for (int i = 0; i <= j + 1; ++i)
    st(W + (int64_t)i * S.n + r, make_double2((i == j + 1 || mod == i) ? 1.0 : 0.0, 0.0));
}

// ---- shifted Hessenberg solves: one workgroup per live system
__global__ __launch_bounds__(kWaves * 64) void k_bsmall(const BSys* __restrict__ sys,
                                                         const int* __restrict__ act, int npoles) {
  const int z = blockIdx.x;
  const BSys& S = sys[z];
  if (act[z] == 0) return;
  __shared__ PoleSet poles;
  if (threadIdx.x == 0) poles.n = npoles;
  for (int i = threadIdx.x; i < npoles; i += blockDim.x) {
    poles.sigma[i] = S.sigma[i];
    poles.omega[i] = S.omega[i];
  }
  __syncthreads();
  fom_small_body(S.arn, S.k, poles, S.rho, S.Y, S.U, S.ucoef, nullptr);
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
                                                int from_b) {
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
    const double2 v = from_b ? S.b[r] : ld(basis<T>(S) + (int64_t)S.k * S.n + r);
    double2 lv[8];   // all loads in flight before any is used
#pragma unroll
    for (int c = 0; c < 8; ++c) lv[c] = S.L[(int64_t)(i0 + min(c, cnt - 1)) * S.n + r];
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (c < cnt) acc[c] = cadd(acc[c], cconjmul(lv[c], v));
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
__global__ __launch_bounds__(kBNT) void k_bproject(const BSys* __restrict__ sys,
                                                   const int* __restrict__ act) {
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
  double2 v = INIT ? S.b[r] : ld(basis<T>(S) + (int64_t)S.k * S.n + r);
  double2 xp = make_double2(0.0, 0.0);
  for (int i = 0; i < mp; ++i) {
    const double2 Ri = S.R[(int64_t)i * S.n + r];
    v = csub(v, cmul(Ri, c[i]));
    if (INIT) xp = cadd(xp, cmul(Ri, fc[i]));
  }
  st(basis<TN>(S) + r, v);
  if (INIT) S.x[r] = xp;
}

__global__ void k_binit(const BSys* __restrict__ sys, int nsys, int npoles) {
  const int z = blockIdx.x;
  if (z >= nsys) return;
  const BSys& S = sys[z];
  const int k = S.k;
  for (int i = threadIdx.x; i < (k + 1) * k; i += blockDim.x) S.arn.H[i] = make_double2(0.0, 0.0);
  for (int i = threadIdx.x; i < k + 2; i += blockDim.x) S.arn.scale[i] = 1.0;
  for (int i = threadIdx.x; i < npoles; i += blockDim.x) S.rho[i] = make_double2(1.0, 0.0);
  for (int i = threadIdx.x; i < 2 * (k + 2); i += blockDim.x) S.sbuf[i] = make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
    CycleState* st = S.arn.st;
    st->beta = st->xnorm2 = st->upd_norm = st->leak = st->hnext = 0.0;
    st->kdone = st->breakdown = st->singular = st->nonfinite = 0;
  }
}

// ---- host side
struct BatchPlan {
  int nsys, ngroups, kmin, kmax, N, mmax;
  int64_t nmax;
  int maxrb_defl;    // most row blocks of the deflation dots (gs_row_blocks is not monotone in n)
  int maxrhs;        // most systems in one group
  bool mixed;
  std::vector<int> kfinal;   // distinct restart lengths (a final pass at each)
  BSys* dsys;        // device descriptors
  BGroup* dgroups;
  int* act;          // device activity mask
  CycleState* st;    // device, nsys contiguous
  double2* poles;    // device, nsys x (sigma[N], omega[N])
};

int sys_k(const sk_batch_system& d, const sk_sign_params* p) { return d.k > 0 ? d.k : p->k; }

size_t carve_batch(Carver& c, int nsys, const sk_batch_system* d, const sk_sign_params* p,
                   std::vector<BSys>* hs, std::vector<BGroup>* hg, BatchPlan* plan) {
  const int N = p->npoles;
  const bool mixed = p->precision == SK_PREC_MIXED;
  // groups: systems sharing links, geometry and mu
  std::vector<BGroup> groups;
  std::vector<int> gid(nsys);
  for (int z = 0; z < nsys; ++z) {
    const sk_operator* o = &d[z].op;
    int found = -1;
    for (size_t q = 0; q < groups.size(); ++q) {
      const sk_operator* r = &d[groups[q].sys[0]].op;
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
  BatchPlan pl;
  pl.maxrhs = 1;
  for (const BGroup& G : groups) pl.maxrhs = std::max(pl.maxrhs, G.nsys);
  pl.nsys = nsys;
  pl.ngroups = (int)groups.size();
  pl.kmin = kMaxK;
  pl.kmax = 0;
  pl.N = N;
  pl.mmax = 0;
  pl.nmax = 0;
  pl.maxrb_defl = 1;
  pl.mixed = mixed;
  pl.dsys = c.take<BSys>(nsys);
  pl.dgroups = c.take<BGroup>(groups.size());
  pl.act = c.take<int>(nsys);
  pl.st = c.take<CycleState>(nsys);
  pl.poles = c.take<double2>((size_t)nsys * 2 * N);
  if (hs) hs->resize(nsys);
  for (int z = 0; z < nsys; ++z) {
    const int64_t n = 12 * volume_of(&d[z].op);
    const int k = sys_k(d[z], p);
    pl.nmax = std::max(pl.nmax, n);
    pl.kmin = std::min(pl.kmin, k);
    pl.kmax = std::max(pl.kmax, k);
    if (std::find(pl.kfinal.begin(), pl.kfinal.end(), k) == pl.kfinal.end()) pl.kfinal.push_back(k);
    pl.mmax = std::max(pl.mmax, d[z].m);
    pl.maxrb_defl = std::max(pl.maxrb_defl, gs_row_blocks(n));
    BSys S;
    std::memset(&S, 0, sizeof(S));
    S.n = n;
    S.k = k;
    S.group = gid[z];
    S.W64 = c.take<double2>((size_t)(k + 1) * n);
    S.W32 = mixed ? c.take<float2>((size_t)(k + 1) * n) : nullptr;
    S.arn.H = c.take<double2>((size_t)(k + 1) * k);
    S.arn.scale = c.take<double>(k + 2);
    S.arn.ldh = k + 1;
    S.arn.st = pl.st ? pl.st + z : nullptr;
    S.gpart = c.take<double2>(gs_part_entries(brow_blocks(n, 1), k));   // any tile
    S.sbuf = c.take<double2>((size_t)2 * (k + 2));
    S.rho = c.take<double2>(N);
    S.Y = c.take<double2>((size_t)N * k);
    S.U = c.take<double2>((size_t)N * k * k);
    S.ucoef = c.take<double2>(k + 1);
    S.sigma = pl.poles ? pl.poles + (size_t)z * 2 * N : nullptr;
    S.omega = pl.poles ? pl.poles + (size_t)z * 2 * N + N : nullptr;
    S.xpart = c.take<double>((n + kBNT - 1) / kBNT);
    S.m = d[z].m;
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

// Per-kernel timing of a batched cycle (plain launches, no graph): the
// host copies of the descriptors and of the activity mask give each launch
// class its algorithmic bytes, summed over the systems live in the cycle.
// A null pointer means no timing.
struct BTiming {
  KTimer* tm;
  const std::vector<BSys>* hs;
  const std::vector<BGroup>* hg;
  const std::vector<int>* act;
  bool on() const { return tm && tm->on(); }
  // sum over live systems of f(system); 0 when timing is off
  template <typename F> double sum(F f) const {
    double t = 0.0;
    if (!on()) return t;
    for (size_t z = 0; z < hs->size(); ++z)
      if ((*act)[z]) t += f((*hs)[z]);
    return t;
  }
  KTimer::Ext ext(int cls, double bytes) const { return on() ? tm->begin_ext(cls, bytes) : KTimer::Ext{}; }
};

// A launch that stamps the timing events when they are set.
template <typename F, typename... Args>
hipError_t blaunch(F kern, dim3 grid, dim3 block, hipStream_t s, hipEvent_t t0, hipEvent_t t1, Args... args) {
  if (t0 || t1) hipExtLaunchKernelGGL(kern, grid, block, 0, s, t0, t1, 0, args...);
  else hipLaunchKernelGGL(kern, grid, block, 0, s, args...);
  return hipGetLastError();
}

// Gram-Schmidt launches of step j: dots, the update of systems still
// stepping, and the final pass of systems whose restart length is j.
template <typename T>
int enqueue_bgs(const BatchPlan& P, const BTile& tile, int j, hipStream_t s, const BTiming& bt = {}) {
  const int maxrb = brow_blocks(P.nmax, tile.rpt, Pk<T>::P);
  const unsigned maxub = (unsigned)brow_blocks(P.nmax, tile.urt, Pk<T>::P);
  const double c = (double)sizeof(T);
  // V_j^H [u z] (j + 2 vectors; the final pass j = k reads k + 1)
  const auto ed = bt.ext(SK_K_GS_DOT, bt.sum([&](const BSys& S) {
    return j <= S.k ? (double)(j < S.k ? j + 2 : j + 1) * S.n * c : 0.0;
  }));
  SK_LAUNCH((blaunch(k_bdot<T>, dim3(maxrb, j > 0 ? (j + 7) / 8 : 1, P.nsys), dim3(kBNT), s, ed.t0, ed.t1,
                     (const BSys*)P.dsys, (const int*)P.act, j, tile)));
  if (gs_reduced(maxrb)) {
    const auto er = bt.ext(SK_K_GS_REDUCE, bt.sum([&](const BSys& S) {
      return j <= S.k ? (double)(brow_blocks(S.n, tile.rpt, Pk<T>::P) + kGsGroups) * (2.0 * j + 2) * 16.0 : 0.0;
    }));
    SK_LAUNCH((blaunch(k_breduce<T>, dim3((2 * j + 2 + 63) / 64, kGsGroups, P.nsys), dim3(kBNT), s, er.t0,
                       er.t1, (const BSys*)P.dsys, (const int*)P.act, j, tile)));
  }
  if (j < P.kmax) {
    // v_j and u_{j+1}: j + 2 reads, 2 writes
    const auto eu = bt.ext(SK_K_GS_UPD_DOT, bt.sum([&](const BSys& S) {
      return j < S.k ? (double)(j + 4) * S.n * c : 0.0;
    }));
    SK_LAUNCH((blaunch(k_bupdate<T, false>, dim3(maxub, 1, P.nsys), dim3(kBNT), s, eu.t0, eu.t1,
                       (const BSys*)P.dsys, (const int*)P.act, j, tile)));
  }
  if (std::find(P.kfinal.begin(), P.kfinal.end(), j) != P.kfinal.end()) {
    // final second pass of v_k: k + 1 reads, 1 write
    const auto ef = bt.ext(SK_K_GS_UPD_NORM, bt.sum([&](const BSys& S) {
      return S.k == j ? (double)(j + 2) * S.n * c : 0.0;
    }));
    SK_LAUNCH((blaunch(k_bupdate<T, true>, dim3(maxub, 1, P.nsys), dim3(kBNT), s, ef.t0, ef.t1,
                       (const BSys*)P.dsys, (const int*)P.act, j, tile)));
  }
  return SK_OK;
}

template <typename T>
int enqueue_bstencil(const BatchPlan& P, const BTile& tile, int j, hipStream_t s, const BTiming& bt = {}) {
  const int maxtiles = (int)((P.nmax / 12 + kSites - 1) / kSites);
  // in + out spinors per stepping system, the links once per group with one
  double bytes = 0.0;
  if (bt.on()) {
    const double c = (double)sizeof(T);
    bytes = bt.sum([&](const BSys& S) { return j < S.k ? 2.0 * S.n * c : 0.0; });
    for (const BGroup& G : *bt.hg) {
      bool stepping = false;
      for (int q = 0; q < G.nsys; ++q) {
        const int z = G.sys[q];
        if ((*bt.act)[z] && j < (*bt.hs)[z].k) stepping = true;
      }
      if (stepping) bytes += 3.0 * (*bt.hs)[G.sys[0]].n * c;   // 36 complex per site = 3 n
    }
  }
  const auto es = bt.ext(SK_K_STENCIL, bytes);
  SK_LAUNCH((blaunch(k_bstencil<T>, dim3(maxtiles, (P.maxrhs + tile.rhs - 1) / tile.rhs, P.ngroups),
                     dim3(kBStencilThreads), s, es.t0, es.t1, (const BGroup*)P.dgroups, (const BSys*)P.dsys,
                     (const int*)P.act, j, tile.rhs)));
  return SK_OK;
}

// One non-final Gram-Schmidt step for the tuner.
template <typename T>
int enqueue_bgs_step(const BatchPlan& P, const BTile& tile, int j, hipStream_t s) {
  const int maxrb = brow_blocks(P.nmax, tile.rpt, Pk<T>::P);
  const unsigned maxub = (unsigned)brow_blocks(P.nmax, tile.urt, Pk<T>::P);
  hipLaunchKernelGGL((k_bdot<T>), dim3(maxrb, j > 0 ? (j + 7) / 8 : 1, P.nsys), dim3(kBNT), 0, s,
                     P.dsys, P.act, j, tile);
  SK_LAUNCH(hipGetLastError());
  if (gs_reduced(maxrb)) {
    hipLaunchKernelGGL((k_breduce<T>), dim3((2 * j + 2 + 63) / 64, kGsGroups, P.nsys), dim3(kBNT), 0, s,
                       P.dsys, P.act, j, tile);
    SK_LAUNCH(hipGetLastError());
  }
  hipLaunchKernelGGL((k_bupdate<T, false>), dim3(maxub, 1, P.nsys), dim3(kBNT), 0, s, P.dsys, P.act, j,
                     tile);
  SK_LAUNCH(hipGetLastError());
  return SK_OK;
}

template <typename T, typename TN>
int enqueue_bcycle(const BatchPlan& P, const BTile& tile, hipStream_t s, const BTiming& bt = {}) {
  const int maxrb = P.maxrb_defl;
  const unsigned maxrows = (unsigned)((P.nmax + kBNT - 1) / kBNT);
  const double c = (double)sizeof(T), cn = (double)sizeof(TN);
  for (int j = 0; j <= P.kmax; ++j) {
    if (j < P.kmax) {
      SK_TRY(enqueue_bstencil<T>(P, tile, j, s, bt));
    }
    SK_TRY(enqueue_bgs<T>(P, tile, j, s, bt));
  }
  const auto em = bt.ext(SK_K_SMALL, 0.0);
  SK_LAUNCH((blaunch(k_bsmall, dim3(P.nsys), dim3(kWaves * 64), s, em.t0, em.t1, (const BSys*)P.dsys,
                     (const int*)P.act, P.N)));
  // x += V_k u: k basis vectors, x read and written in FP64
  const auto ex = bt.ext(SK_K_SOL_UPDATE, bt.sum([&](const BSys& S) {
    return (double)S.k * S.n * c + 2.0 * S.n * 16.0;
  }));
  SK_LAUNCH((blaunch(k_bxupdate<T>, dim3(maxrows, 1, P.nsys), dim3(kBNT), s, ex.t0, nullptr,
                     (const BSys*)P.dsys, (const int*)P.act)));
  SK_LAUNCH((blaunch(k_bxnorm, dim3(P.nsys), dim3(kBNT), s, nullptr, ex.t1, (const BSys*)P.dsys,
                     (const int*)P.act)));
  // L^H v and v - R (L^H v): L and R once each (m > 0), v read twice, the
  // restart vector written in the next cycle's precision
  const auto ep = bt.ext(SK_K_PROJECT, bt.sum([&](const BSys& S) {
    return (S.m > 0 ? 2.0 * S.m * S.n * 16.0 + S.n * c : 0.0) + S.n * c + S.n * cn;
  }));
  if (P.mmax > 0)
    SK_LAUNCH((blaunch(k_bpdot<T>, dim3(maxrb, (P.mmax + 7) / 8, P.nsys), dim3(kBNT), s, ep.t0, nullptr,
                       (const BSys*)P.dsys, (const int*)P.act, 0)));
  SK_LAUNCH((blaunch(k_bproject<T, TN, false>, dim3(maxrows, 1, P.nsys), dim3(kBNT), s,
                     P.mmax > 0 ? nullptr : ep.t0, ep.t1, (const BSys*)P.dsys, (const int*)P.act)));
  return SK_OK;
}

int enqueue_bcycle_kind(int kind, const BatchPlan& P, const BTile& tile, hipStream_t s, const BTiming& bt = {}) {
  if (kind == 0) return enqueue_bcycle<double2, double2>(P, tile, s, bt);
  if (kind == 1) return enqueue_bcycle<double2, float2>(P, tile, s, bt);
  return enqueue_bcycle<float2, float2>(P, tile, s, bt);
}

// The tuner: times the Gram-Schmidt step (dots + update, the bulk of a
// cycle's memory traffic) at j = kmin/2 (every system stepping) for each
// tile candidate on the batch's own workspace, in the precision most cycles
// use, and keeps the fastest.  Results are cached per batch shape for the
// life of the process.
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, BTile> g_tune_cache;
thread_local BTile g_last_tile = {0, 0, 0};
std::atomic<int> g_force_rpt{0}, g_force_urt{0}, g_force_rhs{4};   // rpt 0: use the tuner

std::vector<int64_t> tune_key(const BatchPlan& P, const std::vector<BSys>& hs) {
  std::vector<int64_t> key = {P.mixed ? 1 : 0, P.nsys};
  for (const BSys& S : hs) {
    key.push_back(S.n);
    key.push_back(S.k);
  }
  return key;
}

template <typename T>
int tune_tiles(const BatchPlan& P, hipStream_t s, BTile* best) {
  const int j = P.kmin / 2;
  static const BTile cand[] = {{1, 1, 4}, {2, 1, 4}, {4, 1, 4}, {8, 1, 4}, {2, 2, 4},
                               {4, 2, 4}, {8, 2, 4}, {4, 4, 4}, {8, 4, 4}};
  const dim3 fill_grid((unsigned)brow_blocks(P.nmax, 1), 1, P.nsys);
  hipEvent_t e0, e1;
  SK_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    set_error("hipEventCreate failed");
    return SK_ERR_HIP;
  }
  float tbest = 1e30f;
  int rc = SK_OK;
  for (const BTile& t : cand) {
    float tt = 0.0f;
    for (int rep = 0; rep < 3 && rc == SK_OK; ++rep) {
      // the update rewrites slots j and j+1, so the data is refilled each time
      hipLaunchKernelGGL((k_btune_fill<T>), fill_grid, dim3(kBNT), 0, s, P.dsys, j);
      if (hipGetLastError() != hipSuccess || hipEventRecord(e0, s) != hipSuccess) rc = SK_ERR_HIP;
      if (rc == SK_OK) {
        rc = enqueue_bgs_step<T>(P, t, j, s);
      }
      if (rc == SK_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
        rc = SK_ERR_HIP;
      float ms = 0.0f;
      if (rc == SK_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = SK_ERR_HIP;
      if (rep > 0) tt += ms;   // the first repetition warms caches and code
    }
    if (rc != SK_OK) break;
    if (tt < tbest) {
      tbest = tt;
      *best = t;
    }
  }
  // right-hand sides per stencil block, timed on the same data
  if (rc == SK_OK) {
    float sbest = 1e30f;
    BTile t = *best;
    for (int rhs : {1, 2, 4, 8}) {
      t.rhs = rhs;
      float tt = 0.0f;
      for (int rep = 0; rep < 3 && rc == SK_OK; ++rep) {
        if (hipEventRecord(e0, s) != hipSuccess) rc = SK_ERR_HIP;
        if (rc == SK_OK) rc = enqueue_bstencil<T>(P, t, j, s);
        if (rc == SK_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
          rc = SK_ERR_HIP;
        float ms = 0.0f;
        if (rc == SK_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = SK_ERR_HIP;
        if (rep > 0) tt += ms;
      }
      if (rc != SK_OK) break;
      if (tt < sbest) {
        sbest = tt;
        best->rhs = rhs;
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != SK_OK) set_error("tile tuning failed");
  return rc;
}

int check_batch(int nsys, const sk_batch_system* d, const sk_sign_params* p, char* msg, size_t len) {
  if (nsys < 1 || !d || !p) return snprintf(msg, len, "NULL argument or nsys < 1"), 0;
  if (p->npoles < 1 || p->npoles > kMaxPoles) return snprintf(msg, len, "npoles outside [1, %d]", kMaxPoles), 0;
  if (p->k < 0 || p->k > kMaxK) return snprintf(msg, len, "k = %d outside [1, %d]", p->k, kMaxK), 0;
  if (p->max_cycles < 1 || !(p->tol > 0.0)) return snprintf(msg, len, "max_cycles and tol must be positive"), 0;
  if (p->precision != SK_PREC_FP64 && p->precision != SK_PREC_MIXED) return snprintf(msg, len, "unknown precision"), 0;
  if (p->method != SK_METHOD_FOM) return snprintf(msg, len, "the batched solver runs FOM-LR only"), 0;
  if (p->X_shift) return snprintf(msg, len, "per-shift solutions are not available in the batched solver"), 0;
  if (p->mixed_switch < 0.0) return snprintf(msg, len, "mixed_switch must be >= 0"), 0;
  for (int z = 0; z < nsys; ++z) {
    if (volume_of(&d[z].op) <= 0) return snprintf(msg, len, "system %d: bad lattice dims", z), 0;
    const int k = sys_k(d[z], p);
    if (k < 1 || k > kMaxK || d[z].k < 0)
      return snprintf(msg, len, "system %d: restart length %d outside [1, %d]", z, k, kMaxK), 0;
    if (d[z].m < 0 || d[z].m > kMaxDefl) return snprintf(msg, len, "system %d: m = %d outside [0, %d]", z, d[z].m, kMaxDefl), 0;
    if (!(d[z].sigma || p->sigma) || !(d[z].omega || p->omega))
      return snprintf(msg, len, "system %d: no poles given", z), 0;
  }
  return 1;
}

}  // namespace
}  // namespace sk

using namespace sk;

extern "C" {

size_t sign_apply_batched_workspace_bytes(int nsys, const sk_batch_system* sys, const sk_sign_params* p) {
  char msg[256];
  if (!check_batch(nsys, sys, p, msg, sizeof msg)) return 0;
  Carver c;
  return carve_batch(c, nsys, sys, p, nullptr, nullptr, nullptr);
}

int sk_batched_set_tile(int rows_per_thread_dot, int rows_per_thread_update, int rhs_per_block) {
  const bool off = rows_per_thread_dot == 0 && rows_per_thread_update == 0 && rhs_per_block == 0;
  SK_CHECK(off || (rows_per_thread_dot >= 1 && rows_per_thread_dot <= 8 && rows_per_thread_update >= 1 &&
                   rows_per_thread_update <= 8 && rhs_per_block >= 1 && rhs_per_block <= kMaxGroupRhs),
           "rows per thread must be 1..8 and right-hand sides per block 1..%d (or all 0 for the tuner)",
           kMaxGroupRhs);
  g_force_urt.store(rows_per_thread_update);
  g_force_rhs.store(off ? 4 : rhs_per_block);
  g_force_rpt.store(rows_per_thread_dot);
  return SK_OK;
}

int sk_batched_last_tile(int* rows_per_thread_dot, int* rows_per_thread_update, int* rhs_per_block) {
  SK_CHECK(rows_per_thread_dot && rows_per_thread_update && rhs_per_block, "NULL argument");
  *rows_per_thread_dot = g_last_tile.rpt;
  *rows_per_thread_update = g_last_tile.urt;
  *rhs_per_block = g_last_tile.rhs;
  return SK_OK;
}

int sign_apply_batched(int nsys, const sk_batch_system* d, const sk_sign_params* p, sk_stats* stats,
                       void* ws, size_t ws_bytes, hipStream_t stream) {
  char msg[256];
  SK_CHECK(check_batch(nsys, d, p, msg, sizeof msg), "%s", msg);
  SK_CHECK(ws != nullptr, "workspace is NULL");
  const bool mixed = p->precision == SK_PREC_MIXED;
  for (int z = 0; z < nsys; ++z) {
    SK_TRY(check_operator(&d[z].op, SK_C128));
    if (mixed) SK_TRY(check_operator(&d[z].op, SK_C64));
    SK_CHECK(d[z].b && d[z].x, "system %d: b or x is NULL", z);
    if (d[z].m > 0) SK_CHECK(d[z].R && d[z].L && d[z].F, "system %d: m > 0 needs R, L, F", z);
    const size_t nb = (size_t)12 * volume_of(&d[z].op) * 16;
    SK_CHECK(!overlap(d[z].b, nb, d[z].x, nb), "system %d: b and x overlap", z);
    for (int y = 0; y < z; ++y) {
      const size_t ny = (size_t)12 * volume_of(&d[y].op) * 16;
      SK_CHECK(!overlap(d[y].x, ny, d[z].x, nb) && !overlap(d[y].b, ny, d[z].x, nb) &&
                   !overlap(d[y].x, ny, d[z].b, nb),
               "systems %d and %d share solution memory", y, z);
    }
  }
  const size_t need = sign_apply_batched_workspace_bytes(nsys, d, p);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return SK_ERR_WORKSPACE;
  }
  for (int z = 0; z < nsys; ++z) {
    const size_t nb = (size_t)12 * volume_of(&d[z].op) * 16;
    SK_CHECK(!overlap(ws, need, d[z].x, nb) && !overlap(ws, need, d[z].b, nb),
             "workspace overlaps b or x of system %d", z);
  }
  const int N = p->npoles;
  // per-system pole table: sigma then omega
  std::vector<double2> ptab((size_t)nsys * 2 * N);
  for (int z = 0; z < nsys; ++z) {
    const double* sg = d[z].sigma ? d[z].sigma : p->sigma;
    const double* om = d[z].omega ? d[z].omega : p->omega;
    for (int i = 0; i < N; ++i) {
      SK_CHECK(std::isfinite(sg[2 * i]) && std::isfinite(sg[2 * i + 1]) && std::isfinite(om[2 * i]) &&
                   std::isfinite(om[2 * i + 1]),
               "system %d: pole %d is not finite", z, i);
      ptab[(size_t)z * 2 * N + i] = make_double2(sg[2 * i], sg[2 * i + 1]);
      ptab[(size_t)z * 2 * N + N + i] = make_double2(om[2 * i], om[2 * i + 1]);
    }
  }
  Carver c;
  c.base = (char*)ws;
  std::vector<BSys> hs;
  std::vector<BGroup> hg;
  BatchPlan P;
  carve_batch(c, nsys, d, p, &hs, &hg, &P);
  for (int z = 0; z < nsys; ++z) {
    hs[z].x = (double2*)d[z].x;
    hs[z].b = (const double2*)d[z].b;
    if (hs[z].m > 0) {
      hs[z].R = (const double2*)d[z].R;
      hs[z].L = (const double2*)d[z].L;
      hs[z].F = (const double2*)d[z].F;
    }
  }
  hipStream_t s = stream;
  SK_HIP(hipMemcpyAsync(P.dsys, hs.data(), nsys * sizeof(BSys), hipMemcpyHostToDevice, s));
  SK_HIP(hipMemcpyAsync(P.dgroups, hg.data(), hg.size() * sizeof(BGroup), hipMemcpyHostToDevice, s));
  SK_HIP(hipMemcpyAsync(P.poles, ptab.data(), ptab.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  std::vector<int> act(nsys, 1);
  SK_HIP(hipMemcpyAsync(P.act, act.data(), nsys * sizeof(int), hipMemcpyHostToDevice, s));
  BTile tile = {gs_rpt(P.nmax), 1, 4};
  if (g_force_rpt.load() > 0) {
    tile = {g_force_rpt.load(), g_force_urt.load(), g_force_rhs.load()};
  } else {
    const std::vector<int64_t> key = tune_key(P, hs);
    bool have = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        tile = it->second;
        have = true;
      }
    }
    if (!have && P.kmin >= 2) {
      hipLaunchKernelGGL(k_binit, dim3(nsys), dim3(256), 0, s, P.dsys, nsys, N);
      SK_LAUNCH(hipGetLastError());
      SK_TRY(mixed ? tune_tiles<float2>(P, s, &tile) : tune_tiles<double2>(P, s, &tile));
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune_cache[key] = tile;
    }
  }
  g_last_tile = tile;
  hipLaunchKernelGGL(k_binit, dim3(nsys), dim3(256), 0, s, P.dsys, nsys, N);
  SK_LAUNCH(hipGetLastError());
  const double theta = !mixed ? 0.0 : (p->mixed_switch > 0.0 ? p->mixed_switch : 1e-3);
  bool low = mixed && theta >= 1.0;
  // x = x_P, W_0 = (I - P) b
  const int maxrb = P.maxrb_defl;
  const unsigned maxrows = (unsigned)((P.nmax + kBNT - 1) / kBNT);
  if (P.mmax > 0) {
    hipLaunchKernelGGL((k_bpdot<double2>), dim3(maxrb, (P.mmax + 7) / 8, nsys), dim3(kBNT), 0, s, P.dsys,
                       P.act, 1);
    SK_LAUNCH(hipGetLastError());
  }
  if (low)
    hipLaunchKernelGGL((k_bproject<double2, float2, true>), dim3(maxrows, 1, nsys), dim3(kBNT), 0, s,
                       P.dsys, P.act);
  else
    hipLaunchKernelGGL((k_bproject<double2, double2, true>), dim3(maxrows, 1, nsys), dim3(kBNT), 0, s,
                       P.dsys, P.act);
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
  // per-kernel timing (stats[0].times): plain launches instead of graphs
  KTimer tm;
  if (stats && stats[0].times) {
    tm.out = stats[0].times;
    tm.s = s;
  }
  const BTiming bt = tm.on() ? BTiming{&tm, &hs, &hg, &act} : BTiming{};
  for (int cyc = 0; cyc < p->max_cycles && nact > 0; ++cyc) {
    // the whole batch switches to complex float once every active system
    // meets the switch rule (the next cycle's precision is fixed before this
    // one is enqueued; once low, it stays low)
    bool all_small = true;
    for (int z = 0; z < nsys; ++z)
      if (act[z] && !(cyc > 0 && st[z].upd_norm <= theta * std::sqrt(st[z].xnorm2))) all_small = false;
    const bool low_next = low || (mixed && cyc > 0 && all_small);
    const int kind = !low ? (low_next ? 1 : 0) : 2;
    if (bt.on()) {
      SK_TRY(enqueue_bcycle_kind(kind, P, tile, s, bt));
    } else if (!exec[kind]) {
      hipStream_t cs = batch_capture_stream();
      SK_CHECK(cs != nullptr, "could not create the capture stream");
      SK_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      const int rc = enqueue_bcycle_kind(kind, P, tile, cs);
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
    if (!bt.on()) SK_HIP(hipGraphLaunch(exec[kind], s));
    SK_HIP(hipMemcpyAsync(st.data(), P.st, nsys * sizeof(CycleState), hipMemcpyDeviceToHost, s));
    SK_HIP(hipStreamSynchronize(s));
    tm.flush();
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
