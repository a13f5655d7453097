// Device bodies of the Arnoldi step with delayed reorthogonalisation,
// shared by the single-system kernels (dcgs2.hip) and the batched ones
// (batched.hip).  Internal to libsignkrylov.
#pragma once

#include "sk_internal.h"

namespace sk {
namespace {

constexpr int NT = kTsThreads;
constexpr int NW = NT / 64;
constexpr int VC = 8;

__device__ inline double2 z2() { return make_double2(0.0, 0.0); }

// Row packs: a thread loads P consecutive rows of a vector with one 16-byte
// load (P = 2 for complex float).  n = 12 V is even and every vector starts
// 16-byte aligned, so packs never straddle the end or a vector boundary.
template <typename T> struct Pk;
template <> struct Pk<double2> {
  using type = double2;
  static constexpr int P = 1;
  __device__ static double2 get(const double2& v, int) { return v; }
  __device__ static void set(double2& v, int, double2 x) { v = x; }
};
template <> struct Pk<float2> {
  using type = float4;
  static constexpr int P = 2;
  __device__ static double2 get(const float4& v, int p) {
    return p == 0 ? make_double2((double)v.x, (double)v.y) : make_double2((double)v.z, (double)v.w);
  }
  __device__ static void set(float4& v, int p, double2 x) {
    if (p == 0) {
      v.x = (float)x.x;
      v.y = (float)x.y;
    } else {
      v.z = (float)x.x;
      v.w = (float)x.y;
    }
  }
};

// Column sums of nrows x pr partials (row-major) into sums[0..pr), BT
// threads, scratch of BT entries; fixed order.
template <int BT = NT>
__device__ inline void reduce_cols(const double2* __restrict__ src, int nrows, int pr, double2* sums,
                                   double2* scratch) {
  constexpr int NW = BT / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i0 = 0; i0 < pr; i0 += 64) {
    const int i = i0 + lane;
    double2 acc = z2();
    if (i < pr) {
      // batches of 8 rows per wave, all loads issued before the sums (a
      // partial last batch reads zeros past nrows): the same order of
      // additions as one row at a time, without a chain of dependent loads
      for (int b = wid; b < nrows; b += 8 * NW) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = b + u * NW < nrows ? src[(size_t)(b + u * NW) * pr + i] : z2();
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = cadd(acc, v[u]);
      }
    }
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

// Exchange of a double with lane ^ M: DPP quad permutations for M = 1, 2,
// ds_swizzle (bit mode, within 32 lanes) for M = 4, 8, 16, a permute for 32.
template <int M>
__device__ inline double xor_lane(double v) {
  if constexpr (M == 1) {
    return dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  } else if constexpr (M == 2) {
    return dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  } else if constexpr (M < 32) {
    constexpr int kPat = 0x1F | (M << 10);   // and_mask 31, or_mask 0, xor_mask M
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), kPat);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), kPat);
    return __hiloint2double(hi, lo);
  } else {
    return __shfl_xor(v, M, 64);
  }
}

// Butterfly stages S.. of a reduce-scatter over the wave: at stage S the
// lanes with bit S clear keep the first H = ceil(C/2) of their C values,
// the others the rest (a missing last value reads as 0), and each adds its
// partner's copy of what it keeps.  idx accumulates the position of the
// kept range in the original list, real the number of its entries that
// are not padding.
template <int S, int C, int N>
__device__ inline void scatter_stages(double (&v)[N], int lane, int& idx, int& real) {
  if constexpr (S < 6) {
    constexpr int M = 1 << S, H = (C + 1) / 2;
    const bool up = (lane & M) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double lo = v[i];
      const double hi = (H + i < C) ? v[H + i] : 0.0;
      v[i] = (up ? hi : lo) + xor_lane<M>(up ? lo : hi);
    }
    if (up) {
      idx += H;
      real -= H;
    } else {
      real = min(real, H);
    }
    scatter_stages<S + 1, H, N>(v, lane, idx, real);
  }
}

// Sums over the 64 lanes of N values per lane (N <= 64) with about N
// exchanges instead of the 6 N of one wave_sum per value: afterwards v[0]
// of the returned lane-dependent index d holds the total of value d; every
// d < N is held by exactly one lane, the other lanes return -1.  The order
// of additions is fixed.
template <int N>
__device__ inline int wave_scatter_sum(double (&v)[N], int lane) {
  static_assert(N >= 2 && N <= 64, "one value per lane at most");
  int idx = 0, real = N;
  scatter_stages<0, N, N>(v, lane, idx, real);
  return real > 0 ? idx : -1;
}

constexpr int kRsVals = 4 * VC + 4;   // doubles per lane of the dot kernel

// Rows of one dot block: every load of a row pack is issued before any of
// it is used, so a wave has VC + 2 loads in flight.  FULL: the chunk holds
// VC vectors (no masking); otherwise vectors past cnt re-read a valid
// vector and are masked out.  base, rpt count packs.
template <typename T, bool HAS_Z, bool FULL, int BT>
__device__ inline void dot_rows(const T* __restrict__ W, int64_t ldq, int j, int i0, int cnt, int64_t n,
                                int rpt, int64_t base, bool first, double2 (&at)[VC], double2 (&ap)[VC],
                                double2& aa, double2& ag) {
  using K = Pk<T>;
  using PT = typename K::type;
  const PT* u = reinterpret_cast<const PT*>(W + (int64_t)j * ldq);
  const PT* zv = reinterpret_cast<const PT*>(W + (int64_t)(j + 1) * ldq);
  const int last = cnt > 0 ? cnt - 1 : 0;
  const PT* vb[VC];
#pragma unroll
  for (int c = 0; c < VC; ++c)
    vb[c] = reinterpret_cast<const PT*>(W + (int64_t)(i0 + (FULL ? c : min(c, last))) * ldq);
  for (int q = 0; q < rpt; ++q) {
    const int64_t rp = base + (int64_t)q * BT;
    if (rp * K::P >= n) break;
    PT raw[VC];
    const PT ru = u[rp];
    PT rz;
    if (HAS_Z) rz = zv[rp];
#pragma unroll
    for (int c = 0; c < VC; ++c) raw[c] = vb[c][rp];
#pragma unroll
    for (int p = 0; p < K::P; ++p) {
      const double2 uv = K::get(ru, p);
      const double2 zz = HAS_Z ? K::get(rz, p) : z2();
#pragma unroll
      for (int c = 0; c < VC; ++c)
        if (FULL || c < cnt) {
          const double2 vv = K::get(raw[c], p);
          at[c] = cadd(at[c], cconjmul(vv, uv));
          if (HAS_Z) ap[c] = cadd(ap[c], cconjmul(vv, zz));
        }
      if (first) {
        aa.x += cabs2(uv);
        if (HAS_Z) ag = cadd(ag, cconjmul(uv, zz));
      }
    }
  }
}

// Partial sums of t = V_j^H u, p = V_j^H z (chunk of VC vectors) and, in
// chunk 0, alpha = u^H u and gamma = u^H z.  Layout per row block:
// [t_0..t_{j-1}, p_0..p_{j-1}, alpha, gamma].
// BT: threads of the block (rows of a block: BT * rpt packs).
template <typename T, int BT = NT>
__device__ inline void dc_dot_body(const T* __restrict__ W, int64_t ldq, int j, int has_z,
                                   int64_t n, int rpt, double2* __restrict__ part, int rb, int ch) {
  constexpr int BW = BT / 64;
  const int i0 = ch * VC;
  const int cnt = max(0, min(VC, j - i0));
  double2 at[VC], ap[VC];
  double2 aa = z2(), ag = z2();
#pragma unroll
  for (int q = 0; q < VC; ++q) at[q] = ap[q] = z2();
  const int64_t base = (int64_t)rb * BT * rpt + threadIdx.x;   // in packs
  const bool first = ch == 0;
  if (has_z) {
    if (cnt == VC) dot_rows<T, true, true, BT>(W, ldq, j, i0, cnt, n, rpt, base, first, at, ap, aa, ag);
    else dot_rows<T, true, false, BT>(W, ldq, j, i0, cnt, n, rpt, base, first, at, ap, aa, ag);
  } else {
    if (cnt == VC) dot_rows<T, false, true, BT>(W, ldq, j, i0, cnt, n, rpt, base, first, at, ap, aa, ag);
    else dot_rows<T, false, false, BT>(W, ldq, j, i0, cnt, n, rpt, base, first, at, ap, aa, ag);
  }
  // 4 VC + 4 doubles per lane (t, p, alpha with a zero imaginary part,
  // gamma), summed over the wave by a reduce-scatter, then over the waves
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double v[kRsVals];
#pragma unroll
  for (int c = 0; c < VC; ++c) {
    v[2 * c] = at[c].x;
    v[2 * c + 1] = at[c].y;
    v[2 * (VC + c)] = ap[c].x;
    v[2 * (VC + c) + 1] = ap[c].y;
  }
  v[4 * VC] = aa.x;
  v[4 * VC + 1] = 0.0;
  v[4 * VC + 2] = ag.x;
  v[4 * VC + 3] = ag.y;
  const int d = wave_scatter_sum(v, lane);
  __shared__ double red[BW][kRsVals];
  if (d >= 0) red[wid][d] = v[0];
  __syncthreads();
  const int pr = 2 * j + 2;
  double2* dst = part + (size_t)rb * pr;
  const int t = threadIdx.x;
  if (t < kRsVals) {
    double s = red[0][t];
#pragma unroll
    for (int w = 1; w < BW; ++w) s += red[w][t];
    const int c = t >> 1;   // complex entry, t & 1 its real or imaginary part
    int o = -1;
    if (c < VC) {
      if (c < cnt) o = i0 + c;
    } else if (c < 2 * VC) {
      if (c - VC < cnt) o = j + i0 + (c - VC);
    } else if (ch == 0) {
      o = 2 * j + (c - 2 * VC);
    }
    if (o >= 0) reinterpret_cast<double*>(dst + o)[t & 1] = s;
  }
}

// Fold rows of partial sums (nrb x pr, row-major) into kGsGroups rows:
// block (cx, g) sums rows g*per .. of columns 64 cx + lane, in a fixed
// order, into out[g * pr + col].
__device__ inline void dc_reduce_body(const double2* __restrict__ part, int nrb, int pr,
                                      double2* __restrict__ out, int cx, int g) {
  __shared__ double2 scratch[NT];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int per = (nrb + kGsGroups - 1) / kGsGroups;
  const int r0 = g * per, r1 = min(nrb, r0 + per);
  const int col = cx * 64 + lane;
  double2 acc = z2();
  if (col < pr) {
    int r = r0 + wid;
    for (; r + 3 * NW < r1; r += 4 * NW) {
      double2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = part[(size_t)(r + u * NW) * pr + col];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = cadd(acc, v[u]);
    }
    for (; r < r1; r += NW) acc = cadd(acc, part[(size_t)r * pr + col]);
  }
  scratch[threadIdx.x] = acc;
  __syncthreads();
  if (wid == 0 && col < pr) {
    double2 s = scratch[lane];
#pragma unroll
    for (int w = 1; w < NW; ++w) s = cadd(s, scratch[w * 64 + lane]);
    out[(size_t)g * pr + col] = s;
  }
}

// Second pass of u_j and (unless FINAL) first pass of the next vector.
// `fresh`: first step after a thick restart of the eigensolver, where the
// columns before j already hold the restarted Rayleigh quotient (kept as is).
// The thread updates row packs r0, r0 + BT / SPLIT, ..., urt of them (the
// block's reduction of the partial dots is shared by its BT * urt / SPLIT
// packs).  SPLIT > 1: that many adjacent lanes share a row pack, each
// summing every SPLIT-th basis vector with 16 / SPLIT loads in flight, which
// shortens the chain of dependent loads per thread; they combine their sums
// by exchanges within the quad, the first lane writes v_j and the last one
// u_{j+1}.
template <typename T, bool FINAL, int BT = NT, int SPLIT = 1>
__device__ inline void dc_update_body(T* __restrict__ W, int64_t ldq, int j, int64_t n,
                                      const double2* __restrict__ part, int nrb,
                                      const ArnoldiDev& arn, const double2* __restrict__ s_prev,
                                      double2* __restrict__ s_cur, int fresh, int64_t r0,
                                      int urt, bool writer) {
  constexpr int BW = BT / 64;
  __shared__ double2 sums[2 * kMaxK + 4];
  __shared__ double2 scratch[BT];
  __shared__ double2 ct[kMaxK + 2];   // t
  __shared__ double2 ce[kMaxK + 2];   // e
  __shared__ double2 cs[kMaxK + 2];   // s_j
  __shared__ double red[BW];
  __shared__ double sc[4];            // beta, d/beta (re, im), flag
  __shared__ double2 cd;
  const int pr = 2 * j + 2;
  const int tid = threadIdx.x;
  using K = Pk<T>;
  using PT = typename K::type;
  PT* u = reinterpret_cast<PT*>(W + (int64_t)j * ldq);
  PT* zv = reinterpret_cast<PT*>(W + (int64_t)(j + 1) * ldq);
  // Operands that do not depend on the partial sums are loaded first, so
  // that their latency overlaps the reductions: this thread's entry of
  // s_{j-1}, its first four entries of H_j and its s_{j-1} entry for H_j t,
  // and (with lanes sharing a row pack) u_j, z of its first row pack.
  constexpr int G = BW;   // threads per output of H_j t
  const int lend = (fresh ? j : j - 1);
  const double2 sp_t = (!fresh && tid < j) ? s_prev[tid] : z2();
  const int ih = tid / G, gh = tid % G;
  double2 sp_h = z2();
  double2 hpre[4];
  bool hpre_ok = false;
  if (!FINAL && ih < j) {
    if (!fresh && j > 0 && gh == 0) sp_h = s_prev[ih];
    const int l = max(0, ih - 1) + gh;
    if (l + 3 * G < lend) {
#pragma unroll
      for (int q = 0; q < 4; ++q) hpre[q] = arn.H[(size_t)(l + q * G) * arn.ldh + ih];
      hpre_ok = true;
    }
  }
  PT ru0, rz0;   // (with one lane per row pack the registers are needed for the basis loads)
  if (SPLIT > 1 && r0 * K::P < n) {
    ru0 = u[r0];
    if (!FINAL) rz0 = zv[r0];
  }
  reduce_cols<BT>(part, nrb, pr, sums, scratch);
  // |t|^2 and |s_{j-1}|^2
  double tt = 0.0, ss = 0.0;
  for (int i = tid; i < j; i += BT) {
    ct[i] = sums[i];
    tt += cabs2(sums[i]);
    if (!fresh) ss += cabs2(i == tid ? sp_t : s_prev[i]);
  }
  tt = wave_sum(tt);
  ss = wave_sum(ss);
  if ((tid & 63) == 0) red[tid >> 6] = tt;
  __syncthreads();
  if (tid == 0) {
    double a = 0.0;
    for (int w = 0; w < BW; ++w) a += red[w];
    sc[1] = a;
  }
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = ss;
  __syncthreads();
  if (tid == 0) {
    double sprev = 0.0;
    for (int w = 0; w < BW; ++w) sprev += red[w];
    // ||A v_{j-1}||^2 = alpha + ||s_{j-1}||^2 sets the breakdown scale
    const double alpha = sums[2 * j].x;
    const double b2 = alpha - sc[1];
    const double ref2 = alpha + sprev;
    const bool bad = !isfinite(b2) || !isfinite(ref2);
    const bool brk = bad || !(b2 > kBreakdownTol * kBreakdownTol * ref2);
    sc[0] = brk ? 0.0 : sqrt(b2);
    sc[3] = brk ? 1.0 : 0.0;
    if (writer) {
      if (bad) arn.st->nonfinite = 1;
      if (brk) {
        arn.st->breakdown = 1;
        arn.st->kdone = j;
        if (j > 0 && !fresh) arn.H[(size_t)(j - 1) * arn.ldh + j] = z2();
      } else {
        if (j > 0 && !fresh) arn.H[(size_t)(j - 1) * arn.ldh + j] = make_double2(sc[0], 0.0);
        arn.st->kdone = FINAL ? j : j;   // steps whose columns are final
        if (j == 0) arn.st->beta = sc[0];
      }
    }
  }
  __syncthreads();
  // final column j-1 = s_{j-1} + t (also on breakdown: K_j is invariant)
  if (writer && !fresh)
    for (int i = tid; i < j; i += BT) arn.H[(size_t)(j - 1) * arn.ldh + i] = cadd(s_prev[i], ct[i]);
  if (sc[3] != 0.0) return;
  const double beta = sc[0], ib = 1.0 / beta;
  if (!FINAL) {
    // s_j from the reduced quantities; H_j t uses columns 0..j-2 of H and
    // the final column j-1 = s_{j-1} + t
    const double2 gamma = sums[2 * j + 1];
    // (H_j t)_i over columns l >= i-1 (Hessenberg); the last column is
    // s_{j-1} + t unless the columns came from a thick restart.  G = BW
    // consecutive threads share an output i (strided partial sums, then a
    // fixed-order combination over the group), so the loads of H are
    // spread over the block instead of serialised in j threads.
    for (int i0 = 0; i0 < j; i0 += BT / G) {
      const int i = i0 + tid / G, g = tid % G;
      double2 ht = z2();
      if (i < j) {
        int l = max(0, i - 1) + g;
        if (i0 == 0 && hpre_ok) {   // the first four, loaded at the start
#pragma unroll
          for (int q = 0; q < 4; ++q) ht = cadd(ht, cmul(hpre[q], ct[l + q * G]));
          l += 4 * G;
        }
        for (; l + 3 * G < lend; l += 4 * G) {
          double2 hv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) hv[u] = arn.H[(size_t)(l + u * G) * arn.ldh + i];
#pragma unroll
          for (int u = 0; u < 4; ++u) ht = cadd(ht, cmul(hv[u], ct[l + u * G]));
        }
        for (; l < lend; l += G) ht = cadd(ht, cmul(arn.H[(size_t)l * arn.ldh + i], ct[l]));
      }
#pragma unroll
      for (int off = 1; off < G; off <<= 1) {   // groups of G consecutive lanes (G divides 64)
        ht.x += __shfl_xor(ht.x, off, 64);
        ht.y += __shfl_xor(ht.y, off, 64);
      }
      if (g == 0 && i < j) {
        if (!fresh && j > 0) ht = cadd(ht, cmul(cadd(i0 == 0 ? sp_h : s_prev[i], ct[i]), ct[j - 1]));
        const double2 si = cscale(csub(sums[j + i], ht), ib);     // (p_i - (H_j t)_i) / beta
        cs[i] = si;
        ce[i] = cadd(cscale(ht, ib), si);                         // c_i = (H_j t)_i / beta + s_i
      }
    }
    double2 tp = z2();
    for (int i = tid; i < j; i += BT) tp = cadd(tp, cconjmul(ct[i], sums[j + i]));   // t^H p
    tp.x = wave_sum(tp.x);
    tp.y = wave_sum(tp.y);
    __shared__ double2 tpr[BW];
    if ((tid & 63) == 0) tpr[tid >> 6] = tp;
    __syncthreads();
    if (tid == 0) {
      double2 a = z2();
      for (int w = 0; w < BW; ++w) a = cadd(a, tpr[w]);
      // v_j^H A v_j = ((gamma - t^H p)/beta - beta t_{j-1}) / beta
      double2 vav = cscale(csub(gamma, a), ib);
      if (j > 0) vav = csub(vav, cscale(ct[j - 1], beta));
      vav = cscale(vav, ib);
      cs[j] = vav;
      const double2 d = (j > 0) ? cadd(ct[j - 1], vav) : vav;
      cd = cscale(d, ib);   // d / beta
    }
    __syncthreads();
    for (int i = tid; i < j; i += BT) ce[i] = csub(ce[i], cmul(cd, ct[i]));   // e = c - (d/beta) t
    if (writer)
      for (int i = tid; i <= j; i += BT) {
        s_cur[i] = cs[i];
        arn.H[(size_t)j * arn.ldh + i] = cs[i];   // provisional until step j+1
      }
    __syncthreads();
  }
  static_assert(SPLIT == 1 || SPLIT == 2 || SPLIT == 4, "1, 2 or 4 lanes per row pack");
  const int sub = SPLIT > 1 ? (int)(threadIdx.x & (SPLIT - 1)) : 0;
  for (int q = 0; q < urt; ++q) {
    const int64_t rp = r0 + (int64_t)q * (BT / SPLIT);
    if (rp * K::P >= n) return;   // the lanes of a row pack leave together
    double2 at[K::P], ae[K::P];
#pragma unroll
    for (int p = 0; p < K::P; ++p) at[p] = ae[p] = z2();
    constexpr int B = 16 / SPLIT;   // basis loads in flight per thread
    const PT ru = (SPLIT > 1 && q == 0) ? ru0 : u[rp];
    PT rz;
    if (!FINAL) rz = (SPLIT > 1 && q == 0) ? rz0 : zv[rp];
    int i = sub;   // vectors i, i + SPLIT, ...
    for (; i + SPLIT * (B - 1) < j; i += SPLIT * B) {
      PT raw[B];
#pragma unroll
      for (int b = 0; b < B; ++b)
        raw[b] = reinterpret_cast<const PT*>(W + (int64_t)(i + SPLIT * b) * ldq)[rp];
#pragma unroll
      for (int b = 0; b < B; ++b)
#pragma unroll
        for (int p = 0; p < K::P; ++p) {
          const double2 v = K::get(raw[b], p);
          at[p] = cadd(at[p], cmul(v, ct[i + SPLIT * b]));
          if (!FINAL) ae[p] = cadd(ae[p], cmul(v, ce[i + SPLIT * b]));
        }
    }
    if (i < j) {   // the last vectors of this lane, with clamped (valid) addresses
      PT raw[B];
#pragma unroll
      for (int b = 0; b < B; ++b)
        raw[b] = reinterpret_cast<const PT*>(W + (int64_t)min(i + SPLIT * b, j - 1) * ldq)[rp];
#pragma unroll
      for (int b = 0; b < B; ++b)
        if (i + SPLIT * b < j)
#pragma unroll
          for (int p = 0; p < K::P; ++p) {
            const double2 v = K::get(raw[b], p);
            at[p] = cadd(at[p], cmul(v, ct[i + SPLIT * b]));
            if (!FINAL) ae[p] = cadd(ae[p], cmul(v, ce[i + SPLIT * b]));
          }
    }
    // a + b on one lane, b + a on the other: every lane of the row pack
    // ends with the same sums
    if constexpr (SPLIT >= 2) {
#pragma unroll
      for (int p = 0; p < K::P; ++p) {
        at[p].x += xor_lane<1>(at[p].x);
        at[p].y += xor_lane<1>(at[p].y);
        if (!FINAL) {
          ae[p].x += xor_lane<1>(ae[p].x);
          ae[p].y += xor_lane<1>(ae[p].y);
        }
      }
    }
    if constexpr (SPLIT == 4) {
#pragma unroll
      for (int p = 0; p < K::P; ++p) {
        at[p].x += xor_lane<2>(at[p].x);
        at[p].y += xor_lane<2>(at[p].y);
        if (!FINAL) {
          ae[p].x += xor_lane<2>(ae[p].x);
          ae[p].y += xor_lane<2>(ae[p].y);
        }
      }
    }
    PT vo, uo;
#pragma unroll
    for (int p = 0; p < K::P; ++p) {
      const double2 uv = K::get(ru, p);
      K::set(vo, p, cscale(csub(uv, at[p]), ib));                                 // v_j
      if (!FINAL) K::set(uo, p, csub(csub(cscale(K::get(rz, p), ib), cmul(cd, uv)), ae[p]));   // u_{j+1}
    }
    if (sub == 0) u[rp] = vo;
    if (!FINAL && sub == SPLIT - 1) zv[rp] = uo;
  }
}

}  // namespace
}  // namespace sk
