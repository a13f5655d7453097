// The Wilson kernel H_W = gamma5 D_W(mu) on a structure-of-arrays lattice.
//
// D_W(mu) psi(x) = psi(x) - kappa sum_nu [ e^{+mu d_nu,t} (1 - gamma_nu) U_nu(x) psi(x+nu)
//                                        + e^{-mu d_nu,t} (1 + gamma_nu) U_nu(x-nu)^+ psi(x-nu) ]
// (the operator of Sect. 1; chemical potential on the time hops), chiral
// basis, antiperiodic time boundary optional.  (1 -+ gamma_nu) has rank 2,
// so each hop projects the neighbour spinor to two spin components (a
// half spinor), multiplies those by the 3x3 link, and rebuilds the other
// two spin rows from them.  e^{+-mu}, kappa and the boundary sign are folded
// into one real factor per hop.
//
// Layout: component-major fields, element (c, s) at c*V + s, so the 64
// lanes of a wave read 64 consecutive sites of one component: every load
// and store is coalesced.  Neighbour sites in x are adjacent, in y/z/t
// a fixed stride away, so the halo of one block is shared with its
// neighbours through L2.
#include "sk_internal.h"

#include <cstring>

namespace sk {
namespace {

struct StencilGeom {
  int Lx, Ly, Lz, Lt;
  int V;
  double kf[4];   // forward hop factor: -kappa * e^{+mu} on t
  double kb[4];   // backward hop factor: -kappa * e^{-mu} on t
  double tsign;   // -1 antiperiodic, +1 periodic (applied on the t wrap)
};

// multiply by one of {+1, +i, -1, -i}
template <int P> __device__ inline double2 ph(double2 z) {
  if constexpr (P == 0) return z;
  else if constexpr (P == 1) return make_double2(-z.y, z.x);
  else if constexpr (P == 2) return make_double2(-z.x, -z.y);
  else return make_double2(z.y, -z.x);
}

// Spin structure of (1 + S gamma_nu), S = -1 forward, +1 backward, in the
// chiral basis:  h0 = psi0 + P0 psi_A0,  h1 = psi1 + P1 psi_A1;
// rows 2 and 3 of the projected spinor are Q2 h_B2 and Q3 h_B3.
template <int NU, int S> struct Proj;
// forward (1 - gamma)
template <> struct Proj<0, -1> { static constexpr int A0 = 3, P0 = 1, A1 = 2, P1 = 1, B2 = 1, Q2 = 3, B3 = 0, Q3 = 3; };
template <> struct Proj<1, -1> { static constexpr int A0 = 3, P0 = 0, A1 = 2, P1 = 2, B2 = 1, Q2 = 2, B3 = 0, Q3 = 0; };
template <> struct Proj<2, -1> { static constexpr int A0 = 2, P0 = 1, A1 = 3, P1 = 3, B2 = 0, Q2 = 3, B3 = 1, Q3 = 1; };
template <> struct Proj<3, -1> { static constexpr int A0 = 2, P0 = 2, A1 = 3, P1 = 2, B2 = 0, Q2 = 2, B3 = 1, Q3 = 2; };
// backward (1 + gamma)
template <> struct Proj<0, 1> { static constexpr int A0 = 3, P0 = 3, A1 = 2, P1 = 3, B2 = 1, Q2 = 1, B3 = 0, Q3 = 1; };
template <> struct Proj<1, 1> { static constexpr int A0 = 3, P0 = 2, A1 = 2, P1 = 0, B2 = 1, Q2 = 0, B3 = 0, Q3 = 2; };
template <> struct Proj<2, 1> { static constexpr int A0 = 2, P0 = 3, A1 = 3, P1 = 1, B2 = 0, Q2 = 1, B3 = 1, Q3 = 3; };
template <> struct Proj<3, 1> { static constexpr int A0 = 2, P0 = 0, A1 = 3, P1 = 0, B2 = 0, Q2 = 0, B3 = 1, Q3 = 0; };

// One hop of one site: the projected, link-multiplied half spinor
// (u0, u1) = fac * U (h0, h1) of the neighbour in direction (NU, S).
template <int NU, int S, bool DAG, typename TI, typename TL>
__device__ inline void hop_half(double2 (&u0)[3], double2 (&u1)[3], const TI* __restrict__ in,
                                const TL* __restrict__ U, int V, int nb, int ulink, double fac) {
  using PJ = Proj<NU, S>;
  double2 h0[3], h1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double2 p0 = ld(in + (0 * 3 + c) * V + nb);
    double2 p1 = ld(in + (1 * 3 + c) * V + nb);
    double2 pa = ld(in + (PJ::A0 * 3 + c) * V + nb);
    double2 pb = ld(in + (PJ::A1 * 3 + c) * V + nb);
    h0[c] = cadd(p0, ph<PJ::P0>(pa));
    h1[c] = cadd(p1, ph<PJ::P1>(pb));
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double2 s0 = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double2 u;
      if constexpr (DAG) {
        u = ld(U + ((NU * 3 + b) * 3 + a) * (size_t)V + ulink);
        u.y = -u.y;
      } else {
        u = ld(U + ((NU * 3 + a) * 3 + b) * (size_t)V + ulink);
      }
      s0 = cadd(s0, cmul(u, h0[b]));
      s1 = cadd(s1, cmul(u, h1[b]));
    }
    u0[a] = cscale(s0, fac);
    u1[a] = cscale(s1, fac);
  }
}

// Hop h = 2 nu + d (d = 0 forward, 1 backward) of site s with coordinate
// `coord` along nu; writes its half spinor to LDS.
template <int H, typename TI, typename TL>
__device__ inline void do_hop(double2 (*hs)[64], const TI* in, const TL* U, const StencilGeom& g,
                              int s, int lane, int coord, int ext, int stride) {
  constexpr int NU = H >> 1;
  double2 u0[3], u1[3];
  if constexpr ((H & 1) == 0) {
    const bool wf = (coord == ext - 1);
    const int sf = wf ? s - (ext - 1) * stride : s + stride;
    double ff = g.kf[NU];
    if (NU == 3 && wf) ff *= g.tsign;
    hop_half<NU, -1, false>(u0, u1, in, U, g.V, sf, s, ff);
  } else {
    const bool wb = (coord == 0);
    const int sb = wb ? s + (ext - 1) * stride : s - stride;
    double fb = g.kb[NU];
    if (NU == 3 && wb) fb *= g.tsign;
    hop_half<NU, 1, true>(u0, u1, in, U, g.V, sb, sb, fb);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    hs[a][lane] = u0[a];
    hs[3 + a][lane] = u1[a];
  }
}

// add hop H's contribution to the four spin rows of colour a
template <int H>
__device__ inline void add_hop(double2 (&acc)[4], const double2 (*hs)[64], int a, int lane) {
  using PJ = Proj<(H >> 1), (H & 1) ? 1 : -1>;
  const double2 u0 = hs[a][lane], u1 = hs[3 + a][lane];
  acc[0] = cadd(acc[0], u0);
  acc[1] = cadd(acc[1], u1);
  acc[2] = cadd(acc[2], ph<PJ::Q2>(PJ::B2 == 0 ? u0 : u1));
  acc[3] = cadd(acc[3], ph<PJ::Q3>(PJ::B3 == 0 ? u0 : u1));
}

constexpr int kSitesPerBlock = 64;
constexpr int kStencilThreads = 512;   // 8 waves: one per hop

// Phase 1: wave h computes hop h of the block's 64 sites (coalesced: lanes
// are consecutive sites).  Phase 2: 3 waves (one per colour) add the eight
// half spinors, rebuild the lower spin rows, add the diagonal term and
// apply gamma5.  MODE 0: out = alpha H in;  MODE 1: out = b - (H - sigma) in.
template <int MODE, typename TI, typename TL, typename TO>
__global__ __launch_bounds__(kStencilThreads) void k_wilson(StencilGeom g, const TL* __restrict__ U,
                                                            const TI* __restrict__ in,
                                                            TO* __restrict__ out,
                                                            ScaleSrc src, const int* skip,
                                                            const double2* __restrict__ b,
                                                            double2 sigma) {
  if (skip && *skip) return;
  double sc = 1.0;
  if (MODE == 0) {
    if (src.norm_part) sc = gs_finish_norm(src.norm_part, src.nrb, src.jprev, src.arn, blockIdx.x == 0);
    else if (src.in_scale) sc = *src.in_scale;
    if (src.norm_part && sc == 0.0) return;   // lucky breakdown in the previous step
  }
  __shared__ double2 hs[8][6][64];
  const int lane = threadIdx.x & 63, h = threadIdx.x >> 6;
  const int s = blockIdx.x * kSitesPerBlock + lane;
  const bool act = s < g.V;
  if (act) {
    int r = s;
    const int x = r % g.Lx; r /= g.Lx;
    const int y = r % g.Ly; r /= g.Ly;
    const int z = r % g.Lz;
    const int t = r / g.Lz;
    const int sxy = g.Lx * g.Ly, sxyz = sxy * g.Lz;
    switch (h) {
      case 0: do_hop<0>(hs[0], in, U, g, s, lane, x, g.Lx, 1); break;
      case 1: do_hop<1>(hs[1], in, U, g, s, lane, x, g.Lx, 1); break;
      case 2: do_hop<2>(hs[2], in, U, g, s, lane, y, g.Ly, g.Lx); break;
      case 3: do_hop<3>(hs[3], in, U, g, s, lane, y, g.Ly, g.Lx); break;
      case 4: do_hop<4>(hs[4], in, U, g, s, lane, z, g.Lz, sxy); break;
      case 5: do_hop<5>(hs[5], in, U, g, s, lane, z, g.Lz, sxy); break;
      case 6: do_hop<6>(hs[6], in, U, g, s, lane, t, g.Lt, sxyz); break;
      default: do_hop<7>(hs[7], in, U, g, s, lane, t, g.Lt, sxyz); break;
    }
  }
  __syncthreads();
  if (h >= 3 || !act) return;
  const int a = h;   // colour handled by this wave
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
    const double2 xin = ld(in + c * g.V + s);
    double2 v = cadd(xin, acc[sp]);                    // D_W psi
    if (sp >= 2) v = make_double2(-v.x, -v.y);         // gamma5
    if constexpr (MODE == 0) {
      st(out + c * g.V + s, cscale(v, sc));
    } else {
      v = csub(v, cmul(sigma, xin));
      st(out + c * g.V + s, csub(b[c * g.V + s], v));
    }
  }
}

StencilGeom make_geom(const sk_operator* op, int adjoint) {
  StencilGeom g;
  g.Lx = op->dims[0];
  g.Ly = op->dims[1];
  g.Lz = op->dims[2];
  g.Lt = op->dims[3];
  g.V = (int)volume_of(op);
  const double mu = adjoint ? -op->mu : op->mu;
  for (int nu = 0; nu < 4; ++nu) {
    g.kf[nu] = -op->kappa * (nu == 3 ? std::exp(mu) : 1.0);
    g.kb[nu] = -op->kappa * (nu == 3 ? std::exp(-mu) : 1.0);
  }
  g.tsign = op->t_antiperiodic ? -1.0 : 1.0;
  return g;
}

}  // namespace

static int stencil_blocks(int V) { return (V + kSitesPerBlock - 1) / kSitesPerBlock; }

template <typename TI, typename TL, typename TO>
hipError_t launch_wilson(const sk_operator* op, const TL* links, const TI* in, TO* out, int adjoint,
                         const double* in_scale, const int* skip, hipStream_t s) {
  StencilGeom g = make_geom(op, adjoint);
  ScaleSrc src;
  std::memset(&src, 0, sizeof(src));
  src.in_scale = in_scale;
  hipLaunchKernelGGL((k_wilson<0, TI, TL, TO>), dim3(stencil_blocks(g.V)), dim3(kStencilThreads), 0, s,
                     g, links, in, out, src, skip, (const double2*)nullptr, make_double2(0.0, 0.0));
  return hipGetLastError();
}

template <typename TI, typename TL, typename TO>
hipError_t launch_wilson_arnoldi(const sk_operator* op, const TL* links, const TI* in, TO* out,
                                 int adjoint, const ScaleSrc& src, const int* skip, hipStream_t s) {
  StencilGeom g = make_geom(op, adjoint);
  hipLaunchKernelGGL((k_wilson<0, TI, TL, TO>), dim3(stencil_blocks(g.V)), dim3(kStencilThreads), 0, s,
                     g, links, in, out, src, skip, (const double2*)nullptr, make_double2(0.0, 0.0));
  return hipGetLastError();
}

template <typename TI>
hipError_t launch_wilson_residual(const sk_operator* op, const double2* links, const TI* in,
                                  const double2* b, double2 sigma, double2* out, hipStream_t s) {
  StencilGeom g = make_geom(op, 0);
  ScaleSrc src;
  std::memset(&src, 0, sizeof(src));
  hipLaunchKernelGGL((k_wilson<1, TI, double2, double2>), dim3(stencil_blocks(g.V)),
                     dim3(kStencilThreads), 0, s, g, links, in, out, src,
                     (const int*)nullptr, b, sigma);
  return hipGetLastError();
}

template hipError_t launch_wilson<double2, double2, double2>(const sk_operator*, const double2*,
                                                             const double2*, double2*, int,
                                                             const double*, const int*, hipStream_t);
template hipError_t launch_wilson<float2, float2, float2>(const sk_operator*, const float2*,
                                                          const float2*, float2*, int,
                                                          const double*, const int*, hipStream_t);
template hipError_t launch_wilson_arnoldi<double2, double2, double2>(
    const sk_operator*, const double2*, const double2*, double2*, int, const ScaleSrc&, const int*,
    hipStream_t);
template hipError_t launch_wilson_arnoldi<float2, float2, float2>(
    const sk_operator*, const float2*, const float2*, float2*, int, const ScaleSrc&, const int*,
    hipStream_t);
template hipError_t launch_wilson_residual<double2>(const sk_operator*, const double2*,
                                                    const double2*, const double2*, double2,
                                                    double2*, hipStream_t);
template hipError_t launch_wilson_residual<float2>(const sk_operator*, const double2*,
                                                   const float2*, const double2*, double2,
                                                   double2*, hipStream_t);

}  // namespace sk
