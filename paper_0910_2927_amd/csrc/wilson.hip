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
#include "stencil_dev.h"

#include <hip/hip_ext.h>

#include <cstring>

namespace sk {
namespace {

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
                                                            const double* in_scale, const int* skip,
                                                            const double2* __restrict__ b,
                                                            double2 sigma, double* __restrict__ rpart) {
  if (skip && *skip) return;
  const double sc = (MODE == 0 && in_scale) ? *in_scale : 1.0;
  __shared__ double2 hs[8][6][64];
  const int lane = threadIdx.x & 63, h = threadIdx.x >> 6;
  const int s = xcd_runs(blockIdx.x, gridDim.x) * kSitesPerBlock + lane;
  const bool act = s < g.V;
  // the combining waves load their diagonal terms before the hop phase,
  // so that they are in registers after the barrier
  TI xd[4];
  if (h < 3 && act)
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) xd[sp] = in[(sp * 3 + h) * g.V + s];
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
  if (h >= 3) return;
  const int a = h;   // colour handled by this wave
  double r2 = 0.0;   // MODE 1: this lane's share of ||out||^2
  if (act) {
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
      const double2 xin = cvt(xd[sp]);
      double2 v = cadd(xin, acc[sp]);                    // D_W psi
      if (sp >= 2) v = make_double2(-v.x, -v.y);         // gamma5
      if constexpr (MODE == 0) {
        st(out + c * g.V + s, cscale(v, sc));
      } else {
        v = csub(v, cmul(sigma, xin));
        const double2 r = csub(b[c * g.V + s], v);
        st(out + c * g.V + s, r);
        r2 += cabs2(r);
      }
    }
  }
  // MODE 1: each of a block's three colour waves writes one partial sum
  // (all 64 lanes take part; lanes past the lattice add 0), folded later
  // in a fixed order
  if (MODE == 1 && rpart) {
    const double w = wave_sum(r2);
    if (lane == 0) rpart[(size_t)blockIdx.x * 3 + a] = w;
  }
}

StencilGeom make_geom(const sk_operator* op, int adjoint) { return make_stencil_geom(op, adjoint); }

}  // namespace

static int stencil_blocks(int V) { return (V + kSitesPerBlock - 1) / kSitesPerBlock; }

template <typename TI, typename TL, typename TO>
hipError_t launch_wilson(const sk_operator* op, const TL* links, const TI* in, TO* out, int adjoint,
                         const double* in_scale, const int* skip, hipStream_t s, hipEvent_t t0,
                         hipEvent_t t1) {
  StencilGeom g = make_geom(op, adjoint);
  if (t0 || t1)
    hipExtLaunchKernelGGL((k_wilson<0, TI, TL, TO>), dim3(stencil_blocks(g.V)), dim3(kStencilThreads), 0,
                          s, t0, t1, 0, g, links, in, out, in_scale, skip, (const double2*)nullptr,
                          make_double2(0.0, 0.0), (double*)nullptr);
  else
    hipLaunchKernelGGL((k_wilson<0, TI, TL, TO>), dim3(stencil_blocks(g.V)), dim3(kStencilThreads), 0, s,
                       g, links, in, out, in_scale, skip, (const double2*)nullptr, make_double2(0.0, 0.0),
                       (double*)nullptr);
  return hipGetLastError();
}

template <typename TI>
hipError_t launch_wilson_residual(const sk_operator* op, const double2* links, const TI* in,
                                  const double2* b, double2 sigma, double2* out, double* rpart,
                                  hipStream_t s) {
  StencilGeom g = make_geom(op, 0);
  hipLaunchKernelGGL((k_wilson<1, TI, double2, double2>), dim3(stencil_blocks(g.V)),
                     dim3(kStencilThreads), 0, s, g, links, in, out, (const double*)nullptr,
                     (const int*)nullptr, b, sigma, rpart);
  return hipGetLastError();
}

int wilson_residual_partials(int64_t V) { return 3 * stencil_blocks((int)V); }

template hipError_t launch_wilson<double2, double2, double2>(const sk_operator*, const double2*,
                                                             const double2*, double2*, int,
                                                             const double*, const int*, hipStream_t,
                                                             hipEvent_t, hipEvent_t);
template hipError_t launch_wilson<float2, float2, float2>(const sk_operator*, const float2*,
                                                          const float2*, float2*, int,
                                                          const double*, const int*, hipStream_t,
                                                          hipEvent_t, hipEvent_t);
template hipError_t launch_wilson_residual<double2>(const sk_operator*, const double2*,
                                                    const double2*, const double2*, double2,
                                                    double2*, double*, hipStream_t);
template hipError_t launch_wilson_residual<float2>(const sk_operator*, const double2*,
                                                   const float2*, const double2*, double2,
                                                   double2*, double*, hipStream_t);

}  // namespace sk
