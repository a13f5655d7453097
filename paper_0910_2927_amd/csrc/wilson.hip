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

template <int NU, int S, bool DAG, typename TI, typename TL>
__device__ inline void hop(double2 (&acc)[12], const TI* __restrict__ in, const TL* __restrict__ U,
                           int V, int nb, int ulink, double fac) {
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
  // colour multiply: u0 = U h0, u1 = U h1  (or U^+ for the backward hop)
  double2 u0[3], u1[3];
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
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc[0 * 3 + a] = cadd(acc[0 * 3 + a], u0[a]);
    acc[1 * 3 + a] = cadd(acc[1 * 3 + a], u1[a]);
    const double2 r2 = PJ::B2 == 0 ? u0[a] : u1[a];
    const double2 r3 = PJ::B3 == 0 ? u0[a] : u1[a];
    acc[2 * 3 + a] = cadd(acc[2 * 3 + a], ph<PJ::Q2>(r2));
    acc[3 * 3 + a] = cadd(acc[3 * 3 + a], ph<PJ::Q3>(r3));
  }
}

template <int NU, typename TI, typename TL>
__device__ inline void both_hops(double2 (&acc)[12], const TI* in, const TL* U, const StencilGeom& g,
                                 int s, int coord, int ext, int stride) {
  // forward neighbour x + nu
  const bool wf = (coord == ext - 1);
  const int sf = wf ? s - (ext - 1) * stride : s + stride;
  double ff = g.kf[NU];
  if (NU == 3 && wf) ff *= g.tsign;
  hop<NU, -1, false>(acc, in, U, g.V, sf, s, ff);
  // backward neighbour x - nu, link U_nu(x - nu)^+
  const bool wb = (coord == 0);
  const int sb = wb ? s + (ext - 1) * stride : s - stride;
  double fb = g.kb[NU];
  if (NU == 3 && wb) fb *= g.tsign;
  hop<NU, 1, true>(acc, in, U, g.V, sb, sb, fb);
}

template <typename TI, typename TL, typename TO>
__global__ __launch_bounds__(256) void k_wilson(StencilGeom g, const TL* __restrict__ U,
                                                const TI* __restrict__ in, TO* __restrict__ out,
                                                const double* in_scale, const int* skip) {
  if (skip && *skip) return;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  int r = s;
  const int x = r % g.Lx; r /= g.Lx;
  const int y = r % g.Ly; r /= g.Ly;
  const int z = r % g.Lz;
  const int t = r / g.Lz;
  double2 acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = make_double2(0.0, 0.0);
  both_hops<0>(acc, in, U, g, s, x, g.Lx, 1);
  both_hops<1>(acc, in, U, g, s, y, g.Ly, g.Lx);
  both_hops<2>(acc, in, U, g, s, z, g.Lz, g.Lx * g.Ly);
  both_hops<3>(acc, in, U, g, s, t, g.Lt, g.Lx * g.Ly * g.Lz);
  const double sc = in_scale ? *in_scale : 1.0;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    double2 v = cadd(ld(in + c * g.V + s), acc[c]);   // D_W psi
    if (c >= 6) v = make_double2(-v.x, -v.y);         // gamma5
    st(out + c * g.V + s, cscale(v, sc));
  }
}

// out = b - (H_W - sigma) in, all in double (in may be float: exact upcast)
template <typename TI>
__global__ __launch_bounds__(256) void k_wilson_residual(StencilGeom g, const double2* __restrict__ U,
                                                         const TI* __restrict__ in,
                                                         const double2* __restrict__ b,
                                                         double2 sigma, double2* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  int r = s;
  const int x = r % g.Lx; r /= g.Lx;
  const int y = r % g.Ly; r /= g.Ly;
  const int z = r % g.Lz;
  const int t = r / g.Lz;
  double2 acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = make_double2(0.0, 0.0);
  both_hops<0>(acc, in, U, g, s, x, g.Lx, 1);
  both_hops<1>(acc, in, U, g, s, y, g.Ly, g.Lx);
  both_hops<2>(acc, in, U, g, s, z, g.Lz, g.Lx * g.Ly);
  both_hops<3>(acc, in, U, g, s, t, g.Lt, g.Lx * g.Ly * g.Lz);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double2 xin = ld(in + c * g.V + s);
    double2 v = cadd(xin, acc[c]);
    if (c >= 6) v = make_double2(-v.x, -v.y);
    v = csub(v, cmul(sigma, xin));
    out[c * g.V + s] = csub(b[c * g.V + s], v);
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

template <typename TI, typename TL, typename TO>
hipError_t launch_wilson(const sk_operator* op, const TL* links, const TI* in, TO* out, int adjoint,
                         const double* in_scale, const int* skip, hipStream_t s) {
  StencilGeom g = make_geom(op, adjoint);
  hipLaunchKernelGGL((k_wilson<TI, TL, TO>), dim3((g.V + 255) / 256), dim3(256), 0, s, g, links,
                     in, out, in_scale, skip);
  return hipGetLastError();
}

template <typename TI>
hipError_t launch_wilson_residual(const sk_operator* op, const double2* links, const TI* in,
                                  const double2* b, double2 sigma, double2* out, hipStream_t s) {
  StencilGeom g = make_geom(op, 0);
  hipLaunchKernelGGL((k_wilson_residual<TI>), dim3((g.V + 255) / 256), dim3(256), 0, s, g, links,
                     in, b, sigma, out);
  return hipGetLastError();
}

template hipError_t launch_wilson<double2, double2, double2>(const sk_operator*, const double2*,
                                                             const double2*, double2*, int,
                                                             const double*, const int*, hipStream_t);
template hipError_t launch_wilson<float2, float2, float2>(const sk_operator*, const float2*,
                                                          const float2*, float2*, int,
                                                          const double*, const int*, hipStream_t);
template hipError_t launch_wilson_residual<double2>(const sk_operator*, const double2*,
                                                    const double2*, const double2*, double2,
                                                    double2*, hipStream_t);
template hipError_t launch_wilson_residual<float2>(const sk_operator*, const double2*,
                                                   const float2*, const double2*, double2,
                                                   double2*, hipStream_t);

}  // namespace sk
