// Device pieces of the Wilson stencil shared by the single-field and the
// batched kernels (internal to libsignkrylov).
//
// D_W(mu) psi(x) = psi(x) - kappa sum_nu [ e^{+mu d_nu,t} (1 - gamma_nu) U_nu(x) psi(x+nu)
//                                        + e^{-mu d_nu,t} (1 + gamma_nu) U_nu(x-nu)^+ psi(x-nu) ]
// in the chiral basis; (1 -+ gamma_nu) has rank 2, so a hop projects the
// neighbour spinor to a half spinor, multiplies it by the link and rebuilds
// the other two spin rows.
#pragma once

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

// The hardware deals workgroups to the 8 XCDs in turn (workgroup b to XCD
// b mod 8), and each XCD has its own L2.  Renumbered, XCD x takes runs of
// kRun consecutive site blocks (2048 sites) instead of every 8th block, so
// the neighbours a block reads in y, and mostly in z, are sites its own
// XCD fetched just before.  The 8 runs in flight together stay adjacent in
// memory (whole-range slices per XCD alias at power-of-two volumes and
// were slower at 32^4).  Blocks past the last full set of 8 runs keep their
// number; a bijection of [0, nb).
__device__ inline int xcd_runs(int b, int nb) {
  constexpr int kXcds = 8, kRun = 32;
  if (b >= nb / (kXcds * kRun) * (kXcds * kRun)) return b;
  const int x = b % kXcds, i = b / kXcds;
  return (i / kRun) * (kXcds * kRun) + x * kRun + i % kRun;
}

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

// The link of hop (NU, backward = DAG) into registers: u[a][b] of U or U^+.
template <int NU, bool DAG, typename TL>
__device__ inline void load_link(double2 (&u)[3][3], const TL* __restrict__ U, int V, int ulink) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if constexpr (DAG) {
        double2 x = ld(U + ((NU * 3 + b) * 3 + a) * (size_t)V + ulink);
        u[a][b] = make_double2(x.x, -x.y);
      } else {
        u[a][b] = ld(U + ((NU * 3 + a) * 3 + b) * (size_t)V + ulink);
      }
    }
}

// fac * u (h0, h1) for the neighbour spinor at `nb` with a link in registers.
template <int NU, int S, typename TI>
__device__ inline void half_with_link(double2 (&u0)[3], double2 (&u1)[3], const TI* __restrict__ in,
                                      int V, int nb, const double2 (&u)[3][3], double fac) {
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
      s0 = cadd(s0, cmul(u[a][b], h0[b]));
      s1 = cadd(s1, cmul(u[a][b], h1[b]));
    }
    u0[a] = cscale(s0, fac);
    u1[a] = cscale(s1, fac);
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

// Neighbour of site s (coordinate `coord` along the direction of extent
// `ext`, index stride `stride`) and the hop factor including the t-boundary sign.
__device__ inline void neighbour(int H, const StencilGeom& g, int s, int coord, int ext, int stride,
                                 int& nb, int& ulink, double& fac) {
  const int nu = H >> 1;
  if ((H & 1) == 0) {
    const bool wf = (coord == ext - 1);
    nb = wf ? s - (ext - 1) * stride : s + stride;
    ulink = s;
    fac = g.kf[nu];
    if (nu == 3 && wf) fac *= g.tsign;
  } else {
    const bool wb = (coord == 0);
    nb = wb ? s + (ext - 1) * stride : s - stride;
    ulink = nb;
    fac = g.kb[nu];
    if (nu == 3 && wb) fac *= g.tsign;
  }
}

inline StencilGeom make_stencil_geom(const sk_operator* op, int adjoint) {
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
}  // namespace sk
