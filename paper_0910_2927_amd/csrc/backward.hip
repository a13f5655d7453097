// Gradient of F = Re <eta, g(H_W) b>, g(x) = sum_j omega_j / (x - sigma_j)
// (eq. (g), no deflation), with respect to the gauge links and mu.
//
// With x_j = (H - sigma_j)^{-1} b and z_j = (H^H - conj(sigma_j))^{-1} eta
// (H^H = H_W(-mu), so the adjoint solves are the same multishift method on
// H_W(-mu) with conjugated poles):
//     dF = -Re sum_j omega_j z_j^H (dH) x_j .
// Links move as U_nu(x) -> exp(i theta^a T_a) U_nu(x), T_a = lambda_a / 2, so
// dU = i T_a U in the forward hop of site x and dU^+ = -i U^+ T_a in the
// backward hop of site x+nu.  Per link the kernel builds two 3x3 colour
// matrices, summed over the shifts,
//   B1[c][d] = sum_s conj(z(x)_{s,c})    [gamma5 (1 - gamma_nu) U x(x+nu)]_{s,d}
//   B2[e][d] = sum_s conj((U z(x+nu))_{s,e}) [gamma5 (1 + gamma_nu) x(x)]_{s,d}
// and   dF/dtheta^a = -Re tr(T_a G^T),  G = -kappa (f_+ i B1 - f_- i B2),
// f_+- = e^{+-mu} on time links times the boundary sign.  The mu derivative
// is the sum over time links of -Re(-kappa f_+ tr B1 + kappa f_- tr B2).
#include "sk_internal.h"

namespace sk {
namespace {

template <int P> __device__ inline double2 phz(double2 z) {
  if constexpr (P == 0) return z;
  else if constexpr (P == 1) return make_double2(-z.y, z.x);
  else if constexpr (P == 2) return make_double2(-z.x, -z.y);
  else return make_double2(z.y, -z.x);
}

// spin structure of (1 - gamma_nu) [S = -1] and (1 + gamma_nu) [S = +1]:
// rows 0,1: psi_r + P_r psi_{A_r}; rows 2,3: Q_r * (row B_r)
template <int NU, int S> struct PJ;
template <> struct PJ<0, -1> { static constexpr int A0 = 3, P0 = 1, A1 = 2, P1 = 1, B2 = 1, Q2 = 3, B3 = 0, Q3 = 3; };
template <> struct PJ<1, -1> { static constexpr int A0 = 3, P0 = 0, A1 = 2, P1 = 2, B2 = 1, Q2 = 2, B3 = 0, Q3 = 0; };
template <> struct PJ<2, -1> { static constexpr int A0 = 2, P0 = 1, A1 = 3, P1 = 3, B2 = 0, Q2 = 3, B3 = 1, Q3 = 1; };
template <> struct PJ<3, -1> { static constexpr int A0 = 2, P0 = 2, A1 = 3, P1 = 2, B2 = 0, Q2 = 2, B3 = 1, Q3 = 2; };
template <> struct PJ<0, 1> { static constexpr int A0 = 3, P0 = 3, A1 = 2, P1 = 3, B2 = 1, Q2 = 1, B3 = 0, Q3 = 1; };
template <> struct PJ<1, 1> { static constexpr int A0 = 3, P0 = 2, A1 = 2, P1 = 0, B2 = 1, Q2 = 0, B3 = 0, Q3 = 2; };
template <> struct PJ<2, 1> { static constexpr int A0 = 2, P0 = 3, A1 = 3, P1 = 1, B2 = 0, Q2 = 1, B3 = 1, Q3 = 3; };
template <> struct PJ<3, 1> { static constexpr int A0 = 2, P0 = 0, A1 = 3, P1 = 0, B2 = 0, Q2 = 0, B3 = 1, Q3 = 0; };

// y = gamma5 (1 + S gamma_nu) (M psi): M = U (colour), psi at site `site`.
// Returns the 4 x 3 spinor y[s][c].
template <int NU, int S, bool MUL_U>
__device__ inline void proj_g5(double2 (&y)[4][3], const double2* __restrict__ v, int V, int site,
                               const double2* __restrict__ U, int link) {
  using P = PJ<NU, S>;
  double2 h0[3], h1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h0[c] = cadd(v[(0 * 3 + c) * V + site], phz<P::P0>(v[(P::A0 * 3 + c) * V + site]));
    h1[c] = cadd(v[(1 * 3 + c) * V + site], phz<P::P1>(v[(P::A1 * 3 + c) * V + site]));
  }
  double2 u0[3], u1[3];
  if constexpr (MUL_U) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double2 s0 = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double2 u = U[((NU * 3 + a) * 3 + b) * (size_t)V + link];
        s0 = cadd(s0, cmul(u, h0[b]));
        s1 = cadd(s1, cmul(u, h1[b]));
      }
      u0[a] = s0;
      u1[a] = s1;
    }
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      u0[a] = h0[a];
      u1[a] = h1[a];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    y[0][a] = u0[a];
    y[1][a] = u1[a];
    const double2 r2 = phz<P::Q2>(P::B2 == 0 ? u0[a] : u1[a]);
    const double2 r3 = phz<P::Q3>(P::B3 == 0 ? u0[a] : u1[a]);
    y[2][a] = make_double2(-r2.x, -r2.y);   // gamma5
    y[3][a] = make_double2(-r3.x, -r3.y);
  }
}

struct GradGeom {
  int Lx, Ly, Lz, Lt, V;
  double kappa, emu, emu_inv, tsign;
  int npoles;
  double2 omega[kMaxPoles];
};

template <int NU>
__device__ inline void link_grad(const GradGeom& g, const double2* __restrict__ U, const double2* X,
                                 const double2* Z, int64_t n, int s, int coord, int ext, int stride,
                                 double* __restrict__ grad, double& dmu) {
  const bool wf = (coord == ext - 1);
  const int sf = wf ? s - (ext - 1) * stride : s + stride;
  double fp = -g.kappa, fm = -g.kappa;
  if (NU == 3) {
    fp *= g.emu;
    fm *= g.emu_inv;
    if (wf) {
      fp *= g.tsign;
      fm *= g.tsign;
    }
  }
  double2 B1[3][3], B2[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) B1[c][d] = B2[c][d] = make_double2(0.0, 0.0);
  for (int j = 0; j < g.npoles; ++j) {
    const double2* xj = X + (int64_t)j * n;
    const double2* zj = Z + (int64_t)j * n;
    const double2 om = g.omega[j];
    // B1: conj(z(x)) . gamma5 (1 - gamma) U x(x+nu)
    {
      double2 y[4][3];
      proj_g5<NU, -1, true>(y, xj, g.V, sf, U, s);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        double2 zc[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) zc[c] = cmul(om, make_double2(zj[(sp * 3 + c) * g.V + s].x,
                                                               -zj[(sp * 3 + c) * g.V + s].y));
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int d = 0; d < 3; ++d) B1[c][d] = cadd(B1[c][d], cmul(zc[c], y[sp][d]));
      }
    }
    // B2: conj(U z(x+nu)) . gamma5 (1 + gamma) x(x)
    {
      double2 y[4][3];
      proj_g5<NU, 1, false>(y, xj, g.V, s, U, s);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        double2 w[3];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          double2 acc = make_double2(0.0, 0.0);
#pragma unroll
          for (int c = 0; c < 3; ++c)
            acc = cadd(acc, cmul(U[((NU * 3 + e) * 3 + c) * (size_t)g.V + s], zj[(sp * 3 + c) * g.V + sf]));
          w[e] = cmul(om, make_double2(acc.x, -acc.y));   // omega * conj(U z)
        }
#pragma unroll
        for (int e = 0; e < 3; ++e)
#pragma unroll
          for (int d = 0; d < 3; ++d) B2[e][d] = cadd(B2[e][d], cmul(w[e], y[sp][d]));
      }
    }
  }
  // G = fp * i B1 - fm * i B2 ;  dF/dtheta^a = -Re sum_cd T_a[c][d] G[c][d]
  double2 G[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double2 t = csub(cscale(B1[c][d], fp), cscale(B2[c][d], fm));
      G[c][d] = make_double2(-t.y, t.x);   // i * t
    }
  // Gell-Mann / 2 contracted with G (T_a[c][d] G[c][d])
  const double is3 = 0.57735026918962576451;   // 1/sqrt(3)
  double2 tr[8];
  tr[0] = cadd(G[0][1], G[1][0]);
  tr[1] = cadd(make_double2(G[0][1].y, -G[0][1].x), make_double2(-G[1][0].y, G[1][0].x));  // -i G01 + i G10
  tr[2] = csub(G[0][0], G[1][1]);
  tr[3] = cadd(G[0][2], G[2][0]);
  tr[4] = cadd(make_double2(G[0][2].y, -G[0][2].x), make_double2(-G[2][0].y, G[2][0].x));
  tr[5] = cadd(G[1][2], G[2][1]);
  tr[6] = cadd(make_double2(G[1][2].y, -G[1][2].x), make_double2(-G[2][1].y, G[2][1].x));
  tr[7] = cscale(csub(cadd(G[0][0], G[1][1]), cscale(G[2][2], 2.0)), is3);
#pragma unroll
  for (int a = 0; a < 8; ++a) grad[((size_t)NU * g.V + s) * 8 + a] = -0.5 * tr[a].x;
  if (NU == 3) {
    // dH/dmu: +e^{mu} on the forward time hop, -e^{-mu} on the backward one
    const double2 t1 = cadd(cadd(B1[0][0], B1[1][1]), B1[2][2]);
    const double2 t2 = cadd(cadd(B2[0][0], B2[1][1]), B2[2][2]);
    dmu += -(fp * t1.x - fm * t2.x);
  }
}

__global__ __launch_bounds__(128) void k_grad(GradGeom g, const double2* __restrict__ U,
                                              const double2* __restrict__ X,
                                              const double2* __restrict__ Z, double* __restrict__ grad,
                                              double* __restrict__ mu_part) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double dmu = 0.0;
  if (s < g.V) {
    const int64_t n = 12 * (int64_t)g.V;
    int r = s;
    const int x = r % g.Lx; r /= g.Lx;
    const int y = r % g.Ly; r /= g.Ly;
    const int z = r % g.Lz;
    const int t = r / g.Lz;
    link_grad<0>(g, U, X, Z, n, s, x, g.Lx, 1, grad, dmu);
    link_grad<1>(g, U, X, Z, n, s, y, g.Ly, g.Lx, grad, dmu);
    link_grad<2>(g, U, X, Z, n, s, z, g.Lz, g.Lx * g.Ly, grad, dmu);
    link_grad<3>(g, U, X, Z, n, s, t, g.Lt, g.Lx * g.Ly * g.Lz, grad, dmu);
  }
  dmu = wave_sum(dmu);
  __shared__ double red[2];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dmu;
  __syncthreads();
  if (threadIdx.x == 0) mu_part[blockIdx.x] = red[0] + red[1];
}

}  // namespace

int grad_blocks(int64_t V) { return (int)((V + 127) / 128); }

hipError_t launch_grad(const sk_operator* op, const PoleSet& ps, const double2* X, const double2* Z,
                       double* grad, double* mu_part, hipStream_t s) {
  GradGeom g;
  g.Lx = op->dims[0];
  g.Ly = op->dims[1];
  g.Lz = op->dims[2];
  g.Lt = op->dims[3];
  g.V = (int)volume_of(op);
  g.kappa = op->kappa;
  g.emu = std::exp(op->mu);
  g.emu_inv = std::exp(-op->mu);
  g.tsign = op->t_antiperiodic ? -1.0 : 1.0;
  g.npoles = ps.n;
  for (int i = 0; i < ps.n; ++i) g.omega[i] = ps.omega[i];
  hipLaunchKernelGGL(k_grad, dim3(grad_blocks(g.V)), dim3(128), 0, s, g, (const double2*)op->links,
                     X, Z, grad, mu_part);
  return hipGetLastError();
}

}  // namespace sk
