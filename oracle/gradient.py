"""Oracle: gradients of F = Re <eta, g(H_W) b> (no deflation).

TEST INFRASTRUCTURE ONLY.

g(x) = sum_j omega_j / (x - sigma_j) (eq. (g)).  Links move as
U_nu(x) -> exp(i theta^a T_a) U_nu(x), T_a = lambda_a / 2, evaluated at
theta = 0; mu is the chemical potential of the time hops.

* ``objective``: F by dense solves per pole.
* ``dense_gradient``: dF = -Re sum_j omega_j z_j^H dH x_j with x_j, z_j from
  dense solves, and dH built from the operator definition itself: H_W is
  real-linear in the link field except for the diagonal gamma5, so
  dH = hw(dU) - hw(0) with dU = i T_a U on the one link.  dH/dmu exactly:
  only the time hops carry mu, as e^{+mu} forward and e^{-mu} backward.
* ``fd_link``: central finite difference of F in one coordinate, from the
  exponentiated links (independent of the formula above).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import dirac

__all__ = ["objective", "shift_pairs", "dense_gradient", "directional_dense", "fd_link",
           "rotate_links"]


def _gell_mann():
    g = np.zeros((8, 3, 3), dtype=np.complex128)
    g[0][0, 1] = g[0][1, 0] = 1
    g[1][0, 1], g[1][1, 0] = -1j, 1j
    g[2][0, 0], g[2][1, 1] = 1, -1
    g[3][0, 2] = g[3][2, 0] = 1
    g[4][0, 2], g[4][2, 0] = -1j, 1j
    g[5][1, 2] = g[5][2, 1] = 1
    g[6][1, 2], g[6][2, 1] = -1j, 1j
    g[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return g


T = _gell_mann() / 2


def objective(U, dims, kappa, mu, b, eta, sigma, omega, anti=True):
    A = dirac.hw_dense(U, dims, kappa, mu, anti)
    n = A.shape[0]
    x = np.zeros(n, dtype=np.complex128)
    for s, o in zip(sigma, omega):
        x += o * np.linalg.solve(A - s * np.eye(n), b)
    return float(np.real(np.vdot(eta, x)))


def shift_pairs(A, b, eta, sigma):
    n = A.shape[0]
    X, Z = [], []
    for s in sigma:
        lu = sla.lu_factor(A - s * np.eye(n))
        X.append(sla.lu_solve(lu, b))
        Z.append(sla.lu_solve(lu, eta, trans=2))   # (A - s)^H z = eta
    return np.array(X), np.array(Z)


def dense_gradient(U, dims, kappa, mu, b, eta, sigma, omega, anti=True, coords=None):
    """grad[nu, site, a] (all coordinates, or only `coords` = [(nu, s, a)])
    and dF/dmu."""
    A = dirac.hw_dense(U, dims, kappa, mu, anti)
    X, Z = shift_pairs(A, b, eta, sigma)
    V = U.shape[0]
    zero = np.zeros_like(U)
    H0 = dirac.hw_csr(zero, dims, kappa, mu, anti)
    if coords is None:
        coords = [(nu, s, a) for nu in range(4) for s in range(V) for a in range(8)]
    grad = {}
    for nu, s, a in coords:
        dU = np.zeros_like(U)
        dU[s, nu] = 1j * T[a] @ U[s, nu]
        dH = dirac.hw_csr(dU, dims, kappa, mu, anti) - H0
        grad[(nu, s, a)] = -np.real(sum(o * np.vdot(Z[j], dH @ X[j]) for j, o in enumerate(omega)))
    dHmu = dirac.hw_csr(U, dims, kappa, mu, anti, d_mu=True)
    gmu = -np.real(sum(o * np.vdot(Z[j], dHmu @ X[j]) for j, o in enumerate(omega)))
    return grad, gmu


def directional_dense(U, dims, kappa, mu, b, eta, sigma, omega, theta, anti=True):
    """sum over all links and generators of theta[nu, s, a] dF/dtheta^a_{nu,s}
    (one dH along the whole direction; dH is linear in dU)."""
    A = dirac.hw_dense(U, dims, kappa, mu, anti)
    X, Z = shift_pairs(A, b, eta, sigma)
    gen = np.einsum("nsa,aij->snij", theta, T)          # per-link algebra element
    dU = 1j * np.einsum("snij,snjk->snik", gen, U)
    dH = dirac.hw_csr(dU, dims, kappa, mu, anti) - dirac.hw_csr(np.zeros_like(U), dims, kappa, mu, anti)
    return -np.real(sum(o * np.vdot(Z[j], dH @ X[j]) for j, o in enumerate(omega)))


def rotate_links(U, theta, eps):
    """U_nu(s) -> exp(i eps theta[nu, s, a] T_a) U_nu(s)."""
    gen = np.einsum("nsa,aij->snij", theta, T)
    w, v = np.linalg.eigh(gen)
    E = np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * eps * w), v.conj())
    return np.einsum("snij,snjk->snik", E, U)


def fd_link(U, dims, kappa, mu, b, eta, sigma, omega, nu, s, a, h=1e-5, anti=True):
    theta = np.zeros((4, U.shape[0], 8))
    theta[nu, s, a] = 1.0
    fp = objective(rotate_links(U, theta, h), dims, kappa, mu, b, eta, sigma, omega, anti)
    fm = objective(rotate_links(U, theta, -h), dims, kappa, mu, b, eta, sigma, omega, anti)
    return (fp - fm) / (2 * h)
