"""Oracle: the exact result that restarted FOM-LR converges to.

TEST INFRASTRUCTURE ONLY.

With deflation data (R, L, F) -- R = R_m right eigenvectors, L = L_m left
eigenvectors with L^H R = I_m, F = f(Lambda_m) expressed in the basis R --
and poles/weights (sigma_j, omega_j) of eq. (g), Algorithm 1 computes

    x* = R F L^H b  +  sum_j omega_j (A - sigma_j I)^{-1} (I - R L^H) b .

The first term is x_P of Sect. 4 (computed exactly, with f itself, not g);
the second is the rational approximation applied to the deflated source
(Sect. 4: deflation only replaces b by (I - P) b), which each restarted
shifted FOM converges to (Sect. 3).  With m = 0 it is simply g(A) b.

Two routes to the same definition: dense LU per pole (small n), sparse LU
per pole (moderate n).  Both are plain library solves.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = ["deflated_source", "x_p", "xstar_dense", "xstar_sparse",
           "shift_solutions_dense"]


def deflated_source(b, R=None, L=None):
    """(I - R L^H) b (the r = (I - P) b step of Algorithm 1)."""
    b = np.asarray(b, dtype=np.complex128)
    if R is None or R.shape[1] == 0:
        return b.copy()
    return b - R @ (L.conj().T @ b)


def x_p(b, R=None, L=None, F=None):
    """x_P = R f(Lambda) (L^H b)  (Sect. 4)."""
    b = np.asarray(b, dtype=np.complex128)
    if R is None or R.shape[1] == 0:
        return np.zeros_like(b)
    return R @ (F @ (L.conj().T @ b))


def shift_solutions_dense(A, rhs, sigma):
    """Columns x_j = (A - sigma_j I)^{-1} rhs, by dense LU."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    out = np.empty((len(sigma), n), dtype=np.complex128)
    I = np.eye(n)
    for j, s in enumerate(sigma):
        out[j] = sla.lu_solve(sla.lu_factor(A - s * I), rhs)
    return out


def xstar_dense(A, b, sigma, omega, R=None, L=None, F=None, return_shifts=False):
    rhs = deflated_source(b, R, L)
    X = shift_solutions_dense(A, rhs, sigma)
    x = x_p(b, R, L, F) + np.tensordot(np.asarray(omega), X, axes=(0, 0))
    return (x, X) if return_shifts else x


def xstar_sparse(A, b, sigma, omega, R=None, L=None, F=None, return_shifts=False):
    A = sp.csc_matrix(A)
    n = A.shape[0]
    rhs = deflated_source(b, R, L)
    I = sp.identity(n, dtype=np.complex128, format="csc")
    X = np.empty((len(sigma), n), dtype=np.complex128)
    for j, s in enumerate(sigma):
        X[j] = spla.splu((A - s * I).tocsc()).solve(rhs)
    x = x_p(b, R, L, F) + np.tensordot(np.asarray(omega), X, axes=(0, 0))
    return (x, X) if return_shifts else x
