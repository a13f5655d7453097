"""Oracle: the overlap Dirac operator around the sign function (Sect. 1).

TEST INFRASTRUCTURE ONLY.

The paper's motivation is the inversion of the overlap operator, which
needs sign(H_W) applied to a vector at every step; its definition at
nonzero mu is given by reference.  Here, in the usual normalisation,

    D(m) = (1 - m/2) (1 + gamma5 S) + m,     S = sign(H_W)  (massless at m = 0),

with gamma5 = diag(1, 1, -1, -1) on the spin index.  S is either the exact
dense sign or, to compare with the library, the linear map b -> x*(b) of
Algorithm 1 (rational approximation with deflation, `xstar`).
"""
from __future__ import annotations

import numpy as np

from . import xstar

__all__ = ["gamma5_vec", "gamma5_matrix", "overlap_apply", "overlap_matrix", "sign_map_matrix"]


def gamma5_vec(v):
    """gamma5 v in the canonical layout (index 12 s + 3 spin + colour)."""
    w = np.asarray(v, dtype=np.complex128).reshape(-1, 4, 3).copy()
    w[:, 2:, :] *= -1
    return w.reshape(-1)


def gamma5_matrix(n):
    return np.diag(gamma5_vec(np.ones(n)))


def overlap_apply(sign_apply, b, mass=0.0):
    """D(m) b with sign_apply(v) = S v."""
    b = np.asarray(b, dtype=np.complex128)
    return (1 + 0.5 * mass) * b + (1 - 0.5 * mass) * gamma5_vec(sign_apply(b))


def sign_map_matrix(A, sigma, omega, R=None, L=None, F=None):
    """The matrix of the linear map b -> x*(b) of Algorithm 1:
    R F L^H + sum_j omega_j (A - sigma_j)^{-1} (I - R L^H), by dense LU per pole."""
    import scipy.linalg as sla
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    I = np.eye(n, dtype=np.complex128)
    Q = I if R is None or R.shape[1] == 0 else I - R @ L.conj().T
    G = np.zeros((n, n), dtype=np.complex128) if R is None or R.shape[1] == 0 else R @ F @ L.conj().T
    for s_, o in zip(sigma, omega):
        G += o * sla.lu_solve(sla.lu_factor(A - s_ * I), Q)
    return G


def overlap_matrix(S, mass=0.0):
    n = S.shape[0]
    G5 = gamma5_matrix(n)
    return (1 + 0.5 * mass) * np.eye(n) + (1 - 0.5 * mass) * (G5 @ S)
