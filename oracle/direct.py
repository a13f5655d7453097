"""Oracle: the direct projection methods that Sect. 6 compares FOM-LR with.

TEST INFRASTRUCTURE ONLY.

With P = R L^H the LR projector of Sect. 4, x_P = R f(Lambda) L^H b, and
beta = ||(I - P) b||, the k-th direct approximation of sign(A) b is

    x_k = x_P + beta * V_k sign(H_k) e_1                         (eq. (direct))

with V_k, H_k from k Arnoldi steps on A started at (I - P) b / beta, and
sign(H_k) by Roberts' method, the Newton iteration X <- (X + X^{-1}) / 2
(Sect. 6).  No rational approximation and no restarts are involved: the
error comes only from the Krylov space being too small.

The two-sided Lanczos variant ("2sL" of Fig. 1; the recurrences are the
textbook non-Hermitian Lanczos process, which the paper refers to its
own earlier work for): right and left Krylov spaces of A and A^H from v_1
and w_1 with W_k^H V_k = I, short recurrences, and T_k = W_k^H A V_k
tridiagonal; x_k = x_P + beta V_k sign(T_k) e_1.  The left start is
w_1 = (I - P)^H v_1 = (I - L R^H) v_1, so that the left space avoids the
deflated left subspace just as the right one avoids the right one, and
w_1^H v_1 = 1.
"""
from __future__ import annotations

import numpy as np

from . import krylov, signfun, xstar

__all__ = ["arnoldi_direct", "two_sided_lanczos", "lanczos_direct"]


def arnoldi_direct(matvec, b, k, R=None, L=None, F=None):
    """x_k of eq. (direct).  Returns (x_k, info) with info['k'] (steps done,
    fewer on breakdown), 'H' ((kk+1) x kk) and 'S' = sign(H_kk)."""
    rhs = xstar.deflated_source(b, R, L)
    xp = xstar.x_p(b, R, L, F)
    beta = np.linalg.norm(rhs)
    if beta == 0.0:
        return xp, {"k": 0, "H": np.zeros((1, 0)), "S": np.zeros((0, 0))}
    V, H, kk = krylov.arnoldi(matvec, rhs / beta, k)
    S = signfun.sign_newton(H[:kk, :kk])
    return xp + beta * (V[:, :kk] @ S[:, 0]), {"k": kk, "H": H, "S": S}


def two_sided_lanczos(matvec, rmatvec, v1, w1, k, tol=1e-12):
    """Non-Hermitian Lanczos: V (n x (kk+1)), W, T ((kk+1) x kk) with
    W^H V = I and A V_kk = V_{kk+1} T, A^H W_kk = W_{kk+1} T^H-pattern.

    Normalisation: delta_j = sqrt|w^H v| on the subdiagonal, beta_j =
    (w^H v) / delta_j on the superdiagonal.  Stops early (kk < k) when the
    new right vector vanishes (invariant subspace: exact) and raises on a
    serious breakdown (w^H v = 0 with both nonzero)."""
    n = v1.shape[0]
    V = np.zeros((n, k + 1), dtype=np.complex128)
    W = np.zeros((n, k + 1), dtype=np.complex128)
    T = np.zeros((k + 1, k), dtype=np.complex128)
    s0 = np.vdot(w1, v1)
    V[:, 0] = v1
    W[:, 0] = w1 / np.conj(s0)            # w_1^H v_1 = 1
    beta_prev = delta_prev = 0.0
    for j in range(k):
        z = matvec(V[:, j])
        y = rmatvec(W[:, j])
        alpha = np.vdot(W[:, j], z)
        T[j, j] = alpha
        z = z - alpha * V[:, j]
        y = y - np.conj(alpha) * W[:, j]
        if j > 0:
            z = z - beta_prev * V[:, j - 1]
            y = y - np.conj(delta_prev) * W[:, j - 1]
        zn, yn = np.linalg.norm(z), np.linalg.norm(y)
        if zn <= tol * np.linalg.norm(matvec(V[:, j])):
            return V[:, : j + 1], W[:, : j + 1], T[: j + 1, : j + 1], j + 1
        s = np.vdot(y, z)
        if abs(s) <= tol * zn * yn:
            raise RuntimeError(f"serious breakdown of two-sided Lanczos at step {j + 1}")
        delta = np.sqrt(abs(s))
        beta = s / delta
        V[:, j + 1] = z / delta
        W[:, j + 1] = y / np.conj(beta)
        T[j + 1, j] = delta
        if j + 1 < k:
            T[j, j + 1] = beta
        beta_prev, delta_prev = beta, delta
    return V, W, T, k


def lanczos_direct(matvec, rmatvec, b, k, R=None, L=None, F=None):
    """x_k = x_P + beta V_k sign(T_k) e_1 from two-sided Lanczos."""
    rhs = xstar.deflated_source(b, R, L)
    xp = xstar.x_p(b, R, L, F)
    beta = np.linalg.norm(rhs)
    if beta == 0.0:
        return xp, {"k": 0}
    v1 = rhs / beta
    w1 = v1 if R is None or R.shape[1] == 0 else v1 - L @ (R.conj().T @ v1)
    V, W, T, kk = two_sided_lanczos(matvec, rmatvec, v1, w1, k)
    S = signfun.sign_newton(T[:kk, :kk])
    return xp + beta * (V[:, :kk] @ S[:, 0]), {"k": kk, "T": T, "S": S, "V": V, "W": W}
