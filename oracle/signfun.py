"""Oracle: the matrix sign function of a small dense matrix, three ways.

TEST INFRASTRUCTURE ONLY.

sign(A) for A with no eigenvalue on the imaginary axis (Sect. 1, footnote:
f extended to matrices by the spectral definition).

* ``sign_schur``: sorted complex Schur form A = Z T Z^H with the
  eigenvalues of negative real part first; then sign(T) = [[-I, X], [0, I]],
  where commuting with T forces  T11 X - X T22 = -2 T12  (a Sylvester
  equation).
* ``sign_newton``: Roberts' method, the Newton iteration
  X <- (X + X^{-1}) / 2 started at X = A (Sect. 6 uses it for sign(H_k)).
* ``sign_eig``: A = W diag(lam) W^{-1}, sign = W diag(sign Re lam) W^{-1}
  (brute force for diagonalisable A; only for tiny matrices).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = ["sign_schur", "sign_newton", "sign_eig", "newton_sign_small"]


def sign_schur(A: np.ndarray) -> np.ndarray:
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    T, Z, k = sla.schur(A, output="complex", sort="lhp")
    d = np.diag(T)
    if np.any(np.abs(d.real) == 0):
        raise ValueError("eigenvalue on the imaginary axis: sign undefined")
    S = np.zeros_like(T)
    S[:k, :k] = -np.eye(k)
    S[k:, k:] = np.eye(n - k)
    if 0 < k < n:
        X = sla.solve_sylvester(T[:k, :k], -T[k:, k:], -2.0 * T[:k, k:])
        S[:k, k:] = X
    return Z @ S @ Z.conj().T


def sign_newton(A: np.ndarray, tol: float = 1e-14, maxit: int = 100) -> np.ndarray:
    """Roberts' Newton iteration.  It converges quadratically; in floating
    point the relative change then levels off at about the unit roundoff
    times the conditioning of X, so the loop also ends once the change is
    below 1e-10 and no longer halves (the limit has been reached)."""
    X = np.asarray(A, dtype=np.complex128).copy()
    d_prev = np.inf
    for _ in range(maxit):
        Xn = 0.5 * (X + np.linalg.inv(X))
        d = np.linalg.norm(Xn - X, 1) / np.linalg.norm(Xn, 1)
        X = Xn
        if d < tol or (d < 1e-10 and d > 0.5 * d_prev):
            break
        d_prev = d
    else:
        raise RuntimeError("Newton sign iteration did not converge")
    return X


newton_sign_small = sign_newton


def sign_eig(A: np.ndarray) -> np.ndarray:
    lam, W = np.linalg.eig(np.asarray(A, dtype=np.complex128))
    return W @ np.diag(np.sign(lam.real)) @ np.linalg.inv(W)
