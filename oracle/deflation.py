"""Oracle: LR deflation data (Sect. 4).

TEST INFRASTRUCTURE ONLY.

Sect. 4 deflates m "critical" eigenvalues: R_m holds right eigenvectors,
L_m left ones (L^H A = Lambda L^H), scaled so that L^H R = I_m; then
P = R L^H is the oblique projector onto span(R) and
x_P = R f(Lambda) L^H b.  For f = sign, f(Lambda) = diag(sign Re lambda_i).

Selection: the m eigenvalues of smallest |lambda| ("nearest zero"), or of
smallest |Re lambda| ("nearest the imaginary axis", the paper's wording for
sign); ties broken by arg(lambda), then index.  The paper does not say how
the eigenpairs are obtained (they are inputs of Algorithm 1); here:

* ``lr_dense``: dense eig of A; L^H = the matching rows of W^{-1}, so
  L^H R = I holds by construction.
* ``lr_arpack``: implicitly restarted Arnoldi (scipy/ARPACK) on A^2 for
  its eigenvalues of smallest real part -- the squares of the eigenvalues of
  A nearest 0 lie at the left edge of the spectrum of A^2 -- for right
  vectors, the same on (A^H)^2 for left ones, eigenvalues by Rayleigh
  quotients with A, then L <- L (R^H L)^{-1} for L^H R = I.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

__all__ = ["select_critical", "lr_dense", "lr_arpack", "sign_f_diag",
           "projector_checks"]


def select_critical(lam, m, key="abs", gap_tol=1e-6):
    """Indices of the m critical eigenvalues and the selection gap."""
    lam = np.asarray(lam)
    kv = np.abs(lam) if key == "abs" else np.abs(lam.real)
    order = np.lexsort((np.arange(len(lam)), np.angle(lam), kv))
    sel = order[:m]
    gap = kv[order[m]] - kv[order[m - 1]] if (0 < m < len(lam)) else np.inf
    if gap < gap_tol:
        raise ValueError(f"no selection gap after {m} eigenvalues (gap {gap:.2e})")
    return sel, gap


def sign_f_diag(lam):
    return np.diag(np.sign(np.asarray(lam).real)).astype(np.complex128)


def lr_dense(A, m, key="abs", eig=None):
    """(R, L, Lambda, F) from a dense eigen-decomposition.

    ``eig`` optionally passes a precomputed ``np.linalg.eig(A)``."""
    A = np.asarray(A, dtype=np.complex128)
    lam, W = np.linalg.eig(A) if eig is None else eig
    sel, gap = select_critical(lam, m, key)
    Winv = np.linalg.inv(W)
    R = W[:, sel]
    L = Winv[sel, :].conj().T
    return R, L, lam[sel], sign_f_diag(lam[sel])


def _arpack_sq(A, m, extra, tol):
    n = A.shape[0]
    op = spla.LinearOperator((n, n), matvec=lambda v: A @ (A @ v), dtype=np.complex128)
    mu2, vec = spla.eigs(op, k=m + extra, which="SR", ncv=min(n - 1, 3 * (m + extra) + 20),
                         tol=tol, maxiter=200000)
    vec = vec / np.linalg.norm(vec, axis=0)
    lam = np.array([vec[:, i].conj() @ (A @ vec[:, i]) for i in range(vec.shape[1])])
    return lam, vec, mu2


def lr_arpack(A, AH, m, key="abs", extra=6, tol=1e-13, return_all=False):
    """(R, L, Lambda, F) for a sparse A with AH = A^H, via ARPACK on A^2.

    Completeness: every eigenvalue of A with |lambda| <= |lambda_(m)| has
    Re(lambda^2) <= |lambda|^2, so it is among the computed ones as long as
    the largest computed Re(lambda^2) is at least |lambda_(m)|^2 -- checked.
    (Same argument with |Re lambda| for key="re".)"""
    lam_r, Rr, mu2 = _arpack_sq(A, m, extra, tol)
    lam_l, Ll, _ = _arpack_sq(AH, m, extra, tol)
    sel, _ = select_critical(lam_r, m, key)
    kv = np.abs(lam_r[sel]) if key == "abs" else np.abs(lam_r[sel].real)
    if np.max(mu2.real) < np.max(kv) ** 2:
        raise RuntimeError("ARPACK window too small to certify the selection")
    R = Rr[:, sel]
    lam = lam_r[sel]
    L = np.empty_like(R)
    for i, li in enumerate(lam):
        j = int(np.argmin(np.abs(lam_l.conj() - li)))
        if abs(lam_l[j].conj() - li) > 1e-8 * max(1.0, abs(li)):
            raise RuntimeError("left/right eigenvalue sets do not match")
        L[:, i] = Ll[:, j]
    M = L.conj().T @ R
    L = L @ np.linalg.inv(M).conj().T
    if return_all:
        return R, L, lam, sign_f_diag(lam), lam_r
    return R, L, lam, sign_f_diag(lam)


def projector_checks(A, R, L, lam):
    """Relative eigen-residuals and biorthogonality defect."""
    AR = A @ R
    res_r = np.linalg.norm(AR - R * lam[None, :]) / np.linalg.norm(AR)
    LA = (A.conj().T @ L).conj().T
    res_l = np.linalg.norm(LA - lam[:, None] * L.conj().T) / np.linalg.norm(LA)
    bi = np.linalg.norm(L.conj().T @ R - np.eye(R.shape[1]))
    return res_r, res_l, bi
