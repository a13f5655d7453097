"""Oracle: Arnoldi, multishift FOM and restarted FOM-LR (Algorithm 1), plainly.

TEST INFRASTRUCTURE ONLY.

* ``arnoldi``: the Arnoldi relation A V_k = V_k H_k + h_{k+1,k} v_{k+1} e_k^T
  of Sect. 2, with classical Gram-Schmidt applied twice per step (the paper
  leaves the orthogonalisation variant open; V_k and H_k are unique given
  v_1, whatever the variant, up to rounding).
* ``fom_shifted``: the FOM iterates of Sect. 3,
  y^{(i)} = beta rho^{(i)} (H_k - sigma_i I)^{-1} e_1, and the collinearity
  factors rho^{(i)} <- -h_{k+1,k} e_k^T y^{(i)} (residual r^{(i)} = rho v_{k+1}).
* ``restarted_fom_lr``: Algorithm 1 (restarted FOM-LR(m, k)), step by
  step in the paper's order.  The paper leaves the stopping rule open
  ("not all systems are converged"); the rule here is: stop when the
  cycle's update norm ||sum_i omega_i y^{(i)}||_2 <= tol_update * ||x||_2
  on two consecutive cycles, or on Arnoldi breakdown (exact result).
  Restarted FOM is not monotone: for a short cycle on a spectrum on both
  sides of the imaginary axis, H_k - sigma_i can be nearly singular and the
  iterates blow up; a non-finite update, or one 1e10 times the first,
  ends the loop unconverged.
* ``multishift_fom_unrestarted``: one long Arnoldi run with the FOM iterate
  of every shift, for large n where dense solves are out of reach.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = ["arnoldi", "fom_shifted", "restarted_fom_lr",
           "multishift_fom_unrestarted", "BREAKDOWN_TOL"]

BREAKDOWN_TOL = 1e-12


def arnoldi(matvec, v1, k, V_out=None):
    """k Arnoldi steps from the unit vector v1.

    Returns (V, H, kk): V is n x (kk+1), H is (kk+1) x kk, kk <= k the number
    of steps done (kk < k only on breakdown, where H[kk, kk-1] = 0 exactly).
    A step breaks down when h_{j+1,j} <= BREAKDOWN_TOL * ||A v_j||."""
    n = v1.shape[0]
    V = np.zeros((n, k + 1), dtype=np.complex128) if V_out is None else V_out
    H = np.zeros((k + 1, k), dtype=np.complex128)
    V[:, 0] = v1
    for j in range(k):
        w = matvec(V[:, j])
        wn = np.linalg.norm(w)
        Vj = V[:, : j + 1]
        h = Vj.conj().T @ w
        w = w - Vj @ h
        h2 = Vj.conj().T @ w
        w = w - Vj @ h2
        H[: j + 1, j] = h + h2
        beta = np.linalg.norm(w)
        if beta <= BREAKDOWN_TOL * wn:
            H[j + 1, j] = 0.0
            return V[:, : j + 2], H[: j + 2, : j + 1], j + 1
        H[j + 1, j] = beta
        V[:, j + 1] = w / beta
    return V, H, k


def fom_shifted(H, kk, beta, rho, sigma):
    """FOM iterates of all shifted systems and their new collinearity factors.

    H is (kk+1) x kk.  Returns Y (N x kk) with Y[i] = beta rho_i
    (H_k - sigma_i I)^{-1} e_1 and rho_new[i] = -h_{k+1,k} Y[i, -1]."""
    Hk = H[:kk, :kk]
    e1 = np.zeros(kk, dtype=np.complex128)
    e1[0] = 1.0
    Y = np.empty((len(sigma), kk), dtype=np.complex128)
    for i, s in enumerate(sigma):
        Y[i] = beta * rho[i] * np.linalg.solve(Hk - s * np.eye(kk), e1)
    rho_new = -H[kk, kk - 1] * Y[:, -1]
    return Y, rho_new


def restarted_fom_lr(matvec, b, sigma, omega, k, R=None, L=None, F=None,
                     tol_update=1e-9, max_cycles=200, project_each_cycle=True,
                     keep_shift_solutions=False, history=None):
    """Algorithm 1, restarted FOM-LR(m, k).

    Returns (x, info).  info has 'cycles', 'converged', 'rho', 'update_norms',
    and with keep_shift_solutions the per-shift iterates 'X' (N x n), which
    solve (A - sigma_i) X_i = (I - P) b."""
    b = np.asarray(b, dtype=np.complex128)
    sigma = np.asarray(sigma, dtype=np.complex128)
    omega = np.asarray(omega, dtype=np.complex128)
    N = len(sigma)
    deflate = R is not None and R.shape[1] > 0
    # x = x_P = R f(Lambda) L^H b ;  r = (I - P) b
    if deflate:
        c = L.conj().T @ b
        x = R @ (F @ c)
        r = b - R @ c
    else:
        x = np.zeros_like(b)
        r = b.copy()
    rho = np.ones(N, dtype=np.complex128)
    X = np.zeros((N, b.shape[0]), dtype=np.complex128) if keep_shift_solutions else None
    upd_hist = []
    small = 0
    converged = False
    cycles = 0
    while cycles < max_cycles:
        cycles += 1
        beta = np.linalg.norm(r)
        if beta == 0.0:
            converged = True
            break
        v1 = r / beta
        V, H, kk = arnoldi(matvec, v1, k)
        Y, rho_new = fom_shifted(H, kk, beta, rho, sigma)
        u = omega @ Y                       # sum_i omega_i y^{(i)}
        x = x + V[:, :kk] @ u
        if keep_shift_solutions:
            X += Y @ V[:, :kk].T
        r = V[:, kk].copy()
        rho = rho_new
        if deflate and project_each_cycle:
            r = r - R @ (L.conj().T @ r)   # projection step
        un = np.linalg.norm(u)
        upd_hist.append(un)
        if not np.isfinite(un) or not np.all(np.isfinite(rho)):
            break                           # diverged: restarted FOM is not monotone
        if cycles > 1 and un > 1e10 * upd_hist[0]:
            break                           # same divergence, caught before overflow
        if history is not None:
            history.append({"beta": beta, "rho": rho.copy(), "h_next": H[kk, kk - 1],
                            "update": un, "H": H.copy(), "kk": kk})
        if H[kk, kk - 1] == 0.0:            # breakdown: iterate is exact
            converged = True
            break
        small = small + 1 if un <= tol_update * np.linalg.norm(x) else 0
        if small >= 2:
            converged = True
            break
    info = {"cycles": cycles, "converged": converged, "rho": rho,
            "update_norms": np.array(upd_hist)}
    if keep_shift_solutions:
        info["X"] = X
    return x, info


def multishift_fom_unrestarted(matvec, rhs, sigma, omega, tol=1e-12, kmax=4000,
                               check_every=10, watch=None):
    """Long-recurrence multishift FOM (Sect. 2-3) without restarts.

    Grows one Arnoldi basis for K_k(A, rhs) until every shifted FOM residual
    norm |h_{k+1,k}| |e_k^T y^{(i)}| <= tol * ||rhs||.  Returns
    (sum_i omega_i x^{(i)}, X (N x n), k).

    ``watch`` (indices into sigma) limits the periodic test to those shifts
    -- with many shifts the k x k solves of every test dominate; once they
    pass, every shift is tested and the run goes on unless all pass."""
    rhs = np.asarray(rhs, dtype=np.complex128)
    n = rhs.shape[0]
    beta = np.linalg.norm(rhs)
    V = np.zeros((n, kmax + 1), dtype=np.complex128)
    H = np.zeros((kmax + 1, kmax), dtype=np.complex128)
    V[:, 0] = rhs / beta
    sigma = np.asarray(sigma)
    j = 0
    while j < kmax:
        w = matvec(V[:, j])
        wn = np.linalg.norm(w)
        Vj = V[:, : j + 1]
        h = Vj.conj().T @ w
        w = w - Vj @ h
        h2 = Vj.conj().T @ w
        w = w - Vj @ h2
        H[: j + 1, j] = h + h2
        hb = np.linalg.norm(w)
        j += 1
        done = hb <= BREAKDOWN_TOL * wn
        H[j, j - 1] = 0.0 if done else hb
        if not done:
            V[:, j] = w / hb
        if done or j % check_every == 0 or j == kmax:
            if watch is not None and not done and j < kmax:
                _, rw = fom_shifted(H[: j + 1, :j], j, beta, np.ones(len(watch)), sigma[watch])
                if np.max(np.abs(rw)) > tol * beta:
                    continue
            Y, rho = fom_shifted(H[: j + 1, :j], j, beta, np.ones(len(sigma)), sigma)
            if done or np.max(np.abs(rho)) <= tol * beta:
                break
    X = Y @ V[:, :j].T
    return np.asarray(omega) @ X, X, j
