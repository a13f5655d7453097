"""Oracle: restarted multishift GMRES with LR deflation (GMRES-LR, Sect. 5).

TEST INFRASTRUCTURE ONLY.

The paper names restarted multishift GMRES (Sect. 2 and 3) as the
alternative to FOM and refers its derivation elsewhere.  The method used
here is the standard one for shifted systems (A - sigma_i) x_i = b with
one Krylov space per cycle:

* one "seed" system s is solved by GMRES: over the cycle's Krylov space it
  minimises its residual, y_s = argmin || beta rho_s e_1 - (Hbar_k - sigma_s I~) y ||,
  whose residual is V_{k+1} z with z = beta rho_s e_1 - (Hbar_k - sigma_s I~) y_s;
* every other system is forced to keep its residual collinear with the
  seed's: r_i = rho_i' V_{k+1} z, which for y_i and rho_i' is the square
  (k+1) x (k+1) system [Hbar_k - sigma_i I~, z] [y_i; rho_i'] = beta rho_i e_1
  (I~ = [I_k; 0]);
* the next cycle starts from r = V_{k+1} z (with rho_s = 1), after the same
  projection step r = (I - P) r as Algorithm 1.

The rational approximation adds V_k sum_i omega_i y_i to x each cycle; the
stopping rule is the one of the FOM oracle (update norm below tol * ||x||
on two consecutive cycles).  On a lucky breakdown every system is solved
exactly from the square H_kk.
"""
from __future__ import annotations

import numpy as np

from . import krylov

__all__ = ["gmres_cycle_small", "restarted_gmres_lr"]


def gmres_cycle_small(H, kk, beta, rho, sigma, seed):
    """The small problems of one cycle: returns (Y (N x kk), z (kk+1), rho_new).

    H is (kk+1) x kk (Hbar).  Breakdown (H[kk, kk-1] == 0): FOM solves."""
    N = len(sigma)
    Y = np.zeros((N, kk), dtype=np.complex128)
    Ik = np.vstack([np.eye(kk), np.zeros((1, kk))])
    e1 = np.zeros(kk + 1, dtype=np.complex128)
    e1[0] = 1.0
    if H[kk, kk - 1] == 0.0:
        for i, s in enumerate(sigma):
            Y[i] = beta * rho[i] * np.linalg.solve(H[:kk, :kk] - s * np.eye(kk), e1[:kk])
        return Y, np.zeros(kk + 1, dtype=np.complex128), np.zeros(N, dtype=np.complex128)
    Hs = H - sigma[seed] * Ik
    rhs_s = beta * rho[seed] * e1
    ys, *_ = np.linalg.lstsq(Hs, rhs_s, rcond=None)
    Y[seed] = ys
    z = rhs_s - Hs @ ys
    rho_new = np.zeros(N, dtype=np.complex128)
    rho_new[seed] = 1.0
    for i, s in enumerate(sigma):
        if i == seed:
            continue
        M = np.column_stack([H - s * Ik, z])
        sol = np.linalg.solve(M, beta * rho[i] * e1)
        Y[i] = sol[:kk]
        rho_new[i] = sol[kk]
    return Y, z, rho_new


def restarted_gmres_lr(matvec, b, sigma, omega, k, R=None, L=None, F=None, seed=None,
                       tol_update=1e-9, max_cycles=200, project_each_cycle=True,
                       keep_shift_solutions=False):
    """GMRES-LR(m, k).  seed: index of the GMRES system (default: the pole
    nearest the origin).  Returns (x, info) like krylov.restarted_fom_lr."""
    b = np.asarray(b, dtype=np.complex128)
    sigma = np.asarray(sigma, dtype=np.complex128)
    omega = np.asarray(omega, dtype=np.complex128)
    N = len(sigma)
    if seed is None:
        seed = int(np.argmin(np.abs(sigma)))
    deflate = R is not None and R.shape[1] > 0
    if deflate:
        c = L.conj().T @ b
        x = R @ (F @ c)
        r = b - R @ c
    else:
        x = np.zeros_like(b)
        r = b.copy()
    rho = np.ones(N, dtype=np.complex128)
    X = np.zeros((N, b.shape[0]), dtype=np.complex128) if keep_shift_solutions else None
    upd, small, converged, cycles = [], 0, False, 0
    while cycles < max_cycles:
        cycles += 1
        beta = np.linalg.norm(r)
        if beta == 0.0:
            converged = True
            break
        V, H, kk = krylov.arnoldi(matvec, r / beta, k)
        Y, z, rho_new = gmres_cycle_small(H, kk, beta, rho, sigma, seed)
        u = omega @ Y
        x = x + V[:, :kk] @ u
        if keep_shift_solutions:
            X += Y @ V[:, :kk].T
        un = np.linalg.norm(u)
        upd.append(un)
        if H[kk, kk - 1] == 0.0:
            converged = True
            break
        r = V[:, : kk + 1] @ z
        rho = rho_new
        if deflate and project_each_cycle:
            r = r - R @ (L.conj().T @ r)
        if not np.isfinite(un) or not np.all(np.isfinite(rho)):
            break
        if cycles > 1 and un > 1e10 * upd[0]:
            break                 # the restarted iteration diverges for this k
        small = small + 1 if un <= tol_update * np.linalg.norm(x) else 0
        if small >= 2:
            converged = True
            break
    info = {"cycles": cycles, "converged": converged, "rho": rho, "update_norms": np.array(upd),
            "seed": seed}
    if keep_shift_solutions:
        info["X"] = X
    return x, info
