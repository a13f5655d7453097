"""Write the oracle's reference values for the lattices too large for dense
algebra (8^4, 10^4).  Calls only the CPU oracle and the seeded generators.

For one (config, mu) it computes, in FP64 on the CPU:
  * the m deflated eigenpairs nearest zero (ARPACK on H^2, left and right),
  * the largest |lambda| (ARPACK), hence the pole scale c = (a b)^{-1/2},
  * x* = R sign(Lambda) L^H b + sum_j omega_j (H - sigma_j)^{-1} (I - R L^H) b
    by one long unrestarted multishift FOM run, each shift's residual
    checked with the CSR matrix,
and stores c, the deflated eigenvalues, norms and x* at a fixed sample of
indices (every `stride`-th component, canonical layout) as JSON.

    python tests/golden/make_golden.py c2 0.3        # one job
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as spla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import skinputs as si                       # noqa: E402
from skinputs.configs import CONFIGS       # noqa: E402
from oracle import dirac, rational, deflation, krylov, xstar   # noqa: E402

NSAMPLE = 4096


def sample_indices(n):
    stride = max(1, n // NSAMPLE)
    return np.arange(0, n, stride)[:NSAMPLE]


def run(name, mu, c_override=None):
    cfg = CONFIGS[name]
    t0 = time.time()
    L = cfg.L
    dims = cfg.dims
    U = si.gauge_links(dims, cfg.eps, si.seed_for(L, "gauge"))
    b = si.gaussian_source(cfg.n, si.seed_for(L, "b"))
    A = dirac.hw_csr(U, dims, cfg.kappa, mu, cfg.antiperiodic_t)
    AH = dirac.hw_csr(U, dims, cfg.kappa, -mu, cfg.antiperiodic_t)
    lmax = float(np.max(np.abs(spla.eigs(A, k=4, which="LM", return_eigenvectors=False, tol=1e-8))))
    out = {"config": name, "mu": mu, "dims": list(dims), "eps": cfg.eps, "lambda_max": lmax}
    if cfg.m > 0:
        for extra in (8, 16, 32):   # widen the ARPACK window until the selection is certified
            try:
                R, Lv, lam, F, lam_all = deflation.lr_arpack(A, AH, cfg.m, extra=extra,
                                                             return_all=True)
                break
            except RuntimeError as e:
                if "window" not in str(e) or extra == 32:
                    raise
                print(f"{name}: ARPACK window with {extra} extra too small; widening", flush=True)
        res_r, res_l, bi = deflation.projector_checks(A, R, Lv, lam)
        a = float(np.sort(np.abs(lam_all))[cfg.m])
        order = np.lexsort((np.angle(lam), np.abs(lam)))
        out.update({"eig_re": lam[order].real.tolist(), "eig_im": lam[order].imag.tolist(),
                    "a_next": a, "eig_res_right": res_r, "eig_res_left": res_l,
                    "biorth": bi})
    else:
        R = Lv = F = None
        w = spla.eigs(A @ A, k=6, which="SR", return_eigenvectors=False, tol=1e-10, ncv=60)
        a = float(np.sqrt(np.min(np.abs(w))))
        out["a_next"] = a
    c = float(f"{(a * lmax) ** -0.5:.4g}") if c_override is None else c_override
    out["c"] = c
    sigma, omega = rational.kl_first_order(cfg.s, c)
    rhs = xstar.deflated_source(b, R, Lv)
    xp = xstar.x_p(b, R, Lv, F)
    xs_g, X, kit = krylov.multishift_fom_unrestarted(lambda v: A @ v, rhs, sigma, omega,
                                                     tol=1e-13, kmax=6000)
    x = xp + xs_g
    res = [float(np.linalg.norm(rhs - (A @ X[j] - sigma[j] * X[j])) / np.linalg.norm(rhs))
           for j in range(len(sigma))]
    idx = sample_indices(cfg.n)
    out.update({"fom_iterations": int(kit), "shift_residuals": res,
                "x_norm": float(np.linalg.norm(x)), "xp_norm": float(np.linalg.norm(xp)),
                "b_norm": float(np.linalg.norm(b)),
                "sample_index": idx.tolist(), "x_re": x[idx].real.tolist(),
                "x_im": x[idx].imag.tolist(), "seconds": time.time() - t0})
    path = os.path.join(HERE, f"{name}_mu{mu:g}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"{name} mu={mu}: c={c} a={a:.5g} lmax={lmax:.5g} fom_it={kit} "
          f"max_res={max(res):.2e} {time.time() - t0:.0f}s -> {path}", flush=True)


if __name__ == "__main__":
    run(sys.argv[1], float(sys.argv[2]))
