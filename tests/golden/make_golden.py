"""Write the oracle's reference values for the lattices too large for dense
algebra (8^4, 10^4).  Calls only the CPU oracle and the seeded generators.

For one (config, mu) it computes, in FP64 on the CPU:
  * the m deflated eigenpairs nearest zero (ARPACK on H^2, left and right),
  * the largest |lambda| (ARPACK), hence the pole scale c = (a b)^{-1/2},
  * x* = R sign(Lambda) L^H b + sum_j omega_j (H - sigma_j)^{-1} (I - R L^H) b
    by one long unrestarted multishift FOM run, each shift's residual
    checked with the CSR matrix,
and stores c, the deflated eigenvalues, norms and x* at a fixed sample of
indices (every `stride`-th component, canonical layout) as JSON, and the
whole x* (canonical layout, complex128) as `<config>_mu<mu>_x.npy`.

Configurations that differ only in the Kenney-Laub order s (c3 and the
sign-accurate c3s) share the deflation and one Krylov run: list them after
--with.  --order-check also computes x* with twice each order, 2s, and
records the relative difference ||x*(s) - x*(2s)|| / ||x*(2s)||, an
estimate of the rational approximation's own error next to the scalar
bound 2 rho^{2s}, rho = (sqrt(q) - 1)/(sqrt(q) + 1), q = lambda_max / a of
Sect. 6's scaled approximation on the real segment [a, lambda_max].

    python tests/golden/make_golden.py c2 0.3                     # one job
    python tests/golden/make_golden.py c3 0.3 --with c3s --order-check
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


def kl_bound(a, lmax, s):
    q = lmax / a
    rho = (np.sqrt(q) - 1) / (np.sqrt(q) + 1)
    return float(2 * rho ** (2 * s))


def run(name, mu, also=(), order_check=False, c_override=None):
    cfg = CONFIGS[name]
    group = [cfg] + [CONFIGS[o] for o in also]
    for o in group[1:]:
        assert (o.dims, o.eps, o.m, o.kappa, o.antiperiodic_t) == \
            (cfg.dims, cfg.eps, cfg.m, cfg.kappa, cfg.antiperiodic_t), o.name
    t0 = time.time()
    L = cfg.L
    dims = cfg.dims
    U = si.gauge_links(dims, cfg.eps, si.seed_for(L, "gauge"))
    b = si.gaussian_source(cfg.n, si.seed_for(L, "b"))
    A = dirac.hw_csr(U, dims, cfg.kappa, mu, cfg.antiperiodic_t)
    AH = dirac.hw_csr(U, dims, cfg.kappa, -mu, cfg.antiperiodic_t)
    lmax = float(np.max(np.abs(spla.eigs(A, k=4, which="LM", return_eigenvectors=False, tol=1e-8))))
    common = {"mu": mu, "dims": list(dims), "eps": cfg.eps, "lambda_max": lmax}
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
        common.update({"eig_re": lam[order].real.tolist(), "eig_im": lam[order].imag.tolist(),
                       "a_next": a, "eig_res_right": res_r, "eig_res_left": res_l,
                       "biorth": bi})
    else:
        R = Lv = F = None
        w = spla.eigs(A @ A, k=6, which="SR", return_eigenvectors=False, tol=1e-10, ncv=60)
        a = float(np.sqrt(np.min(np.abs(w))))
        common["a_next"] = a
    c = float(f"{(a * lmax) ** -0.5:.4g}") if c_override is None else c_override
    print(f"{name} mu={mu}: a={a:.6g} lmax={lmax:.6g} c={c} ({time.time() - t0:.0f}s)", flush=True)
    # every pole set of the group (and 2s for the order check) in one Krylov run
    orders = []
    for o in group:
        orders.append(o.s)
        if order_check:
            orders.append(2 * o.s)
    orders = sorted(set(orders))
    sig_all, om_all, spans = [], [], {}
    for s_ in orders:
        sg, om = rational.kl_first_order(s_, c)
        spans[s_] = (len(sig_all), len(sig_all) + len(sg))
        sig_all += list(sg)
        om_all += list(om)
    sig_all = np.array(sig_all)
    om_all = np.array(om_all)
    watch = np.argsort(np.abs(sig_all))[:2]     # the shifts nearest the spectrum converge last
    rhs = xstar.deflated_source(b, R, Lv)
    xp = xstar.x_p(b, R, Lv, F)
    _, X, kit = krylov.multishift_fom_unrestarted(lambda v: A @ v, rhs, sig_all, om_all,
                                                  tol=1e-13, kmax=6000, watch=watch)
    res = np.array([float(np.linalg.norm(rhs - (A @ X[j] - sig_all[j] * X[j]))
                          / np.linalg.norm(rhs)) for j in range(len(sig_all))])
    xs = {}
    for s_ in orders:
        lo, hi = spans[s_]
        xs[s_] = xp + om_all[lo:hi] @ X[lo:hi]
    for o in group:
        lo, hi = spans[o.s]
        x = xs[o.s]
        idx = sample_indices(o.n)
        out = dict(common)
        out.update({"config": o.name, "s": o.s, "c": c, "fom_iterations": int(kit),
                    "shift_residuals": res[lo:hi].tolist(),
                    "kl_bound": kl_bound(a, lmax, o.s),
                    "x_norm": float(np.linalg.norm(x)), "xp_norm": float(np.linalg.norm(xp)),
                    "b_norm": float(np.linalg.norm(b)),
                    "sample_index": idx.tolist(), "x_re": x[idx].real.tolist(),
                    "x_im": x[idx].imag.tolist(), "seconds": time.time() - t0})
        if order_check:
            x2 = xs[2 * o.s]
            out["order_check"] = {"s2": 2 * o.s,
                                  "rel_diff": float(np.linalg.norm(x - x2) / np.linalg.norm(x2)),
                                  "kl_bound_s2": kl_bound(a, lmax, 2 * o.s),
                                  "max_shift_residual_s2": float(res[spans[2 * o.s][0]:
                                                                     spans[2 * o.s][1]].max())}
        path = os.path.join(HERE, f"{o.name}_mu{mu:g}.json")
        with open(path, "w") as f:
            json.dump(out, f)
        np.save(os.path.join(HERE, f"{o.name}_mu{mu:g}_x.npy"), x)
        print(f"{o.name} mu={mu}: s={o.s} c={c} fom_it={kit} max_res={res[lo:hi].max():.2e} "
              + (f"x(s) vs x(2s) {out['order_check']['rel_diff']:.2e} " if order_check else "")
              + f"{time.time() - t0:.0f}s -> {path}", flush=True)


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("config")
    ap.add_argument("mu", type=float)
    ap.add_argument("--with", dest="also", nargs="*", default=[])
    ap.add_argument("--order-check", action="store_true")
    ap.add_argument("--c", type=float, default=None, help="use this pole scale")
    a = ap.parse_args()
    run(a.config, a.mu, a.also, a.order_check, a.c)
