"""GMRES-LR (restarted multishift GMRES with LR deflation, Sect. 2, 3, 5)
through sign_apply(method = GMRES) against the oracle's same algorithm,
cycle for cycle, and against x* once converged."""
import numpy as np
import pytest

import skinputs as si
from oracle import dirac, rational, deflation, xstar, gmres
from tests.gpu_util import make_op, to_dev, from_dev, vecs_to_dev, rel, announce, torch_dev

pytestmark = pytest.mark.gpu


def _run(dims, k, m, seed, cycles, tol=1e-12):
    import torch
    from paper_0910_2927_amd import api
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.5, seed)
    b = si.gaussian_source(12 * V, seed + 1)
    A = dirac.hw_csr(U, dims, 0.25, 0.3)
    R = L = F = None
    kw = {}
    if m:
        R, L, lam, F = deflation.lr_dense(A.toarray(), m)
        kw = dict(R=vecs_to_dev(R, V), Lv=vecs_to_dev(L, V), F=torch.from_numpy(F).to(torch_dev()))
    sig, om = rational.kl_first_order(6, 1.3)
    ref, info = gmres.restarted_gmres_lr(lambda v: A @ v, b, sig, om, k, R, L, F, tol_update=tol,
                                         max_cycles=cycles)
    op = make_op(U, dims, 0.25, 0.3)
    announce(f"sign_apply GMRES-LR dims={dims} k={k} m={m} cycles<={cycles}")
    res = api.SignSolver(op, sig, om, k, tol=tol, max_cycles=cycles, method="gmres", **kw)(
        to_dev(b, V), raise_on_error=False)
    return res, ref, info, (A, b, sig, om, R, L, F, V)


@pytest.mark.parametrize("dims,k,m", [((4, 4, 4, 4), 24, 0), ((3, 4, 5, 6), 30, 12)])
def test_gmres_lr_matches_oracle_cycle_for_cycle(dims, k, m):
    res, ref, info, ctx = _run(dims, k, m, 900 + k, 3)
    err = rel(from_dev(res.x, ctx[-1]), ref)
    print(f"GMRES-LR 3 cycles: rel err vs oracle {err:.2e}")
    assert res.cycles == info["cycles"] == 3
    assert err <= 1e-10
    assert np.allclose(res.rho_hist[-1], np.abs(info["rho"]), rtol=1e-6, atol=1e-12)


def test_gmres_lr_converges_to_xstar():
    res, ref, info, ctx = _run((4, 4, 4, 4), 40, 12, 950, 400)
    A, b, sig, om, R, L, F, V = ctx
    xs = xstar.xstar_sparse(A, b, sig, om, R, L, F)
    err = rel(from_dev(res.x, V), xs)
    print(f"GMRES-LR converged in {res.cycles} cycles (oracle {info['cycles']}): rel err vs x* {err:.2e}")
    assert res.converged and info["converged"]
    assert err <= 1e-8
