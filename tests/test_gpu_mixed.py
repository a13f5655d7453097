"""Mixed precision (complex-float basis and stencil, FP64 accumulators,
FP64 anchor cycles) against the oracle, with the error of each variant
stated: FP64, mixed, and complex float throughout (no FP64 cycles)."""
import json
import os

import numpy as np
import pytest

import skinputs as si
from skinputs.configs import CONFIGS
from oracle import dirac, rational, xstar, deflation
from tests.gpu_util import make_op, to_dev, from_dev, vecs_to_dev, rel, announce, torch_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 4, 5, 6)])
def test_mixed_precision_error_table(dims):
    import torch
    from paper_0910_2927_amd import api
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.7, 400 + V)
    b = si.gaussian_source(12 * V, 401 + V)
    A = dirac.hw_dense(U, dims, 0.25, 0.3)
    R, L, lam, F = deflation.lr_dense(A, 12)
    sig, om = rational.kl_first_order(8, 1.6)
    ref = xstar.xstar_dense(A, b, sig, om, R, L, F)
    op = make_op(U, dims, 0.25, 0.3)
    kw = dict(tol=1e-11, max_cycles=600, R=vecs_to_dev(R, V), Lv=vecs_to_dev(L, V),
              F=torch.from_numpy(F).to(torch_dev()))
    errs = {}
    for prec in ("fp64", "mixed", "mixed_c64_only"):
        announce(f"sign_apply {prec} dims={dims}")
        res = api.sign_apply(op, to_dev(b, V), sig, om, 30, precision=prec, **kw)
        errs[prec] = (rel(from_dev(res.x, V), ref), res.cycles, res.cycles_c64)
    print("error vs oracle x* (rel 2-norm), cycles, complex-float cycles:", errs)
    assert errs["fp64"][0] <= 1e-8
    assert errs["mixed"][0] <= 1e-8          # after the FP64 anchor cycles
    assert errs["mixed"][2] >= errs["mixed"][1] // 2   # most cycles in complex float
    assert errs["mixed_c64_only"][0] <= 1e-6  # complex float throughout
    assert errs["mixed_c64_only"][2] == errs["mixed_c64_only"][1]


def test_config_c2_mixed_with_gpu_deflation():
    from paper_0910_2927_amd import api
    cfg = CONFIGS["c2"]
    mu = 0.1
    g = json.load(open(os.path.join(GOLDEN, f"c2_mu{mu:g}.json")))
    U = si.gauge_links(cfg.dims, cfg.eps, si.seed_for(cfg.L, "gauge"))
    b = si.gaussian_source(cfg.n, si.seed_for(cfg.L, "b"))
    op = make_op(U, cfg.dims, cfg.kappa, mu)
    announce("eigensolve c2 8^4 mu=0.1")
    R, L, F, lam, st = api.deflation_eigensolve(op, cfg.m, nev_extra=16, tol=1e-12)
    refl = np.array(g["eig_re"]) + 1j * np.array(g["eig_im"])
    assert np.allclose(np.sort_complex(lam), np.sort_complex(refl), rtol=0, atol=1e-9)
    sig, om = api.kl_poles(cfg.s, cfg.scales[mu])
    idx = np.array(g["sample_index"])
    xs = np.array(g["x_re"]) + 1j * np.array(g["x_im"])
    for prec in ("fp64", "mixed"):
        announce(f"sign_apply c2 8^4 mu=0.1 {prec}")
        res = api.sign_apply(op, to_dev(b, cfg.V), sig, om, cfg.k, tol=cfg.tol,
                             max_cycles=cfg.max_cycles, R=R, Lv=L, F=F, precision=prec)
        assert res.converged
        err = rel(from_dev(res.x, cfg.V)[idx], xs)
        print(f"c2 mu=0.1 {prec}: sampled rel err {err:.2e}, cycles {res.cycles} "
              f"(complex float {res.cycles_c64})")
        assert err <= 1e-8
