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
        # complex float throughout cannot carry residuals below its own
        # rounding: its FP64 check is run at that level
        rt = 1e-5 if prec == "mixed_c64_only" else 0.0
        res = api.sign_apply(op, to_dev(b, V), sig, om, 30, precision=prec, resid_tol=rt, **kw)
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


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 4, 5, 6)])
def test_mixed_result_checked_by_fp64_true_residuals(dims):
    """Mixed precision ends with an FP64 check inside the library: N
    complex-double stencil applications give the true residuals of the
    shifted systems, (I-P)b - (A - sigma_i) X_i, which must stay within
    10 |rho_i| + resid_tol ||(I-P)b||.  The library's residual norms are
    compared with the same residuals formed on the CPU from the returned
    per-shift solutions."""
    import torch
    from paper_0910_2927_amd import api
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.7, 410 + V)
    b = si.gaussian_source(12 * V, 411 + V)
    A = dirac.hw_csr(U, dims, 0.25, 0.3)
    R, L, lam, F = deflation.lr_dense(A.toarray(), 12)
    sig, om = rational.kl_first_order(8, 1.6)
    op = make_op(U, dims, 0.25, 0.3)
    announce(f"sign_apply mixed with FP64 residual check dims={dims}")
    res = api.sign_apply(op, to_dev(b, V), sig, om, 30, precision="mixed", tol=1e-11, max_cycles=600,
                         R=vecs_to_dev(R, V), Lv=vecs_to_dev(L, V), F=torch.from_numpy(F).to(torch_dev()),
                         keep_shift_solutions=True, residuals=True)
    assert res.converged and res.resid_ok
    rhs = xstar.deflated_source(b, R, L)
    X = res.X_shift.cpu().numpy()
    cpu = np.array([np.linalg.norm(rhs - (A @ si.canonical_from_soa(X[i], V) - sig[i] * si.canonical_from_soa(X[i], V)))
                    for i in range(len(sig))]) / np.linalg.norm(rhs)
    print("true residuals (library, CPU) and implicit:", res.shift_resid, cpu, res.shift_resid_implicit)
    assert np.all(res.shift_resid <= 10 * res.shift_resid_implicit + 100 * 1e-11)
    big = cpu > 1e-13
    assert np.allclose(res.shift_resid[big], cpu[big], rtol=1e-2, atol=0)
    assert np.all(res.shift_resid[~big] < 1e-12)
    # and the rho history is recorded per cycle and ends at the implicit residuals
    assert res.rho_hist.shape == (res.cycles, len(sig))


def test_mixed_check_failure_is_reported():
    """Complex float from the first cycle to a tolerance below what complex
    float can carry, with resid_tol forced tiny from the host: the FP64
    check must reject the result with SK_ERR_NOCONV (x still holds the
    iterate, the residuals are reported)."""
    from paper_0910_2927_amd import api, _lib
    dims = (4, 4, 4, 4)
    V = 256
    U = si.gauge_links(dims, 0.7, 420)
    b = si.gaussian_source(12 * V, 421)
    sig, om = rational.kl_first_order(5, 1.3)
    op = make_op(U, dims, 0.25, 0.3)
    announce("sign_apply mixed_c64_only with resid_tol 1e-300 (check must fail)")
    res = api.sign_apply(op, to_dev(b, V), sig, om, 20, precision="mixed_c64_only", tol=1e-9,
                         max_cycles=600, resid_tol=1e-300, residuals=True, raise_on_error=False)
    assert res.status == _lib.SK_ERR_NOCONV
    assert res.resid_ok is False
    assert np.max(res.shift_resid) > 1e-9       # complex-float rounding shows in the residuals


def test_arnoldi_and_rho_errors_of_complex_float_against_fp64():
    """The error statements of the mixed path for H_k and rho: one Arnoldi
    cycle and one multishift FOM step from the same start vector, with the
    basis in complex float against complex double."""
    import torch
    from paper_0910_2927_amd import api
    dims = (4, 4, 4, 6)
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.7, 430)
    b = si.gaussian_source(12 * V, 431)
    op = make_op(U, dims, 0.25, 0.3, with_c64=True)
    k = 30
    announce("arnoldi_cycle c128 and c64, k=30")
    V64, H64, kd64 = api.arnoldi_cycle(op, to_dev(b, V), k)
    V32, H32, kd32 = api.arnoldi_cycle(op, to_dev(b, V, torch.complex64), k)
    assert kd64 == kd32 == k
    eH = float(torch.linalg.matrix_norm(H32 - H64) / torch.linalg.matrix_norm(H64))
    sig, om = rational.kl_first_order(8, 1.6)
    out = {}
    for name, Vb, H in (("c128", V64, H64), ("c64", V32, H32)):
        beta = torch.tensor([np.linalg.norm(b)], dtype=torch.float64, device=torch_dev())
        rho = torch.ones(len(sig), dtype=torch.complex128, device=torch_dev())
        x = torch.zeros(12 * V, dtype=torch.complex128, device=torch_dev())
        api.multishift_fom_restart(H, k, sig, om, beta, rho, Vb, x)
        out[name] = (rho.cpu().numpy(), from_dev(x, V))
    erho = float(np.max(np.abs(out["c64"][0] - out["c128"][0]) / np.abs(out["c128"][0])))
    ex = rel(out["c64"][1], out["c128"][1])
    print(f"complex float vs complex double: H_k {eH:.2e}, rho {erho:.2e}, x after one cycle {ex:.2e}")
    assert eH <= 1e-5 and erho <= 1e-4 and ex <= 1e-5
    assert eH >= 1e-9          # the complex-float basis really is in complex float
