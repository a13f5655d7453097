"""GPU parity of sign_apply (Algorithm 1, restarted FOM-LR) against the
oracle's x* = R sign(Lambda) L^H b + sum_j omega_j (H - sigma_j)^{-1}(I - R L^H) b,
on lattices small enough for dense algebra."""
import ctypes as C

import numpy as np
import pytest

import skinputs as si
from skinputs.configs import CONFIGS
from oracle import dirac, rational, xstar, deflation
from tests.gpu_util import make_op, to_dev, from_dev, vecs_to_dev, rel, announce, torch_dev

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-8   # relative 2-norm error bound of the FP64 path


def _problem(dims, eps, mu, seed_g, seed_b):
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, eps, seed_g)
    b = si.gaussian_source(12 * V, seed_b)
    A = dirac.hw_dense(U, dims, 0.25, mu)
    return V, U, b, A


def test_config_c1_matches_oracle():
    from paper_0910_2927_amd import api
    cfg = CONFIGS["c1"]
    mu = cfg.mus[0]
    V, U, b, A = _problem(cfg.dims, cfg.eps, mu, si.seed_for(cfg.L, "gauge"), si.seed_for(cfg.L, "b"))
    sig, om = rational.kl_first_order(cfg.s, cfg.scales[mu])
    announce("sign_apply c1 4^4 k=20 N=10")
    op = make_op(U, cfg.dims, cfg.kappa, mu)
    res = api.sign_apply(op, to_dev(b, V), sig, om, cfg.k, tol=cfg.tol, max_cycles=cfg.max_cycles)
    assert res.converged
    ref = xstar.xstar_dense(A, b, sig, om)
    err = rel(from_dev(res.x, V), ref)
    print(f"c1: cycles={res.cycles} matvecs={res.matvecs} err={err:.2e}")
    assert err <= TOL_FP64


@pytest.mark.parametrize("k", [12, 37])
def test_ragged_lattice_with_deflation(k):
    from paper_0910_2927_amd import api
    import torch
    dims = (3, 4, 5, 6)
    V, U, b, A = _problem(dims, 0.6, 0.3, 91, 92)
    R, L, lam, F = deflation.lr_dense(A, 24)
    sig, om = rational.kl_first_order(8, 1.5)
    announce(f"sign_apply ragged 3x4x5x6 m=24 k={k}")
    op = make_op(U, dims, 0.25, 0.3)
    res = api.sign_apply(op, to_dev(b, V), sig, om, k, tol=1e-11, max_cycles=400,
                         R=vecs_to_dev(R, V), Lv=vecs_to_dev(L, V),
                         F=torch.from_numpy(F).to(torch_dev()))
    assert res.converged
    ref = xstar.xstar_dense(A, b, sig, om, R, L, F)
    err = rel(from_dev(res.x, V), ref)
    print(f"ragged k={k}: cycles={res.cycles} err={err:.2e} leak={res.leaks[-1]:.1e}")
    assert err <= TOL_FP64


def test_per_shift_solutions_match_dense_solves():
    from paper_0910_2927_amd import api
    dims = (2, 3, 4, 5)
    V, U, b, A = _problem(dims, 0.5, 0.3, 93, 94)
    sig, om = rational.kl_first_order(5, 1.2)
    announce("sign_apply keep_shift_solutions 2x3x4x5")
    op = make_op(U, dims, 0.25, 0.3)
    res = api.sign_apply(op, to_dev(b, V), sig, om, 16, tol=1e-12, max_cycles=400,
                         keep_shift_solutions=True)
    assert res.converged
    ref, Xref = xstar.xstar_dense(A, b, sig, om, return_shifts=True)
    for i in range(len(sig)):
        assert rel(from_dev(res.X_shift[i], V), Xref[i]) <= 1e-9
    # the combination sum omega_i X_i is the returned x
    comb = sum(om[i] * from_dev(res.X_shift[i], V) for i in range(len(sig)))
    assert rel(comb, from_dev(res.x, V)) < 1e-12


def test_plane_wave_source_ends_in_one_cycle_with_closed_form():
    from paper_0910_2927_amd import api
    dims = (4, 4, 4, 4)
    V = 256
    s = np.arange(V)
    x, z, t = s % 4, (s // 16) % 4, s // 64
    ph = np.exp(1j * (np.pi / 2 * x + np.pi * z + (np.pi / 4 + np.pi / 2) * t))
    b = (ph[:, None, None] * si.gaussian_source(12, 15).reshape(4, 3)[None]).reshape(-1)
    sig, om = rational.kl_first_order(5, 0.7)
    announce("sign_apply plane-wave breakdown")
    op = make_op(si.unit_links(dims), dims, 0.25, 0.3)
    res = api.sign_apply(op, to_dev(b, V), sig, om, 10, tol=1e-10)
    assert res.converged and res.breakdown and res.cycles == 1 and res.matvecs == 2
    ref = dirac.free_field_function(b, dims, 0.25, 0.3, lambda l: rational.kl_closed_form(0.7 * l, 5))
    assert rel(from_dev(res.x, V), ref) < 1e-12


def test_restart_length_independence_and_divergence():
    """Converged results do not depend on k.  Restarted FOM is not monotone:
    on this problem k = 25 diverges -- in the CPU oracle too -- and the
    library must say so instead of returning garbage."""
    from paper_0910_2927_amd import api, _lib
    from oracle import krylov
    dims = (4, 4, 4, 4)
    V, U, b, A = _problem(dims, 0.5, 0.3, 95, 96)
    sig, om = rational.kl_first_order(6, 1.4)
    op = make_op(U, dims, 0.25, 0.3)
    ref = xstar.xstar_dense(A, b, sig, om)
    for k in (10, 60):
        announce(f"sign_apply restart length k={k}")
        res = api.sign_apply(op, to_dev(b, V), sig, om, k, tol=1e-11, max_cycles=1000)
        assert res.converged
        assert rel(from_dev(res.x, V), ref) <= TOL_FP64
    _, info = krylov.restarted_fom_lr(lambda v: A @ v, b, sig, om, k=25, tol_update=1e-11,
                                      max_cycles=1000)
    assert not info["converged"]
    announce("sign_apply restart length k=25 (diverges)")
    res = api.sign_apply(op, to_dev(b, V), sig, om, 25, tol=1e-11, max_cycles=1000,
                         raise_on_error=False)
    assert res.status == _lib.SK_ERR_NOCONV and not res.converged
    # (the exact cycle at which growth passes 1e10 is rounding-sensitive in a
    # divergent iteration, so only the outcome is compared)


def test_error_paths_forced_from_the_host():
    from paper_0910_2927_amd import api, _lib
    dims = (2, 2, 2, 4)
    V, U, b, A = _problem(dims, 0.5, 0.3, 97, 98)
    sig, om = rational.kl_first_order(5, 1.2)
    op = make_op(U, dims, 0.25, 0.3)
    announce("sign_apply error paths")
    # non-convergence: one cycle only, x holds the iterate
    res = api.sign_apply(op, to_dev(b, V), sig, om, 4, tol=1e-14, max_cycles=1, raise_on_error=False)
    assert res.status == _lib.SK_ERR_NOCONV and res.cycles == 1 and not res.converged
    assert np.all(np.isfinite(from_dev(res.x, V)))
    # NaN in the source
    bn = b.copy()
    bn[5] = np.nan
    res = api.sign_apply(op, to_dev(bn, V), sig, om, 8, tol=1e-10, raise_on_error=False)
    assert res.status == _lib.SK_ERR_NAN
    # bad restart length is rejected before any launch
    with pytest.raises(_lib.SkError) as e:
        api.sign_apply(op, to_dev(b, V), sig, om, 0, tol=1e-10)
    assert e.value.status == _lib.SK_ERR_ARG
    # undersized workspace: refused on the host, nothing launched
    solver = api.SignSolver(op, sig, om, 8, tol=1e-10)
    lib = _lib.load()
    bd = to_dev(b, V)
    xd = bd.clone()
    st = lib.sign_apply(C.byref(solver.opstruct), C.byref(solver.params), C.c_void_p(bd.data_ptr()),
                        C.c_void_p(xd.data_ptr()), None, C.c_void_p(solver.ws.data_ptr()), 16, None)
    assert st == _lib.SK_ERR_WORKSPACE


def test_zero_source_and_deterministic_repeat():
    from paper_0910_2927_amd import api
    dims = (2, 2, 3, 4)
    V, U, b, A = _problem(dims, 0.5, 0.3, 99, 100)
    sig, om = rational.kl_first_order(5, 1.2)
    op = make_op(U, dims, 0.25, 0.3)
    announce("sign_apply zero source / repeat")
    res = api.sign_apply(op, to_dev(np.zeros_like(b), V), sig, om, 8, tol=1e-10)
    assert res.converged and float(res.x.abs().max()) == 0.0
    r1 = api.sign_apply(op, to_dev(b, V), sig, om, 8, tol=1e-10)
    r2 = api.sign_apply(op, to_dev(b, V), sig, om, 8, tol=1e-10)
    assert bool((r1.x == r2.x).all())   # fixed reduction order: bitwise repeatable


def test_graph_replay_matches_plain_launches():
    """Every restart cycle replays a captured HIP graph; with per-kernel
    timing on, the same cycles run as plain launches.  Both must give the
    same iterate bit for bit, in FP64 and in mixed precision (three graph
    kinds: double->double, double->float, float->float)."""
    import ctypes as C
    import torch
    from paper_0910_2927_amd import api, _lib
    dims = (3, 4, 5, 6)
    V, U, b, A = _problem(dims, 0.6, 0.3, 120, 121)
    sig, om = rational.kl_first_order(8, 1.5)
    op = make_op(U, dims, 0.25, 0.3)
    lib = _lib.load()
    for prec in ("fp64", "mixed"):
        announce(f"graph vs plain launches {prec}")
        solver = api.SignSolver(op, sig, om, 20, tol=1e-11, max_cycles=400, precision=prec)
        bd = to_dev(b, V)
        r1 = solver(bd)
        x1 = r1.x.clone()
        times = _lib.SkKernelTimes()
        st = _lib.SkStats()
        st.times = C.pointer(times)
        x2 = torch.empty_like(bd)
        s = lib.sign_apply(C.byref(solver.opstruct), C.byref(solver.params), C.c_void_p(bd.data_ptr()),
                           C.c_void_p(x2.data_ptr()), C.byref(st), C.c_void_p(solver.ws.data_ptr()),
                           solver.ws.numel(), C.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert s == 0 and st.cycles == r1.cycles and st.cycles_c64 == r1.cycles_c64
        assert bool((x1 == x2).all())
        if prec == "mixed":
            assert 0 < r1.cycles_c64 < r1.cycles


def test_projection_step_keeps_the_deflated_part_out():
    """Sect. 4/5: without the projection step after every cycle the
    deflated directions leak back into the restart vector (||L^H r|| grows
    cycle by cycle); with it the leak stays at rounding level and the
    result matches the oracle's x*."""
    from paper_0910_2927_amd import api
    import torch
    dims = (3, 4, 5, 6)
    V, U, b, A = _problem(dims, 0.6, 0.3, 95, 96)
    R, L, lam, F = deflation.lr_dense(A, 24)
    sig, om = rational.kl_first_order(8, 1.5)
    op = make_op(U, dims, 0.25, 0.3)
    kw = dict(tol=1e-11, max_cycles=400, R=vecs_to_dev(R, V), Lv=vecs_to_dev(L, V),
              F=torch.from_numpy(F).to(torch_dev()))
    ref = xstar.xstar_dense(A, b, sig, om, R, L, F)
    announce("sign_apply with and without the projection step")
    on = api.sign_apply(op, to_dev(b, V), sig, om, 20, project_each_cycle=True, **kw)
    off = api.sign_apply(op, to_dev(b, V), sig, om, 20, project_each_cycle=False, raise_on_error=False,
                         **kw)
    err_on = rel(from_dev(on.x, V), ref)
    err_off = rel(from_dev(off.x, V), ref)
    print(f"projection on: err {err_on:.2e}, max leak/beta {np.max(on.leaks / on.betas):.1e}; "
          f"off: err {err_off:.2e}, leak/beta first {off.leaks[0] / off.betas[0]:.1e} "
          f"last {off.leaks[-1] / off.betas[-1]:.1e}")
    assert on.converged and err_on <= TOL_FP64
    assert np.max(on.leaks / on.betas) < 1e-9
    assert off.leaks[-1] / off.betas[-1] > 100 * np.max(on.leaks / on.betas)


@pytest.mark.parametrize("k,s", [(130, 8), (256, 32)])
def test_longest_restart_and_most_poles(k, s):
    """The size limits of the library: k up to 256 (four columns per lane in
    the small solves) and 64 first-order poles, against the oracle."""
    from paper_0910_2927_amd import api
    dims = (2, 3, 4, 5)
    V, U, b, A = _problem(dims, 0.5, 0.3, 97, 98)
    sig, om = rational.kl_first_order(s, 1.3)
    announce(f"sign_apply 2x3x4x5 k={k} poles={2 * s}")
    op = make_op(U, dims, 0.25, 0.3)
    res = api.sign_apply(op, to_dev(b, V), sig, om, k, tol=1e-12, max_cycles=100)
    assert res.converged
    err = rel(from_dev(res.x, V), xstar.xstar_dense(A, b, sig, om))
    print(f"k={k} N={2 * s}: cycles={res.cycles} err={err:.2e}")
    assert err <= TOL_FP64


def test_largest_deflation_space():
    """m = 128, the library's limit for the deflation space (coefficients of
    the projection held in LDS, 16 chunks of 8 columns in the dots), with 64
    poles, against the oracle's x* with the same LR deflation."""
    import torch
    from paper_0910_2927_amd import api
    dims = (4, 4, 4, 4)
    V, U, b, A = _problem(dims, 0.6, 0.3, 131, 132)
    R, L, lam, F = deflation.lr_dense(A, 128)
    sig, om = rational.kl_first_order(32, 1.2)
    announce("sign_apply 4^4 m=128 poles=64 k=40")
    op = make_op(U, dims, 0.25, 0.3)
    res = api.sign_apply(op, to_dev(b, V), sig, om, 40, tol=1e-11, max_cycles=400,
                         R=vecs_to_dev(R, V), Lv=vecs_to_dev(L, V), F=torch.from_numpy(F).to(torch_dev()))
    assert res.converged
    err = rel(from_dev(res.x, V), xstar.xstar_dense(A, b, sig, om, R, L, F))
    print(f"m=128: cycles={res.cycles} err={err:.2e} leak={res.leaks[-1]:.1e}")
    assert err <= TOL_FP64


def test_shifted_residuals_stay_collinear_across_restarts():
    """Sect. 3: after every restart the residuals of all shifted systems are
    multiples of one vector (the restart vector), which is what lets one
    Krylov space serve every pole.  Checked on the GPU iterates after 3
    cycles (not yet converged) with the dense matrix."""
    from paper_0910_2927_amd import api
    dims = (2, 3, 4, 5)
    V, U, b, A = _problem(dims, 0.5, 0.3, 99, 100)
    sig, om = rational.kl_first_order(5, 1.2)
    announce("sign_apply 3 cycles with per-shift solutions, 2x3x4x5")
    op = make_op(U, dims, 0.25, 0.3)
    res = api.sign_apply(op, to_dev(b, V), sig, om, 8, tol=1e-14, max_cycles=3,
                         keep_shift_solutions=True, raise_on_error=False)
    assert res.cycles == 3 and not res.converged
    R = np.array([b - (A @ from_dev(res.X_shift[i], V) - sig[i] * from_dev(res.X_shift[i], V))
                  for i in range(len(sig))])
    norms = np.linalg.norm(R, axis=1)
    # poles already converged to rounding carry only rounding noise: compare
    # the ones whose residual is well above it (6 of the 10 here)
    live = np.flatnonzero(norms > 1e-6 * np.linalg.norm(b))
    assert len(live) >= 6
    ref = R[np.argmax(norms)] / norms.max()
    for i in live:
        u = R[i] / norms[i]
        phase = np.vdot(ref, u)
        dev = np.linalg.norm(u - phase * ref)
        print(f"pole {i}: |r_i|/|b| = {norms[i] / np.linalg.norm(b):.3e}, off-line part {dev:.1e}")
        assert dev < 1e-8                                  # parallel up to a phase
