"""The overlap operator D(m) = (1 - m/2)(1 + gamma5 sign(H_W)) + m around the
library's sign_apply (Sect. 1: its inversion is what the sign function is
needed for), and its inversion by the outer restarted GMRES, against the
oracle's dense operator built from the same rational approximation and
deflation."""
import numpy as np
import pytest

import skinputs as si
from oracle import dirac, rational, deflation, xstar, overlap
from tests.gpu_util import make_op, to_dev, from_dev, vecs_to_dev, rel, announce, torch_dev

pytestmark = pytest.mark.gpu


def _solver(op, V, sig, om, k, R=None, L=None, F=None, tol=1e-12):
    import torch
    from paper_0910_2927_amd import api
    kw = {}
    if R is not None:
        kw = dict(R=vecs_to_dev(R, V), Lv=vecs_to_dev(L, V), F=torch.from_numpy(F).to(torch_dev()))
    return api.SignSolver(op, sig, om, k, tol=tol, max_cycles=800, **kw)


@pytest.mark.parametrize("mass", [0.0, 0.1])
def test_overlap_apply_matches_oracle(mass):
    from paper_0910_2927_amd import api
    dims = (4, 4, 4, 4)
    V = 256
    U = si.gauge_links(dims, 0.5, 800)
    b = si.gaussian_source(12 * V, 801)
    A = dirac.hw_csr(U, dims, 0.25, 0.3)
    R, L, lam, F = deflation.lr_dense(A.toarray(), 10)
    sig, om = rational.kl_first_order(5, 1.3)
    ref = overlap.overlap_apply(lambda v: xstar.xstar_sparse(A, v, sig, om, R, L, F), b, mass)
    op = make_op(U, dims, 0.25, 0.3)
    D = api.OverlapOperator(_solver(op, V, sig, om, 20, R, L, F), mass=mass)
    announce(f"overlap_apply 4^4 mass={mass}")
    y = D.apply(to_dev(b, V))
    err = rel(from_dev(y, V), ref)
    print(f"overlap_apply mass={mass}: rel err {err:.2e}")
    assert err <= 1e-9


def test_overlap_solve_matches_dense_inverse():
    """Small lattice: x = D(m)^{-1} b with D built densely from the same
    poles and deflation (the map b -> x*(b) of Algorithm 1)."""
    from paper_0910_2927_amd import api
    dims = (3, 3, 3, 4)
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.5, 810)
    b = si.gaussian_source(12 * V, 811)
    A = dirac.hw_dense(U, dims, 0.25, 0.3)
    R, L, lam, F = deflation.lr_dense(A, 8)
    sig, om = rational.kl_first_order(6, 1.3)
    mass = 0.1
    Dm = overlap.overlap_matrix(overlap.sign_map_matrix(A, sig, om, R, L, F), mass)
    ref = np.linalg.solve(Dm, b)
    op = make_op(U, dims, 0.25, 0.3)
    D = api.OverlapOperator(_solver(op, V, sig, om, 20, R, L, F), mass=mass, k_outer=40)
    announce("overlap_solve 3x3x3x4 mass=0.1")
    x, st = D.solve(to_dev(b, V), tol=1e-10)
    err = rel(from_dev(x, V), ref)
    print(f"overlap_solve: rel err {err:.2e}, {st}")
    assert st["converged"] and err <= 1e-8


def test_overlap_solve_residual_at_4x4():
    """4^4, mu = 0.3, deflated: the returned x satisfies D x = b to the outer
    tolerance, checked with the oracle's D (sparse LU per pole)."""
    from paper_0910_2927_amd import api
    dims = (4, 4, 4, 4)
    V = 256
    U = si.gauge_links(dims, 0.5, 820)
    b = si.gaussian_source(12 * V, 821)
    A = dirac.hw_csr(U, dims, 0.25, 0.3)
    R, L, lam, F = deflation.lr_dense(A.toarray(), 12)
    sig, om = rational.kl_first_order(6, 1.3)
    mass = 0.05
    op = make_op(U, dims, 0.25, 0.3)
    D = api.OverlapOperator(_solver(op, V, sig, om, 20, R, L, F), mass=mass, k_outer=30)
    announce("overlap_solve 4^4 mass=0.05")
    x, st = D.solve(to_dev(b, V), tol=1e-9)
    xc = from_dev(x, V)
    res = b - overlap.overlap_apply(lambda v: xstar.xstar_sparse(A, v, sig, om, R, L, F), xc, mass)
    print(f"overlap_solve 4^4: oracle residual {np.linalg.norm(res) / np.linalg.norm(b):.2e}, {st}")
    assert st["converged"] and np.linalg.norm(res) <= 1e-8 * np.linalg.norm(b)
    assert st["restarts"] >= 1 and st["inner_matvecs"] > st["outer_iters"]


def test_overlap_solve_reports_nonconvergence():
    from paper_0910_2927_amd import api, _lib
    dims = (4, 4, 4, 4)
    V = 256
    U = si.gauge_links(dims, 0.5, 830)
    b = si.gaussian_source(12 * V, 831)
    sig, om = rational.kl_first_order(5, 1.3)
    op = make_op(U, dims, 0.25, 0.3)
    D = api.OverlapOperator(_solver(op, V, sig, om, 20), mass=0.0, k_outer=10)
    announce("overlap_solve max_outer=3 (must not converge)")
    x, st = D.solve(to_dev(b, V), tol=1e-12, max_outer=3, raise_on_error=False)
    assert st["status"] == _lib.SK_ERR_NOCONV and not st["converged"]
