"""GPU parity of the individual entry points against the CPU oracle.

Sizes span several 256-site blocks with ragged tails (3x4x5x6 = 360 sites,
5x4x3x7 = 420) as well as the paper's lattices 4^4 .. 10^4.
"""
import numpy as np
import pytest

import skinputs as si
from oracle import dirac, krylov, deflation, xstar, rational
from tests.gpu_util import make_op, to_dev, from_dev, vecs_to_dev, rel, announce, torch_dev

pytestmark = pytest.mark.gpu

DIMS = [(2, 2, 2, 2), (3, 4, 5, 6), (5, 4, 3, 7), (4, 4, 4, 4), (8, 8, 8, 8), (10, 10, 10, 10)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("mu", [0.0, 0.3])
@pytest.mark.parametrize("adjoint", [False, True])
def test_wilson_apply_c128_matches_csr(dims, mu, adjoint):
    from paper_0910_2927_amd import api
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.6, 31 + V)
    psi = si.gaussian_source(12 * V, 32 + V)
    anti = V % 2 == 0
    announce(f"wilson c128 dims={dims} mu={mu} adjoint={adjoint}")
    op = make_op(U, dims, 0.23, mu, anti)
    out = from_dev(api.wilson_apply(op, to_dev(psi, V), adjoint=adjoint), V)
    A = dirac.hw_csr(U, dims, 0.23, -mu if adjoint else mu, anti)
    ref = A @ psi
    assert np.max(np.abs(out - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("dims", [(3, 4, 5, 6), (10, 10, 10, 10)])
def test_wilson_apply_c64_matches_csr(dims):
    import torch
    from paper_0910_2927_amd import api
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.7, 41)
    psi = si.gaussian_source(12 * V, 42)
    announce(f"wilson c64 dims={dims}")
    op = make_op(U, dims, 0.25, 0.3, True, with_c64=True)
    out = from_dev(api.wilson_apply(op, to_dev(psi, V, torch.complex64)), V)
    ref = dirac.hw_csr(U, dims, 0.25, 0.3) @ psi
    # float storage: inputs rounded to 2^-24 relative, ~50 terms per row
    assert np.max(np.abs(out - ref)) <= 2e-6 * np.max(np.abs(ref))


def test_wilson_free_field_closed_form_10x4():
    from paper_0910_2927_amd import api
    dims = (10, 10, 10, 10)
    V = si.lattice_volume(dims)
    psi = si.gaussian_source(12 * V, 51)
    announce("wilson free field 10^4")
    op = make_op(si.unit_links(dims), dims, 0.25, 0.3, True)
    out = from_dev(api.wilson_apply(op, to_dev(psi, V)), V)
    ref = dirac.free_field_apply(psi, dims, 0.25, 0.3, True)
    assert rel(out, ref) < 1e-13


@pytest.mark.parametrize("dims,k", [((4, 4, 4, 4), 20), ((3, 4, 5, 6), 33)])
@pytest.mark.parametrize("mu", [0.3, 0.0])
def test_arnoldi_cycle_matches_oracle(dims, k, mu):
    from paper_0910_2927_amd import api
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.5, 61)
    b = si.gaussian_source(12 * V, 62)
    announce(f"arnoldi dims={dims} k={k} mu={mu}")
    op = make_op(U, dims, 0.25, mu, True)
    Vd, Hd, kd = api.arnoldi_cycle(op, to_dev(b, V), k)
    H = Hd.cpu().numpy()
    A = dirac.hw_csr(U, dims, 0.25, mu)
    Vo, Ho, ko = krylov.arnoldi(lambda v: A @ v, b / np.linalg.norm(b), k)
    assert kd == ko == k
    assert np.max(np.abs(H - Ho)) <= 1e-10 * np.max(np.abs(Ho))
    Vb = np.stack([from_dev(Vd[j], V) for j in range(k + 1)], axis=1)
    assert np.linalg.norm(Vb.conj().T @ Vb - np.eye(k + 1)) < 1e-12
    assert np.linalg.norm(A @ Vb[:, :k] - Vb @ H) < 1e-12 * np.linalg.norm(H)
    if mu == 0.0:
        assert np.linalg.norm(np.triu(H[:k, :k], 2)) < 1e-12


def test_arnoldi_plane_wave_breakdown():
    from paper_0910_2927_amd import api
    dims = (4, 4, 4, 4)
    V = 256
    s = np.arange(V)
    x, z, t = s % 4, (s // 16) % 4, s // 64
    ph = np.exp(1j * (np.pi / 2 * x + np.pi * z + (np.pi / 4 + np.pi / 2) * t))
    chi = si.gaussian_source(12, 15).reshape(4, 3)
    b = (ph[:, None, None] * chi[None]).reshape(-1)
    announce("arnoldi plane-wave breakdown")
    op = make_op(si.unit_links(dims), dims, 0.25, 0.3, True)
    _, Hd, kd = api.arnoldi_cycle(op, to_dev(b, V), 10)
    assert kd == 2
    assert abs(Hd.cpu().numpy()[2, 1]) == 0.0


def test_multishift_fom_restart_matches_oracle():
    import torch
    from paper_0910_2927_amd import api
    dims = (3, 4, 5, 6)
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.5, 71)
    b = si.gaussian_source(12 * V, 72)
    A = dirac.hw_csr(U, dims, 0.25, 0.3)
    k = 24
    Vo, Ho, _ = krylov.arnoldi(lambda v: A @ v, b / np.linalg.norm(b), k)
    sig, om = rational.kl_first_order(8, 1.3)
    rho0 = np.exp(1j * np.linspace(0, 1, len(sig))) * np.linspace(0.5, 2, len(sig))
    beta = 1.7
    Y, rho_new = krylov.fom_shifted(Ho, k, beta, rho0, sig)
    x0 = si.gaussian_source(12 * V, 73)
    dev = torch_dev()
    Vd = torch.stack([to_dev(Vo[:, j], V) for j in range(k)])
    Hd = torch.from_numpy(Ho).to(dev)
    betad = torch.tensor([beta], dtype=torch.float64, device=dev)
    rhod = torch.from_numpy(rho0.astype(np.complex128)).to(dev)
    xd = to_dev(x0, V)
    Xd = torch.zeros((len(sig), 12 * V), dtype=torch.complex128, device=dev)
    announce("multishift_fom_restart 3x4x5x6 k=24 N=16")
    upd = api.multishift_fom_restart(Hd, k, sig, om, betad, rhod, Vd, xd, Xd)
    u = om @ Y
    assert abs(upd - np.linalg.norm(u)) <= 1e-12 * np.linalg.norm(u)
    assert rel(rhod.cpu().numpy(), rho_new) < 1e-11
    assert rel(from_dev(xd, V), x0 + Vo[:, :k] @ u) < 1e-12
    Xo = Y @ Vo[:, :k].T
    for i in range(len(sig)):
        assert rel(from_dev(Xd[i], V), Xo[i]) < 1e-11


def test_deflate_project_matches_oracle():
    from paper_0910_2927_amd import api
    import torch
    dims = (2, 2, 3, 4)
    V = si.lattice_volume(dims)
    Ad = dirac.hw_dense(si.gauge_links(dims, 0.5, 81), dims, 0.25, 0.3)
    R, L, lam, F = deflation.lr_dense(Ad, 17)
    b = si.gaussian_source(12 * V, 82)
    announce("deflate_project 2x2x3x4 m=17")
    r, coeff, xp = api.deflate_project(vecs_to_dev(R, V), vecs_to_dev(L, V), to_dev(b, V),
                                       torch.from_numpy(F).to(torch_dev()))
    assert rel(coeff.cpu().numpy(), L.conj().T @ b) < 1e-12
    assert rel(from_dev(r, V), xstar.deflated_source(b, R, L)) < 1e-12
    assert rel(from_dev(xp, V), xstar.x_p(b, R, L, F)) < 1e-12


# 11 x 12 x 13 x 14 = 24 024 sites: 376 stencil blocks of 64 sites, so the
# first 256 run in the per-XCD order and the rest (with a ragged last block)
# in plain order; n = 288 288 rows fills the update grid with one lane per
# row pack in both precisions (the smaller lattices above take two).
BIG = (11, 12, 13, 14)


@pytest.mark.parametrize("adjoint", [False, True])
def test_wilson_apply_renumbered_blocks(adjoint):
    import torch
    from paper_0910_2927_amd import api
    V = si.lattice_volume(BIG)
    U = si.gauge_links(BIG, 0.7, 71)
    psi = si.gaussian_source(12 * V, 72)
    A = dirac.hw_csr(U, BIG, 0.25, -0.3 if adjoint else 0.3)
    ref = A @ psi
    announce(f"wilson 11x12x13x14 adjoint={adjoint}")
    op = make_op(U, BIG, 0.25, 0.3, True, with_c64=True)
    out = from_dev(api.wilson_apply(op, to_dev(psi, V), adjoint=adjoint), V)
    assert rel(out, ref) < 1e-14
    out64 = from_dev(api.wilson_apply(op, to_dev(psi, V, torch.complex64), adjoint=adjoint), V)
    assert np.max(np.abs(out64 - ref)) <= 2e-6 * np.max(np.abs(ref))   # float storage


def test_arnoldi_cycle_one_lane_update_path():
    import torch
    from paper_0910_2927_amd import api
    V = si.lattice_volume(BIG)
    k = 12
    U = si.gauge_links(BIG, 0.7, 73)
    b = si.gaussian_source(12 * V, 74)
    A = dirac.hw_csr(U, BIG, 0.25, 0.3)
    Vo, Ho, ko = krylov.arnoldi(lambda v: A @ v, b / np.linalg.norm(b), k)
    announce(f"arnoldi 11x12x13x14 k={k} complex double and complex float")
    op = make_op(U, BIG, 0.25, 0.3, True, with_c64=True)
    for dt, tol_h, tol_o in ((torch.complex128, 1e-10, 1e-12), (torch.complex64, 1e-5, 1e-5)):
        Vd, Hd, kd = api.arnoldi_cycle(op, to_dev(b, V, dt), k)
        H = Hd.cpu().numpy()
        assert kd == ko == k
        err_h = np.max(np.abs(H - Ho)) / np.max(np.abs(Ho))
        Vb = np.stack([from_dev(Vd[j], V) for j in range(k + 1)], axis=1)
        err_o = np.linalg.norm(Vb.conj().T @ Vb - np.eye(k + 1))
        err_r = np.linalg.norm(A @ Vb[:, :k] - Vb @ H) / np.linalg.norm(H)
        print(f"{dt}: H {err_h:.1e}, orthonormality {err_o:.1e}, Arnoldi relation {err_r:.1e}")
        assert err_h <= tol_h and err_o < tol_o and err_r < tol_o


def test_singular_shifted_hessenberg_is_reported():
    """Forced from the host: a Hessenberg matrix whose shifted leading block
    H_k - sigma_0 I is exactly singular (zero first column), passed to the
    per-cycle multishift step; the library must return SK_ERR_SINGULAR and
    not a non-finite iterate."""
    import torch
    from paper_0910_2927_amd import api, _lib
    dev = torch_dev()
    k, n = 2, 12 * 16
    H = torch.zeros((k + 1, k), dtype=torch.complex128)
    H[0, 0], H[1, 1], H[2, 1] = 1.0, 2.0, 0.5          # h_{2,1} = 0
    sig = np.array([1.0 + 0j, 3.0 + 0j])
    om = np.array([0.5 + 0j, 0.5 + 0j])
    Vb = torch.from_numpy(np.linalg.qr(si.gaussian_source(n * k, 90).reshape(n, k))[0].T.copy()).to(dev)
    beta = torch.tensor([1.0], dtype=torch.float64, device=dev)
    rho = torch.ones(2, dtype=torch.complex128, device=dev)
    x = torch.zeros(n, dtype=torch.complex128, device=dev)
    announce("multishift_fom_restart with a singular shifted H_k")
    with pytest.raises(_lib.SkError) as e:
        api.multishift_fom_restart(H.to(dev), k, sig, om, beta, rho, Vb, x)
    assert e.value.status == _lib.SK_ERR_SINGULAR
