"""The direct projection methods of Sect. 6 (eq. (direct)):
x_k = x_P + ||(I-P)b|| V_k sign(M_k) e_1 with M_k = H_k (Arnoldi) or the
two-sided Lanczos T_k ("2sL" of Fig. 1), sign(M_k) by Roberts' Newton
iteration on the device, against the oracle's same construction, and the
approximation error against the dense sign(A) b decreasing with k."""
import numpy as np
import pytest

import skinputs as si
from oracle import dirac, direct, signfun, deflation, rational
from tests.gpu_util import make_op, to_dev, from_dev, vecs_to_dev, rel, announce, torch_dev

pytestmark = pytest.mark.gpu


def _setup(dims, seed, m=0, mu=0.3):
    import torch
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.5, seed)
    b = si.gaussian_source(12 * V, seed + 1)
    A = dirac.hw_csr(U, dims, 0.25, mu)
    AH = dirac.hw_csr(U, dims, 0.25, -mu)
    defl = dev = None
    if m:
        R, L, lam, F = deflation.lr_dense(A.toarray(), m)
        defl = (R, L, F)
        dev = (vecs_to_dev(R, V), vecs_to_dev(L, V), torch.from_numpy(F).to(torch_dev()))
    return V, U, b, A, AH, defl, dev


@pytest.mark.parametrize("dims,k,m", [((4, 4, 4, 4), 20, 0), ((4, 4, 4, 4), 60, 10),
                                      ((3, 4, 5, 6), 33, 12), ((4, 4, 4, 4), 128, 0)])
def test_direct_arnoldi_matches_oracle(dims, k, m):
    from paper_0910_2927_amd import api
    V, U, b, A, AH, defl, dev = _setup(dims, 600 + k, m)
    R, L, F = defl if m else (None, None, None)
    ref, info = direct.arnoldi_direct(lambda v: A @ v, b, k, R, L, F)
    op = make_op(U, dims, 0.25, 0.3)
    announce(f"direct_sign_apply arnoldi dims={dims} k={k} m={m}")
    kw = dict(R=dev[0], Lv=dev[1], F=dev[2]) if m else {}
    x, st, S = api.direct_sign_apply(op, to_dev(b, V), k, "arnoldi", return_sign=True, **kw)
    err = rel(from_dev(x, V), ref)
    eS = rel(S.cpu().numpy(), info["S"])
    print(f"arnoldi k={k} m={m}: rel err {err:.2e}, sign(H_k) {eS:.2e}, newton {st['newton_iters']} its")
    assert st["k_done"] == info["k"] == k
    assert err <= 1e-9 and eS <= 1e-9


@pytest.mark.parametrize("dims,k,m", [((4, 4, 4, 4), 20, 0), ((4, 4, 4, 4), 40, 10),
                                      ((3, 4, 5, 6), 30, 12)])
def test_direct_lanczos_matches_oracle(dims, k, m):
    from paper_0910_2927_amd import api
    V, U, b, A, AH, defl, dev = _setup(dims, 700 + k, m)
    R, L, F = defl if m else (None, None, None)
    ref, info = direct.lanczos_direct(lambda v: A @ v, lambda v: AH @ v, b, k, R, L, F)
    op = make_op(U, dims, 0.25, 0.3)
    announce(f"direct_sign_apply lanczos dims={dims} k={k} m={m}")
    kw = dict(R=dev[0], Lv=dev[1], F=dev[2]) if m else {}
    x, st, S = api.direct_sign_apply(op, to_dev(b, V), k, "lanczos", return_sign=True, **kw)
    err = rel(from_dev(x, V), ref)
    eS = rel(S.cpu().numpy(), info["S"])
    print(f"lanczos k={k} m={m}: rel err {err:.2e}, sign(T_k) {eS:.2e}, newton {st['newton_iters']} its")
    assert st["k_done"] == info["k"] == k
    assert err <= 1e-8 and eS <= 1e-8


def test_direct_methods_converge_to_dense_sign():
    """The approximation error against sign(A) b (dense sorted-Schur sign)
    decreases with k for both direct methods, with deflation."""
    from paper_0910_2927_amd import api
    dims = (4, 4, 4, 4)
    V, U, b, A, AH, defl, dev = _setup(dims, 640, 16)
    ex = signfun.sign_schur(A.toarray()) @ b
    op = make_op(U, dims, 0.25, 0.3)
    errs = {"arnoldi": [], "lanczos": []}
    for k in (20, 60, 120):
        for mth in errs:
            announce(f"direct {mth} k={k} vs dense sign")
            x, st = api.direct_sign_apply(op, to_dev(b, V), k, mth, R=dev[0], Lv=dev[1], F=dev[2])
            errs[mth].append(rel(from_dev(x, V), ex))
    print("error vs dense sign(A) b at k = 20, 60, 120:", errs)
    for mth, e in errs.items():
        assert e[0] > e[1] > e[2], mth
    assert errs["arnoldi"][-1] < 1e-3


def test_direct_hermitian_limit_lanczos_equals_arnoldi():
    """mu = 0, no deflation: H_W is Hermitian, two-sided Lanczos with
    w_1 = v_1 is Hermitian Lanczos and T_k = H_k, so both direct methods
    give the same x_k."""
    from paper_0910_2927_amd import api
    dims = (4, 4, 4, 4)
    V, U, b, A, AH, _, _ = _setup(dims, 650, 0, mu=0.0)
    op = make_op(U, dims, 0.25, 0.0)
    announce("direct arnoldi vs lanczos at mu=0")
    xa, _ = api.direct_sign_apply(op, to_dev(b, V), 30, "arnoldi")
    xl, _ = api.direct_sign_apply(op, to_dev(b, V), 30, "lanczos")
    assert rel(from_dev(xl, V), from_dev(xa, V)) < 1e-10


def test_direct_plane_wave_is_exact_after_two_steps():
    """Free field: the Krylov space of a plane wave has dimension 2, both
    methods stop there and give sign(H(p)) b exactly (closed form)."""
    from paper_0910_2927_amd import api
    dims = (4, 4, 4, 4)
    V = 256
    chi = si.gaussian_source(12, 15).reshape(4, 3)
    s = np.arange(V)
    x_, z_, t_ = s % 4, (s // 16) % 4, s // 64
    ph = np.exp(1j * (2 * np.pi / 4 * x_ + np.pi * z_ + (np.pi / 4 + np.pi / 2) * t_))
    b = (ph[:, None, None] * chi[None]).reshape(-1)
    ref = dirac.free_field_function(b, dims, 0.25, 0.3, lambda l: np.sign(l.real))
    op = make_op(si.unit_links(dims), dims, 0.25, 0.3)
    for mth in ("arnoldi", "lanczos"):
        announce(f"direct {mth} plane wave")
        x, st = api.direct_sign_apply(op, to_dev(b, V), 10, mth)
        assert st["k_done"] == 2 and st["breakdown"]
        assert rel(from_dev(x, V), ref) < 1e-12
