"""Pins for the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: textbook
identities (Clifford algebra, gauge covariance, sign(A)^2 = I), closed forms
(free field in momentum space, Kenney-Laub closed form), special cases
(mu = 0 Hermitian limit, Arnoldi breakdown on a plane wave) and brute force
on tiny lattices.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import skinputs as si
from oracle import dirac, rational, signfun, xstar, krylov, deflation

RAGGED = (3, 4, 5, 6)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


# ---------------------------------------------------------------- gamma algebra
def test_gamma_clifford_and_gamma5():
    g = dirac.gammas()
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            ac = g[a] @ g[b] + g[b] @ g[a]
            assert np.allclose(ac, 2 * np.eye(4) * (a == b))
    g5 = dirac.gamma5()
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))
    for a in range(4):
        assert np.allclose(g5 @ g[a] + g[a] @ g5, 0)


# ---------------------------------------------------------------- Kenney-Laub
@pytest.mark.parametrize("s", [3, 5, 8, 10])
def test_kl_partial_fractions_match_closed_form(s):
    rng = np.random.default_rng(s)
    t = rng.normal(size=200) * 2 + 1j * rng.normal(size=200) * 2
    t = t[np.abs(t.real) > 0.05]
    g0 = rational.kl_closed_form(t, s)
    g1 = rational.kl_t2_form(t, s)
    sig, om = rational.kl_first_order(s, 1.0)
    g2 = rational.g_first_order(t, sig, om)
    assert np.max(np.abs(g1 - g0)) < 1e-12
    assert np.max(np.abs(g2 - g0)) < 1e-12
    # scaled form: g_s(c x) from first-order poles at +-i tau/c, weights w/(2c)
    c = 0.37
    sig, om = rational.kl_first_order(s, c)
    assert np.max(np.abs(rational.g_first_order(t, sig, om) - rational.kl_closed_form(c * t, s))) < 1e-12


@pytest.mark.parametrize("s", [4, 8])
def test_kl_structural_identities(s):
    t = np.array([0.3 + 0.2j, 1.7 - 0.4j, 5.0 + 1.0j, -2.0 + 0.1j])
    g = lambda u: rational.kl_closed_form(u, s)
    assert abs(g(np.array([1.0]))[0] - 1) < 1e-15        # g_s(1) = 1
    assert np.allclose(g(-t), -g(t))                     # odd
    assert np.allclose(g(1 / t), g(t))                   # g_s(1/t) = g_s(t)
    sig, om = rational.kl_first_order(s)
    assert np.allclose(np.sort_complex(sig.conj()), np.sort_complex(sig))  # conjugation closed
    assert np.allclose(om.imag, 0)
    # sign-like: approaches +-1 exponentially in s on the positive / negative axis
    x = np.linspace(0.2, 5, 50)
    assert np.max(np.abs(rational.kl_closed_form(x, 40) - 1)) < 1e-10


# ---------------------------------------------------------------- Wilson operator
@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), RAGGED])
@pytest.mark.parametrize("mu", [0.0, 0.3])
@pytest.mark.parametrize("anti", [True, False])
def test_free_field_csr_matches_momentum_space(dims, mu, anti):
    V = si.lattice_volume(dims)
    A = dirac.hw_csr(si.unit_links(dims), dims, 0.25, mu, anti)
    psi = si.gaussian_source(12 * V, 5)
    ff = dirac.free_field_apply(psi, dims, 0.25, mu, anti)
    assert rel(A @ psi, ff) < 1e-13


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), RAGGED])
def test_gamma5_hermiticity_and_mu_zero_limit(dims):
    U = si.gauge_links(dims, 0.5, 11)
    A = dirac.hw_csr(U, dims, 0.2, 0.3)
    B = dirac.hw_csr(U, dims, 0.2, -0.3)
    assert abs(A.conj().T - B).max() < 1e-15        # H(mu)^H = H(-mu)
    A0 = dirac.hw_csr(U, dims, 0.2, 0.0)
    assert abs(A0.conj().T - A0).max() < 1e-15       # Hermitian at mu = 0
    assert abs(A - A.conj().T).max() > 1e-3          # and not at mu != 0


def _random_su3_field(V, seed):
    return si.gauge_links((V, 1, 1, 1), 1.3, seed)[:, 0]


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), RAGGED])
def test_gauge_covariance(dims):
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.7, 3)
    Om = _random_su3_field(V, 4)                      # Omega(x)
    fwd, _, _, _ = dirac.neighbours(dims)
    Ug = np.einsum("sab,snbc,sndc->snad", Om, U, Om[fwd].conj())  # Om(x) U Om(x+nu)^+
    psi = si.gaussian_source(12 * V, 6).reshape(V, 4, 3)
    gpsi = np.einsum("sab,sib->sia", Om, psi).reshape(-1)
    A = dirac.hw_csr(U, dims, 0.21, 0.4)
    Ag = dirac.hw_csr(Ug, dims, 0.21, 0.4)
    lhs = Ag @ gpsi
    rhs = np.einsum("sab,sib->sia", Om, (A @ psi.reshape(-1)).reshape(V, 4, 3)).reshape(-1)
    assert rel(lhs, rhs) < 1e-13


def test_direct_site_loop_matches_csr_2x4():
    """Brute force on 2x2x2x2 plus one odd extent: H_W applied by explicit
    Python loops over sites and directions (a second, unvectorised reading
    of the definition) equals the CSR matrix."""
    dims = (2, 3, 2, 2)
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.6, 21)
    psi = si.gaussian_source(12 * V, 22).reshape(V, 4, 3)
    kappa, mu = 0.23, 0.35
    g = dirac.gammas()
    g5 = dirac.gamma5()
    Lx, Ly, Lz, Lt = dims
    out = np.zeros_like(psi)
    for t in range(Lt):
        for z in range(Lz):
            for y in range(Ly):
                for x in range(Lx):
                    s = ((t * Lz + z) * Ly + y) * Lx + x
                    acc = psi[s].copy()
                    c = [x, y, z, t]
                    for nu in range(4):
                        cf = list(c); cf[nu] = (c[nu] + 1) % dims[nu]
                        cb = list(c); cb[nu] = (c[nu] - 1) % dims[nu]
                        sf = ((cf[3] * Lz + cf[2]) * Ly + cf[1]) * Lx + cf[0]
                        sb = ((cb[3] * Lz + cb[2]) * Ly + cb[1]) * Lx + cb[0]
                        ef = np.exp(mu) if nu == 3 else 1.0
                        eb = np.exp(-mu) if nu == 3 else 1.0
                        if nu == 3 and c[3] == Lt - 1:
                            ef = -ef
                        if nu == 3 and c[3] == 0:
                            eb = -eb
                        hop_f = (np.eye(4) - g[nu]) @ (U[s, nu] @ psi[sf].T).T
                        hop_b = (np.eye(4) + g[nu]) @ (U[sb, nu].conj().T @ psi[sb].T).T
                        acc = acc - kappa * (ef * hop_f + eb * hop_b)
                    out[s] = g5 @ acc
    A = dirac.hw_csr(U, dims, kappa, mu)
    assert rel(A @ psi.reshape(-1), out.reshape(-1)) < 1e-14


# ---------------------------------------------------------------- sign function
@pytest.fixture(scope="module")
def small_hw():
    dims = (2, 2, 2, 2)
    U = si.gauge_links(dims, 0.5, 2007)
    return dirac.hw_dense(U, dims, 0.25, 0.3), dims, U


def test_sign_schur_newton_eig_agree(small_hw):
    A, _, _ = small_hw
    S1 = signfun.sign_schur(A)
    S2 = signfun.sign_newton(A)
    S3 = signfun.sign_eig(A)
    assert rel(S1, S2) < 1e-12
    assert rel(S1, S3) < 1e-10
    n = A.shape[0]
    assert np.linalg.norm(S1 @ S1 - np.eye(n)) / np.sqrt(n) < 1e-12
    assert np.linalg.norm(S1 @ A - A @ S1) / np.linalg.norm(A) < 1e-12


def test_sign_mu_zero_limit_is_eigh():
    dims = (2, 2, 2, 2)
    A = dirac.hw_dense(si.gauge_links(dims, 0.5, 9), dims, 0.25, 0.0)
    w, W = np.linalg.eigh(A)
    ref = (W * np.sign(w)) @ W.conj().T
    assert rel(signfun.sign_schur(A), ref) < 1e-12
    assert rel(signfun.sign_newton(A), ref) < 1e-12


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 3, 2, 4)])
def test_free_field_sign_closed_form(dims):
    V = si.lattice_volume(dims)
    A = dirac.hw_dense(si.unit_links(dims), dims, 0.25, 0.3)
    b = si.gaussian_source(12 * V, 7)
    ref = dirac.free_field_function(b, dims, 0.25, 0.3, lambda l: np.sign(l.real))
    assert rel(signfun.sign_schur(A) @ b, ref) < 1e-12


# ---------------------------------------------------------------- x* and rational g
def test_xstar_free_field_closed_form_4x4():
    dims = (4, 4, 4, 4)
    V = si.lattice_volume(dims)
    A = dirac.hw_dense(si.unit_links(dims), dims, 0.25, 0.3)
    b = si.gaussian_source(12 * V, 8)
    s, c = 5, 0.8
    sig, om = rational.kl_first_order(s, c)
    x = xstar.xstar_dense(A, b, sig, om)
    ref = dirac.free_field_function(b, dims, 0.25, 0.3, lambda l: rational.kl_closed_form(c * l, s))
    assert rel(x, ref) < 1e-12
    # sparse LU route agrees too
    Asp = dirac.hw_csr(si.unit_links(dims), dims, 0.25, 0.3)
    assert rel(xstar.xstar_sparse(Asp, b, sig, om), ref) < 1e-12


def test_xstar_brute_force_2x4(small_hw):
    """At 2^4 compute g(A) b from the eigendecomposition and compare."""
    A, dims, _ = small_hw
    b = si.gaussian_source(A.shape[0], 9)
    sig, om = rational.kl_first_order(5, 0.9)
    lam, W = np.linalg.eig(A)
    ref = W @ (rational.g_first_order(lam, sig, om) * np.linalg.solve(W, b))
    assert rel(xstar.xstar_dense(A, b, sig, om), ref) < 1e-11


# ---------------------------------------------------------------- deflation
def test_lr_deflation_projector_properties(small_hw):
    A, _, _ = small_hw
    R, L, lam, F = deflation.lr_dense(A, 12)
    P = R @ L.conj().T
    assert np.linalg.norm(P @ P - P) < 1e-11
    assert np.linalg.norm(A @ P - P @ A) / np.linalg.norm(A) < 1e-11
    assert np.linalg.norm(L.conj().T @ R - np.eye(12)) < 1e-11
    res_r, res_l, bi = deflation.projector_checks(A, R, L, lam)
    assert max(res_r, res_l, bi) < 1e-11
    # the selected eigenvalues are the 12 of smallest modulus
    allv = np.sort(np.abs(np.linalg.eigvals(A)))
    assert np.allclose(np.sort(np.abs(lam)), allv[:12])
    # x_P = sign(A) P b exactly
    b = si.gaussian_source(A.shape[0], 10)
    assert rel(xstar.x_p(b, R, L, F), signfun.sign_schur(A) @ (P @ b)) < 1e-11


def test_deflated_xstar_equals_sign_on_deflated_part(small_hw):
    """Deflating every eigenvalue makes x* = sign(A) b exactly."""
    A, _, _ = small_hw
    n = A.shape[0]
    R, L, lam, F = deflation.lr_dense(A, n - 1)
    b = si.gaussian_source(n, 12)
    sig, om = rational.kl_first_order(8, 1.0)
    x = xstar.xstar_dense(A, b, sig, om, R, L, F)
    # remaining one-dimensional part is handled by g: compare on the split
    P = R @ L.conj().T
    ref = signfun.sign_schur(A) @ (P @ b) + xstar.xstar_dense(A, b - P @ b, sig, om)
    assert rel(x, ref) < 1e-11


# ---------------------------------------------------------------- Krylov
def test_arnoldi_relation_and_hermitian_limit():
    dims = (2, 2, 2, 4)
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.5, 13)
    b = si.gaussian_source(12 * V, 14)
    for mu in (0.3, 0.0):
        A = dirac.hw_csr(U, dims, 0.25, mu)
        Vb, H, kk = krylov.arnoldi(lambda v: A @ v, b / np.linalg.norm(b), 15)
        assert kk == 15
        assert np.linalg.norm(Vb.conj().T @ Vb - np.eye(16)) < 1e-13
        assert np.linalg.norm(A @ Vb[:, :15] - Vb @ H) < 1e-13
        if mu == 0.0:
            Hk = H[:15, :15]
            assert np.linalg.norm(np.triu(Hk, 2)) < 1e-12      # tridiagonal
            assert np.linalg.norm(Hk - Hk.conj().T) < 1e-12
        else:
            assert np.linalg.norm(np.triu(H[:15, :15], 2)) > 1e-3


def test_plane_wave_breaks_down_at_step_two():
    """Free field: H(p)^2 = lam^2, so K(H, e^{ipx} chi) has dimension 2."""
    dims = (4, 4, 4, 4)
    V = si.lattice_volume(dims)
    n = 12 * V
    A = dirac.hw_csr(si.unit_links(dims), dims, 0.25, 0.3)
    chi = si.gaussian_source(12, 15).reshape(4, 3)
    # momentum p = (2pi/4, 0, 2pi*2/4, pi/4 + 2pi/4) with antiperiodic time
    Lx, Ly, Lz, Lt = dims
    s = np.arange(V)
    x, y, z, t = s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)
    ph = np.exp(1j * (2 * np.pi / 4 * x + np.pi * z + (np.pi / 4 + np.pi / 2) * t))
    b = (ph[:, None, None] * chi[None]).reshape(-1)
    Vb, H, kk = krylov.arnoldi(lambda v: A @ v, b / np.linalg.norm(b), 10)
    assert kk == 2
    sig, om = rational.kl_first_order(5, 0.7)
    x_rs, info = krylov.restarted_fom_lr(lambda v: A @ v, b, sig, om, k=10)
    assert info["converged"] and info["cycles"] == 1
    ref = dirac.free_field_function(b, dims, 0.25, 0.3, lambda l: rational.kl_closed_form(0.7 * l, 5))
    assert rel(x_rs, ref) < 1e-12


@pytest.mark.parametrize("k", [8, 12, 40])
def test_restarted_fom_converges_to_xstar_any_k(k):
    dims = (2, 2, 3, 4)
    V = si.lattice_volume(dims)
    A = dirac.hw_csr(si.gauge_links(dims, 0.5, 16), dims, 0.25, 0.3)
    b = si.gaussian_source(12 * V, 17)
    sig, om = rational.kl_first_order(5, 0.9)
    ref = xstar.xstar_dense(A.toarray(), b, sig, om)
    x, info = krylov.restarted_fom_lr(lambda v: A @ v, b, sig, om, k=k, tol_update=1e-12)
    assert info["converged"]
    assert rel(x, ref) < 1e-10
    # collinear residuals: true per-shift residuals are rho_i * r
    x2, info2 = krylov.restarted_fom_lr(lambda v: A @ v, b, sig, om, k=k, max_cycles=2,
                                         keep_shift_solutions=True)
    X = info2["X"]
    res = [b - (A @ X[i] - sig[i] * X[i]) for i in range(len(sig))]
    r0 = res[0] / np.linalg.norm(res[0])
    for ri in res[1:]:
        # the part of r_i off the common direction is rounding-sized
        off = ri - np.vdot(r0, ri) * r0
        assert np.linalg.norm(off) < 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(res[0]) > 1e-8 * np.linalg.norm(b)   # not yet converged


def test_restarted_fom_short_cycle_divergence_is_reported():
    """Restarted FOM with k = 5 diverges on this indefinite spectrum (both
    half-planes occupied): the loop must stop and report non-convergence."""
    dims = (2, 2, 3, 4)
    V = si.lattice_volume(dims)
    A = dirac.hw_csr(si.gauge_links(dims, 0.5, 16), dims, 0.25, 0.3)
    b = si.gaussian_source(12 * V, 17)
    sig, om = rational.kl_first_order(5, 0.9)
    with np.errstate(all="ignore"):
        x, info = krylov.restarted_fom_lr(lambda v: A @ v, b, sig, om, k=5, max_cycles=2000)
    assert not info["converged"]


def test_restarted_fom_lr_with_deflation_matches_xstar():
    dims = (2, 2, 3, 4)
    V = si.lattice_volume(dims)
    Ad = dirac.hw_dense(si.gauge_links(dims, 0.5, 18), dims, 0.25, 0.3)
    b = si.gaussian_source(12 * V, 19)
    R, L, lam, F = deflation.lr_dense(Ad, 10)
    sig, om = rational.kl_first_order(8, 0.9)
    ref = xstar.xstar_dense(Ad, b, sig, om, R, L, F)
    x, info = krylov.restarted_fom_lr(lambda v: Ad @ v, b, sig, om, k=8, R=R, L=L, F=F,
                                       tol_update=1e-12)
    assert info["converged"]
    assert rel(x, ref) < 1e-10


def test_unrestarted_multishift_fom_matches_dense():
    dims = (2, 2, 3, 4)
    V = si.lattice_volume(dims)
    A = dirac.hw_csr(si.gauge_links(dims, 0.5, 20), dims, 0.25, 0.3)
    b = si.gaussian_source(12 * V, 21)
    sig, om = rational.kl_first_order(8, 0.9)
    x, X, k = krylov.multishift_fom_unrestarted(lambda v: A @ v, b, sig, om, tol=1e-13)
    ref, Xref = xstar.xstar_dense(A.toarray(), b, sig, om, return_shifts=True)
    assert rel(x, ref) < 1e-11
    assert rel(X, Xref) < 1e-11


# ---------------------------------------------------------------- gradient
def test_oracle_gradient_matches_finite_differences_2x4():
    """The dense gradient formula against central differences of F with
    exponentiated links, on coordinates of every direction, and dF/dmu
    against a central difference in mu."""
    from oracle import gradient
    dims = (2, 2, 2, 2)
    V = 16
    U = si.gauge_links(dims, 0.5, 500)
    b = si.gaussian_source(12 * V, 501)
    eta = si.gaussian_source(12 * V, 502)
    sig, om = rational.kl_first_order(4, 1.2)
    coords = [(0, 3, 0), (1, 7, 1), (2, 11, 4), (3, 0, 7), (3, 15, 2), (0, 9, 6)]
    grad, gmu = gradient.dense_gradient(U, dims, 0.25, 0.3, b, eta, sig, om, coords=coords)
    for c in coords:
        fd = gradient.fd_link(U, dims, 0.25, 0.3, b, eta, sig, om, *c, h=1e-5)
        assert abs(fd - grad[c]) <= 1e-7 * max(1.0, abs(fd)), (c, fd, grad[c])
    h = 1e-5
    fdmu = (gradient.objective(U, dims, 0.25, 0.3 + h, b, eta, sig, om)
            - gradient.objective(U, dims, 0.25, 0.3 - h, b, eta, sig, om)) / (2 * h)
    assert abs(fdmu - gmu) <= 1e-7 * max(1.0, abs(fdmu))
    # the directional form agrees with the coordinate gradient
    theta = np.zeros((4, V, 8))
    for c in coords:
        theta[c] = 0.7 + 0.1 * c[2]
    dd = gradient.directional_dense(U, dims, 0.25, 0.3, b, eta, sig, om, theta)
    assert abs(dd - sum(theta[c] * grad[c] for c in coords)) < 1e-10 * max(1, abs(dd))


# ---------------------------------------------------------------- ARPACK deflation vs dense
@pytest.mark.parametrize("dims,m", [((4, 4, 4, 4), 10), (RAGGED, 16)])
def test_lr_arpack_matches_dense_eig(dims, m):
    """Sect. 4: the sparse route (ARPACK on A^2, left vectors from A^H, pairing
    by conjugate eigenvalue, L <- L (R^H L)^{-1}) selects the same eigenvalues
    as a dense eigendecomposition and builds the same oblique projector
    P = R L^H and deflated start x_P = R sign(Lambda) L^H b, for both
    selection keys (|lambda| and |Re lambda|).  P and x_P are unique
    (eigenvector phases and scales cancel), so they are compared directly;
    a wrong pairing of left with right vectors, a wrong selection or a
    missing biorthonormalisation changes them at O(1)."""
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.5, 31)
    A = dirac.hw_csr(U, dims, 0.25, 0.3)
    AH = dirac.hw_csr(U, dims, 0.25, -0.3)
    eig = np.linalg.eig(A.toarray())
    rng = np.random.default_rng(7)
    Z = rng.standard_normal((12 * V, 4)) + 1j * rng.standard_normal((12 * V, 4))
    b = si.gaussian_source(12 * V, 32)
    for key in ("abs", "re"):
        Rd, Ld, lamd, Fd = deflation.lr_dense(A.toarray(), m, key=key, eig=eig)
        Ra, La, lama, Fa = deflation.lr_arpack(A, AH, m, key=key, extra=12)
        # same eigenvalue set
        sd = np.sort_complex(lamd)
        sa = np.sort_complex(lama)
        assert np.max(np.abs(sd - sa)) < 1e-10 * np.max(np.abs(sd)), key
        # biorthonormal and an invariant pair
        assert np.linalg.norm(La.conj().T @ Ra - np.eye(m)) < 1e-10
        res_r, res_l, _ = deflation.projector_checks(A, Ra, La, lama)
        assert max(res_r, res_l) < 1e-10
        # same projector, applied to random vectors; same deflated start
        assert rel(Ra @ (La.conj().T @ Z), Rd @ (Ld.conj().T @ Z)) < 1e-10, key
        assert rel(xstar.x_p(b, Ra, La, Fa), xstar.x_p(b, Rd, Ld, Fd)) < 1e-10, key
    # the two keys really select different sets on this spectrum
    s_abs = np.sort_complex(deflation.lr_dense(A.toarray(), m, key="abs", eig=eig)[2])
    s_re = np.sort_complex(deflation.lr_dense(A.toarray(), m, key="re", eig=eig)[2])
    assert np.max(np.abs(s_abs - s_re)) > 1e-3


def test_lr_arpack_pairing_survives_shuffled_left_vectors(monkeypatch):
    """The pairing of left with right vectors must follow the eigenvalues,
    not the order ARPACK returns them in: reverse the left set and the
    projector must not change."""
    dims = (4, 4, 4, 4)
    U = si.gauge_links(dims, 0.5, 33)
    A = dirac.hw_csr(U, dims, 0.25, 0.3)
    AH = dirac.hw_csr(U, dims, 0.25, -0.3)
    Ra, La, lama, _ = deflation.lr_arpack(A, AH, 10, extra=10)
    orig = deflation._arpack_sq
    calls = {"n": 0}

    def shuffled(M, m, extra, tol):
        lam, vec, mu2 = orig(M, m, extra, tol)
        calls["n"] += 1
        if calls["n"] == 2:                       # the left (A^H) solve
            return lam[::-1], vec[:, ::-1], mu2[::-1]
        return lam, vec, mu2

    monkeypatch.setattr(deflation, "_arpack_sq", shuffled)
    Rb, Lb, lamb, _ = deflation.lr_arpack(A, AH, 10, extra=10)
    z = si.gaussian_source(A.shape[0], 34)
    assert rel(Rb @ (Lb.conj().T @ z), Ra @ (La.conj().T @ z)) < 1e-10


@pytest.mark.parametrize("anti", [True, False])
def test_exact_mu_derivative_of_hw(anti):
    """dH_W/dmu written from the definition (only the time hops carry mu)
    against a central difference of the matrix itself, and against the
    free-field symbol's derivative in momentum space."""
    dims = RAGGED
    U = si.gauge_links(dims, 0.6, 41)
    mu, h = 0.3, 1e-5
    dH = dirac.hw_csr(U, dims, 0.25, mu, anti, d_mu=True)
    fd = (dirac.hw_csr(U, dims, 0.25, mu + h, anti) - dirac.hw_csr(U, dims, 0.25, mu - h, anti)) / (2 * h)
    assert abs(dH - fd).max() < 1e-9
    assert abs(dH).max() > 0.1
    # derivative is nonzero only on time hops: zero spatial links leave it unchanged
    U0 = U.copy()
    U0[:, :3] = 0
    assert abs(dirac.hw_csr(U0, dims, 0.25, mu, anti, d_mu=True) - dH).max() == 0.0


# ---------------------------------------------------------------- direct projection methods
def test_direct_arnoldi_full_space_is_exact(small_hw):
    """eq. (direct) with the whole space (k = n, 2^4) is sign(A) b exactly;
    with deflation too (the deflated part is x_P exactly)."""
    from oracle import direct
    A, _, _ = small_hw
    n = A.shape[0]
    b = si.gaussian_source(n, 60)
    ex = signfun.sign_schur(A) @ b
    x, info = direct.arnoldi_direct(lambda v: A @ v, b, n)
    assert rel(x, ex) < 1e-12
    R, L, lam, F = deflation.lr_dense(A, 20)
    # (I - P) b lies in an invariant subspace of dimension n - 20
    x, info = direct.arnoldi_direct(lambda v: A @ v, b, n - 20, R, L, F)
    assert rel(x, ex) < 1e-11


def test_two_sided_lanczos_relations_and_hermitian_limit(small_hw):
    from oracle import direct
    A, dims, U = small_hw
    n = A.shape[0]
    b = si.gaussian_source(n, 61)
    v1 = b / np.linalg.norm(b)
    w1 = si.gaussian_source(n, 62)
    V, W, T, kk = direct.two_sided_lanczos(lambda v: A @ v, lambda v: A.conj().T @ v, v1, w1, 15)
    assert kk == 15
    assert np.linalg.norm(W.conj().T @ V - np.eye(16)) < 1e-10          # biorthogonal
    assert np.linalg.norm(A @ V[:, :15] - V @ T) < 1e-12 * np.linalg.norm(A)
    assert np.linalg.norm(np.triu(T[:15, :15], 2)) == 0 and np.linalg.norm(np.tril(T, -2)) == 0
    # mu = 0, w_1 = v_1: Hermitian Lanczos, which is Arnoldi (unique H_k)
    A0 = dirac.hw_dense(U, dims, 0.25, 0.0)
    V, W, T, kk = direct.two_sided_lanczos(lambda v: A0 @ v, lambda v: A0.conj().T @ v, v1, v1, 25)
    Va, H, ka = krylov.arnoldi(lambda v: A0 @ v, v1, 25)
    assert np.abs(T - H).max() < 1e-13 and np.abs(V - Va).max() < 1e-12


def test_lanczos_left_space_avoids_the_deflated_left_subspace(small_hw):
    """With LR deflation the left start (I - L R^H) v_1 keeps R^H W = 0
    (A^H maps ker R^H into itself), the right space keeps L^H V = 0."""
    from oracle import direct
    A, _, _ = small_hw
    n = A.shape[0]
    R, L, lam, F = deflation.lr_dense(A, 12)
    b = si.gaussian_source(n, 63)
    x, info = direct.lanczos_direct(lambda v: A @ v, lambda v: A.conj().T @ v, b, 20, R, L, F)
    assert np.linalg.norm(R.conj().T @ info["W"]) < 1e-10
    assert np.linalg.norm(L.conj().T @ info["V"]) < 1e-10
    assert abs(np.vdot(info["W"][:, 0], info["V"][:, 0]) - 1) < 1e-13


def test_direct_methods_on_a_plane_wave():
    """Free field: both direct methods stop after 2 steps with the exact
    momentum-space sign."""
    from oracle import direct
    dims = (4, 4, 4, 4)
    V = 256
    A = dirac.hw_csr(si.unit_links(dims), dims, 0.25, 0.3)
    AH = dirac.hw_csr(si.unit_links(dims), dims, 0.25, -0.3)
    chi = si.gaussian_source(12, 15).reshape(4, 3)
    s = np.arange(V)
    x_, z_, t_ = s % 4, (s // 16) % 4, s // 64
    ph = np.exp(1j * (2 * np.pi / 4 * x_ + np.pi * z_ + (np.pi / 4 + np.pi / 2) * t_))
    b = (ph[:, None, None] * chi[None]).reshape(-1)
    ref = dirac.free_field_function(b, dims, 0.25, 0.3, lambda l: np.sign(l.real))
    xa, ia = direct.arnoldi_direct(lambda v: A @ v, b, 10)
    xl, il = direct.lanczos_direct(lambda v: A @ v, lambda v: AH @ v, b, 10)
    assert ia["k"] == 2 and il["k"] == 2
    assert rel(xa, ref) < 1e-12 and rel(xl, ref) < 1e-12


def test_newton_sign_stops_at_rounding_level():
    """Roberts' iteration on an ill-conditioned matrix: the change levels
    off near roundoff; the iteration still returns sign(A) (checked against
    the sorted-Schur sign)."""
    rng = np.random.default_rng(5)
    n = 40
    Q = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))[0]
    lam = np.concatenate([rng.uniform(0.01, 2, n // 2), -rng.uniform(0.01, 2, n // 2)]) + 1j * rng.normal(size=n)
    T = np.diag(lam) + np.triu(rng.normal(size=(n, n)) * 0.5, 1)
    A = Q @ T @ Q.conj().T
    S = signfun.sign_newton(A)
    assert rel(S, signfun.sign_schur(A)) < 1e-8
    assert np.linalg.norm(S @ S - np.eye(n)) / np.sqrt(n) < 1e-8


# ---------------------------------------------------------------- overlap operator
def test_overlap_operator_identities(small_hw):
    """With the exact sign: Ginsparg-Wilson relation of the massless operator
    (gamma5 D + D gamma5 = D gamma5 D, which holds for any S with S^2 = I and
    fails if gamma5 is misplaced), gamma5-hermiticity gamma5 D(mu) gamma5 =
    D(-mu)^H, and the mass term D(m) = (1 - m/2) D(0) + m."""
    from oracle import overlap
    A, dims, U = small_hw
    n = A.shape[0]
    S = signfun.sign_schur(A)
    D = overlap.overlap_matrix(S)
    G5 = overlap.gamma5_matrix(n)
    assert np.linalg.norm(G5 @ D + D @ G5 - D @ G5 @ D) / np.linalg.norm(D) < 1e-12
    Sm = signfun.sign_schur(dirac.hw_dense(U, dims, 0.25, -0.3))
    assert np.linalg.norm(G5 @ D @ G5 - overlap.overlap_matrix(Sm).conj().T) / np.linalg.norm(D) < 1e-12
    m = 0.2
    assert np.linalg.norm(overlap.overlap_matrix(S, m) - ((1 - m / 2) * D + m * np.eye(n))) < 1e-12
    b = si.gaussian_source(n, 70)
    assert rel(overlap.overlap_apply(lambda v: S @ v, b, m), overlap.overlap_matrix(S, m) @ b) < 1e-14


def test_overlap_free_field_closed_form():
    """Free field: D(0) b = b + gamma5 sign(H(p)) b in momentum space."""
    from oracle import overlap
    dims = (2, 2, 2, 4)
    b = si.gaussian_source(12 * 32, 71)
    sb = dirac.free_field_function(b, dims, 0.25, 0.3, lambda l: np.sign(l.real))
    ref = b + overlap.gamma5_vec(sb)
    A = dirac.hw_dense(si.unit_links(dims), dims, 0.25, 0.3)
    S = signfun.sign_schur(A)
    assert rel(overlap.overlap_apply(lambda v: S @ v, b), ref) < 1e-12


def test_sign_map_matrix_columns_are_xstar(small_hw):
    from oracle import overlap
    A, _, _ = small_hw
    n = A.shape[0]
    R, L, lam, F = deflation.lr_dense(A, 8)
    sig, om = rational.kl_first_order(5, 0.9)
    G = overlap.sign_map_matrix(A, sig, om, R, L, F)
    b = si.gaussian_source(n, 72)
    assert rel(G @ b, xstar.xstar_dense(A, b, sig, om, R, L, F)) < 1e-12


# ---------------------------------------------------------------- GMRES-LR
def test_gmres_seed_minimises_its_residual_and_others_stay_collinear():
    """One GMRES-LR cycle: the seed iterate minimises ||b - (A - sigma_s) x||
    over the Krylov space (checked by a least-squares solve on the explicit
    basis), and every other shifted residual is a multiple of the seed's."""
    from oracle import gmres
    dims = (2, 2, 3, 4)
    V = 48
    A = dirac.hw_csr(si.gauge_links(dims, 0.5, 16), dims, 0.25, 0.3)
    b = si.gaussian_source(12 * V, 17)
    sig, om = rational.kl_first_order(5, 0.9)
    k = 12
    x, info = gmres.restarted_gmres_lr(lambda v: A @ v, b, sig, om, k, max_cycles=1,
                                       keep_shift_solutions=True)
    X, s = info["X"], info["seed"]
    Vb, H, kk = krylov.arnoldi(lambda v: A @ v, b / np.linalg.norm(b), k)
    M = A @ Vb[:, :k] - sig[s] * Vb[:, :k]
    y = np.linalg.lstsq(M, b, rcond=None)[0]
    assert rel(X[s], Vb[:, :k] @ y) < 1e-10
    rs = b - (A @ X[s] - sig[s] * X[s])
    for i in range(len(sig)):
        ri = b - (A @ X[i] - sig[i] * X[i])
        off = ri - np.vdot(rs, ri) / np.vdot(rs, rs) * rs
        assert np.linalg.norm(off) < 1e-10 * np.linalg.norm(b)
        assert abs(np.vdot(rs, ri) / np.vdot(rs, rs) - info["rho"][i]) < 1e-9 * max(1, abs(info["rho"][i]))


@pytest.mark.parametrize("k,m", [(20, 0), (40, 0), (12, 10)])
def test_gmres_lr_converges_to_xstar(k, m):
    from oracle import gmres
    dims = (2, 2, 3, 4)
    V = 48
    Ad = dirac.hw_dense(si.gauge_links(dims, 0.5, 16), dims, 0.25, 0.3)
    b = si.gaussian_source(12 * V, 17)
    sig, om = rational.kl_first_order(5, 0.9)
    R = L = F = None
    if m:
        R, L, lam, F = deflation.lr_dense(Ad, m)
    ref = xstar.xstar_dense(Ad, b, sig, om, R, L, F)
    x, info = gmres.restarted_gmres_lr(lambda v: Ad @ v, b, sig, om, k, R, L, F, tol_update=1e-12,
                                       max_cycles=500)
    assert info["converged"] and rel(x, ref) < 1e-10


def test_gmres_lr_short_cycle_divergence_is_reported():
    from oracle import gmres
    dims = (2, 2, 3, 4)
    V = 48
    A = dirac.hw_csr(si.gauge_links(dims, 0.5, 16), dims, 0.25, 0.3)
    b = si.gaussian_source(12 * V, 17)
    sig, om = rational.kl_first_order(5, 0.9)
    with np.errstate(all="ignore"):
        x, info = gmres.restarted_gmres_lr(lambda v: A @ v, b, sig, om, 8, max_cycles=2000)
    assert not info["converged"]


def test_rational_approximation_error_against_dense_sign():
    """How close x* (the fixed point of Algorithm 1) is to sign(A) b itself:
    with the two-circle scale c = (a b)^{-1/2} from the deflated spectrum,
    the error falls with the Kenney-Laub order s as the scalar bound
    2 rho^{2s} does, rho = (sqrt(q) - 1)/(sqrt(q) + 1), q = b / a."""
    dims = (2, 2, 3, 4)
    V = si.lattice_volume(dims)
    A = dirac.hw_dense(si.gauge_links(dims, 0.5, 16), dims, 0.25, 0.3)
    b = si.gaussian_source(12 * V, 17)
    R, L, lam, F = deflation.lr_dense(A, 10)
    ev = np.linalg.eigvals(A)
    a = np.sort(np.abs(ev))[10]
    bmax = np.max(np.abs(ev))
    c = (a * bmax) ** -0.5
    q = bmax / a
    rho = (np.sqrt(q) - 1) / (np.sqrt(q) + 1)
    ex = signfun.sign_schur(A) @ b
    errs = []
    for s in (4, 8, 16, 32):
        sig, om = rational.kl_first_order(s, c)
        e = rel(xstar.xstar_dense(A, b, sig, om, R, L, F), ex)
        errs.append(e)
        assert e <= 10 * 2 * rho ** (2 * s) + 1e-13, (s, e, 2 * rho ** (2 * s))
    assert errs[0] > errs[1] > errs[2]
    assert errs[-1] < 1e-10
