"""Oracle: the Wilson operator H_W = gamma5 D_W(mu), written out plainly.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this.

The paper (Sect. 1) takes H_W = gamma5 D_W with D_W the Wilson-Dirac
operator at quark chemical potential mu, non-Hermitian for mu != 0, and
defers the definition to its own reference list.  This file uses the
standard form with the chemical potential in the time hops:

    D_W(mu) psi(x) = psi(x) - kappa * sum_nu [ e^{+mu d_{nu,t}} (1 - gamma_nu) U_nu(x) psi(x + nu)
                                              + e^{-mu d_{nu,t}} (1 + gamma_nu) U_nu(x - nu)^+ psi(x - nu) ]

with kappa = 1/(2 m_W + 8), periodic boundaries in space and (by default)
antiperiodic ones in time (a hop across the t boundary picks up -1).
The Dirac matrices are the chiral Euclidean basis

    gamma_k = [[0, -i s_k], [i s_k, 0]],  gamma_t = [[0, 1], [1, 0]],
    gamma5 = gamma_1 gamma_2 gamma_3 gamma_t = diag(1, 1, -1, -1).

With this form H_W(mu)^dagger = H_W(-mu), and H_W is Hermitian at mu = 0
(the Hermitian / non-Hermitian split of Sect. 1).

Two independent constructions are given: a sparse CSR matrix assembled site
by site from the definition, and the free-field (U = 1) closed form in
momentum space, applied through FFTs.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = ["gammas", "gamma5", "kappa_from_mass", "neighbours", "hw_csr",
           "hw_dense", "free_field_symbol", "free_field_apply",
           "free_field_function"]

_SIGMA = [np.array([[0, 1], [1, 0]], dtype=np.complex128),
          np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
          np.array([[1, 0], [0, -1]], dtype=np.complex128)]


def gammas() -> np.ndarray:
    """gamma_nu for nu = x, y, z, t in the chiral basis, shape (4, 4, 4)."""
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    Z = np.zeros((2, 2), dtype=np.complex128)
    I2 = np.eye(2, dtype=np.complex128)
    for k in range(3):
        g[k] = np.block([[Z, -1j * _SIGMA[k]], [1j * _SIGMA[k], Z]])
    g[3] = np.block([[Z, I2], [I2, Z]])
    return g


def gamma5() -> np.ndarray:
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]


def kappa_from_mass(m_w: float) -> float:
    return 1.0 / (2.0 * m_w + 8.0)


def neighbours(dims):
    """Forward / backward neighbour site indices and boundary signs.

    Returns fwd[s, nu], bwd[s, nu] (int64) and bc_fwd[s, nu], bc_bwd[s, nu]
    (+1 or -1: -1 only for t hops that cross the time boundary when the
    caller asks for antiperiodic time)."""
    Lx, Ly, Lz, Lt = dims
    V = Lx * Ly * Lz * Lt
    s = np.arange(V)
    x = s % Lx
    y = (s // Lx) % Ly
    z = (s // (Lx * Ly)) % Lz
    t = s // (Lx * Ly * Lz)
    coords = [x, y, z, t]
    ext = [Lx, Ly, Lz, Lt]

    def idx(c):
        return ((c[3] * Lz + c[2]) * Ly + c[1]) * Lx + c[0]

    fwd = np.empty((V, 4), dtype=np.int64)
    bwd = np.empty((V, 4), dtype=np.int64)
    wrap_f = np.zeros((V, 4), dtype=bool)
    wrap_b = np.zeros((V, 4), dtype=bool)
    for nu in range(4):
        cf = list(coords)
        cf[nu] = (coords[nu] + 1) % ext[nu]
        fwd[:, nu] = idx(cf)
        wrap_f[:, nu] = coords[nu] == ext[nu] - 1
        cb = list(coords)
        cb[nu] = (coords[nu] - 1) % ext[nu]
        bwd[:, nu] = idx(cb)
        wrap_b[:, nu] = coords[nu] == 0
    return fwd, bwd, wrap_f, wrap_b


def hw_csr(U: np.ndarray, dims, kappa: float, mu: float,
           antiperiodic_t: bool = True, d_mu: bool = False) -> sp.csr_matrix:
    """H_W = gamma5 D_W(mu) as a CSR matrix of size 12V, from the definition.

    U has the canonical shape (V, 4, 3, 3); row/column index 12 s + 3 spin + colour.

    With ``d_mu`` the exact derivative dH_W/dmu instead: mu enters only
    through the time-hop factors e^{+mu} (forward) and e^{-mu} (backward),
    whose derivatives are e^{+mu} and -e^{-mu}; the diagonal and the spatial
    hops drop out."""
    dims = tuple(int(d) for d in dims)
    V = int(np.prod(dims))
    U = np.asarray(U, dtype=np.complex128).reshape(V, 4, 3, 3)
    fwd, bwd, wrap_f, wrap_b = neighbours(dims)
    g = gammas()
    g5 = gamma5()
    I4 = np.eye(4, dtype=np.complex128)
    rows, cols, vals = [], [], []
    base_r = np.arange(12)
    sites = np.arange(V)
    # diagonal: gamma5 (x) 1_colour
    diag = np.kron(g5, np.eye(3)) * (0.0 if d_mu else 1.0)
    for a in range(12):
        for b in range(12):
            if diag[a, b] != 0:
                rows.append(12 * sites + a)
                cols.append(12 * sites + b)
                vals.append(np.full(V, diag[a, b]))
    for nu in range(4):
        if d_mu and nu != 3:
            continue
        ph_f = np.exp(mu) if nu == 3 else 1.0
        ph_b = np.exp(-mu) if nu == 3 else 1.0
        if d_mu:
            ph_b = -ph_b
        sgn_f = np.ones(V)
        sgn_b = np.ones(V)
        if nu == 3 and antiperiodic_t:
            sgn_f[wrap_f[:, 3]] = -1.0
            sgn_b[wrap_b[:, 3]] = -1.0
        Pm = g5 @ (I4 - g[nu])          # gamma5 (1 - gamma_nu)
        Pp = g5 @ (I4 + g[nu])          # gamma5 (1 + gamma_nu)
        Uf = U[:, nu]                                   # U_nu(x)
        Ub = np.conj(np.transpose(U[bwd[:, nu], nu], (0, 2, 1)))  # U_nu(x-nu)^+
        for sa in range(4):
            for sb in range(4):
                cf = Pm[sa, sb]
                cb = Pp[sa, sb]
                for ca in range(3):
                    for cc in range(3):
                        r = 12 * sites + 3 * sa + ca
                        if cf != 0:
                            rows.append(r)
                            cols.append(12 * fwd[:, nu] + 3 * sb + cc)
                            vals.append(-kappa * ph_f * sgn_f * cf * Uf[:, ca, cc])
                        if cb != 0:
                            rows.append(r)
                            cols.append(12 * bwd[:, nu] + 3 * sb + cc)
                            vals.append(-kappa * ph_b * sgn_b * cb * Ub[:, ca, cc])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    n = 12 * V
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


def hw_dense(U, dims, kappa, mu, antiperiodic_t=True) -> np.ndarray:
    return hw_csr(U, dims, kappa, mu, antiperiodic_t).toarray()


# ---- free field (U = 1): closed form in momentum space -------------------

def _momenta(dims, antiperiodic_t):
    """Momentum components p_nu on the FFT grid (axes t, z, y, x) and the
    time twist e^{i pi t / Lt} used to map antiperiodic fields to periodic."""
    Lx, Ly, Lz, Lt = dims
    px = 2 * np.pi * np.fft.fftfreq(Lx) * 1.0
    py = 2 * np.pi * np.fft.fftfreq(Ly)
    pz = 2 * np.pi * np.fft.fftfreq(Lz)
    pt = 2 * np.pi * np.fft.fftfreq(Lt) + (np.pi / Lt if antiperiodic_t else 0.0)
    P = np.meshgrid(pt, pz, py, px, indexing="ij")
    return [P[3], P[2], P[1], P[0]]


def free_field_symbol(dims, kappa, mu, antiperiodic_t=True):
    """a(p) and b_nu(p) with D_W(p) = a + i sum_nu b_nu gamma_nu for U = 1:
    a = 1 - 2 kappa sum cos(pt_nu), b_nu = 2 kappa sin(pt_nu), where
    pt_nu = p_nu except pt_t = p_t - i mu.  H(p)^2 = (a^2 + sum b^2) * 1."""
    p = _momenta(dims, antiperiodic_t)
    pt = [p[0], p[1], p[2], p[3] - 1j * mu]
    a = 1 - 2 * kappa * sum(np.cos(q) for q in pt)
    b = [2 * kappa * np.sin(q) for q in pt]
    return a, b


def _to_momentum(psi, dims, antiperiodic_t):
    Lx, Ly, Lz, Lt = dims
    f = np.asarray(psi, dtype=np.complex128).reshape(Lt, Lz, Ly, Lx, 4, 3)
    if antiperiodic_t:
        tw = np.exp(-1j * np.pi * np.arange(Lt) / Lt)
        f = f * tw[:, None, None, None, None, None]
    return np.fft.fftn(f, axes=(0, 1, 2, 3))


def _from_momentum(ft, dims, antiperiodic_t):
    Lx, Ly, Lz, Lt = dims
    f = np.fft.ifftn(ft, axes=(0, 1, 2, 3))
    if antiperiodic_t:
        tw = np.exp(1j * np.pi * np.arange(Lt) / Lt)
        f = f * tw[:, None, None, None, None, None]
    return f.reshape(-1)


def free_field_apply(psi, dims, kappa, mu, antiperiodic_t=True):
    """H_W psi for U = 1, via FFT: H(p) = gamma5 (a + i b.gamma)."""
    return free_field_function(psi, dims, kappa, mu, None, antiperiodic_t)


def free_field_function(psi, dims, kappa, mu, f, antiperiodic_t=True):
    """f(H_W) psi for U = 1 and a scalar function f (None -> identity).

    In momentum space H(p)^2 = lam^2 * 1 with lam^2 = a^2 + sum b_nu^2, so
    H(p) has eigenvalues +-lam and, for any f,
        f(H(p)) = (f(lam) + f(-lam))/2 * 1 + (f(lam) - f(-lam))/(2 lam) * H(p),
    with lam the principal square root of lam^2."""
    dims = tuple(int(d) for d in dims)
    ft = _to_momentum(psi, dims, antiperiodic_t)
    a, b = free_field_symbol(dims, kappa, mu, antiperiodic_t)
    g = gammas()
    g5 = gamma5()
    # H(p) chi: apply gamma5 (a + i b.gamma) to the spin index
    Hchi = a[..., None, None] * ft
    for nu in range(4):
        Hchi = Hchi + 1j * b[nu][..., None, None] * np.einsum("ij,...jc->...ic", g[nu], ft)
    Hchi = np.einsum("ij,...jc->...ic", g5, Hchi)
    if f is None:
        out = Hchi
    else:
        lam2 = a * a + sum(q * q for q in b)
        lam = np.sqrt(lam2)
        fp = f(lam)
        fm = f(-lam)
        c0 = 0.5 * (fp + fm)
        c1 = 0.5 * (fp - fm) / lam
        out = c0[..., None, None] * ft + c1[..., None, None] * Hchi
    return _from_momentum(out, dims, antiperiodic_t)
