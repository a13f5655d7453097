"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only draws random numbers and arranges them into arrays: gauge
links, sources and test directions.  It holds none of the method's
arithmetic (no Dirac operator, no rational function, no Krylov step), so the
oracle and the HIP path can both take their inputs from here without sharing
any computation.

Canonical host layout (used by every function here and by the oracle):

* lattice dims ``(Lx, Ly, Lz, Lt)``; site index
  ``s = ((t*Lz + z)*Ly + y)*Lx + x`` (x fastest);
* direction index ``nu = 0,1,2,3`` for x, y, z, t (t carries the chemical
  potential);
* links ``U[s, nu, a, b]`` -- complex128 SU(3) matrix on the link from ``s``
  to ``s + nu_hat``;
* spinors ``psi[s, spin, colour]`` flattened to index ``12*s + 3*spin +
  colour`` (n = 12 V complex entries).

The paper's experiments use lattice gauge configurations that are not part
of the paper (Sect. 6 names only the lattice sizes 4^4 .. 10^4 and mu = 0.3).
They are replaced here by random SU(3) links ``U = exp(i eps Q)`` with
``Q = sum_a q_a lambda_a / 2``, ``q_a ~ N(0, 1)``; ``eps`` controls the
roughness (eps -> 0 is the free field).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "lattice_volume",
    "gell_mann",
    "gauge_links",
    "unit_links",
    "gaussian_source",
    "z2_source",
    "point_source",
    "su3_directions",
    "seed_for",
    "soa_from_canonical",
    "canonical_from_soa",
    "links_soa_from_canonical",
]


def lattice_volume(dims) -> int:
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or min(dims) < 1:
        raise ValueError(f"need four positive lattice extents, got {dims}")
    return dims[0] * dims[1] * dims[2] * dims[3]


def seed_for(L: int, what: str, idx: int = 0) -> int:
    """Fixed seed recipe: gauge 1000L+7, b 1000L+11, eta 1000L+13,
    Z2 sources 1000L+17+idx, derivative directions 99."""
    base = {"gauge": 7, "b": 11, "eta": 13, "z2": 17}
    if what == "dir":
        return 99 + idx
    return 1000 * int(L) + base[what] + (idx if what == "z2" else 0)


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    g = np.zeros((8, 3, 3), dtype=np.complex128)
    g[0][0, 1] = g[0][1, 0] = 1
    g[1][0, 1] = -1j
    g[1][1, 0] = 1j
    g[2][0, 0] = 1
    g[2][1, 1] = -1
    g[3][0, 2] = g[3][2, 0] = 1
    g[4][0, 2] = -1j
    g[4][2, 0] = 1j
    g[5][1, 2] = g[5][2, 1] = 1
    g[6][1, 2] = -1j
    g[6][2, 1] = 1j
    g[7][0, 0] = g[7][1, 1] = 1 / np.sqrt(3)
    g[7][2, 2] = -2 / np.sqrt(3)
    return g


def _exp_i_hermitian(Q: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps Q) for a stack of Hermitian 3x3 matrices, via eigh, so the
    result is unitary to rounding."""
    w, v = np.linalg.eigh(Q)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", v, ph, v.conj())


def gauge_links(dims, eps: float, seed: int) -> np.ndarray:
    """Random SU(3) links U = exp(i eps Q), Q = sum_a q_a lambda_a/2.

    Draw order: ``rng.standard_normal((V, 4, 8))`` from
    ``numpy.random.Generator(PCG64(seed))``; site-major, then direction,
    then generator index.
    Returns complex128 array of shape (V, 4, 3, 3)."""
    V = lattice_volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    q = rng.standard_normal((V, 4, 8))
    Q = np.einsum("sna,aij->snij", q, gell_mann()) * 0.5
    return _exp_i_hermitian(Q, float(eps))


def unit_links(dims) -> np.ndarray:
    V = lattice_volume(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1
    return U


def gaussian_source(n: int, seed: int) -> np.ndarray:
    """Complex Gaussian vector, Re and Im ~ N(0, 1/2) (drawn as one
    (2, n) block: first row real parts, second row imaginary parts)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((2, int(n)))
    return (z[0] + 1j * z[1]) / np.sqrt(2.0)


def z2_source(n: int, seed: int) -> np.ndarray:
    """Real +-1 noise on every component."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (2.0 * rng.integers(0, 2, size=int(n)) - 1.0).astype(np.complex128)


def point_source(n: int, site: int, spin: int, colour: int) -> np.ndarray:
    b = np.zeros(int(n), dtype=np.complex128)
    b[12 * site + 3 * spin + colour] = 1.0
    return b


def su3_directions(V: int, seed: int) -> np.ndarray:
    """Random real coefficient field theta[nu, s, a] ~ N(0,1), shape (4, V, 8)
    (a tangent direction in su(3)^(4V), used for derivative checks)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((4, int(V), 8))


# ---- layout helpers: pure index permutations, no arithmetic ---------------

def soa_from_canonical(psi: np.ndarray, V: int) -> np.ndarray:
    """Canonical [V][12] -> component-major [12][V] (site fastest)."""
    return np.ascontiguousarray(np.asarray(psi).reshape(V, 12).T).reshape(-1)


def canonical_from_soa(psi: np.ndarray, V: int) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(psi).reshape(12, V).T).reshape(-1)


def links_soa_from_canonical(U: np.ndarray) -> np.ndarray:
    """Canonical [V][4][3][3] -> [4][3][3][V] (site fastest)."""
    return np.ascontiguousarray(np.transpose(np.asarray(U), (1, 2, 3, 0)))
