"""The library's host FP64 dense routines (used by the deflation
eigensolver) against textbook properties and the oracle."""
import numpy as np
import pytest

from oracle import signfun


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 150])
@pytest.mark.parametrize("key", ["re", "abs", "absre"])
def test_schur_form_unitary_triangular_sorted(n, key):
    from paper_0910_2927_amd import api
    rng = np.random.default_rng(n)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    T, Q = api.dense_schur(A, key)
    assert np.abs(Q.conj().T @ Q - np.eye(n)).max() < 1e-13
    assert np.abs(Q @ T @ Q.conj().T - A).max() < 1e-12 * max(1, np.abs(A).max()) * n
    assert np.abs(np.tril(T, -1)).max() == 0.0
    d = np.diag(T)
    kf = {"re": lambda z: z.real, "abs": np.abs, "absre": lambda z: np.abs(z.real)}[key]
    assert np.all(np.diff(kf(d)) >= -1e-12)
    ref = np.linalg.eigvals(A)
    assert np.allclose(np.sort_complex(d), np.sort_complex(ref), atol=1e-10)


def test_schur_of_normal_and_defective_like_matrices():
    from paper_0910_2927_amd import api
    # Hermitian: real eigenvalues; upper triangular input stays exact
    rng = np.random.default_rng(3)
    B = rng.normal(size=(30, 30)) + 1j * rng.normal(size=(30, 30))
    H = B + B.conj().T
    T, Q = api.dense_schur(H, "re")
    assert np.allclose(np.diag(T), np.sort(np.linalg.eigvalsh(H)), atol=1e-11)
    U = np.triu(B)
    T, Q = api.dense_schur(U, "re", count=0)
    assert np.allclose(np.sort_complex(np.diag(T)), np.sort_complex(np.diag(U)))


@pytest.mark.parametrize("n", [1, 4, 25, 60])
def test_newton_sign_matches_oracle(n):
    from paper_0910_2927_amd import api
    rng = np.random.default_rng(10 + n)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)) + 0.5 * np.eye(n)
    S = api.dense_sign(A)
    assert np.abs(S - signfun.sign_schur(A)).max() < 1e-10
    assert np.abs(S @ S - np.eye(n)).max() < 1e-10


def test_sign_refuses_imaginary_axis():
    from paper_0910_2927_amd import api, _lib
    A = np.diag([1j, 2.0, -1.0])
    with pytest.raises(_lib.SkError):
        api.dense_sign(A)
