"""Pins for the oracle's Householder tridiagonalisation and QR eigenvalues.

Independent library routines: LAPACK through numpy.linalg.eigvalsh (zheevd)
and scipy.linalg.eigvalsh_tridiagonal (dstemr/dstebz family), plus exact
special cases and sum rules.
"""

import numpy as np
import pytest
import scipy.linalg

import oracle


def rand_herm(rng, n):
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return A + A.conj().T


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 31, 64, 129])
def test_random_hermitian_vs_lapack(n):
    rng = np.random.default_rng(n)
    A = rand_herm(rng, n)
    w = oracle.eigvalsh(A)
    ref = np.linalg.eigvalsh(A)
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(w - ref).max() < 1e-13 * n * scale
    assert abs(w.sum() - np.trace(A).real) < 1e-12 * n * scale
    assert abs((w ** 2).sum() - (np.abs(A) ** 2).sum()) < 1e-11 * n * scale ** 2


@pytest.mark.parametrize("n", [2, 5, 40])
def test_tridiagonal_form_preserves_spectrum(n):
    rng = np.random.default_rng(100 + n)
    A = rand_herm(rng, n)
    d, e = oracle.tridiagonalize(A)
    assert (e >= 0).all()
    ref = scipy.linalg.eigvalsh_tridiagonal(d, e)
    assert np.abs(np.sort(ref) - np.linalg.eigvalsh(A)).max() < 1e-12 * n
    assert np.abs(oracle.tridiag_eigvals(d, e) - ref).max() < 1e-12 * n


def test_special_matrices():
    assert oracle.eigvalsh(np.zeros((0, 0))).shape == (0,)
    assert np.all(oracle.eigvalsh(np.zeros((6, 6))) == 0)
    D = np.diag([3.0, -1.0, 2.0, 2.0, 0.0])
    assert np.array_equal(oracle.eigvalsh(D), np.sort(np.diag(D)))
    assert np.allclose(oracle.eigvalsh(2.5 * np.eye(7)), 2.5, atol=0, rtol=1e-15)
    # already tridiagonal (real) -> eigenvalues of the tridiagonal
    d = np.array([1.0, -2.0, 0.5, 4.0])
    e = np.array([0.3, 0.0, 1.7])
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    assert np.abs(oracle.eigvalsh(T) - np.linalg.eigvalsh(T)).max() < 1e-14


def test_degenerate_spectrum():
    rng = np.random.default_rng(7)
    n = 24
    lam = np.repeat([-3.0, 0.0, 0.0, 1.5], 6)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
    A = (Q * lam) @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    assert np.abs(oracle.eigvalsh(A) - np.sort(lam)).max() < 1e-13


def test_tridiag_qr_graded_and_glued():
    # graded diagonal and tiny off-diagonals exercise deflation
    d = np.array([1e6, 1.0, 1e-6, -1.0, 3.0])
    e = np.array([1e-3, 1e-12, 0.5, 0.0])
    ref = scipy.linalg.eigvalsh_tridiagonal(d, e)
    assert np.abs(oracle.tridiag_eigvals(d, e) - ref).max() < 1e-9
    # Wilkinson's W21+ matrix: pairs of nearly equal eigenvalues
    d = np.abs(np.arange(-10, 11)).astype(float)
    e = np.ones(20)
    ref = scipy.linalg.eigvalsh_tridiagonal(d, e)
    assert np.abs(oracle.tridiag_eigvals(d, e) - ref).max() < 1e-13
