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


def cluster_projectors(w, V, tol):
    """Orthogonal projectors onto the eigenspaces of clusters of eigenvalues closer than tol."""
    out, i = [], 0
    while i < len(w):
        j = i + 1
        while j < len(w) and w[j] - w[j - 1] <= tol:
            j += 1
        out.append((i, j, V[:, i:j] @ V[:, i:j].conj().T))
        i = j
    return out


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (33, 3), (64, 4)])
def test_eigh_random_hermitian(n, seed):
    """Eigenstates of random Hermitian matrices: H V = V diag(w), V unitary,
    w equal to LAPACK's, and each eigenvector LAPACK's up to a phase."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = X + X.conj().T
    w, V = oracle.eigh(H)
    wl, Vl = np.linalg.eigh(H)
    scale = max(1.0, np.abs(wl).max())
    assert np.abs(w - wl).max() <= 1e-12 * scale
    assert np.abs(H @ V - V * w).max() <= 1e-12 * scale * n
    assert np.abs(V.conj().T @ V - np.eye(n)).max() <= 1e-12 * n
    overlaps = np.abs(np.sum(V.conj() * Vl, axis=0))   # |<v_i, v_i^LAPACK>|, simple spectrum
    assert np.abs(overlaps - 1.0).max() <= 1e-9


def test_eigh_degenerate_graphene_supercell(glat):
    """Eigenstates of a graphene supercell with vacancies at a zone-corner
    point (exactly degenerate levels, zero modes): residual and unitarity, and
    the projector onto each degenerate eigenspace equal to LAPACK's."""
    N = 4
    mask = np.zeros((N, N, 2), dtype=np.uint8)
    mask[0, 0, 0] = mask[2, 1, 0] = mask[1, 3, 0] = 1      # three A sites vacant: 3 zero modes
    H = oracle.build_hamiltonian(glat, N, mask, np.array([0.0, 0.0]))
    n = H.shape[0]
    w, V = oracle.eigh(H)
    wl, Vl = np.linalg.eigh(H)
    assert np.abs(w - wl).max() <= 1e-12 * 8.1
    assert np.abs(H @ V - V * w).max() <= 1e-12 * 8.1 * n
    assert np.abs(V.conj().T @ V - np.eye(n)).max() <= 1e-12 * n
    assert np.sum(np.abs(w) < 1e-10) >= 3
    for (i, j, P), (il, jl, Pl) in zip(cluster_projectors(w, V, 1e-8), cluster_projectors(wl, Vl, 1e-8)):
        assert (i, j) == (il, jl)
        assert np.abs(P - Pl).max() <= 1e-9


def test_eigh_pristine_bands_closed_form(glat):
    """Pristine supercell: eigenvalues are the folded bands; each eigenvector
    of a simple level is a Bloch wave of the primitive cell (its modulus is
    the same on every cell of a sublattice)."""
    N = 3
    kappa = np.array([0.21, -0.37])
    H = oracle.build_hamiltonian(glat, N, np.zeros((N, N, 2), dtype=np.uint8), kappa)
    w, V = oracle.eigh(H)
    t = 2.7
    ks = [((kappa[0] + m) / N, (kappa[1] + q) / N) for m in range(N) for q in range(N)]
    f = [abs(1 + np.exp(2j * np.pi * k1) + np.exp(2j * np.pi * k2)) for k1, k2 in ks]
    bands = np.sort(np.concatenate([-t * np.array(f), t * np.array(f)]))
    assert np.abs(w - bands).max() <= 1e-12
    gaps = np.diff(w)
    for i in range(len(w)):
        isolated = (i == 0 or gaps[i - 1] > 1e-6) and (i == len(w) - 1 or gaps[i] > 1e-6)
        if isolated:
            mod = np.abs(V[:, i]).reshape(N * N, 2)
            assert np.abs(mod - mod[0]).max() <= 1e-10
