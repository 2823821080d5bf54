"""GPU parity of the non-orthogonal (overlap) path: S(k) assembly, the
batched generalised eigensolver (Cholesky + two-sided reduction on the GPU)
and a level call on the graphene overlap model of Section 3.1, against the
FP64 oracle and LAPACK."""

import sys

import numpy as np
import pytest
import scipy.linalg

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from mlmc_inputs import energy_grid, graphene, graphene_overlap  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_1611_09784_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def odev(B):
    d = B.DeviceLattice(graphene_overlap(eps_2p=0.3), 0)
    yield d
    d.close()


def check_eigs(got, want_list, sizes, rel):
    for u, m in enumerate(sizes):
        if m == 0:
            continue
        want = want_list[u]
        assert np.abs(got[u, :m] - want).max() <= rel * max(1.0, np.abs(want).max()), (u, m)


@pytest.mark.parametrize("N,p", [(3, 0.3), (1, 0.0), (5, 0.2)])
def test_build_overlaps(B, odev, N, p):
    say(f"[overlap build] N={N} p={p}")
    mask = B.mlmc_sample_vacancies(odev, N, p, 5, odev.tag(N), 0, 3)
    kred, _ = B.mlmc_kgrid(0, 2)
    S, n = B.mlmc_build_overlaps(odev, N, mask, kred)
    Sc, nc, m = S.cpu().numpy(), n.cpu().numpy(), mask.cpu().numpy()
    kr = kred.cpu().numpy()
    for u in range(Sc.shape[0]):
        s, k = divmod(u, kr.shape[0])
        want = oracle.build_overlap(odev.lat, N, m[s], kr[k])
        got = Sc[u].T[: nc[u], : nc[u]]
        assert want.shape[0] == nc[u]
        assert np.abs(got - want).max() < 1e-14


@pytest.mark.parametrize("N,K", [(4, 2), (12, 1)])
def test_generalized_eigvalsh_lattice(B, odev, N, K):
    say(f"[generalized lattice] N={N} K={K}")
    mask = B.mlmc_sample_vacancies(odev, N, 0.1, 9, odev.tag(N), 0, 2)
    kred, _ = B.mlmc_kgrid(1, K)
    H, n = B.mlmc_build_hamiltonians(odev, N, mask, kred)
    S, _ = B.mlmc_build_overlaps(odev, N, mask, kred)
    Hc, Sc, nc = H.cpu().numpy(), S.cpu().numpy(), n.cpu().numpy()
    w = B.mlmc_batched_eigvalsh_generalized(H, S, n).cpu().numpy()
    want = [oracle.eigvalsh_generalized(Hc[u].T[: nc[u], : nc[u]], Sc[u].T[: nc[u], : nc[u]]) for u in range(len(nc))]
    check_eigs(w, want, nc, 1e-9)


@pytest.mark.parametrize("ld,sizes", [(40, [40, 17, 1, 0]), (200, [200, 199, 33, 2]), (700, [700, 531, 640])])
@pytest.mark.parametrize("prec", [0, 1])
def test_generalized_eigvalsh_random_pencils(B, ld, sizes, prec):
    say(f"[generalized random] ld={ld} sizes={sizes} prec={prec}")
    rng = np.random.default_rng(ld + 7 * prec)
    batch = len(sizes)
    Hs = np.zeros((batch, ld, ld), np.complex128)
    Ss = np.zeros((batch, ld, ld), np.complex128)
    want = []
    for u, m in enumerate(sizes):
        A = rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))
        A = (A + A.conj().T) / 2
        E = rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))
        Sm = np.eye(m) + 0.3 * (E @ E.conj().T) / max(m, 1)        # well-conditioned, positive definite
        Hs[u, :m, :m] = A.T
        Ss[u, :m, :m] = Sm.T
        want.append(scipy.linalg.eigh(A, Sm, eigvals_only=True) if m else np.zeros(0))
    tdt = torch.complex128 if prec == 0 else torch.complex64
    H = torch.as_tensor(Hs, device=DEV).to(tdt)
    S = torch.as_tensor(Ss, device=DEV).to(tdt)
    n = torch.as_tensor(np.array(sizes, np.int32), device=DEV)
    w = B.mlmc_batched_eigvalsh_generalized(H, S, n).cpu().numpy()
    check_eigs(w, want, sizes, 1e-9 if prec == 0 else 5e-5)


@pytest.mark.parametrize("N,coupled,K,Kc,kind,prec,chunk", [(4, False, 2, 2, 0, 0, None), (8, True, 2, 4, 1, 0, None),
                                                            (4, False, 2, 2, 0, 1, None), (16, False, 1, 1, 1, 0, None),
                                                            (16, True, 1, 2, 1, 0, 1)])
def test_overlap_level_parity(B, odev, N, coupled, K, Kc, kind, prec, chunk):
    say(f"[overlap level] N={N} coupled={coupled} prec={prec} chunk={chunk}")
    eps = energy_grid(-9.0, 18.0, 201)
    M = 3
    got = B.mlmc_level_estimate(odev, N, coupled, 0.1, K, Kc, kind, 77, 2, M, torch.as_tensor(eps, device=DEV), 0.1,
                                prec=prec, chunk_samples=chunk).cpu().numpy()
    want = oracle.level_estimate(odev.lat, N, coupled, 0.1, K, Kc, kind, 77, 2, M, eps, 0.1, 0, n_threads=8)
    tol = 1e-10 if prec == 0 else 1e-5
    assert np.abs(got[0] - want[0]).max() <= M * tol
    assert np.abs(got[2] - want[2]).max() <= M * tol


def test_overlap_level_alternating_streams(B, odev):
    """Consecutive level calls of the overlap model with one pipeline context
    on one workspace, alternating between two streams (the Cholesky-reduction workspace shared
    by the chunks of both calls): bit-identical to the same calls on one
    stream, and the oracle's sums over all samples."""
    say("[overlap level, alternating streams]")
    eps = energy_grid(-9.0, 18.0, 201)
    N, K, kind, prec = 16, 1, 1, 0
    d_eps = torch.as_tensor(eps, device=DEV)
    need = B.mlmc_level_workspace(odev, N, False, K, K, kind, 1, prec, eps.size)
    work = torch.empty((need,), dtype=torch.uint8, device=DEV)
    calls = [(0, 2), (2, 2), (4, 1)]

    def run(streams, ctx=None):
        stats = torch.zeros((4, eps.size), dtype=torch.float64, device=DEV)
        torch.cuda.synchronize()
        for i, (first, M) in enumerate(calls):
            B.mlmc_level_estimate(odev, N, False, 0.1, K, K, kind, 31, first, M, d_eps, 0.1, prec=prec, stats=stats,
                                  work=work, ctx=ctx, stream=streams[i % len(streams)])
        torch.cuda.synchronize()
        return stats.cpu().numpy()

    one = run([torch.cuda.current_stream()])
    with B.Context() as ctx:
        two = run([torch.cuda.current_stream(), torch.cuda.Stream(DEV)], ctx)
    assert np.array_equal(one, two)
    want = oracle.level_estimate(odev.lat, N, False, 0.1, K, K, kind, 31, 0, 5, eps, 0.1, 0, n_threads=8)
    assert np.abs(two[0] - want[0]).max() <= 5 * 1e-10
    assert np.abs(two[2] - want[2]).max() <= 5 * 1e-10


def test_overlap_errors(B):
    d = B.DeviceLattice(graphene(), 0)
    try:
        mask = B.mlmc_sample_vacancies(d, 2, 0.0, 1, d.tag(2), 0, 1)
        kred, _ = B.mlmc_kgrid(0, 1)
        with pytest.raises(B.MLMCError):
            B.mlmc_build_overlaps(d, 2, mask, kred)
    finally:
        d.close()


@pytest.mark.timeout(900)
def test_generalized_eigvalsh_n32_overlap_model(B, odev):
    """The overlap model at the size of the paper's bi-level graphene run
    (32 x 32 supercell, ld = 2048): the panel substitution of the reduction to
    standard form runs in two 1024-row segments.  One outcome, one k-point,
    against the oracle (Cholesky + Householder + QR)."""
    N = 32
    say("[generalized N=32 overlap model, ld=2048]")
    mask = B.mlmc_sample_vacancies(odev, N, 0.02, 13, odev.tag(N), 0, 1)
    kred = torch.as_tensor(np.array([[0.0, 0.0]]), device=DEV)
    H, n = B.mlmc_build_hamiltonians(odev, N, mask, kred)
    S, _ = B.mlmc_build_overlaps(odev, N, mask, kred)
    nc = n.cpu().numpy()
    Hc, Sc = H.cpu().numpy()[0].T[: nc[0], : nc[0]], S.cpu().numpy()[0].T[: nc[0], : nc[0]]
    w = B.mlmc_batched_eigvalsh_generalized(H, S, n).cpu().numpy()
    want = oracle.eigvalsh_generalized(np.ascontiguousarray(Hc), np.ascontiguousarray(Sc))
    check_eigs(w, [want], nc, 1e-9)


@pytest.mark.parametrize("prec", [0, 1])
def test_generalized_eigvalsh_random_pencils_two_segments(B, prec):
    """Random pencils above 1024 rows (ld 1500): the substitution's second
    segment reads the first segment's solution back from H."""
    ld, sizes = 1500, [1500, 1100]
    say(f"[generalized random two segments] ld={ld} prec={prec}")
    rng = np.random.default_rng(99 + prec)
    Hs = np.zeros((len(sizes), ld, ld), np.complex128)
    Ss = np.zeros((len(sizes), ld, ld), np.complex128)
    want = []
    for u, m in enumerate(sizes):
        A = rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))
        A = (A + A.conj().T) / 2
        E = rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))
        Sm = np.eye(m) + 0.3 * (E @ E.conj().T) / m
        Hs[u, :m, :m] = A.T
        Ss[u, :m, :m] = Sm.T
        want.append(scipy.linalg.eigh(A, Sm, eigvals_only=True))
    tdt = torch.complex128 if prec == 0 else torch.complex64
    H = torch.as_tensor(Hs, device=DEV).to(tdt)
    S = torch.as_tensor(Ss, device=DEV).to(tdt)
    n = torch.as_tensor(np.array(sizes, np.int32), device=DEV)
    w = B.mlmc_batched_eigvalsh_generalized(H, S, n).cpu().numpy()
    check_eigs(w, want, sizes, 1e-9 if prec == 0 else 5e-5)


def _full_from_lower(Hcm_u, m):
    """The Hermitian matrix whose lower triangle the column-major block holds."""
    A = np.array(Hcm_u[:m, :m].T)
    return np.tril(A) + np.tril(A, -1).conj().T


@pytest.mark.parametrize("N,p,K,prec", [(4, 0.2, 2, 0), (8, 0.05, 1, 0), (12, 0.1, 1, 0), (8, 0.05, 1, 1),
                                        (12, 0.1, 1, 1)])
def test_eigh_generalized(B, odev, N, p, K, prec):
    """Eigenstates of the overlap model's pencils (H(k), S(k)) with vacancies:
    eigenvalues against the oracle's generalised eigenvalues, residuals
    ||H c - E S c|| and S-orthonormality c^H S c = I within bounds scaled by
    the condition of S; sides 32 and 128 (LDS-resident) and 288 (banded)."""
    say(f"[eigh generalized] N={N} p={p} K={K} prec={prec}")
    mask = B.mlmc_sample_vacancies(odev, N, p, 77, odev.tag(N), 0, 1)
    kred, _ = B.mlmc_kgrid(0, K)
    H, n = B.mlmc_build_hamiltonians(odev, N, mask, kred, B.MLMC_C128)
    S, _ = B.mlmc_build_overlaps(odev, N, mask, kred)
    dt = torch.complex128 if prec == 0 else torch.complex64
    Hd, Sd = H.to(dt), S.to(dt)
    Hin, Sin = Hd.cpu().numpy().astype(np.complex128), Sd.cpu().numpy().astype(np.complex128)  # what the GPU saw
    w, V = B.mlmc_batched_eigh_generalized(Hd.clone(), Sd.clone(), n)
    torch.cuda.synchronize()
    wc, Vc, nc = w.cpu().numpy(), V.cpu().numpy().astype(np.complex128), n.cpu().numpy()
    eps = np.finfo(np.float64 if prec == 0 else np.float32).eps
    for u in range(Hin.shape[0]):
        m = int(nc[u])
        A, Sm = _full_from_lower(Hin[u], m), _full_from_lower(Sin[u], m)
        wo = oracle.eigvalsh_generalized(A, Sm)
        scale = max(1.0, np.abs(wo).max())
        err = np.abs(wc[u, :m] - wo).max()
        assert err <= (1e-9 if prec == 0 else 2e-5) * scale, f"unit {u}: eigenvalue error {err:.3e}"
        X = Vc[u][:m, :m].T  # column i: the eigenvector of w[u, i]
        kappa = np.linalg.cond(Sm)
        hn = np.abs(A).sum(axis=0).max() + np.abs(wc[u, :m]).max() * np.abs(Sm).sum(axis=0).max()
        res = np.linalg.norm(A @ X - (Sm @ X) * wc[u, :m][None, :], axis=0).max()
        orth = np.abs(X.conj().T @ Sm @ X - np.eye(m)).max()
        say(f"  unit {u}: n={m} kappa(S)={kappa:.2f} res/(n eps (|H|+|E||S|))={res / (m * eps * hn):.3f} "
            f"orth/(n eps kappa)={orth / (m * eps * kappa):.3f}")
        assert res <= 16 * m * eps * hn * kappa, f"unit {u}: residual {res:.3e}"
        assert orth <= 16 * m * eps * kappa, f"unit {u}: S-orthonormality {orth:.3e}"
