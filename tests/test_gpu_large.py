"""GPU parity at the largest matrix sizes of the workloads.

* MoS2-shaped N = 16 (ld 2816, n ~ 2785): eigenvalues of one outcome at two
  k-points, FP64 and mixed, against the oracle; and the coupled N = 16 level
  (fine K = 1, quarters on the K = 2 grid) against the oracle's level sums.
* Graphene N = 32 (n ~ 2007), the finest level of the graphene hierarchy,
  coupled (fine K = 1, quarters N = 16 on K = 2), FP64 and mixed against the
  oracle's level sums.  Both coupled levels also run on a pipeline context
  (reductions on the caller's stream, chases on the chase stream, bisections
  on the back stream), equal to the single-stream call bit for bit.
* MoS2-shaped N = 32 (ld 11264, 2 GB per complex128 matrix, the largest
  matrix of the served stream): the pristine supercell's spectrum is the
  union of the primitive 11 x 11 spectra at the N^2 folded wave vectors, an
  exact property at any size; with vacancies, the trace identities
  sum E = Tr H and sum E^2 = ||H||_F^2 and the eigenvalue count.

Tolerances as in test_gpu_parity: eigenvalues 1e-9 max|E| (FP64), 2e-5 max|E|
(mixed); level sums 1e-10 (FP64) and 1e-5 (mixed) per sample.  The oracle's
eigensolves at n ~ 2800 take about a minute each on one host core, so these
tests run them once per module, in parallel threads.
"""

import concurrent.futures as cf
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from mlmc_inputs import energy_grid, graphene, mos2_shaped  # noqa: E402

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
def mlat():
    return mos2_shaped()


@pytest.fixture(scope="module")
def mdev(B, mlat):
    d = B.DeviceLattice(mlat, 0)
    yield d
    d.close()


@pytest.fixture(scope="module")
def gdev(B):
    d = B.DeviceLattice(graphene(), 0)
    yield d
    d.close()


def check_eigs(w, ref, n, rel):
    for u, r in enumerate(ref):
        if n[u] == 0:
            continue
        scale = max(1.0, np.abs(r).max())
        err = np.abs(w[u, : n[u]] - r).max()
        assert err <= rel * scale, f"unit {u}: n={n[u]} err={err:.3e} (bound {rel * scale:.3e})"


def compare_stats(got, want, M, tol):
    ymax = max(1.0, np.abs(want[0]).max() / M, np.abs(want[2]).max() / M)
    assert np.abs(got[0] - want[0]).max() <= M * tol
    assert np.abs(got[2] - want[2]).max() <= M * tol
    assert np.abs(got[1] - want[1]).max() <= M * 2.5 * ymax * tol
    assert np.abs(got[3] - want[3]).max() <= M * 2.5 * ymax * tol


MOS2_KAPPA = np.array([[0.0, 0.0], [0.35, -0.2]])


@pytest.fixture(scope="module")
def mos2_n16(B, mdev, mlat):
    """One MoS2-shaped N = 16 outcome at two k-points: matrices and the
    oracle's eigenvalues (two oracle solves in parallel threads)."""
    N = 16
    mask = B.mlmc_sample_vacancies(mdev, N, 0.02, 404, mdev.tag(N), 7, 1)
    kred = torch.as_tensor(MOS2_KAPPA, device=DEV)
    H128, n = B.mlmc_build_hamiltonians(mdev, N, mask, kred, B.MLMC_C128)
    nc = n.cpu().numpy()
    Hc = H128.cpu().numpy()
    say(f"[mos2 N=16] n = {nc.tolist()}; oracle eigensolves ...")
    with cf.ThreadPoolExecutor(max_workers=2) as ex:
        ref = list(ex.map(lambda u: oracle.eigvalsh(np.ascontiguousarray(Hc[u][: nc[u], : nc[u]].T)), range(2)))
    del Hc
    return mask, kred, n, nc, ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [0, 1])
def test_eigvalsh_mos2_n16(B, mdev, mos2_n16, prec):
    mask, kred, n, nc, ref = mos2_n16
    say(f"[eigvalsh mos2 N=16 ld=2816] prec={prec}")
    code = B.MLMC_C128 if prec == 0 else B.MLMC_C64
    H, _ = B.mlmc_build_hamiltonians(mdev, 16, mask, kred, code)
    w = B.mlmc_batched_eigvalsh(H, n, prec=prec).cpu().numpy()
    check_eigs(w, ref, nc, 1e-9 if prec == 0 else 2e-5)


@pytest.fixture(scope="module")
def mos2_n16_level(mlat):
    b = mlat.hop_magnitude_bound() + 1.0
    eps = energy_grid(-b, b, 201)
    say("[mos2 N=16 level] oracle level sums ...")
    want = oracle.level_estimate(mlat, 16, True, 0.02, 1, 2, 1, 404, 3, 1, eps, 0.1, 0, n_threads=1)
    return eps, want


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [0, 1])
def test_level_mos2_n16_coupled(B, mdev, mos2_n16_level, prec):
    """MoS2-shaped N = 16 coupled level (fine n ~ 2785 at Gamma, quarters
    n ~ 700 on the 2 x 2 Gamma grid), one sample."""
    eps, want = mos2_n16_level
    say(f"[level mos2 N=16 coupled] prec={prec}")
    got = B.mlmc_level_estimate(mdev, 16, True, 0.02, 1, 2, 1, 404, 3, 1, torch.as_tensor(eps, device=DEV), 0.1,
                                prec=prec).cpu().numpy()
    compare_stats(got, want, 1, 1e-10 if prec == 0 else 1e-5)
    # on a pipeline context: reductions on the caller's stream, chases on the
    # chase stream, bisections and sums on the back stream
    with B.Context() as ctx:
        piped = B.mlmc_level_estimate(mdev, 16, True, 0.02, 1, 2, 1, 404, 3, 1, torch.as_tensor(eps, device=DEV), 0.1,
                                      prec=prec, ctx=ctx).cpu().numpy()
    assert np.array_equal(piped, got)


@pytest.fixture(scope="module")
def graphene_n32_level():
    eps = energy_grid(-9.0, 9.0, 401)
    say("[graphene N=32 coupled level] oracle level sums ...")
    want = oracle.level_estimate(graphene(), 32, True, 0.02, 1, 2, 1, 303, 11, 2, eps, 0.05, 0, n_threads=2)
    return eps, want


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [0, 1])
def test_level_graphene_n32_coupled(B, gdev, graphene_n32_level, prec):
    """The finest level of the graphene hierarchy as the MLMC runs use it:
    fine N = 32 (n ~ 2007) at Gamma, quarters N = 16 on the 2 x 2 Gamma
    grid, two samples."""
    eps, want = graphene_n32_level
    say(f"[level graphene N=32 coupled] prec={prec}")
    got = B.mlmc_level_estimate(gdev, 32, True, 0.02, 1, 2, 1, 303, 11, 2, torch.as_tensor(eps, device=DEV), 0.05,
                                prec=prec).cpu().numpy()
    compare_stats(got, want, 2, 1e-10 if prec == 0 else 1e-5)
    # One sample per chunk on a pipeline context (the first chunk chased on
    # the chase stream's share of the CUs beside the second chunk's reduction,
    # the last chunk on the whole device) against the same chunks on one
    # stream, bit for bit.
    d_eps = torch.as_tensor(eps, device=DEV)
    one = B.mlmc_level_estimate(gdev, 32, True, 0.02, 1, 2, 1, 303, 11, 2, d_eps, 0.05, prec=prec,
                                chunk_samples=1).cpu().numpy()
    with B.Context() as ctx:
        piped = B.mlmc_level_estimate(gdev, 32, True, 0.02, 1, 2, 1, 303, 11, 2, d_eps, 0.05, prec=prec,
                                      chunk_samples=1, ctx=ctx).cpu().numpy()
    assert np.array_equal(piped, one)
    compare_stats(piped, want, 2, 1e-10 if prec == 0 else 1e-5)


def folded_primitive_bands(lat, N, kappa):
    """Spectrum of the pristine N x N supercell at reduced wave vector kappa:
    the union of the primitive-cell spectra at (kappa + (m, q)) / N."""
    out = []
    G = lat.n_groups
    for m in range(N):
        for q in range(N):
            Hp = oracle.build_hamiltonian(lat, 1, np.zeros((1, 1, G), np.uint8),
                                          ((kappa[0] + m) / N, (kappa[1] + q) / N))
            out.append(np.linalg.eigvalsh(Hp))
    return np.sort(np.concatenate(out))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [0, 1])
def test_eigvalsh_mos2_n32_pristine_folding(B, mdev, mlat, prec):
    """ld = n = 11264: the pristine MoS2-shaped N = 32 supercell (2 GB in
    complex128) against its folded primitive bands."""
    N = 32
    kappa = (0.3, 0.1)
    say(f"[eigvalsh mos2 N=32 pristine, n=11264] prec={prec}")
    mask = torch.zeros((1, N, N, mlat.n_groups), dtype=torch.uint8, device=DEV)
    kred = torch.as_tensor(np.array([kappa]), device=DEV)
    H, n = B.mlmc_build_hamiltonians(mdev, N, mask, kred, B.MLMC_C128 if prec == 0 else B.MLMC_C64)
    assert int(n[0]) == 11 * N * N
    w = B.mlmc_batched_eigvalsh(H, n, prec=prec).cpu().numpy()
    del H
    torch.cuda.empty_cache()
    ref = folded_primitive_bands(mlat, N, kappa)
    check_eigs(w, [ref], [ref.size], 1e-9 if prec == 0 else 2e-5)


@pytest.mark.timeout(900)
def test_eigvalsh_mos2_n32_with_vacancies_trace_identities(B, mdev, mlat):
    """MoS2-shaped N = 32 with vacancies (p = 0.02, ld 11264, FP64):
    sum E = Tr H, sum E^2 = ||H||_F^2 (every Hermitian matrix), n_b
    eigenvalues in ascending order."""
    N = 32
    say("[eigvalsh mos2 N=32 with vacancies, ld=11264]")
    mask = B.mlmc_sample_vacancies(mdev, N, 0.02, 404, mdev.tag(N), 0, 1)
    kred = torch.as_tensor(np.array([[0.25, 0.5]]), device=DEV)
    H, n = B.mlmc_build_hamiltonians(mdev, N, mask, kred, B.MLMC_C128)
    nb = int(n[0])
    A = H[0, :nb, :nb]  # [column][row]: the lower triangle of the matrix is the upper one of this view
    tr = float(torch.diagonal(A).real.sum())
    low = torch.tril(A.transpose(0, 1))  # the stored lower triangle, with the diagonal
    fro2 = float(2.0 * (low.abs() ** 2).sum() - (torch.diagonal(A).real ** 2).sum())
    del A, low
    w = B.mlmc_batched_eigvalsh(H, n).cpu().numpy()[0]
    del H
    torch.cuda.empty_cache()
    assert nb < 11 * N * N
    E = w[:nb]
    assert np.all(np.diff(E) >= 0)
    emax = np.abs(E).max()
    # each eigenvalue within 1e-9 max|E| gives these bounds on the sums
    assert abs(E.sum() - tr) <= nb * 1e-9 * emax
    assert abs((E * E).sum() - fro2) <= 2.0 * nb * 1e-9 * emax * emax


def known_spectrum_matrix(n, seed):
    """Dense Hermitian H = P3 P2 P1 diag(lam) P1 P2 P3 with random Householder
    reflectors P = I - 2 v v^H (every entry of H nonzero) and a spectrum lam
    known by construction: random values, a three-fold zero, a three-fold
    1.5 and a pair 1e-9 apart."""
    rng = np.random.default_rng(seed)
    lam = np.sort(np.concatenate([rng.uniform(-6.0, 6.0, n - 8), [0.0] * 3, [1.5] * 3, [2.0, 2.0 + 1e-9]]))
    A = np.diag(lam).astype(np.complex128)
    for _ in range(3):
        v = rng.normal(size=n) + 1j * rng.normal(size=n)
        v /= np.linalg.norm(v)
        w = A @ v
        A -= 2.0 * np.outer(v, w.conj())
        A -= 2.0 * np.outer(w, v.conj())
        A += (4.0 * np.vdot(v, w).real) * np.outer(v, v.conj())
    return A, lam


@pytest.mark.parametrize("n,prec", [(5200, 0), (9000, 0), (9000, 1)])
def test_eigvalsh_tall_panels_known_spectrum(B, n, prec):
    """Dense matrices whose dense-to-band panels are taller than 4096 rows
    (the register-blocked panel QR with 16 rows per thread, and 32 in
    complex64; above 8192 rows in complex128 the global-memory panel QR):
    every eigenvalue against the spectrum known by construction, within
    1e-9 max|E| (FP64) and 5e-5 max|E| (mixed, a single-precision reduction of
    side 9000)."""
    say(f"[eigvalsh known spectrum] n={n} prec={prec}")
    A, lam = known_spectrum_matrix(n, 1000 + n)
    dt = torch.complex128 if prec == 0 else torch.complex64
    H = torch.as_tensor(np.ascontiguousarray(A.T)[None], device=DEV).to(dt)  # column-major storage
    del A
    nn = torch.full((1,), n, dtype=torch.int32, device=DEV)
    w = B.mlmc_batched_eigvalsh(H, nn, prec=prec).cpu().numpy()[0]
    err = np.abs(w - lam).max()
    tol = (1e-9 if prec == 0 else 5e-5) * np.abs(lam).max()
    say(f"  max error {err:.3e} (bound {tol:.3e})")
    assert err <= tol
