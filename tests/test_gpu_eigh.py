"""GPU parity of mlmc_batched_eigh (eigenvalues and eigenvectors of
LDS-resident Hermitian matrices) against the oracle's eigh.

An eigenvector is fixed only up to a phase, and inside a degenerate or
tightly clustered eigenvalue only the eigenspace is fixed, so the tests
compare what is unique and check that the rest is valid:
  * eigenvalues: max|E - E_oracle| <= 1e-9 max|E| (complex128 path),
    2e-5 max|E| (complex64 path);
  * residuals: max_i ||H v_i - E_i v_i||_2 <= 16 n eps ||H||_1, eps the
    compute type's unit roundoff;
  * orthonormality: max |V^H V - I| <= 16 n eps;
  * spectral projectors: for every group of eigenvalues separated from the
    rest of the spectrum by a gap g (groups split where consecutive oracle
    eigenvalues differ by more than 1e-6 ||H||), the projector V_G V_G^H
    against the oracle's, within 32 n eps ||H||_1 / g (the Davis-Kahan bound
    for two residuals of the size above) plus 16 n eps.
"""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from mlmc_inputs import graphene, mos2_shaped  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
EPS = {0: np.finfo(np.float64).eps, 1: np.finfo(np.float32).eps}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_1611_09784_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def devs(B):
    g = B.DeviceLattice(graphene(), 0)
    m = B.DeviceLattice(mos2_shaped(), 0)
    yield {"graphene": g, "mos2": m}
    g.close()
    m.close()


def full_from_lower(Hcm_u, m):
    """The Hermitian matrix whose lower triangle the column-major block holds."""
    A = np.array(Hcm_u[:m, :m].T)
    L = np.tril(A)
    return L + np.tril(A, -1).conj().T


def groups(w, tol):
    """Index ranges of w (ascending) split where neighbours differ by > tol."""
    out, s = [], 0
    for i in range(1, len(w) + 1):
        if i == len(w) or w[i] - w[i - 1] > tol:
            out.append((s, i))
            s = i
    return out


def check_eigh(A, w, V, prec, label, projectors=True):
    """One matrix: eigenvalues, residuals, orthonormality, projectors (those
    only with `projectors`: they cost n^3 per group)."""
    m = A.shape[0]
    if m == 0:
        return
    eps = EPS[prec]
    wo, Vo = oracle.eigh(A)
    hn = max(np.abs(A).sum(axis=0).max(), 1e-300)
    scale = max(1.0, np.abs(wo).max())
    ev_tol = 1e-9 if prec == 0 else 2e-5
    err_w = np.abs(w - wo).max()
    assert err_w <= ev_tol * scale, f"{label}: eigenvalue error {err_w:.3e}"
    res = np.linalg.norm(A @ V - V * w[None, :], axis=0).max()
    orth = np.abs(V.conj().T @ V - np.eye(m)).max()
    say(f"  {label}: n={m} res/(n eps |H|)={res / (m * eps * hn):.3f} orth/(n eps)={orth / (m * eps):.3f}")
    assert res <= 16 * m * eps * hn, f"{label}: residual {res:.3e}"
    assert orth <= 16 * m * eps, f"{label}: orthonormality {orth:.3e}"
    if not projectors:
        return
    worst = 0.0
    for a, b in groups(wo, 1e-6 * hn):
        if b - a == m:
            continue  # the whole space: nothing to compare
        gap = min(wo[a] - wo[a - 1] if a > 0 else np.inf, wo[b] - wo[b - 1] if b < m else np.inf)
        P = V[:, a:b] @ V[:, a:b].conj().T
        Po = Vo[:, a:b] @ Vo[:, a:b].conj().T
        d = np.abs(P - Po).max()
        bound = 32 * m * eps * hn / gap + 16 * m * eps
        worst = max(worst, d / bound)
        assert d <= bound, f"{label}: projector of eigenvalues {a}..{b - 1} off by {d:.3e} (bound {bound:.3e})"
    say(f"  {label}: worst projector error / bound = {worst:.3f}")


def run_and_check(B, Hs, sizes, prec, label, projectors=True):
    """Hs: [batch][ld][ld] column-major complex128 (lower triangles used)."""
    n = torch.as_tensor(np.array(sizes, np.int32), device=DEV)
    dt = torch.complex128 if prec == 0 else torch.complex64
    H = torch.as_tensor(Hs, device=DEV).to(dt)
    H0 = H.clone()
    w, V = B.mlmc_batched_eigh(H, n)
    torch.cuda.synchronize()
    assert torch.equal(H, H0), "the matrices must be left unchanged"
    wc, Vc = w.cpu().numpy(), V.cpu().numpy()
    Hin = H0.cpu().numpy().astype(np.complex128)  # what the kernel saw, rounded to its type
    for u, m in enumerate(sizes):
        A = full_from_lower(Hin[u], m)
        Vu = Vc[u][:m, :m].T.astype(np.complex128)  # column i = eigenvector i
        check_eigh(A, wc[u, :m], Vu, prec, f"{label}[{u}]", projectors)
    return w, V


def clustered_spectrum(m, rng):
    """Exact multiplicities (four-fold levels, a three-fold zero), a cluster
    1e-13 wide, a pair 1e-9 apart, and simple random values."""
    lam = [0.0, 0.0, 0.0, 1.0, 1.0 + 1e-13, 1.0 + 2e-13, 2.5, 2.5 + 1e-9]
    for v in (-3.2, -1.1, 0.7, 4.4):
        lam += [v] * 4
    lam += list(rng.uniform(-6.0, 6.0, size=max(0, m - len(lam))))
    return np.sort(np.array(lam[:m]))


@pytest.mark.parametrize("ld,sizes,prec", [(64, [0, 1, 2, 3, 17, 64], 0), (128, [128, 127, 5], 0),
                                           (127, [127, 60, 1], 0), (33, [33, 20, 2], 1),   # odd sides
                                           (64, [1, 2, 33, 64], 1), (180, [180, 179, 7], 1)])
def test_eigh_random(B, ld, sizes, prec):
    say(f"[eigh random] ld={ld} sizes={sizes} prec={prec}")
    rng = np.random.default_rng(1000 + ld + prec)
    Hs = np.zeros((len(sizes), ld, ld), np.complex128)
    for u, m in enumerate(sizes):
        A = rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))
        Hs[u, :m, :m] = (A + A.conj().T).T
    run_and_check(B, Hs, sizes, prec, "random")


@pytest.mark.parametrize("ld,sizes,prec", [(128, [96, 40, 128], 0), (128, [96, 40], 1)])
def test_eigh_clustered(B, ld, sizes, prec):
    """H = U diag(lam) U^H with degenerate and clustered lam: the cluster
    treatment of the inverse iteration (eigenspaces, not vectors, compared)."""
    say(f"[eigh clustered] ld={ld} sizes={sizes} prec={prec}")
    rng = np.random.default_rng(77 + prec)
    Hs = np.zeros((len(sizes), ld, ld), np.complex128)
    for u, m in enumerate(sizes):
        lam = clustered_spectrum(m, rng)
        Q, _ = np.linalg.qr(rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m)))
        A = (Q * lam) @ Q.conj().T
        Hs[u, :m, :m] = (0.5 * (A + A.conj().T)).T
    run_and_check(B, Hs, sizes, prec, "clustered")


def test_eigh_diagonal_and_block(B):
    """Special cases: a diagonal matrix (every reflector the identity, the
    vectors unit vectors up to phase), a zero matrix (one n-fold eigenvalue)
    and a 2 x 2 with a complex off-diagonal entry (closed form)."""
    say("[eigh special cases]")
    ld = 32
    Hs = np.zeros((3, ld, ld), np.complex128)
    d = np.array([3.0, -1.0, 2.0, 0.5, -4.0, 1.5, 0.25, -2.5])
    Hs[0, np.arange(8), np.arange(8)] = d
    a, b, c = 1.25, -0.5, 0.75 - 2.0j
    Hs[2, 0, 0], Hs[2, 1, 1], Hs[2, 0, 1] = a, b, c  # column 0 row 1: H[1, 0] = c
    w, V = run_and_check(B, Hs, [8, 5, 2], 0, "special")
    wc, Vc = w.cpu().numpy(), V.cpu().numpy()
    assert np.abs(wc[0, :8] - np.sort(d)).max() <= 1e-12
    order = np.argsort(d)
    for i in range(8):
        v = Vc[0, i, :8]
        assert abs(abs(v[order[i]]) - 1.0) <= 1e-15 and np.abs(np.delete(v, order[i])).max() <= 1e-15
    assert np.abs(wc[1, :5]).max() <= 1e-12
    r = np.sqrt(((a - b) / 2) ** 2 + abs(c) ** 2)
    assert np.allclose(wc[2, :2], [(a + b) / 2 - r, (a + b) / 2 + r], rtol=0, atol=1e-12)


@pytest.mark.parametrize("name,N,p,K,prec", [("graphene", 4, 0.1, 3, 0), ("graphene", 8, 0.05, 1, 0),
                                             ("mos2", 3, 0.2, 2, 0), ("graphene", 8, 0.05, 1, 1),
                                             ("mos2", 4, 0.1, 1, 1)])
def test_eigh_hamiltonians(B, devs, name, N, p, K, prec):
    """H(k) with vacancies: zero modes of the honeycomb (exactly degenerate
    at E = 0), band degeneracies at high-symmetry k, ragged sides."""
    say(f"[eigh H(k)] {name} N={N} p={p} K={K} prec={prec}")
    dl = devs[name]
    mask = B.mlmc_sample_vacancies(dl, N, p, 31, dl.tag(N), 0, 2)
    kred, _ = B.mlmc_kgrid(1, K)
    H, n = B.mlmc_build_hamiltonians(dl, N, mask, kred, B.MLMC_C128)
    run_and_check(B, H.cpu().numpy(), [int(x) for x in n.cpu().numpy()], prec, f"{name}N{N}")


def test_eigh_ragged_offsets_bit_exact(B):
    """Matrices packed at caller offsets (ld * n_b elements each, reversed and
    with gaps) give the fixed-stride results bit for bit; two calls agree bit
    for bit; a side outside [0, ld] gives NaN eigenvalues."""
    say("[eigh ragged offsets]")
    rng = np.random.default_rng(4242)
    ld, sizes = 96, [96, 1, 50, 0, 73]
    Hs = np.zeros((len(sizes), ld, ld), np.complex128)
    for u, m in enumerate(sizes):
        A = rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))
        Hs[u, :m, :m] = (A + A.conj().T).T
    n = torch.as_tensor(np.array(sizes, np.int32), device=DEV)
    H = torch.as_tensor(Hs, device=DEV)
    w1, V1 = B.mlmc_batched_eigh(H, n)
    w2, V2 = B.mlmc_batched_eigh(H, n)
    assert torch.equal(w1, w2) and torch.equal(V1, V2)
    offs, flat, at = [], [], 0
    for u in reversed(range(len(sizes))):
        at += 7 * ld  # a gap
        offs.append(at)
        flat.append((u, at))
        at += ld * sizes[u]
    order = list(reversed(offs))
    buf = torch.zeros((at + ld,), dtype=torch.complex128, device=DEV)
    for u, o in flat:
        buf[o:o + ld * sizes[u]] = H[u, : sizes[u], :].reshape(-1)
    off_t = torch.as_tensor(np.array(order, np.int64), device=DEV)
    w3, V3 = B.mlmc_batched_eigh(buf, n, offsets=off_t, ld=ld)
    for u, m in enumerate(sizes):
        assert torch.equal(w3[u, :m], w1[u, :m])
        assert torch.equal(V3[u, :m, :m], V1[u, :m, :m])
    bad = torch.as_tensor(np.array([ld + 1, 3], np.int32), device=DEV)
    w4, _ = B.mlmc_batched_eigh(H[:2].clone(), bad)
    assert torch.isnan(w4[0]).all() and not torch.isnan(w4[1, :3]).any()


def test_eigh_errors(B):
    """The banded path runs up to side 4096 in both precisions."""
    say("[eigh errors]")
    for prec, cap in ((0, 4096), (1, 4096)):
        dt = torch.complex128 if prec == 0 else torch.complex64
        H = torch.zeros((1, cap + 1, cap + 1), dtype=dt, device=DEV)
        n = torch.ones((1,), dtype=torch.int32, device=DEV)
        with pytest.raises(RuntimeError):
            B.mlmc_batched_eigh(H, n)


# Above 128 (complex128) or 180 (complex64) the banded path runs: stage 1 to
# half-bandwidth 16 with each panel's reflector kept, chase + bisection for
# the eigenvalues, inverse iteration on the band, back-transformation through
# the panels (in double; complex64 input is widened, the vectors rounded).
# Sides 17 and 18 give no panel and a panel of one reflector.

@pytest.mark.parametrize("ld,sizes,prec", [(300, [300, 257, 129, 1, 0], 0), (160, [160, 17, 18, 33, 2], 0),
                                           (300, [300, 181, 17, 1], 1)])
def test_eigh_large_random(B, ld, sizes, prec):
    say(f"[eigh large random] ld={ld} sizes={sizes} prec={prec}")
    rng = np.random.default_rng(5000 + ld + prec)
    Hs = np.zeros((len(sizes), ld, ld), np.complex128)
    for u, m in enumerate(sizes):
        A = rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))
        Hs[u, :m, :m] = (A + A.conj().T).T
    run_and_check(B, Hs, sizes, prec, "large-random")


@pytest.mark.parametrize("prec", [0, 1])
def test_eigh_large_clustered(B, prec):
    say(f"[eigh large clustered] prec={prec}")
    rng = np.random.default_rng(91)
    ld, sizes = 256, [256, 200]
    Hs = np.zeros((len(sizes), ld, ld), np.complex128)
    for u, m in enumerate(sizes):
        lam = clustered_spectrum(m, rng)
        Q, _ = np.linalg.qr(rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m)))
        A = (Q * lam) @ Q.conj().T
        Hs[u, :m, :m] = (0.5 * (A + A.conj().T)).T
    run_and_check(B, Hs, sizes, prec, "large-clustered")


@pytest.mark.parametrize("name,N,p,K,prec", [("graphene", 16, 0.05, 1, 0), ("graphene", 12, 0.1, 2, 0),
                                             ("mos2", 5, 0.1, 1, 0), ("graphene", 16, 0.05, 1, 1),
                                             ("mos2", 5, 0.1, 1, 1)])
def test_eigh_large_hamiltonians(B, devs, name, N, p, K, prec):
    """H(k) with vacancies above the LDS bound: zero modes, the degeneracies
    of the Gamma point (K = 1) and of a 2 x 2 grid."""
    say(f"[eigh large H(k)] {name} N={N} p={p} K={K} prec={prec}")
    dl = devs[name]
    mask = B.mlmc_sample_vacancies(dl, N, p, 57, dl.tag(N), 0, 1)
    kred, _ = B.mlmc_kgrid(1, K)
    H, n = B.mlmc_build_hamiltonians(dl, N, mask, kred, B.MLMC_C128)
    run_and_check(B, H.cpu().numpy(), [int(x) for x in n.cpu().numpy()], prec, f"{name}N{N}")


def test_eigh_large_n2000(B, devs):
    """Graphene N = 32 at Gamma (n ~ 2000, the blocked panel kernels of stage 1):
    eigenvalues, residuals and orthonormality against the oracle."""
    say("[eigh large n~2000] graphene N=32")
    dl = devs["graphene"]
    mask = B.mlmc_sample_vacancies(dl, 32, 0.05, 58, dl.tag(32), 0, 1)
    kred, _ = B.mlmc_kgrid(1, 1)
    H, n = B.mlmc_build_hamiltonians(dl, 32, mask, kred, B.MLMC_C128)
    run_and_check(B, H.cpu().numpy(), [int(x) for x in n.cpu().numpy()], 0, "grapheneN32", projectors=False)


def test_eigh_large_ragged_offsets_bit_exact(B):
    """The banded path at caller offsets gives the fixed-stride results bit for
    bit, and two calls agree bit for bit."""
    say("[eigh large ragged offsets]")
    rng = np.random.default_rng(4343)
    ld, sizes = 200, [200, 150, 0, 170]
    Hs = np.zeros((len(sizes), ld, ld), np.complex128)
    for u, m in enumerate(sizes):
        A = rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))
        Hs[u, :m, :m] = (A + A.conj().T).T
    n = torch.as_tensor(np.array(sizes, np.int32), device=DEV)
    H = torch.as_tensor(Hs, device=DEV)
    w1, V1 = B.mlmc_batched_eigh(H, n)
    w2, V2 = B.mlmc_batched_eigh(H, n)
    assert torch.equal(w1, w2) and torch.equal(V1, V2)
    offs, at = [0] * len(sizes), 0
    for u in reversed(range(len(sizes))):
        at += 5 * ld
        offs[u] = at
        at += ld * sizes[u]
    buf = torch.zeros((at + ld,), dtype=torch.complex128, device=DEV)
    for u, m in enumerate(sizes):
        buf[offs[u]:offs[u] + ld * m] = H[u, :m, :].reshape(-1)
    off_t = torch.as_tensor(np.array(offs, np.int64), device=DEV)
    w3, V3 = B.mlmc_batched_eigh(buf, n, offsets=off_t, ld=ld)
    for u, m in enumerate(sizes):
        assert torch.equal(w3[u, :m], w1[u, :m])
        assert torch.equal(V3[u, :m, :m], V1[u, :m, :m])
    bad = torch.as_tensor(np.array([3, ld + 1], np.int32), device=DEV)
    w4, _ = B.mlmc_batched_eigh(H[:2].clone(), bad)
    assert torch.isnan(w4[1]).all() and not torch.isnan(w4[0, :3]).any()
