"""The no-allocation eigensolver entry point (mlmc_batched_eigvalsh_noalloc)
against mlmc_batched_eigvalsh, through the C ABI: same matrices, bit-identical
eigenvalues, on two calls in a row (the second smaller, so that it finds the
first call's contents in the library's scratch), on the LDS-resident path,
the two-stage path with several scratch chunks, and in mixed precision."""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from mlmc_inputs import graphene, mos2_shaped  # noqa: E402

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


def hamiltonians(B, dl, N, p, seed, first, ns, kappa, dtype):
    mask = B.mlmc_sample_vacancies(dl, N, p, seed, dl.tag(N), first, ns)
    kred = torch.as_tensor(np.asarray(kappa, dtype=np.float64), device=DEV)
    return B.mlmc_build_hamiltonians(dl, N, mask, kred, dtype)


# (lattice, N, precision, outcomes in the first call, outcomes in the second)
CASES = [
    ("graphene", 4, 0, 40, 7),      # n <= 32: LDS-resident path, no scratch
    ("graphene", 16, 0, 200, 9),    # ld 512: 94 matrices per scratch chunk -> three chunks, then one
    ("graphene", 16, 1, 400, 5),    # mixed precision, ld 512: 186 per chunk
    ("mos2", 8, 0, 150, 3),         # ld 704 (MoS2-shaped): 68 per chunk
    ("graphene", 32, 0, 50, 2),     # ld 2048: 23 per chunk
]


@pytest.mark.parametrize("name,N,prec,n1,n2", CASES)
def test_noalloc_matches_workspace_entry_point(B, name, N, prec, n1, n2):
    say(f"[noalloc] {name} N={N} prec={prec} calls of {n1} and {n2} matrices")
    lat = graphene() if name == "graphene" else mos2_shaped()
    dl = B.DeviceLattice(lat, 0)
    try:
        dtype = B.MLMC_C128 if prec == 0 else B.MLMC_C64
        kappa = [[0.25, -0.25]]
        for call, (ns, first) in enumerate(((n1, 0), (n2, 1000))):
            H, n = hamiltonians(B, dl, N, 0.05, 77 + call, first, ns, kappa, dtype)
            H2 = H.clone()
            want = B.mlmc_batched_eigvalsh(H, n, prec=prec)
            got = B.mlmc_batched_eigvalsh_noalloc(H2, n, prec=prec)
            torch.cuda.synchronize()
            w, g = want.cpu().numpy(), got.cpu().numpy()
            nn = n.cpu().numpy()
            for u in range(ns):
                assert np.array_equal(g[u, :nn[u]], w[u, :nn[u]]), f"call {call} matrix {u}"
            del H, H2
    finally:
        dl.close()


def test_noalloc_rejects_bad_arguments(B):
    H = torch.zeros((1, 600, 600), dtype=torch.complex128, device=DEV)
    n = torch.full((1,), 600, dtype=torch.int32, device=DEV)
    w = torch.zeros((1, 600), dtype=torch.float64, device=DEV)
    lib = B.lib()
    # ldw below ld, a dtype/precision pair the library does not run, and a side beyond the library's limit
    assert lib.mlmc_batched_eigvalsh_noalloc(B.MLMC_C128, B.MLMC_PREC_FP64, B._ptr(H), 600, B._ptr(n), 1, B._ptr(w),
                                             599, None) == B.MLMC_ERR_INVALID_ARG
    assert lib.mlmc_batched_eigvalsh_noalloc(B.MLMC_C128, B.MLMC_PREC_MIXED, B._ptr(H), 600, B._ptr(n), 1, B._ptr(w),
                                             600, None) == B.MLMC_ERR_UNSUPPORTED
    assert lib.mlmc_batched_eigvalsh_noalloc(B.MLMC_C128, B.MLMC_PREC_FP64, B._ptr(H), 16385, B._ptr(n), 1,
                                             B._ptr(w), 16385, None) == B.MLMC_ERR_UNSUPPORTED
