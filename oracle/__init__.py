"""FP64 CPU oracle for the per-sample spectral hot path (test infrastructure).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it.  The GPU library
never calls it and shares no code with it; the only inputs both sides take
from a common place are the seeded lattice descriptions and grids of
``mlmc_inputs`` (data, no arithmetic of the method).

The numerical work lives in ``oracle.c`` (built by ``oracle/build.py`` with
gcc); this module only marshals numpy arrays to it.  See ``oracle.c`` for
the paper passage each routine follows.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OK = 0
ERR_ARG = -1
ERR_NOT_CONVERGED = -5


class OracleError(RuntimeError):
    pass


class _OraLattice(C.Structure):
    _fields_ = [
        ("lattice_id", C.c_int32), ("n_orb", C.c_int32), ("n_groups", C.c_int32), ("n_hops", C.c_int32),
        ("cell_area", C.c_double),
        ("orb_frac", C.c_void_p), ("orb_group", C.c_void_p), ("removable", C.c_void_p),
        ("hop_R", C.c_void_p), ("hop_from", C.c_void_p), ("hop_to", C.c_void_p),
        ("hop_re", C.c_void_p), ("hop_im", C.c_void_p),
        ("has_overlap", C.c_int32), ("n_ovl", C.c_int32),
        ("ovl_R", C.c_void_p), ("ovl_from", C.c_void_p), ("ovl_to", C.c_void_p),
        ("ovl_re", C.c_void_p), ("ovl_im", C.c_void_p),
    ]


def lib():
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        P = C.c_void_p
        L.ora_philox4x64_10.argtypes = [P, P, P]
        L.ora_philox4x64_10.restype = None
        L.ora_sample_vacancies.argtypes = [P, C.c_int32, C.c_double, C.c_uint64, C.c_uint64, C.c_int64,
                                           C.c_int64, P]
        L.ora_partition_masks.argtypes = [C.c_int32, C.c_int32, P, P]
        L.ora_kgrid.argtypes = [C.c_int32, C.c_int32, P, P]
        L.ora_build_overlap.argtypes = [P, C.c_int32, P, C.c_double, C.c_double, P, C.c_int64, P]
        L.ora_cholesky.argtypes = [C.c_int32, P, C.c_int64]
        L.ora_eigvalsh_generalized.argtypes = [C.c_int32, P, P, C.c_int64, P]
        L.ora_kgrid_points.argtypes = [C.c_int32, C.c_int32]
        L.ora_kgrid_points.restype = C.c_int32
        L.ora_build_hamiltonian.argtypes = [P, C.c_int32, P, C.c_double, C.c_double, P, C.c_int64, P]
        L.ora_tridiagonalize.argtypes = [C.c_int32, P, C.c_int64, P, P]
        L.ora_tridiag_eigvals.argtypes = [C.c_int32, P, P, P]
        L.ora_eigvalsh.argtypes = [C.c_int32, P, C.c_int64, P]
        L.ora_eigh.argtypes = [C.c_int32, P, C.c_int64, P, P, C.c_int64]
        L.ora_smooth_step.argtypes = [C.c_int32, C.c_double]
        L.ora_smooth_step.restype = C.c_double
        L.ora_idos.argtypes = [P, C.c_int64, P, C.c_int32, P, C.c_double, P, C.c_int32, C.c_double,
                               C.c_int32, P]
        L.ora_sample_qoi.argtypes = [P, C.c_int32, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P,
                                     C.c_int32, C.c_double, C.c_int32, P, P]
        L.ora_level_estimate.argtypes = [P, C.c_int32, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                         C.c_int32, C.c_uint64, C.c_int64, C.c_int64, P, C.c_int32,
                                         C.c_double, C.c_int32, C.c_int32, P, P, P]
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _check(st, what):
    if st != OK:
        raise OracleError(f"{what} failed with status {st}")


class OracleLattice:
    """Keeps the numpy arrays alive while C holds pointers into them."""

    def __init__(self, lat):
        self.lat = lat
        self.frac = np.ascontiguousarray(lat.orb_frac, dtype=np.float64)
        self.group = np.ascontiguousarray(lat.orb_group, dtype=np.int32)
        self.removable = np.ascontiguousarray(lat.group_removable, dtype=np.uint8)
        h = lat.hops
        self.R = np.ascontiguousarray(np.stack([h["R1"], h["R2"]], axis=1), dtype=np.int32)
        self.frm = np.ascontiguousarray(h["frm"], dtype=np.int32)
        self.to = np.ascontiguousarray(h["to"], dtype=np.int32)
        self.re = np.ascontiguousarray(h["re"], dtype=np.float64)
        self.im = np.ascontiguousarray(h["im"], dtype=np.float64)
        o = lat.overlap if lat.overlap is not None else np.zeros(0, dtype=h.dtype)
        self.oR = np.ascontiguousarray(np.stack([o["R1"], o["R2"]], axis=1).reshape(-1, 2), dtype=np.int32)
        self.ofrm = np.ascontiguousarray(o["frm"], dtype=np.int32)
        self.oto = np.ascontiguousarray(o["to"], dtype=np.int32)
        self.ore = np.ascontiguousarray(o["re"], dtype=np.float64)
        self.oim = np.ascontiguousarray(o["im"], dtype=np.float64)
        self.s = _OraLattice(lat.lattice_id, lat.n_orb, lat.n_groups, lat.n_hops, lat.cell_area,
                             _ptr(self.frac).value, _ptr(self.group).value, _ptr(self.removable).value,
                             _ptr(self.R).value, _ptr(self.frm).value, _ptr(self.to).value,
                             _ptr(self.re).value, _ptr(self.im).value,
                             1 if lat.overlap is not None else 0, int(o.shape[0]),
                             _ptr(self.oR).value, _ptr(self.ofrm).value, _ptr(self.oto).value,
                             _ptr(self.ore).value, _ptr(self.oim).value)

    @property
    def ref(self):
        return C.cast(C.pointer(self.s), C.c_void_p)


_LAT_CACHE = {}


def _olat(lat):
    key = id(lat)
    ol = _LAT_CACHE.get(key)
    if ol is None or ol.lat is not lat:
        ol = OracleLattice(lat)
        _LAT_CACHE[key] = ol
    return ol


def stream_tag(lat, N: int) -> int:
    """Vacancy-stream tag of a lattice at supercell side N."""
    return (int(lat.lattice_id) << 32) | int(N)


def philox4x64_10(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().ora_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def sample_vacancies(lat, N, p, seed, tag, first_sample, n_samples) -> np.ndarray:
    out = np.zeros((n_samples, N, N, lat.n_groups), dtype=np.uint8)
    _check(lib().ora_sample_vacancies(_olat(lat).ref, N, p, seed, tag, first_sample, n_samples, _ptr(out)),
           "sample_vacancies")
    return out


def partition_masks(mask: np.ndarray) -> np.ndarray:
    """mask [N][N][G] -> quarters [4][N/2][N/2][G]."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    N, _, G = mask.shape
    out = np.zeros((4, N // 2, N // 2, G), dtype=np.uint8)
    _check(lib().ora_partition_masks(N, G, _ptr(mask), _ptr(out)), "partition_masks")
    return out


def kgrid_points(kind: int, K: int) -> int:
    n = lib().ora_kgrid_points(kind, K)
    if n < 0:
        raise ValueError(f"kgrid_points: kind {kind}, K {K}")
    return n


def kgrid(kind: int, K: int):
    nk = kgrid_points(kind, K)
    kred = np.zeros((nk, 2))
    kw = np.zeros(nk)
    _check(lib().ora_kgrid(kind, K, _ptr(kred), _ptr(kw)), "kgrid")
    return kred, kw


def build_hamiltonian(lat, N, mask, kappa) -> np.ndarray:
    """Dense Hermitian H(k) of one outcome; returns an n x n complex128 array."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    nmax = lat.n_orb * N * N
    H = np.zeros((nmax, nmax), dtype=np.complex128, order="F")
    n = C.c_int32(0)
    _check(lib().ora_build_hamiltonian(_olat(lat).ref, N, _ptr(mask), float(kappa[0]), float(kappa[1]),
                                       _ptr(H), nmax, C.byref(n)), "build_hamiltonian")
    return np.array(H[: n.value, : n.value])


def build_overlap(lat, N, mask, kappa) -> np.ndarray:
    """Overlap matrix S(k) of one outcome (unit matrix plus the Bloch sum of the
    overlap table); n x n complex128."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    nmax = lat.n_orb * N * N
    S = np.zeros((nmax, nmax), dtype=np.complex128, order="F")
    n = C.c_int32(0)
    _check(lib().ora_build_overlap(_olat(lat).ref, N, _ptr(mask), float(kappa[0]), float(kappa[1]),
                                   _ptr(S), nmax, C.byref(n)), "build_overlap")
    return np.array(S[: n.value, : n.value])


def cholesky(S: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor of a Hermitian positive definite matrix."""
    A = np.array(S, dtype=np.complex128, order="F")
    n = A.shape[0]
    _check(lib().ora_cholesky(n, _ptr(A), max(n, 1)), "cholesky")
    return np.tril(A)


def eigvalsh_generalized(H: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Eigenvalues of the Hermitian-definite pencil (H, S), ascending."""
    A = np.array(H, dtype=np.complex128, order="F")
    Bm = np.array(S, dtype=np.complex128, order="F")
    n = A.shape[0]
    w = np.zeros(n)
    _check(lib().ora_eigvalsh_generalized(n, _ptr(A), _ptr(Bm), max(n, 1), _ptr(w)), "eigvalsh_generalized")
    return w


def tridiagonalize(A: np.ndarray):
    A = np.array(A, dtype=np.complex128, order="F")
    n = A.shape[0]
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 0) + 1)
    _check(lib().ora_tridiagonalize(n, _ptr(A), max(n, 1), _ptr(d), _ptr(e)), "tridiagonalize")
    return d, e[: max(n - 1, 0)]


def tridiag_eigvals(d, e) -> np.ndarray:
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = d.shape[0]
    e = np.ascontiguousarray(np.append(np.asarray(e, dtype=np.float64), 0.0))
    w = np.zeros(n)
    _check(lib().ora_tridiag_eigvals(n, _ptr(d), _ptr(e), _ptr(w)), "tridiag_eigvals")
    return w


def eigvalsh(A: np.ndarray) -> np.ndarray:
    A = np.array(A, dtype=np.complex128, order="F")
    n = A.shape[0]
    w = np.zeros(n)
    _check(lib().ora_eigvalsh(n, _ptr(A), max(n, 1), _ptr(w)), "eigvalsh")
    return w


def eigh(A: np.ndarray):
    """(w ascending, V) with A V[:, i] = w[i] V[:, i], V unitary (column i the
    unit eigenvector of w[i])."""
    A = np.array(A, dtype=np.complex128, order="F")
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n), dtype=np.complex128, order="F")
    _check(lib().ora_eigh(n, _ptr(A), max(n, 1), _ptr(w), _ptr(V), max(n, 1)), "eigh")
    return w, V


def smooth_step(smoother: int, x: float) -> float:
    return lib().ora_smooth_step(smoother, float(x))


def idos(w: np.ndarray, n: np.ndarray, kweight: np.ndarray, area: float, eps: np.ndarray, delta: float,
         smoother: int) -> np.ndarray:
    """w [n_k][ldw] eigenvalues (first n[k] valid) -> I[n_eps]."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.int32)
    kweight = np.ascontiguousarray(kweight, dtype=np.float64)
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    out = np.zeros(eps.shape[0])
    _check(lib().ora_idos(_ptr(w), w.shape[1], _ptr(n), w.shape[0], _ptr(kweight), float(area), _ptr(eps),
                          eps.shape[0], float(delta), int(smoother), _ptr(out)), "idos")
    return out


def sample_qoi(lat, N, mask, coupled, K_fine, K_coarse, kind, eps, delta, smoother):
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    qf = np.zeros(eps.shape[0])
    qq = np.zeros((4, eps.shape[0])) if coupled else None
    _check(lib().ora_sample_qoi(_olat(lat).ref, N, _ptr(mask), int(coupled), K_fine, K_coarse, kind,
                                _ptr(eps), eps.shape[0], float(delta), int(smoother), _ptr(qf), _ptr(qq)),
           "sample_qoi")
    return (qf, qq) if coupled else qf


def level_estimate(lat, N, coupled, p, K_fine, K_coarse, kind, seed, first_sample, M, eps, delta, smoother,
                   n_threads=1, per_sample=False):
    """Per-level sums [4][n_eps] (sum Y, sum Y^2, sum Q_f, sum Q_f^2)."""
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    ne = eps.shape[0]
    stats = np.zeros((4, ne))
    Y = np.zeros((M, ne)) if per_sample else None
    Qf = np.zeros((M, ne)) if per_sample else None
    _check(lib().ora_level_estimate(_olat(lat).ref, N, int(coupled), float(p), K_fine, K_coarse, kind, seed,
                                    first_sample, M, _ptr(eps), ne, float(delta), int(smoother), int(n_threads),
                                    _ptr(stats), _ptr(Y), _ptr(Qf)), "level_estimate")
    if per_sample:
        return stats, Y, Qf
    return stats
