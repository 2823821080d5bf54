"""ctypes binding of ``include/mlmc.h`` (argument marshalling only).

Every computation happens in ``libmlmc.so`` (HIP kernels for gfx950).  This
module converts torch tensors to device pointers, picks the current HIP
stream, checks status codes and allocates output tensors with torch.  It
never computes any step of the method itself, and it raises if the library
has not been built: there is no CPU fallback.
"""

from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmlmc.so")

MLMC_OK = 0
MLMC_ERR_INVALID_ARG = -1
MLMC_ERR_UNSUPPORTED = -2
MLMC_ERR_WORKSPACE = -3
MLMC_ERR_HIP = -4

MLMC_C128 = 0
MLMC_C64 = 1
MLMC_PREC_FP64 = 0
MLMC_PREC_MIXED = 1
MLMC_KGRID_MP = 0
MLMC_KGRID_GAMMA = 1
MLMC_KGRID_RHOMBI = 2
MLMC_SMOOTH_GAUSS = 0
MLMC_SMOOTH_CUBIC = 1
MLMC_OP_BATCHED_EIGVALSH = 0
MLMC_OP_BATCHED_EIGVALSH_GENERALIZED = 1
MLMC_OP_LEVEL_ESTIMATE = 2
MLMC_OP_LEVEL_OUTCOMES_SINGLE_PASS = 3
MLMC_OP_BATCHED_EIGH = 4
MLMC_OP_BATCHED_EIGH_GENERALIZED = 5

# Largest matrix side of the LDS-resident fused path / of the device-memory path.
SMALL_MAX = {MLMC_PREC_FP64: 128, MLMC_PREC_MIXED: 180}
LARGE_MAX = {MLMC_PREC_FP64: 16384, MLMC_PREC_MIXED: 16384}


class MLMCError(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__(f"{where}: {status_string(status)} ({status}): {detail}")
        self.status = status


class _Hop(C.Structure):
    _fields_ = [("R", C.c_int32 * 2), ("from_orb", C.c_int32), ("to_orb", C.c_int32),
                ("re", C.c_double), ("im", C.c_double)]


class _LatticeDesc(C.Structure):
    _fields_ = [("lattice_id", C.c_uint32), ("n_orb", C.c_int32), ("n_groups", C.c_int32), ("n_hops", C.c_int32),
                ("cell_area", C.c_double), ("orb_frac", C.c_void_p), ("orb_group", C.c_void_p),
                ("group_removable", C.c_void_p), ("hops", C.c_void_p),
                ("n_overlap", C.c_int32), ("overlap", C.c_void_p)]


class _LaunchConfig(C.Structure):
    _fields_ = [("chase_workgroups", C.c_int64), ("bisect_workgroups", C.c_int64), ("update_tile_rows", C.c_int32)]


class _WorkspaceRequest(C.Structure):
    _fields_ = [("op", C.c_int), ("dtype", C.c_int), ("prec", C.c_int), ("ld", C.c_int64), ("batch", C.c_int64),
                ("lat", C.c_void_p), ("N_fine", C.c_int32), ("coupled", C.c_int32), ("K_fine", C.c_int32),
                ("K_coarse", C.c_int32), ("kgrid", C.c_int), ("chunk_samples", C.c_int64), ("n_eps", C.c_int32)]


_LIB = None
P = C.c_void_p
I32, I64, U64, DBL, SZ = C.c_int32, C.c_int64, C.c_uint64, C.c_double, C.c_size_t

# name -> (restype, argtypes); mirrors include/mlmc.h
SIGNATURES = {
    "mlmc_status_string": (C.c_char_p, [C.c_int]),
    "mlmc_last_error": (C.c_char_p, []),
    "mlmc_lattice_create": (C.c_int, [P, P]),
    "mlmc_lattice_destroy": (C.c_int, [P]),
    "mlmc_lattice_max_orbitals": (C.c_int, [P, I32, P]),
    "mlmc_sample_vacancies": (C.c_int, [P, I32, DBL, U64, U64, I64, I64, P, P]),
    "mlmc_partition_masks": (C.c_int, [P, I32, P, I64, P, P]),
    "mlmc_kgrid_points": (C.c_int, [C.c_int, I32, P]),
    "mlmc_kgrid": (C.c_int, [C.c_int, I32, P, P, P]),
    "mlmc_build_hamiltonians": (C.c_int, [P, I32, P, I64, P, I32, C.c_int, P, I64, P, P]),
    "mlmc_workspace_bytes": (C.c_int, [P, P]),
    "mlmc_batched_eigvalsh": (C.c_int, [C.c_int, C.c_int, P, I64, P, P, I64, P, I64, P, SZ, P]),
    "mlmc_batched_eigvalsh_noalloc": (C.c_int, [C.c_int, C.c_int, P, I64, P, I64, P, I64, P]),
    "mlmc_batched_eigh": (C.c_int, [C.c_int, C.c_int, P, I64, P, P, I64, P, I64, P, I64, P, SZ, P]),
    "mlmc_batched_eigh_generalized": (C.c_int, [C.c_int, C.c_int, P, P, I64, P, I64, P, I64, P, I64, P, SZ, P]),
    "mlmc_build_overlaps": (C.c_int, [P, I32, P, I64, P, I32, C.c_int, P, I64, P, P]),
    "mlmc_batched_eigvalsh_generalized": (C.c_int, [C.c_int, C.c_int, P, P, I64, P, I64, P, I64, P, SZ, P]),
    "mlmc_idos": (C.c_int, [P, I64, P, I64, I32, P, DBL, P, I32, DBL, C.c_int, P, P]),
    "mlmc_level_stats": (C.c_int, [P, P, I64, I32, P, P]),
    "mlmc_level_estimate": (C.c_int, [P, I32, I32, DBL, I32, I32, C.c_int, U64, I64, I64, P, I32, DBL, C.c_int,
                                      C.c_int, P, P, SZ, P, P, P]),
    "mlmc_level_outcomes": (C.c_int, [P, I32, I32, I32, I32, C.c_int, P, I64, P, I32, DBL, C.c_int, C.c_int,
                                      P, P, P, P, SZ, P, P]),
    "mlmc_context_create": (C.c_int, [P]),
    "mlmc_context_destroy": (C.c_int, [P]),
    "mlmc_context_timer": (C.c_int, [P, I64, C.c_int32]),
    "mlmc_context_configure": (C.c_int, [P, P]),
    "mlmc_context_stream": (C.c_int, [P, I32, P]),
    "mlmc_context_timer_read": (C.c_int, [P, C.c_char_p, P, P, P]),
    "mlmc_optimal_samples": (C.c_int, [I32, P, P, DBL, DBL, DBL, P]),
    "mlmc_dos": (C.c_int, [I32, P, P, P]),
    "mlmc_chase_cus": (C.c_int, [C.c_int, P]),
}


def lib() -> C.CDLL:
    """Load libmlmc.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                               f"g.build()'` (there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def status_string(st: int) -> str:
    try:
        return lib().mlmc_status_string(st).decode()
    except Exception:  # pragma: no cover - only when the library itself is missing
        return str(st)


def _check(st: int, where: str):
    if st != MLMC_OK:
        raise MLMCError(st, where, lib().mlmc_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if t.numel() == 0:
            return None
        if not t.is_contiguous():
            raise ValueError("tensor arguments must be contiguous")
        return C.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    raise TypeError(type(t))


def _dev(t: torch.Tensor, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def stream_tag(lattice_id: int, N: int) -> int:
    """Vacancy-stream tag used by mlmc_level_estimate: (lattice_id << 32) | N."""
    return (int(lattice_id) << 32) | int(N)


def _hop_rows(table):
    rows = np.zeros(table.shape[0], dtype=np.dtype([("R", np.int32, 2), ("from_orb", np.int32),
                                                    ("to_orb", np.int32), ("re", np.float64), ("im", np.float64)]))
    rows["R"][:, 0] = table["R1"]
    rows["R"][:, 1] = table["R2"]
    rows["from_orb"] = table["frm"]
    rows["to_orb"] = table["to"]
    rows["re"] = table["re"]
    rows["im"] = table["im"]
    return rows


# Handles still open when the interpreter exits are released before the HIP
# runtime shuts down (at process exit, after the atexit hooks).
_OPEN_HANDLES = weakref.WeakSet()


@atexit.register
def _close_open_handles():
    for h in list(_OPEN_HANDLES):
        try:
            h.close()
        except Exception:
            pass


class DeviceLattice:
    """Device-resident lattice handle (mlmc_lattice_create / _destroy)."""

    def __init__(self, lat, device=None):
        self.lat = lat
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        hops = _hop_rows(lat.hops)
        ovl = _hop_rows(lat.overlap) if getattr(lat, "overlap", None) is not None else None
        frac = np.ascontiguousarray(lat.orb_frac, dtype=np.float64)
        group = np.ascontiguousarray(lat.orb_group, dtype=np.int32)
        rem = np.ascontiguousarray(lat.group_removable, dtype=np.uint8)
        desc = _LatticeDesc(lat.lattice_id, lat.n_orb, lat.n_groups, lat.n_hops, lat.cell_area,
                            _ptr(frac), _ptr(group), _ptr(rem), _ptr(hops),
                            0 if ovl is None else ovl.shape[0], None if ovl is None else _ptr(ovl))
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().mlmc_lattice_create(C.byref(desc), C.byref(handle)), "mlmc_lattice_create")
        self._h = handle
        _OPEN_HANDLES.add(self)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("lattice handle already closed")
        return self._h

    def max_orbitals(self, N: int) -> int:
        out = C.c_int64()
        _check(lib().mlmc_lattice_max_orbitals(self.handle, N, C.byref(out)), "mlmc_lattice_max_orbitals")
        return out.value

    def tag(self, N: int) -> int:
        return stream_tag(self.lat.lattice_id, N)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().mlmc_lattice_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """Pipeline context of level estimates (mlmc_context_create / _destroy):
    the chase and back streams, their events and the buffer-set rotation of
    consecutive calls, on the device current at creation."""

    def __init__(self, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().mlmc_context_create(C.byref(handle)), "mlmc_context_create")
        self._h = handle
        _OPEN_HANDLES.add(self)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("context already closed")
        return self._h

    def stream(self, index: int):
        """Caller stream `index` (0 or 1) owned by the context, as a torch stream."""
        out = C.c_void_p()
        _check(lib().mlmc_context_stream(self.handle, int(index), C.byref(out)), "mlmc_context_stream")
        return torch.cuda.ExternalStream(out.value, device=self.device)

    def configure(self, chase_workgroups: int = 0, bisect_workgroups: int = 0, update_tile_rows: int = 0):
        """Launch choices of this context's level calls (0: the library's default)."""
        cfg = _LaunchConfig(int(chase_workgroups), int(bisect_workgroups), int(update_tile_rows))
        _check(lib().mlmc_context_configure(self.handle, C.byref(cfg)), "mlmc_context_configure")

    def timer(self, capacity: int, detail: bool = False):
        """Create `capacity` start/stop event pairs (0: destroy them); the
        level calls of this context then time their kernel launches (with
        `detail` also the dense-to-band stage's kernels one by one)."""
        _check(lib().mlmc_context_timer(self.handle, int(capacity), int(bool(detail))), "mlmc_context_timer")

    def timer_read(self, name: str):
        """(total milliseconds, launches, dropped) of kernel `name` since the timer was (re)set."""
        ms, count, dropped = C.c_double(), C.c_int64(), C.c_int64()
        _check(lib().mlmc_context_timer_read(self.handle, name.encode(), C.byref(ms), C.byref(count),
                                             C.byref(dropped)), "mlmc_context_timer_read")
        return ms.value, count.value, dropped.value

    def close(self):
        if getattr(self, "_h", None) is not None:
            with torch.cuda.device(self.device):
                st = lib().mlmc_context_destroy(self._h)
            self._h = None
            _check(st, "mlmc_context_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ctx(ctx):
    return None if ctx is None else ctx.handle


# ---------------------------------------------------------------------------
# One wrapper per C entry point (same names).
# ---------------------------------------------------------------------------

def mlmc_sample_vacancies(dlat, N, p, seed, tag, first_sample, n_samples, out=None, stream=None):
    if out is None:
        out = torch.empty((n_samples, N, N, dlat.lat.n_groups), dtype=torch.uint8, device=dlat.device)
    _dev(out, torch.uint8, "mask")
    _check(lib().mlmc_sample_vacancies(dlat.handle, N, float(p), int(seed) & (2**64 - 1), int(tag) & (2**64 - 1),
                                       first_sample, n_samples, _ptr(out), _stream(stream)), "mlmc_sample_vacancies")
    return out


def mlmc_partition_masks(dlat, N, mask, out=None, stream=None):
    _dev(mask, torch.uint8, "mask")
    ns = mask.shape[0]
    h = N // 2
    if out is None:
        out = torch.empty((ns, 4, h, h, dlat.lat.n_groups), dtype=torch.uint8, device=mask.device)
    _check(lib().mlmc_partition_masks(dlat.handle, N, _ptr(mask), ns, _ptr(out), _stream(stream)),
           "mlmc_partition_masks")
    return out


def mlmc_kgrid_points(kind, K) -> int:
    out = C.c_int32()
    _check(lib().mlmc_kgrid_points(kind, K, C.byref(out)), "mlmc_kgrid_points")
    return out.value


def mlmc_kgrid(kind, K, device=None, stream=None):
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    nk = mlmc_kgrid_points(kind, K)
    kred = torch.empty((nk, 2), dtype=torch.float64, device=dev)
    kw = torch.empty((nk,), dtype=torch.float64, device=dev)
    _check(lib().mlmc_kgrid(kind, K, _ptr(kred), _ptr(kw), _stream(stream)), "mlmc_kgrid")
    return kred, kw


def mlmc_build_hamiltonians(dlat, N, mask, kred, dtype=MLMC_C128, ld=None, H=None, n_out=None, stream=None):
    _dev(mask, torch.uint8, "mask")
    _dev(kred, torch.float64, "kred")
    ns = mask.shape[0]
    nk = kred.shape[0]
    ld = dlat.max_orbitals(N) if ld is None else ld
    tdt = torch.complex128 if dtype == MLMC_C128 else torch.complex64
    if H is None:
        H = torch.empty((ns * nk, ld, ld), dtype=tdt, device=mask.device)
    if n_out is None:
        n_out = torch.empty((ns * nk,), dtype=torch.int32, device=mask.device)
    _dev(H, tdt, "H")
    _dev(n_out, torch.int32, "n")
    _check(lib().mlmc_build_hamiltonians(dlat.handle, N, _ptr(mask), ns, _ptr(kred), nk, dtype, _ptr(H), ld,
                                         _ptr(n_out), _stream(stream)), "mlmc_build_hamiltonians")
    return H, n_out


def mlmc_build_overlaps(dlat, N, mask, kred, dtype=MLMC_C128, ld=None, S=None, n_out=None, stream=None):
    _dev(mask, torch.uint8, "mask")
    _dev(kred, torch.float64, "kred")
    ns = mask.shape[0]
    nk = kred.shape[0]
    ld = dlat.max_orbitals(N) if ld is None else ld
    tdt = torch.complex128 if dtype == MLMC_C128 else torch.complex64
    if S is None:
        S = torch.empty((ns * nk, ld, ld), dtype=tdt, device=mask.device)
    if n_out is None:
        n_out = torch.empty((ns * nk,), dtype=torch.int32, device=mask.device)
    _dev(S, tdt, "S")
    _dev(n_out, torch.int32, "n")
    _check(lib().mlmc_build_overlaps(dlat.handle, N, _ptr(mask), ns, _ptr(kred), nk, dtype, _ptr(S), ld,
                                     _ptr(n_out), _stream(stream)), "mlmc_build_overlaps")
    return S, n_out


def mlmc_workspace_bytes(op, dtype=MLMC_C128, prec=MLMC_PREC_FP64, ld=0, batch=0, dlat=None, N_fine=0, coupled=0,
                         K_fine=0, K_coarse=0, kgrid=MLMC_KGRID_MP, chunk_samples=0, n_eps=0) -> int:
    req = _WorkspaceRequest(op, dtype, prec, ld, batch, None if dlat is None else dlat.handle, N_fine, int(coupled),
                            K_fine, K_coarse, kgrid, chunk_samples, n_eps)
    out = C.c_size_t()
    _check(lib().mlmc_workspace_bytes(C.byref(req), C.byref(out)), "mlmc_workspace_bytes")
    return out.value


def mlmc_generalized_workspace(dtype, prec, ld, batch) -> int:
    return mlmc_workspace_bytes(MLMC_OP_BATCHED_EIGVALSH_GENERALIZED, dtype, prec, ld, batch)


def mlmc_batched_eigvalsh_generalized(H, S, n, prec=None, w=None, ldw=None, work=None, stream=None):
    """Eigenvalues of the pencils (H, S); H and S are overwritten."""
    dtype = MLMC_C128 if H.dtype == torch.complex128 else MLMC_C64
    if prec is None:
        prec = MLMC_PREC_FP64 if dtype == MLMC_C128 else MLMC_PREC_MIXED
    _dev(H, None, "H")
    _dev(S, H.dtype, "S")
    _dev(n, torch.int32, "n")
    batch, ld = H.shape[0], H.shape[1]
    if S.shape != H.shape:
        raise ValueError("H and S must have the same shape")
    ldw = ld if ldw is None else ldw
    if w is None:
        w = torch.zeros((batch, ldw), dtype=torch.float64, device=H.device)
    _dev(w, torch.float64, "w")
    need = mlmc_generalized_workspace(dtype, prec, ld, batch)
    if work is None and need > 0:
        work = torch.empty((need,), dtype=torch.uint8, device=H.device)
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(lib().mlmc_batched_eigvalsh_generalized(dtype, prec, _ptr(H), _ptr(S), ld, _ptr(n), batch, _ptr(w), ldw,
                                                   _ptr(work), wb, _stream(stream)),
           "mlmc_batched_eigvalsh_generalized")
    return w


def mlmc_eigvalsh_workspace(dtype, prec, ld, batch) -> int:
    return mlmc_workspace_bytes(MLMC_OP_BATCHED_EIGVALSH, dtype, prec, ld, batch)


def mlmc_batched_eigvalsh(H, n, prec=None, w=None, ldw=None, work=None, stream=None, offsets=None, ld=None):
    """H: [batch][ld][ld] column-major (torch stores [u][c][r]); overwritten.
    Ragged layout: `offsets` (int64 device tensor [batch]) gives each matrix's
    first element in the flat buffer H, with leading dimension `ld`."""
    if H.dtype == torch.complex128:
        dtype = MLMC_C128
    elif H.dtype == torch.complex64:
        dtype = MLMC_C64
    else:
        raise ValueError("H must be complex64 or complex128")
    if prec is None:
        prec = MLMC_PREC_FP64 if dtype == MLMC_C128 else MLMC_PREC_MIXED
    _dev(H, None, "H")
    _dev(n, torch.int32, "n")
    if offsets is None:
        batch, ld = H.shape[0], H.shape[1]
    else:
        _dev(offsets, torch.int64, "offsets")
        if ld is None:
            raise ValueError("a ragged layout needs ld")
        batch = offsets.shape[0]
    ldw = ld if ldw is None else ldw
    if w is None:
        w = torch.zeros((batch, ldw), dtype=torch.float64, device=H.device)
    _dev(w, torch.float64, "w")
    need = mlmc_eigvalsh_workspace(dtype, prec, ld, batch)
    if work is None and need > 0:
        work = torch.empty((need,), dtype=torch.uint8, device=H.device)
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(lib().mlmc_batched_eigvalsh(dtype, prec, _ptr(H), ld, _ptr(offsets), _ptr(n), batch, _ptr(w), ldw,
                                       _ptr(work), wb, _stream(stream)), "mlmc_batched_eigvalsh")
    return w


def mlmc_eigh_workspace(dtype, prec, ld, batch) -> int:
    return mlmc_workspace_bytes(MLMC_OP_BATCHED_EIGH, dtype, prec, ld, batch)


def mlmc_batched_eigh(H, n, prec=None, w=None, V=None, work=None, stream=None, offsets=None, ld=None):
    """Eigenvalues and eigenvectors of Hermitian matrices (up to side 4096).
    H: [batch][ld][ld] column-major (torch [u][c][r]), read only; or a flat
    buffer with `offsets` and `ld` as in mlmc_batched_eigvalsh.  Returns
    (w [batch][ld], V [batch][ld][ld]) with V[b, i, :n_b] the unit
    eigenvector of w[b, i] (column i of the column-major matrix)."""
    if H.dtype == torch.complex128:
        dtype = MLMC_C128
    elif H.dtype == torch.complex64:
        dtype = MLMC_C64
    else:
        raise ValueError("H must be complex64 or complex128")
    if prec is None:
        prec = MLMC_PREC_FP64 if dtype == MLMC_C128 else MLMC_PREC_MIXED
    _dev(H, None, "H")
    _dev(n, torch.int32, "n")
    if offsets is None:
        batch, ld = H.shape[0], H.shape[1]
    else:
        _dev(offsets, torch.int64, "offsets")
        if ld is None:
            raise ValueError("a ragged layout needs ld")
        batch = offsets.shape[0]
    if w is None:
        w = torch.zeros((batch, ld), dtype=torch.float64, device=H.device)
    _dev(w, torch.float64, "w")
    if V is None:
        V = torch.zeros((batch, ld, ld), dtype=H.dtype, device=H.device)
    _dev(V, H.dtype, "V")
    if V.dim() != 3 or V.shape[0] != batch or V.shape[1] != V.shape[2] or not V.is_contiguous():
        raise ValueError("V must be a contiguous [batch][ldv][ldv] tensor")
    need = mlmc_eigh_workspace(dtype, prec, ld, batch)
    if work is None and need > 0:
        work = torch.empty((need,), dtype=torch.uint8, device=H.device)
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(lib().mlmc_batched_eigh(dtype, prec, _ptr(H), ld, _ptr(offsets), _ptr(n), batch, _ptr(w), w.shape[1],
                                   _ptr(V), V.shape[1], _ptr(work), wb, _stream(stream)), "mlmc_batched_eigh")
    return w, V


def mlmc_eigh_generalized_workspace(dtype, prec, ld, batch) -> int:
    return mlmc_workspace_bytes(MLMC_OP_BATCHED_EIGH_GENERALIZED, dtype, prec, ld, batch)


def mlmc_batched_eigh_generalized(H, S, n, prec=None, w=None, V=None, work=None, stream=None):
    """Eigenvalues and S-orthonormal eigenvectors of the pencils (H, S) (up to
    side 2048).  H, S: [batch][ld][ld] column-major (torch [u][c][r]), both
    overwritten.  Returns (w [batch][ld], V [batch][ld][ld]) with V[b, i, :n_b]
    the eigenvector of w[b, i]."""
    if H.dtype == torch.complex128:
        dtype = MLMC_C128
    elif H.dtype == torch.complex64:
        dtype = MLMC_C64
    else:
        raise ValueError("H must be complex64 or complex128")
    if prec is None:
        prec = MLMC_PREC_FP64 if dtype == MLMC_C128 else MLMC_PREC_MIXED
    _dev(H, None, "H")
    _dev(S, H.dtype, "S")
    _dev(n, torch.int32, "n")
    if S.shape != H.shape or H.dim() != 3:
        raise ValueError("H and S must be [batch][ld][ld] of one shape")
    batch, ld = H.shape[0], H.shape[1]
    if w is None:
        w = torch.zeros((batch, ld), dtype=torch.float64, device=H.device)
    _dev(w, torch.float64, "w")
    if V is None:
        V = torch.zeros((batch, ld, ld), dtype=H.dtype, device=H.device)
    _dev(V, H.dtype, "V")
    if V.dim() != 3 or V.shape[0] != batch or V.shape[1] != V.shape[2] or not V.is_contiguous():
        raise ValueError("V must be a contiguous [batch][ldv][ldv] tensor")
    need = mlmc_eigh_generalized_workspace(dtype, prec, ld, batch)
    if work is None and need > 0:
        work = torch.empty((need,), dtype=torch.uint8, device=H.device)
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(lib().mlmc_batched_eigh_generalized(dtype, prec, _ptr(H), _ptr(S), ld, _ptr(n), batch, _ptr(w), w.shape[1],
                                               _ptr(V), V.shape[1], _ptr(work), wb, _stream(stream)),
           "mlmc_batched_eigh_generalized")
    return w, V


def mlmc_batched_eigvalsh_noalloc(H, n, prec=None, w=None, ldw=None, stream=None):
    """mlmc_batched_eigvalsh on the library's static device scratch (no
    workspace argument, no allocation in the library); H is overwritten."""
    if H.dtype == torch.complex128:
        dtype = MLMC_C128
    elif H.dtype == torch.complex64:
        dtype = MLMC_C64
    else:
        raise ValueError("H must be complex64 or complex128")
    if prec is None:
        prec = MLMC_PREC_FP64 if dtype == MLMC_C128 else MLMC_PREC_MIXED
    _dev(H, None, "H")
    _dev(n, torch.int32, "n")
    batch, ld = H.shape[0], H.shape[1]
    ldw = ld if ldw is None else ldw
    if w is None:
        w = torch.zeros((batch, ldw), dtype=torch.float64, device=H.device)
    _dev(w, torch.float64, "w")
    _check(lib().mlmc_batched_eigvalsh_noalloc(dtype, prec, _ptr(H), ld, _ptr(n), batch, _ptr(w), ldw,
                                               _stream(stream)), "mlmc_batched_eigvalsh_noalloc")
    return w


def mlmc_idos(w, n, n_k, kweight, area, eps, delta, smoother=MLMC_SMOOTH_GAUSS, out=None, stream=None):
    _dev(w, torch.float64, "w")
    _dev(n, torch.int32, "n")
    _dev(kweight, torch.float64, "kweight")
    _dev(eps, torch.float64, "eps")
    ns = w.shape[0] // n_k
    if out is None:
        out = torch.empty((ns, eps.shape[0]), dtype=torch.float64, device=w.device)
    _check(lib().mlmc_idos(_ptr(w), w.shape[1], _ptr(n), ns, n_k, _ptr(kweight), float(area), _ptr(eps),
                           eps.shape[0], float(delta), smoother, _ptr(out), _stream(stream)), "mlmc_idos")
    return out


def mlmc_level_stats(idos_fine, idos_quarters=None, stats=None, stream=None):
    _dev(idos_fine, torch.float64, "idos_fine")
    ns, ne = idos_fine.shape
    if idos_quarters is not None:
        _dev(idos_quarters, torch.float64, "idos_quarters")
    if stats is None:
        stats = torch.zeros((4, ne), dtype=torch.float64, device=idos_fine.device)
    _check(lib().mlmc_level_stats(_ptr(idos_fine), _ptr(idos_quarters), ns, ne, _ptr(stats), _stream(stream)),
           "mlmc_level_stats")
    return stats


def mlmc_level_workspace(dlat, N, coupled, K_fine, K_coarse, kind, chunk_samples, prec, n_eps) -> int:
    return mlmc_workspace_bytes(MLMC_OP_LEVEL_ESTIMATE, prec=prec, dlat=dlat, N_fine=N, coupled=coupled,
                                K_fine=K_fine, K_coarse=K_coarse, kgrid=kind, chunk_samples=chunk_samples,
                                n_eps=n_eps)


def mlmc_level_outcomes_workspace(dlat, N, coupled, K_fine, K_coarse, kind, n_outcomes, prec, n_eps) -> int:
    """Workspace bytes for mlmc_level_outcomes on n_outcomes outcomes in one pass."""
    return mlmc_workspace_bytes(MLMC_OP_LEVEL_OUTCOMES_SINGLE_PASS, prec=prec, dlat=dlat, N_fine=N, coupled=coupled,
                                K_fine=K_fine, K_coarse=K_coarse, kgrid=kind, chunk_samples=n_outcomes, n_eps=n_eps)


def mlmc_level_estimate(dlat, N, coupled, p, K_fine, K_coarse, kind, seed, first_sample, M, eps, delta,
                        smoother=MLMC_SMOOTH_GAUSS, prec=MLMC_PREC_FP64, stats=None, work=None, chunk_samples=None,
                        ctx=None, stream=None, first_counter=None):
    """One level's sums ([4][n_eps]: sum Y, sum Y^2, sum Q, sum Q^2, accumulated
    into `stats`).  ctx: a Context (pipelined over its streams) or None (all on
    `stream`).  first_counter: an int64 device tensor [1] added to first_sample
    on the device and advanced by M (for graph capture)."""
    if first_counter is not None:
        _dev(first_counter, torch.int64, "first_counter")
    _dev(eps, torch.float64, "eps")
    ne = eps.shape[0]
    if stats is None:
        stats = torch.zeros((4, ne), dtype=torch.float64, device=eps.device)
    _dev(stats, torch.float64, "stats")
    if work is None:
        chunk = max(1, min(M, 64) if chunk_samples is None else chunk_samples)
        need = mlmc_level_workspace(dlat, N, coupled, K_fine, K_coarse, kind, chunk, prec, ne)
        work = torch.empty((need,), dtype=torch.uint8, device=eps.device)
    _check(lib().mlmc_level_estimate(dlat.handle, N, int(coupled), float(p), K_fine, K_coarse, kind,
                                     int(seed) & (2**64 - 1), first_sample, M, _ptr(eps), ne, float(delta), smoother,
                                     prec, _ptr(stats), _ptr(work), work.numel(), _ptr(first_counter), _ctx(ctx),
                                     _stream(stream)), "mlmc_level_estimate")
    return stats


def mlmc_level_outcomes(dlat, N, coupled, K_fine, K_coarse, kind, mask, eps, delta, smoother=MLMC_SMOOTH_GAUSS,
                        prec=MLMC_PREC_FP64, stats=None, Y=None, Q=None, work=None, chunk_samples=None, ctx=None,
                        stream=None, want_stats=True, want_rows=True):
    """The level over given outcomes `mask` ([M][N][N][G]): per-outcome rows
    Y, Q ([M][n_eps]) and/or the accumulated level sums."""
    _dev(eps, torch.float64, "eps")
    _dev(mask, torch.uint8, "mask")
    ne = eps.shape[0]
    M = mask.shape[0]
    if want_stats and stats is None:
        stats = torch.zeros((4, ne), dtype=torch.float64, device=eps.device)
    if want_rows and Y is None:
        Y = torch.empty((M, ne), dtype=torch.float64, device=eps.device)
    if want_rows and Q is None:
        Q = torch.empty((M, ne), dtype=torch.float64, device=eps.device)
    for t, name in ((stats, "stats"), (Y, "Y"), (Q, "Q")):
        if t is not None:
            _dev(t, torch.float64, name)
    if work is None:
        if chunk_samples is None:  # all outcomes in one pass
            need = mlmc_level_outcomes_workspace(dlat, N, coupled, K_fine, K_coarse, kind, max(1, M), prec, ne)
        else:
            need = mlmc_level_workspace(dlat, N, coupled, K_fine, K_coarse, kind, chunk_samples, prec, ne)
        work = torch.empty((need,), dtype=torch.uint8, device=eps.device)
    _check(lib().mlmc_level_outcomes(dlat.handle, N, int(coupled), K_fine, K_coarse, kind, _ptr(mask), M, _ptr(eps),
                                     ne, float(delta), smoother, prec, _ptr(stats), _ptr(Y), _ptr(Q), _ptr(work),
                                     work.numel(), _ctx(ctx), _stream(stream)), "mlmc_level_outcomes")
    return stats, Y, Q


def mlmc_optimal_samples(V, W, C_alpha, theta, tol) -> np.ndarray:
    V = np.ascontiguousarray(V, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    out = np.zeros_like(V)
    _check(lib().mlmc_optimal_samples(V.shape[0], _ptr(V), _ptr(W), float(C_alpha), float(theta), float(tol),
                                      _ptr(out)), "mlmc_optimal_samples")
    return out


def mlmc_dos(eps, idos) -> np.ndarray:
    """Density of states from an IDoS on an increasing energy grid (host arrays)."""
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    idos = np.ascontiguousarray(idos, dtype=np.float64)
    if eps.shape != idos.shape or eps.ndim != 1:
        raise ValueError("mlmc_dos: eps and idos must be 1-d arrays of one length")
    out = np.zeros_like(idos)
    _check(lib().mlmc_dos(eps.shape[0], _ptr(eps), _ptr(idos), _ptr(out)), "mlmc_dos")
    return out


def mlmc_chase_cus(prec) -> int:
    """CUs (one chase workgroup each) that a level estimate's chase occupies on the current device."""
    out = C.c_int64()
    _check(lib().mlmc_chase_cus(prec, C.byref(out)), "mlmc_chase_cus")
    return out.value
