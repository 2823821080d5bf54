"""Honeycomb lattice descriptions used as inputs (tight-binding data only).

Section 3.1 of the paper defines the tight-binding model on a honeycomb
lattice with two sublattice sites A and B per primitive cell; Section 3.2
defines vacancies as removal of all orbitals of a site.

A lattice is described by

* primitive vectors ``a1, a2`` (Angstrom) and the primitive cell area |F|,
* orbital positions in fractional coordinates of (a1, a2),
* a group id per orbital (a group is the set of orbitals removed together
  when a vacancy occurs) and a removable flag per group,
* a hopping table: each row ``(R1, R2, from, to, re, im)`` contributes
  ``h * exp(i k . (R + r_to - r_from))`` to ``H[from, to]`` and the complex
  conjugate to ``H[to, from]``.  A row with ``R = 0`` and ``from == to`` is an
  on-site energy and is added once.

Two lattices are provided:

* ``graphene``: one p_z orbital per atom, nearest-neighbour hopping
  t = -2.7 eV, on-site 0, orthogonal basis (overlap S = I).  Each of the two
  atoms is its own removable group.  The lattice constant a = 2.46 A only
  sets |F|.
* ``mos2_shaped``: a synthetic stand-in with the orbital and vacancy
  structure of a MoS2 monolayer (11 orbitals per cell: Mo d x5 on site A,
  top-S p x3 and bottom-S p x3 on site B).  Its parameters are random
  (iid uniform on [-1.5, 1.5] eV), drawn once from ``param_seed`` in the fixed
  order documented in :func:`mos2_shaped`.  Mo is never removed; each S site
  is its own 3-orbital removable group, or (``s_pairs``) the two S of a cell
  are removed together as one 6-orbital group.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

HOP_DTYPE = np.dtype(
    [("R1", np.int32), ("R2", np.int32), ("frm", np.int32), ("to", np.int32),
     ("re", np.float64), ("im", np.float64)]
)


@dataclass(frozen=True)
class Lattice:
    name: str
    lattice_id: int            # used in the vacancy-RNG stream tag
    a1: tuple
    a2: tuple
    cell_area: float           # |F| in Angstrom^2
    orb_frac: np.ndarray       # [n_orb, 2] float64
    orb_group: np.ndarray      # [n_orb] int32
    group_removable: np.ndarray  # [n_groups] uint8
    hops: np.ndarray           # [n_hops] HOP_DTYPE
    # Non-orthogonal basis: S(k) = I + Bloch sum of this table (HOP_DTYPE), or
    # None for an orthogonal basis (S = I).
    overlap: np.ndarray = None

    @property
    def n_orb(self) -> int:
        return int(self.orb_frac.shape[0])

    @property
    def n_groups(self) -> int:
        return int(self.group_removable.shape[0])

    @property
    def n_hops(self) -> int:
        return int(self.hops.shape[0])

    @property
    def has_overlap(self) -> bool:
        return self.overlap is not None

    def max_orbitals(self, N: int) -> int:
        """Matrix side of the pristine N x N supercell."""
        return self.n_orb * N * N

    def hop_magnitude_bound(self) -> float:
        """Largest per-orbital sum of |h| over hopping-table rows touching it.

        Used only to choose an energy window that covers every spectrum."""
        s = np.zeros(self.n_orb)
        for h in self.hops:
            mag = math.hypot(h["re"], h["im"])
            onsite = h["R1"] == 0 and h["R2"] == 0 and h["frm"] == h["to"]
            if onsite:
                s[h["frm"]] += mag
            else:
                s[h["frm"]] += mag
                s[h["to"]] += mag
        return float(s.max())


def _hops(rows):
    arr = np.zeros(len(rows), dtype=HOP_DTYPE)
    for i, (R1, R2, f, t, re, im) in enumerate(rows):
        arr[i] = (R1, R2, f, t, re, im)
    return arr


def graphene(t: float = -2.7, a: float = 2.46) -> Lattice:
    """Nearest-neighbour pi-band graphene (orthogonal form, eps_2p = 0).

    A at fractional (0, 0), B at (1/3, 1/3); the three A->B bonds go to B in
    cells (0, 0), (-1, 0) and (0, -1)."""
    rows = [(0, 0, 0, 1, t, 0.0), (-1, 0, 0, 1, t, 0.0), (0, -1, 0, 1, t, 0.0)]
    return Lattice(
        name="graphene",
        lattice_id=1,
        a1=(a, 0.0),
        a2=(0.5 * a, 0.5 * math.sqrt(3.0) * a),
        cell_area=0.5 * math.sqrt(3.0) * a * a,
        orb_frac=np.array([[0.0, 0.0], [1.0 / 3.0, 1.0 / 3.0]]),
        orb_group=np.array([0, 1], dtype=np.int32),
        group_removable=np.array([1, 1], dtype=np.uint8),
        hops=_hops(rows),
    )


def graphene_overlap(t: float = -3.033, s: float = 0.129, eps_2p: float = 0.0, a: float = 2.46) -> Lattice:
    """Graphene in the non-orthogonal nearest-neighbour model of Section 3.1:
    hopping t and overlap s on the three A-B bonds, on-site energy eps_2p and
    unit on-site overlap, i.e. the generalised problem H c = E S c with
    S = I + s (bond Bloch sum).  Groups and geometry as in ``graphene``; its
    own lattice id, so its vacancy stream is independent."""
    rows = [(0, 0, 0, 1, t, 0.0), (-1, 0, 0, 1, t, 0.0), (0, -1, 0, 1, t, 0.0)]
    if eps_2p != 0.0:
        rows += [(0, 0, 0, 0, eps_2p, 0.0), (0, 0, 1, 1, eps_2p, 0.0)]
    ovl = [(0, 0, 0, 1, s, 0.0), (-1, 0, 0, 1, s, 0.0), (0, -1, 0, 1, s, 0.0)]
    return Lattice(
        name="graphene_overlap",
        lattice_id=4,
        a1=(a, 0.0),
        a2=(0.5 * a, 0.5 * math.sqrt(3.0) * a),
        cell_area=0.5 * math.sqrt(3.0) * a * a,
        orb_frac=np.array([[0.0, 0.0], [1.0 / 3.0, 1.0 / 3.0]]),
        orb_group=np.array([0, 1], dtype=np.int32),
        group_removable=np.array([1, 1], dtype=np.uint8),
        hops=_hops(rows),
        overlap=_hops(ovl),
    )


MOS2_MO = list(range(0, 5))      # Mo d orbitals (site A)
MOS2_S = list(range(5, 11))      # top-S p x3 (5,6,7) then bottom-S p x3 (8,9,10) (site B)
NN_DIRS = [(0, 0), (-1, 0), (0, -1)]          # A -> B nearest-neighbour cells
SAME_SUBLATTICE_DIRS = [(1, 0), (0, 1), (-1, 1)]  # a1, a2, a2 - a1


def mos2_shaped(param_seed: int = 4040, a: float = 3.19, scale: float = 1.5, s_pairs: bool = False) -> Lattice:
    """MoS2-shaped 11-orbital honeycomb model with random real parameters.

    Vacancy groups: Mo (never removed) and, by default, each S site on its
    own (3 orbitals).  With ``s_pairs`` the top and bottom S of a cell form one
    6-orbital group removed together (the S-pair vacancies of Section 3.2);
    that lattice has its own id, so its vacancy stream is independent.

    Draw order (one ``Generator(Philox(param_seed)).uniform(-scale, scale)``
    stream, consumed in this order):

    1. Mo on-site 5x5 symmetric block: entries (m, m') with m <= m', row-major.
    2. S on-site 6x6 symmetric block, same order (orbitals 5..10).
    3. Mo -> S blocks 5x6 for the nearest-neighbour cells (0,0), (-1,0),
       (0,-1), each block row-major.
    4. Mo -> Mo blocks 5x5 for R = a1, a2, a2 - a1, each row-major.
    5. S -> S blocks 6x6 for the same three R, each row-major.

    The reverse directions (-R) are implied by the Hermitian rule of the
    hopping table."""
    rng = np.random.Generator(np.random.Philox(param_seed))
    rows = []

    def u():
        return float(rng.uniform(-scale, scale))

    for block in (MOS2_MO, MOS2_S):
        for ii, m in enumerate(block):
            for mp in block[ii:]:
                rows.append((0, 0, m, mp, u(), 0.0))
    for (R1, R2) in NN_DIRS:
        for m in MOS2_MO:
            for mp in MOS2_S:
                rows.append((R1, R2, m, mp, u(), 0.0))
    for block in (MOS2_MO, MOS2_S):
        for (R1, R2) in SAME_SUBLATTICE_DIRS:
            for m in block:
                for mp in block:
                    rows.append((R1, R2, m, mp, u(), 0.0))
    frac = np.array([[0.0, 0.0]] * 5 + [[1.0 / 3.0, 1.0 / 3.0]] * 6)
    if s_pairs:
        group = np.array([0] * 5 + [1] * 6, dtype=np.int32)
        removable = np.array([0, 1], dtype=np.uint8)
    else:
        group = np.array([0] * 5 + [1] * 3 + [2] * 3, dtype=np.int32)
        removable = np.array([0, 1, 1], dtype=np.uint8)
    return Lattice(
        name="mos2_shaped_spairs" if s_pairs else "mos2_shaped",
        lattice_id=3 if s_pairs else 2,
        a1=(a, 0.0),
        a2=(0.5 * a, 0.5 * math.sqrt(3.0) * a),
        cell_area=0.5 * math.sqrt(3.0) * a * a,
        orb_frac=frac,
        orb_group=group,
        group_removable=removable,
        hops=_hops(rows),
    )


def lattice_by_name(name: str) -> Lattice:
    if name == "graphene":
        return graphene()
    if name in ("mos2_shaped", "mos2"):
        return mos2_shaped()
    if name in ("mos2_shaped_spairs", "mos2_spairs"):
        return mos2_shaped(s_pairs=True)
    if name == "graphene_overlap":
        return graphene_overlap()
    raise ValueError(f"unknown lattice {name!r}")
