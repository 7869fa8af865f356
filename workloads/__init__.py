"""Seeded synthetic inputs for the ChFSI hot path.

This module only draws inputs: atom positions and parameters of the
synthetic Gaussian systems, random start blocks and Lanczos start vectors.
It holds none of the method's arithmetic (no finite-element tables, no
operator, no filter).  Both the oracle and the HIP library consume what it
produces, so they see identical inputs.

The workloads stand in for the paper's ONCV-pseudopotential Mo/Al/InP
benchmark systems (Section 5), which need pseudopotential files and
reference codes that are not available here.  They keep the paper's
discretisation scale: spectral elements of order 4-6 on cells of about
2 bohr (Tables of Section 5.1 use h of about 2 bohr at p = 6-7).

Draw order per system (one ``numpy.random.default_rng(seed)`` stream):
positions uniform in [0, L)^3, one atom at a time, each candidate rejected
while its minimum-image distance to an accepted atom is below ``d_min``;
then Z ~ U[1, 4] for all atoms, s ~ U[0.5, 1.0]; if the system has
projectors, w ~ U[0.8, 1.5], h_s ~ U[-2, 2], h_p ~ U[-2, 2].
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "System", "Config", "CONFIGS", "make_system", "start_block",
    "lanczos_start", "kpoints_mp4", "config", "small_system",
]


@dataclasses.dataclass
class System:
    """A periodic cube [0, L)^3 meshed by ``ncell``^3 hex cells of order ``p``.

    Atoms carry a Gaussian local potential -Z exp(-r^2 / (2 s^2)) and, when
    ``has_proj`` is set, one s and three p Gaussian-radial projectors of
    width ``w`` with couplings ``h_s`` and ``h_p`` (Ha).  ``k`` is the Bloch
    wave vector (bohr^-1); k = 0 is the real Gamma-point problem.
    """

    L: float
    ncell: int
    p: int
    pos: np.ndarray            # (na, 3) bohr
    Z: np.ndarray              # (na,)
    s: np.ndarray              # (na,) bohr
    has_proj: bool = False
    w: Optional[np.ndarray] = None      # (na,) bohr
    h_s: Optional[np.ndarray] = None    # (na,) Ha
    h_p: Optional[np.ndarray] = None    # (na,) Ha
    k: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    seed: int = 0

    @property
    def natoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n(self) -> int:
        """Unique nodes per direction on the periodic mesh."""
        return self.ncell * self.p

    @property
    def M(self) -> int:
        return self.n ** 3

    @property
    def E(self) -> int:
        return self.ncell ** 3

    @property
    def mcell(self) -> int:
        return (self.p + 1) ** 3

    @property
    def is_complex(self) -> bool:
        return bool(np.any(np.asarray(self.k) != 0.0))

    def with_k(self, k) -> "System":
        return dataclasses.replace(self, k=np.asarray(k, dtype=np.float64))


@dataclasses.dataclass
class Config:
    name: str
    L: float
    ncell: int
    p: int
    natoms: int
    d_min: float
    has_proj: bool
    nwanted: int
    block: int
    degree: int
    passes: Optional[int]
    seed: int


def _min_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def make_system(L: float, ncell: int, p: int, natoms: int, seed: int,
                d_min: float = 1.0, has_proj: bool = False,
                k: Sequence[float] = (0.0, 0.0, 0.0)) -> System:
    """Draw one seeded synthetic system (draw order in the module docstring)."""
    rng = np.random.default_rng(seed)
    pos: List[np.ndarray] = []
    tries = 0
    while len(pos) < natoms:
        cand = rng.uniform(0.0, L, size=3)
        tries += 1
        if tries > 1_000_000:
            raise RuntimeError("could not place atoms with the requested separation")
        ok = True
        for q in pos:
            if np.linalg.norm(_min_image(cand - q, L)) < d_min:
                ok = False
                break
        if ok:
            pos.append(cand)
    P = np.array(pos, dtype=np.float64).reshape(natoms, 3)
    Z = rng.uniform(1.0, 4.0, size=natoms)
    s = rng.uniform(0.5, 1.0, size=natoms)
    w = h_s = h_p = None
    if has_proj:
        w = rng.uniform(0.8, 1.5, size=natoms)
        h_s = rng.uniform(-2.0, 2.0, size=natoms)
        h_p = rng.uniform(-2.0, 2.0, size=natoms)
    return System(L=float(L), ncell=int(ncell), p=int(p), pos=P, Z=Z, s=s,
                  has_proj=has_proj, w=w, h_s=h_s, h_p=h_p,
                  k=np.asarray(k, dtype=np.float64), seed=int(seed))


def kpoints_mp4(L: float) -> np.ndarray:
    """Shifted 2x2x2 Monkhorst-Pack grid reduced by time reversal to 4 points.

    Each carries weight 1/4; they are (2 pi / L) / 4 times (1,1,1), (1,1,-1),
    (1,-1,1), (-1,1,1).
    """
    f = 2.0 * math.pi / L * 0.25
    return f * np.array([[1, 1, 1], [1, 1, -1], [1, -1, 1], [-1, 1, 1]], dtype=np.float64)


# The five workloads.  c2 reuses c1's operator; c3 is a list of 8 systems.
CONFIGS = {
    "c0": Config("c0_fp64_gamma_p4_4096", L=10.0, ncell=4, p=4, natoms=2, d_min=1.0,
                 has_proj=False, nwanted=32, block=32, degree=20, passes=10, seed=0),
    "c1": Config("c1_fp64_gamma_p6_2985984", L=48.0, ncell=24, p=6, natoms=64, d_min=2.0,
                 has_proj=True, nwanted=256, block=128, degree=30, passes=None, seed=1000),
    "c2": Config("c2_mixed_p6_2985984_n1024", L=48.0, ncell=24, p=6, natoms=64, d_min=2.0,
                 has_proj=True, nwanted=1024, block=128, degree=30, passes=None, seed=1000),
    "c4": Config("c4_learned_p5_216000", L=24.0, ncell=12, p=5, natoms=16, d_min=1.0,
                 has_proj=True, nwanted=128, block=128, degree=30, passes=None, seed=4000),
}

# (ncell, natoms, nwanted) for the 8 batched systems; h = 2 bohr, p = 5.
C3_SYSTEMS = [(8, 8, 64), (10, 12, 96), (11, 16, 128), (13, 24, 160),
              (15, 28, 224), (17, 36, 256), (18, 40, 320), (20, 48, 384)]


# (ncell, natoms, nwanted) for a batch of small p = 5 boxes (h = 2 bohr), each
# at the 4 Monkhorst-Pack k-points: problems far too small to fill the GPU
# one at a time (M = 3,375 .. 27,000).
SMALL_BATCH_SYSTEMS = [(3, 2, 16), (3, 3, 24), (4, 2, 16), (4, 3, 24), (4, 4, 32), (5, 3, 24),
                       (5, 4, 32), (5, 5, 40), (6, 4, 32), (6, 5, 40), (6, 6, 48), (3, 2, 24),
                       (4, 5, 40), (5, 6, 48), (6, 3, 24), (4, 2, 16)]


def config(name: str, index: int = 0) -> System:
    """The seeded system of workload ``name`` (``index`` selects c3/c4 members)."""
    if name == "c3":
        nc, na, _ = C3_SYSTEMS[index]
        return make_system(2.0 * nc, nc, 5, na, seed=3000 + index, d_min=1.0, has_proj=True)
    if name == "small_batch":
        nc, na, _ = SMALL_BATCH_SYSTEMS[index]
        return make_system(2.0 * nc, nc, 5, na, seed=6000 + index, d_min=1.0, has_proj=True)
    c = CONFIGS[name]
    seed = c.seed + index
    return make_system(c.L, c.ncell, c.p, c.natoms, seed=seed, d_min=c.d_min,
                       has_proj=c.has_proj)


def small_system(ncell: int, p: int, natoms: int, seed: int, L: Optional[float] = None,
                 has_proj: bool = False, k=(0.0, 0.0, 0.0)) -> System:
    """A small seeded system for parity tests (h = 2 bohr unless L is given)."""
    if L is None:
        L = 2.0 * ncell
    return make_system(L, ncell, p, natoms, seed=seed, d_min=1.0, has_proj=has_proj, k=k)


def start_block(M: int, N: int, seed: int, complex_: bool = False) -> np.ndarray:
    """Random N(0,1) start block, row-major M x N (C order).

    Complex blocks draw a real plane then an imaginary plane, each scaled by
    1/sqrt(2).
    """
    rng = np.random.default_rng(seed)
    if not complex_:
        return rng.standard_normal((M, N))
    re = rng.standard_normal((M, N))
    im = rng.standard_normal((M, N))
    return (re + 1j * im) / math.sqrt(2.0)


def lanczos_start(M: int, seed: int, complex_: bool = False) -> np.ndarray:
    """Seeded N(0,1) vector used to start the Lanczos bound (not normalised)."""
    return start_block(M, 1, seed, complex_)[:, 0].copy()
