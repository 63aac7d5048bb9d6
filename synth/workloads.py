"""Grid recipes, method options and seeded draws for the synthetic Poisson problems.

Every random quantity is drawn from ``numpy.random.default_rng(seed)`` (PCG64)
in a fixed order: grid parameters first, then the right-hand side, then the
initial guess.  Vectors are produced in the library's element-major GLL order
(element index e = m1 + N1*(m2 + N2*m3), x fastest inside an element), which is
a pure indexing convention and involves no node coordinates.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

DIRICHLET = "dirichlet"
PERIODIC = "periodic"


@dataclass
class Grid:
    """Cartesian tensor-product grid: per-direction element sizes."""

    dim: int
    dx: Tuple[np.ndarray, ...]          # one array of element sizes per direction
    periodic: Tuple[bool, ...]          # per direction

    @property
    def n(self) -> Tuple[int, ...]:
        return tuple(len(d) for d in self.dx)

    @property
    def n_elem(self) -> int:
        return int(np.prod(self.n))

    def n_dof(self, P: int) -> int:
        return self.n_elem * (P + 1) ** self.dim

    def n_lattice(self, P: int) -> int:
        """Unknowns of the continuous counterpart: per direction the N P element
        boundary and interior node positions, less the two ends when Dirichlet."""
        out = 1
        for d in range(self.dim):
            out *= len(self.dx[d]) * P - (0 if self.periodic[d] else 1)
        return out

    def aspect_ratio(self) -> float:
        """Largest ratio of two element sizes within any single element."""
        if self.dim == 1:
            return 1.0
        mx = max(float(np.max(d)) for d in self.dx)
        mn = min(float(np.min(d)) for d in self.dx)
        return mx / mn


@dataclass
class Method:
    """Solver options (names follow the paper's notation).

    flux: "ip" or "ldg"; beta: per-direction LDG parameter; mu_star: penalty
    factor; smoother: "EA" / "FA" (element- / face-centred weighted additive)
    or "EM" / "FM" (element- / face-centred multiplicative); overlap: "level"
    (N_O = 1 + P_l/8 rounded), "level_floor", "zero", or an int; weighting:
    "quintic", "cubic", "arith", "none" (additive smoothers only); vcycle:
    "classical" or "variable"; precision: "fp64" or "mixed"; order: subdomain
    order of the multiplicative smoothers, "lex" (lexicographic, direction 1
    fastest) or "colour" (colour classes of mutually independent subdomains);
    disc: "dg" or "se" (the continuous spectral-element counterpart, with the
    element-centred additive smoother).
    """

    P: int
    flux: str = "ip"
    beta: Tuple[float, ...] = (0.0, 0.0, 0.0)
    mu_star: float = 1.0
    smoother: str = "EA"
    overlap: object = "level"
    weighting: str = "quintic"
    vcycle: str = "classical"
    ns: Tuple[int, int] = (1, 1)
    precision: str = "fp64"
    krylov: bool = True
    order: str = "lex"
    disc: str = "dg"


@dataclass
class Workload:
    name: str
    grid: Grid
    method: Method
    seed: Optional[int]
    rhs_kind: str                      # "uniform" (i.i.d. U[-1,1]) or "manufactured"
    tol: float = 1e-10

    @property
    def n_dof(self) -> int:
        if self.method.disc == "se":
            return self.grid.n_lattice(self.method.P)
        return self.grid.n_dof(self.method.P)


def uniform_grid(dim: int, n: Sequence[int] | int, lengths: Sequence[float] | float = 1.0,
                 periodic: bool | Sequence[bool] = False) -> Grid:
    if isinstance(n, int):
        n = (n,) * dim
    if isinstance(lengths, (int, float)):
        lengths = (float(lengths),) * dim
    if isinstance(periodic, bool):
        periodic = (periodic,) * dim
    dx = tuple(np.full(int(n[d]), float(lengths[d]) / int(n[d])) for d in range(dim))
    return Grid(dim=dim, dx=dx, periodic=tuple(bool(p) for p in periodic))


def geometric_spacing(n: int, first: float, total: float = 1.0) -> np.ndarray:
    """Sizes first*q**k, k = 0..n-1, with the ratio q chosen so that they sum to total."""
    def s(q):
        return first * (q ** n - 1.0) / (q - 1.0) if abs(q - 1.0) > 1e-14 else first * n
    lo, hi = 1.0 + 1e-12, 4.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if s(mid) < total:
            lo = mid
        else:
            hi = mid
    q = 0.5 * (lo + hi)
    h = first * q ** np.arange(n, dtype=np.float64)
    return h * (total / h.sum())


def random_spacing(rng: np.random.Generator, n: int, max_log2: float = 5.0,
                   total: float = 1.0) -> np.ndarray:
    """Sizes proportional to 2**U(0, max_log2), normalised to sum to total."""
    h = 2.0 ** rng.uniform(0.0, max_log2, size=n)
    return h * (total / h.sum())


def rhs_uniform(seed: int, n_dof: int, rng: Optional[np.random.Generator] = None) -> np.ndarray:
    """Right-hand side with i.i.d. U[-1, 1] entries (element-major order)."""
    rng = np.random.default_rng(seed) if rng is None else rng
    return rng.uniform(-1.0, 1.0, size=n_dof)


def guess_uniform01(seed: int, n_dof: int) -> np.ndarray:
    """Random initial guess in [0, 1] as used for the paper's convergence tables."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=n_dof)


# --------------------------------------------------------------------------- configs

def c1_poisson2d_p4() -> Workload:
    """2D Poisson on [0,1]^2, 4x4 elements, SIPG P=4, Dirichlet, manufactured RHS, EA_l."""
    g = uniform_grid(2, 4, 1.0, False)
    m = Method(P=4, flux="ip", beta=(0.0, 0.0), smoother="EA", overlap="level")
    return Workload("poisson2d_4x4_p4_sipg_ea", g, m, None, "manufactured")


def c2_poisson3d_p8(n: int = 16) -> Workload:
    """3D Poisson on [0,1]^3, n^3 elements, SIPG P=8, Dirichlet, U[-1,1] RHS, FA_l, FP64."""
    g = uniform_grid(3, n, 1.0, False)
    m = Method(P=8, flux="ip", beta=(0.0, 0.0, 0.0), smoother="FA", overlap="level")
    return Workload(f"poisson3d_{n}^3_p8_sipg_fa_fp64", g, m, 2, "uniform")


def c3_ldg3d_stretched(n: int = 32, ar: float = 32.0) -> Workload:
    """3D LDG (beta = 1/2), n^3 elements, z geometrically stretched (first size 1/(n*ar)), mixed."""
    dz = geometric_spacing(n, 1.0 / (n * ar), 1.0)
    g = Grid(3, (np.full(n, 1.0 / n), np.full(n, 1.0 / n), dz), (False, False, False))
    m = Method(P=8, flux="ldg", beta=(0.5, 0.5, 0.5), smoother="FA", overlap="level",
               precision="mixed")
    return Workload(f"ldg3d_{n}^3_zstretch{int(ar)}_p8_fa_mixed", g, m, 3, "uniform")


def c4_batched(seed: int = 4, count: int = 64, n_range=(4, 16),
               orders=(4, 6, 8, 12, 16)) -> List[Workload]:
    """Independent 3D SIPG grids: N ~ U{n_range}, P ~ orders, domain lengths 2**U(0,3)."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        P = int(rng.choice(orders))
        lengths = 2.0 ** rng.uniform(0.0, 3.0, size=3)
        lengths = lengths / lengths.min()
        g = uniform_grid(3, n, tuple(lengths), False)
        m = Method(P=P, flux="ip", beta=(0.0, 0.0, 0.0), smoother="FA", overlap="level",
                   precision="mixed")
        out.append(Workload(f"batch{b}_{n}^3_p{P}", g, m, seed * 1000 + b, "uniform"))
    return out


def c5_poisson3d_p32(seed: int = 5, n: int = 8) -> Workload:
    """3D SIPG P=32 on n^3 elements with random per-direction sizes (aspect ratios up to 32)."""
    rng = np.random.default_rng(seed)
    dx = tuple(random_spacing(rng, n, 5.0, 1.0) for _ in range(3))
    g = Grid(3, dx, (False, False, False))
    m = Method(P=32, flux="ip", beta=(0.0, 0.0, 0.0), smoother="FA", overlap="level",
               precision="mixed")
    return Workload(f"poisson3d_{n}^3_p32_fa", g, m, seed, "uniform")


def paper_periodic_2d(P: int, n: int = 16, ar: int = 1, smoother: str = "EA",
                      overlap: object = "level", beta: float = 0.0, weighting: str = "quintic",
                      krylov: bool = True, vcycle: str = "classical", order: str = "lex") -> Workload:
    """The paper's test case: periodic (0, 2AR) x (0, 2), n x n equal elements."""
    g = uniform_grid(2, n, (2.0 * ar, 2.0), True)
    m = Method(P=P, flux="ip" if beta == 0.0 else "ldg", beta=(beta, beta), smoother=smoother,
               overlap=overlap, weighting=weighting, krylov=krylov, vcycle=vcycle, order=order)
    return Workload(f"periodic2d_{n}x{n}_ar{ar}_p{P}_{smoother}", g, m, 0, "manufactured")


def se_poisson3d_p8(n: int = 16) -> Workload:
    """The continuous spectral-element counterpart of EA_l on the 3D grid of
    poisson3d_16^3_p8: [0,1]^3, n^3 elements, P = 8, Dirichlet, U[-1,1] RHS, FP64."""
    g = uniform_grid(3, n, 1.0, False)
    m = Method(P=8, smoother="EA", overlap="level", disc="se")
    return Workload(f"se_poisson3d_{n}^3_p8_ea_fp64", g, m, 6, "uniform")


def paper_fig6_2d(P: int, disc: str = "dg") -> Workload:
    """The workload of Fig. 6: (256/P)^2 square elements of order P on the paper's
    periodic domain (0, 2)^2, EA_l (DG or its continuous counterpart)."""
    w = paper_periodic_2d(P, n=256 // P, smoother="EA")
    return Workload(f"fig6_{disc}_{256 // P}x{256 // P}_p{P}_ea", w.grid, replace(w.method, disc=disc), 7, "uniform")


def with_method(w: Workload, **kw) -> Workload:
    return replace(w, method=replace(w.method, **kw))
