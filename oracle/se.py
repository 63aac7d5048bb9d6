"""Continuous spectral-element (SE) counterpart of the DG solver (oracle; test
infrastructure only).

Sec. 4.3 (Fig. 6) compares the DG multigrid with the corresponding method for
the continuous spectral element discretisation on the same Cartesian grids; the
DG smoothers of Sec. 3.1 are presented as adaptations of the SE ones.  This
module restates that continuous method from its definitions.

Discretisation.  C0 piecewise polynomials of degree P on the elements, nodal
basis on the GLL points (Sec. 2.4), GLL quadrature.  Global unknowns are the
lattice nodes: per direction the node positions g = 0 .. N P (element m holds
g = m P .. m P + P, neighbours share g = m P).  Homogeneous Dirichlet directions
drop g = 0 and g = N P (stored index g - 1, n = N P - 1 unknowns); periodic ones
identify g with g mod N P (n = N P).  Vectors are lexicographic over the stored
lattice, direction 1 fastest.

System matrix (the definition, ``assemble``): direct stiffness summation
A = sum_e Q_e^T A_e Q_e of the element matrices of the Laplacian with GLL
quadrature, A_e = sum_d (x)_{d' != d} M^e_{d'} (x) L^e_d with the 1D element
mass M^e = (dx/2) diag(rho) and stiffness L^e = (2/dx) L^s (Sec. 2.4).

Multigrid: the V-cycle of Alg. 1 (the DG paper repeats the continuous one) and
MGCG of Alg. 2 are shared with ``multigrid``; levels P_l by halving; coarse
operators rediscretised; prolongation = the embedded interpolation (a
continuous coarse function evaluated at the fine nodes), restriction its
transpose; exact coarse solve.

Smoother: the SE version of EA (weighted additive element-centred Schwarz).
Readings (the paper gives the SE smoother only by reference):
* the subdomain of element m holds the element's nodes plus N_O node layers of
  each neighbour beyond the shared boundary node, g in [m P - N_O, m P + P + N_O];
* the overlap width is the distance from the element boundary to the nearest
  excluded node layer, as for DG: dxi_O = eta_{N_O + 1} + 1;
* N_O = (the DG overlap rule) - 1: the DG subdomain counts the neighbour's
  boundary node, which coincides with the element's own, as a layer of its own
  (Sec. 3.1), so this choice covers the same region and excludes the same node
  layer as the DG subdomain with the rule's N_O; the rule's N_O = 0 (no overlap)
  has no continuous counterpart and is rejected;
* weights: the hat function w_H of eq. (weight function:ec) at the node's
  position relative to the core element; on a Dirichlet side of a boundary
  element the missing term is 1 (as for DG).  With these weights the
  subdomains sum to one at every unknown.
Local problems A_ss = R_s A R_s^T, solved densely (the definition) or by fast
diagonalisation of the restricted 1D matrices (exact on Cartesian grids).

Pins (tests/test_oracle_se.py): closed-form P = 1 matrices; element-loop
assembly against the Kronecker form of independently assembled 1D matrices;
the exact energy of a polynomial; the order of convergence for a manufactured
solution; polynomial reproduction and the 1D Galerkin identity of the
transfers; partition of unity; dense against fast-diagonalisation solves; the
convergence rates Sec. 4.3 quotes for the SE method.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .gll import gll, interp_matrix, stiffness_std
from .multigrid import Hierarchy, level_orders
from .schwarz import overlap_for, w_hat


# --------------------------------------------------------------------------- lattice

def lattice_size(P: int, N: int, periodic: bool) -> int:
    return N * P if periodic else N * P - 1


def stored_index(g, P: int, N: int, periodic: bool):
    """Stored index of lattice position(s) g (-1 for a dropped Dirichlet node)."""
    g = np.asarray(g, dtype=np.int64)
    if periodic:
        return np.mod(g, N * P)
    return np.where((g >= 1) & (g <= N * P - 1), g - 1, -1)


def element_map_1d(P: int, N: int, periodic: bool) -> np.ndarray:
    """(N, P+1) stored indices of every element's nodes (-1: Dirichlet node)."""
    g = np.arange(N)[:, None] * P + np.arange(P + 1)[None, :]
    return stored_index(g, P, N, periodic)


def lattice_shape(grid, P: int):
    """Shape of the lexicographic lattice array (slowest direction first)."""
    return tuple(lattice_size(P, grid.n[d], grid.periodic[d]) for d in reversed(range(grid.dim)))


def n_dof(grid, P: int) -> int:
    return int(np.prod(lattice_shape(grid, P)))


def node_coords_1d(dx: np.ndarray, P: int, periodic: bool) -> np.ndarray:
    """Physical coordinates of the stored lattice nodes of one direction."""
    eta, _ = gll(P)
    dx = np.asarray(dx, dtype=np.float64)
    N = len(dx)
    left = np.concatenate(([0.0], np.cumsum(dx)[:-1]))
    x = np.zeros(N * P + 1)
    for m in range(N):
        x[m * P: m * P + P + 1] = left[m] + 0.5 * (1.0 + eta) * dx[m]
    return x[np.arange(N * P)] if periodic else x[1:N * P]


# --------------------------------------------------------------------------- matrices

def element_matrices_1d(P: int, h: float):
    """1D element mass (diagonal, as a vector) and stiffness with GLL quadrature."""
    _, rho = gll(P)
    return 0.5 * h * rho, (2.0 / h) * stiffness_std(P)


def assemble_1d(P: int, dx, periodic: bool):
    """Assembled 1D (M diagonal vector, L dense) by direct stiffness summation."""
    dx = np.asarray(dx, dtype=np.float64)
    N = len(dx)
    n = lattice_size(P, N, periodic)
    emap = element_map_1d(P, N, periodic)
    M = np.zeros(n)
    L = np.zeros((n, n))
    for m in range(N):
        me, le = element_matrices_1d(P, dx[m])
        for i in range(P + 1):
            a = emap[m, i]
            if a < 0:
                continue
            M[a] += me[i]
            for k in range(P + 1):
                b = emap[m, k]
                if b >= 0:
                    L[a, b] += le[i, k]
    return M, L


def _element_matrix(P: int, h_per_dir) -> np.ndarray:
    """A_e = sum_d (x)_{d' != d} M^e_{d'} (x) L^e_d, local lex order (direction 1 fastest)."""
    dim = len(h_per_dir)
    mats = [element_matrices_1d(P, h) for h in h_per_dir]
    A = None
    for d in range(dim):
        term = np.ones((1, 1))
        for dd in reversed(range(dim)):
            B = mats[dd][1] if dd == d else np.diag(mats[dd][0])
            term = np.kron(term, B)
        A = term if A is None else A + term
    return A


def _element_global_indices(grid, P: int, m_multi) -> np.ndarray:
    """Stored global (flat) indices of one element's local nodes (lex, direction 1
    fastest); -1 where any direction's node is a dropped Dirichlet node."""
    dim = grid.dim
    shape = lattice_shape(grid, P)          # slowest first
    strides = [1] * dim
    for d in range(1, dim):
        strides[d] = strides[d - 1] * shape[dim - d]
    maps = [element_map_1d(P, grid.n[d], grid.periodic[d])[m_multi[d]] for d in range(dim)]
    idx = np.zeros((P + 1,) * dim, dtype=np.int64)   # axes: slowest direction first
    bad = np.zeros((P + 1,) * dim, dtype=bool)
    for d in range(dim):
        sh = [1] * dim
        sh[dim - 1 - d] = P + 1
        a = maps[d].reshape(sh)
        idx = idx + a * strides[d]
        bad = bad | (a < 0)
    return np.where(bad, -1, idx).reshape(-1)


def _elements(grid):
    return np.ndindex(*[grid.n[d] for d in reversed(range(grid.dim))])


def assemble(grid, P: int) -> sp.csr_matrix:
    """A = sum_e Q_e^T A_e Q_e (element loop; the definition)."""
    dim = grid.dim
    n = n_dof(grid, P)
    rows, cols, vals = [], [], []
    for rev in _elements(grid):
        m = tuple(reversed(rev))
        Ae = _element_matrix(P, [float(grid.dx[d][m[d]]) for d in range(dim)])
        gi = _element_global_indices(grid, P, m)
        ok = gi >= 0
        sub = Ae[np.ix_(ok, ok)]
        r, c = np.meshgrid(gi[ok], gi[ok], indexing="ij")
        rows.append(r.reshape(-1))
        cols.append(c.reshape(-1))
        vals.append(sub.reshape(-1))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return A.tocsr()


def assemble_kron(grid, P: int) -> sp.csr_matrix:
    """The same matrix as ``assemble`` in the Kronecker form of the assembled 1D
    matrices, sum_d (x)_{d' != d} M_{d'} (x) L_d (the elements are tensor cells;
    equality with the element loop is pinned by the tests).  Sparse, so it also
    serves grids whose dense element matrices would be too large."""
    dim = grid.dim
    ops = [assemble_1d(P, grid.dx[d], grid.periodic[d]) for d in range(dim)]
    A = None
    for d in range(dim):
        t = sp.identity(1, format="csr")
        for dd in reversed(range(dim)):
            B = sp.csr_matrix(ops[dd][1]) if dd == d else sp.diags(ops[dd][0])
            t = sp.kron(t, B, format="csr")
        A = t if A is None else A + t
    return A.tocsr()


def apply_kron(grid, P: int, u: np.ndarray, ops=None) -> np.ndarray:
    """A u in the Kronecker form, axis by axis with the assembled 1D matrices
    (the same operator as ``assemble_kron``; for grids too large to assemble)."""
    dim = grid.dim
    if ops is None:
        ops = [assemble_1d(P, grid.dx[d], grid.periodic[d]) for d in range(dim)]
    U = np.asarray(u, dtype=np.float64).reshape(lattice_shape(grid, P))
    y = np.zeros_like(U)
    for d in range(dim):
        ax = dim - 1 - d
        t = np.moveaxis(np.moveaxis(U, ax, -1) @ ops[d][1].T, -1, ax)
        for dd in range(dim):
            if dd != d:
                sh = [1] * dim
                sh[dim - 1 - dd] = -1
                t = t * ops[dd][0].reshape(sh)
        y += t
    return y.reshape(-1)


def apply(grid, P: int, u: np.ndarray) -> np.ndarray:
    """A u matrix-free: per element gather, local operator, scatter-add."""
    dim = grid.dim
    y = np.zeros(n_dof(grid, P))
    u = np.asarray(u, dtype=np.float64)
    for rev in _elements(grid):
        m = tuple(reversed(rev))
        gi = _element_global_indices(grid, P, m)
        ok = gi >= 0
        ue = np.where(ok, u[np.where(ok, gi, 0)], 0.0).reshape((P + 1,) * dim)
        ye = np.zeros_like(ue)
        mats = [element_matrices_1d(P, float(grid.dx[d][m[d]])) for d in range(dim)]
        for d in range(dim):
            ax = dim - 1 - d
            t = np.moveaxis(np.moveaxis(ue, ax, -1) @ mats[d][1].T, -1, ax)
            for dd in range(dim):
                if dd != d:
                    sh = [1] * dim
                    sh[dim - 1 - dd] = P + 1
                    t = t * mats[dd][0].reshape(sh)
            ye += t
        np.add.at(y, gi[ok], ye.reshape(-1)[ok])
    return y


def mass_vector(grid, P: int) -> np.ndarray:
    """Diagonal of the assembled (GLL-lumped) mass matrix, lex order."""
    vecs = [assemble_1d(P, grid.dx[d], grid.periodic[d])[0] for d in range(grid.dim)]
    out = vecs[grid.dim - 1]
    for d in reversed(range(grid.dim - 1)):
        out = np.kron(out, vecs[d])
    return out


# --------------------------------------------------------------------------- transfers

def interp_1d(Pf: int, Pc: int, N: int, periodic: bool) -> np.ndarray:
    """Global 1D embedded interpolation (n_f x n_c): row of fine node = the element
    interpolation J of an element containing it (all such elements agree)."""
    J = interp_matrix(Pf, Pc)
    nf, nc = lattice_size(Pf, N, periodic), lattice_size(Pc, N, periodic)
    ef, ec = element_map_1d(Pf, N, periodic), element_map_1d(Pc, N, periodic)
    I = np.zeros((nf, nc))
    for m in range(N):
        for i in range(Pf + 1):
            a = ef[m, i]
            if a < 0:
                continue
            row = np.zeros(nc)
            for k in range(Pc + 1):
                if ec[m, k] >= 0:
                    row[ec[m, k]] += J[i, k]
            I[a] = row
    return I


def interp(grid, Pf: int, Pc: int) -> sp.csr_matrix:
    """nD interpolation: tensor product of the 1D global interpolations (the
    elements are tensor cells, so this is the element-wise J (x) J (x) J)."""
    mats = [sp.csr_matrix(interp_1d(Pf, Pc, grid.n[d], grid.periodic[d])) for d in range(grid.dim)]
    out = mats[grid.dim - 1]
    for d in reversed(range(grid.dim - 1)):
        out = sp.kron(out, mats[d], format="csr")
    return out


# --------------------------------------------------------------------------- smoother

def se_overlap(P_l: int, overlap) -> int:
    """N_O of the continuous subdomains: the DG rule's value minus one."""
    n = overlap_for(P_l, overlap) - 1
    if n < 0:
        raise ValueError("the continuous subdomains need the DG overlap N_O >= 1")
    return n


@dataclass
class Patch1D:
    idx: np.ndarray      # stored indices, patch order
    pos: np.ndarray      # tile positions t = g - (m P - N_O)
    w: np.ndarray


def ec_patches_1d(P: int, N: int, periodic: bool, n_o: int, kind: str) -> List[Patch1D]:
    eta, _ = gll(P)
    if n_o + 1 > P:
        raise ValueError("overlap reaches beyond the neighbouring element")
    dxi_o = eta[n_o + 1] + 1.0
    out = []
    for m in range(N):
        g = np.arange(m * P - n_o, m * P + P + n_o + 1)
        s = stored_index(g, P, N, periodic)
        keep = s >= 0
        gk = g[keep]
        mm = np.floor_divide(gk, P)
        mm = np.where(gk == m * P + P, m, mm)       # the right boundary node in the core's coordinates
        i = gk - mm * P
        xi_h = eta[i] + 2.0 * (mm - m)
        lb = (not periodic) and m == 0
        rb = (not periodic) and m == N - 1
        w = w_hat(xi_h, dxi_o, kind, lb, rb)
        out.append(Patch1D(s[keep].astype(np.int64), np.nonzero(keep)[0], w))
    return out


def _gen_eig(L: np.ndarray, M: np.ndarray):
    """L S = diag(M) S Lambda with S^T diag(M) S = I."""
    msq = 1.0 / np.sqrt(M)
    lam, V = np.linalg.eigh(msq[:, None] * L * msq[None, :])
    return lam, msq[:, None] * V


class SESmoother:
    """Weighted additive element-centred Schwarz on one SE level."""

    def __init__(self, grid, P: int, n_o: int, kind: str, A: Optional[sp.csr_matrix], mode: str = "fdm"):
        self.grid, self.P, self.n_o, self.mode = grid, P, n_o, mode
        self.A = A
        self.dim = grid.dim
        self.shape = lattice_shape(grid, P)
        self.p1 = [ec_patches_1d(P, grid.n[d], grid.periodic[d], n_o, kind) for d in range(grid.dim)]
        self.ops1 = [assemble_1d(P, grid.dx[d], grid.periodic[d]) for d in range(grid.dim)]
        self._eig = {}

    def _eig1(self, d, m):
        key = (d, m)
        if key not in self._eig:
            M, L = self.ops1[d]
            ix = self.p1[d][m].idx
            self._eig[key] = _gen_eig(L[np.ix_(ix, ix)], M[ix])
        return self._eig[key]

    def patches(self):
        return np.ndindex(*[self.grid.n[d] for d in reversed(range(self.dim))])

    def solve_patch(self, m, r_patch: np.ndarray, flat_idx: np.ndarray) -> np.ndarray:
        """A_ss^-1 r_s (r_patch shaped slowest direction first)."""
        if self.mode == "dense":
            As = self.A[flat_idx][:, flat_idx].toarray()
            return np.linalg.solve(As, r_patch.reshape(-1)).reshape(r_patch.shape)
        dim = self.dim
        eigs = [self._eig1(d, m[d]) for d in range(dim)]
        t = r_patch
        for d in range(dim):                       # forward: S_d^T along each axis
            ax = dim - 1 - d
            t = np.moveaxis(np.moveaxis(t, ax, -1) @ eigs[d][1], -1, ax)
        den = np.zeros(t.shape)
        for d in range(dim):
            sh = [1] * dim
            sh[dim - 1 - d] = -1
            den = den + eigs[d][0].reshape(sh)
        t = t / den
        for d in range(dim):                       # backward: S_d along each axis
            ax = dim - 1 - d
            t = np.moveaxis(np.moveaxis(t, ax, -1) @ eigs[d][1].T, -1, ax)
        return t

    def patch_index(self, m):
        """Flat stored indices (patch lex order) and the tensor weight of patch m."""
        dim = self.dim
        shape = self.shape
        strides = [1] * dim
        for d in range(1, dim):
            strides[d] = strides[d - 1] * shape[dim - d]
        flat = np.zeros([1] * dim, dtype=np.int64)
        w = np.ones([1] * dim)
        for d in range(dim):
            sh = [1] * dim
            pd = self.p1[d][m[d]]
            sh[dim - 1 - d] = len(pd.idx)
            flat = flat + pd.idx.reshape(sh) * strides[d]
            w = w * pd.w.reshape(sh)
        return flat, w

    def sweep(self, u: np.ndarray, f: np.ndarray, applyA) -> np.ndarray:
        """u + sum_s R_s^T (w_s A_ss^-1 R_s (f - A u))."""
        r = f - applyA(u)
        du = np.zeros_like(u)
        for rev in self.patches():
            m = tuple(reversed(rev))
            flat, w = self.patch_index(m)
            us = self.solve_patch(m, r[flat], flat.reshape(-1))
            np.add.at(du, flat.reshape(-1), (w * us).reshape(-1))
        return u + du

    def weight_sum(self) -> np.ndarray:
        tot = np.zeros(int(np.prod(self.shape)))
        for rev in self.patches():
            flat, w = self.patch_index(tuple(reversed(rev)))
            np.add.at(tot, flat.reshape(-1), np.broadcast_to(w, flat.shape).reshape(-1))
        return tot


# --------------------------------------------------------------------------- hierarchy

@dataclass
class SELevel:
    P: int
    A: Optional[sp.csr_matrix]
    smoother: Optional[SESmoother]


class SEHierarchy:
    """Levels of the SE problem with the interface ``multigrid.mgcg`` drives."""

    vcycle = Hierarchy.vcycle

    def __init__(self, grid, method, patch_mode: str = "fdm", assemble_all: bool = True):
        if method.smoother != "EA":
            raise ValueError("the SE counterpart uses the element-centred additive smoother")
        self.grid, self.method = grid, method
        self.orders = level_orders(method.P)
        self.levels: List[SELevel] = []
        for l, Pl in enumerate(self.orders):
            A = assemble_kron(grid, Pl) if (assemble_all or l == 0 or patch_mode == "dense") else None
            sm = None
            if l > 0:
                sm = SESmoother(grid, Pl, se_overlap(Pl, method.overlap), method.weighting, A, patch_mode)
            self.levels.append(SELevel(Pl, A, sm))
        self._I = {l: interp(grid, self.orders[l], self.orders[l - 1]) for l in range(1, len(self.orders))}
        A0 = self.levels[0].A
        self.periodic_all = all(grid.periodic)
        if self.periodic_all:
            self._lu0 = spla.splu(sp.csc_matrix(A0[1:, 1:]))
        else:
            self._lu0 = spla.splu(sp.csc_matrix(A0))

    @property
    def L(self):
        return len(self.orders) - 1

    def apply(self, l: int, u: np.ndarray) -> np.ndarray:
        lev = self.levels[l]
        if lev.A is not None:
            return lev.A @ u
        return apply_kron(self.grid, lev.P, u, ops=lev.smoother.ops1 if lev.smoother is not None else None)

    def prolong(self, l: int, uc: np.ndarray) -> np.ndarray:
        return self._I[l] @ uc

    def restrict(self, l: int, rf: np.ndarray) -> np.ndarray:
        return self._I[l].T @ rf

    def coarse_solve(self, f0: np.ndarray) -> np.ndarray:
        if self.periodic_all:
            f = f0 - f0.mean()
            x = np.zeros_like(f)
            x[1:] = self._lu0.solve(f[1:])
            return x - x.mean()
        return self._lu0.solve(f0)

    def smooth(self, l: int, u, f, steps: int, start: int = 0):
        for _ in range(steps):
            u = self.levels[l].smoother.sweep(u, f, lambda v: self.apply(l, v))
        return u
