"""p-multigrid V-cycle (Alg. 1) and inexact MG-preconditioned CG (Alg. 2) (oracle).

Level series: P_L = P and P_{l-1} = floor(P_l / 2) down to P_0 = 1 (Sec. 3.2
gives P_l = 2^l; the halving rule is the reading used for other orders).
Coarse operators are rediscretisations at order P_l with the same grid,
fluxes and mu_star.  Transfers: prolongation by the element-local tensor
product of the embedded interpolation J_l, restriction by its transpose.

Coarse solve u_0 = A_0^+ f_0 (Alg. 1): exact, by sparse LU.  For periodic grids
the right side is made orthogonal to the constants and the minimum-norm
(mean-free) solution is returned.

MGCG (Alg. 2) is implemented as printed, with one reading: the update of the
search-direction coefficient uses the preconditioned residual,
beta = z^T (r - r_old) / delta (the flexible CG of Golub and Ye; the printed
q^T(...) is a misprint).  r_old starts at zero as printed.  Exit test:
Euclidean norm of the recursively updated residual <= tol * ||r_0||, confirmed
by the true residual g - A u (Alg. 2 stops on r_max; the recursion and the
true residual drift apart by rounding): when the recursive norm passes but the
true one does not, r is replaced by the true residual and the iteration goes on.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .gll import interp_matrix
from .operator import apply_kron, assemble_kron, lex_shape, operators_1d, _betas
from .schwarz import SmootherLevel, overlap_for


def level_orders(P: int) -> List[int]:
    """[P_0 = 1, ..., P_L = P] by repeated halving."""
    out = [P]
    while out[-1] > 1:
        out.append(out[-1] // 2)
    return list(reversed(out))


def ns_for(method, L: int, l: int):
    """Smoothing counts (N_S1, N_S2) on level l: classical (1,1) or variable 2^(L-l)."""
    if method.vcycle == "variable":
        k = 2 ** (L - l)
        return (k * method.ns[0], k * method.ns[1])
    return tuple(method.ns)


def _prolong_axis(u, J, N, ax):
    """Apply blockdiag_N(J) along axis ``ax`` of u."""
    u = np.moveaxis(u, ax, -1)
    sh = u.shape[:-1]
    nc = J.shape[1]
    v = u.reshape(sh + (N, nc)) @ J.T
    return np.moveaxis(v.reshape(sh + (N * J.shape[0],)), -1, ax)


def _restrict_axis(u, J, N, ax):
    u = np.moveaxis(u, ax, -1)
    sh = u.shape[:-1]
    nf = J.shape[0]
    v = u.reshape(sh + (N, nf)) @ J
    return np.moveaxis(v.reshape(sh + (N * J.shape[1],)), -1, ax)


@dataclass
class Level:
    P: int
    A: Optional[sp.csr_matrix]
    smoother: Optional[SmootherLevel]
    ops: list


class Hierarchy:
    """All levels of one problem; vectors are lexicographic flat FP64 arrays."""

    def __init__(self, grid, method, patch_mode: str = "fdm", assemble: bool = True, face_params=None,
                 coarse: bool = True):
        """face_params: optional {level: [(theta[nf], omega[nf]) per direction]} for the
        face-centred normal weights (learned-weight variant; see fc_patches_1d).
        coarse=False skips the coarse LU and assembly (level operations only, for
        grids too large for a sparse direct solve)."""
        self.grid = grid
        self.method = method
        self.orders = level_orders(method.P)
        betas = _betas(method.beta, grid.dim)
        self.levels: List[Level] = []
        for l, Pl in enumerate(self.orders):
            ops = [operators_1d(Pl, np.asarray(grid.dx[d]), grid.periodic[d], betas[d], method.mu_star)
                   for d in range(grid.dim)]
            A = assemble_kron(grid, Pl, betas, method.mu_star) if (assemble or (l == 0 and coarse)) else None
            sm = None
            if l > 0:
                if A is not None:
                    applyA = (lambda A_: (lambda u: A_ @ u))(A)
                else:
                    applyA = (lambda P_, ops_: (lambda u: apply_kron(grid, P_, u, ops=ops_)))(Pl, ops)
                sm = SmootherLevel(grid, Pl, overlap_for(Pl, method.overlap), method.weighting,
                                   method.smoother, applyA, A, ops, mode=patch_mode,
                                   face_params=None if face_params is None else face_params.get(l),
                                   order=getattr(method, "order", "lex"))
            self.levels.append(Level(Pl, A, sm, ops))
        A0 = self.levels[0].A
        self.periodic_any = all(grid.periodic)
        if not coarse:
            self._lu0 = None
        elif self.periodic_any:
            # pin the first unknown, solve, then remove the mean (min-norm solution)
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
        return apply_kron(self.grid, lev.P, u, ops=lev.ops)

    def prolong(self, l: int, uc: np.ndarray) -> np.ndarray:
        """I_l u_{l-1}: element-local tensor-product interpolation from P_{l-1} to P_l."""
        J = interp_matrix(self.orders[l], self.orders[l - 1])
        dim = self.grid.dim
        u = uc.reshape(lex_shape(self.grid.n, self.orders[l - 1]))
        for d in range(dim):
            u = _prolong_axis(u, J, self.grid.n[d], dim - 1 - d)
        return u.reshape(-1)

    def restrict(self, l: int, rf: np.ndarray) -> np.ndarray:
        """I_l^T r_l."""
        J = interp_matrix(self.orders[l], self.orders[l - 1])
        dim = self.grid.dim
        u = rf.reshape(lex_shape(self.grid.n, self.orders[l]))
        for d in range(dim):
            u = _restrict_axis(u, J, self.grid.n[d], dim - 1 - d)
        return u.reshape(-1)

    def coarse_solve(self, f0: np.ndarray) -> np.ndarray:
        if self.periodic_any:
            f = f0 - f0.mean()
            x = np.zeros_like(f)
            x[1:] = self._lu0.solve(f[1:])
            return x - x.mean()
        return self._lu0.solve(f0)

    def smooth(self, l: int, u, f, steps: int, start: int = 0):
        """`steps` smoothing iterations on level l (the multiplicative smoothers
        alternate their direction within the call, starting forwards)."""
        if steps <= 0:
            return u
        return self.levels[l].smoother.smooth(u, f, steps, start)

    def vcycle(self, u: np.ndarray, f: np.ndarray) -> np.ndarray:
        """MultigridCycle(u, f, N_S) of Alg. 1."""
        L = self.L
        us = [None] * (L + 1)
        fs = [None] * (L + 1)
        us[L] = u.copy()
        fs[L] = f.copy()
        for l in range(L, 0, -1):
            if l < L:
                us[l] = np.zeros_like(fs[l])
            us[l] = self.smooth(l, us[l], fs[l], ns_for(self.method, L, l)[0])
            fs[l - 1] = self.restrict(l, fs[l] - self.apply(l, us[l]))
        us[0] = self.coarse_solve(fs[0])
        for l in range(1, L + 1):
            us[l] = us[l] + self.prolong(l, us[l - 1])
            us[l] = self.smooth(l, us[l], fs[l], ns_for(self.method, L, l)[1])
        return us[L]


@dataclass
class SolveResult:
    x: np.ndarray
    iterations: int
    history: List[float] = field(default_factory=list)   # ||r_i||, i = 0..n
    converged: bool = False


def mgcg(h: Hierarchy, f: np.ndarray, u0: np.ndarray, tol: float = 1e-10, i_max: int = 200,
         precond=None, callback=None) -> SolveResult:
    """MGCG(u, f, N_S, i_max, r_max) of Alg. 2 with r_max = tol * ||f - A u0||.
    callback(i, u), if given, sees every iterate after its update (read only)."""
    M = precond if precond is not None else (lambda r: h.vcycle(np.zeros_like(r), r))
    u = u0.copy()
    L = h.L
    r_old = np.zeros_like(f)
    r = f - h.apply(L, u)
    r0 = float(np.linalg.norm(r))
    hist = [r0]
    r_max = tol * r0
    if r0 == 0.0:
        return SolveResult(u, 0, hist, True)
    p = M(r)
    delta = float(p @ r)
    for i in range(1, i_max + 1):
        q = h.apply(L, p)
        alpha = delta / float(p @ q)
        u = u + alpha * p
        r = r - alpha * q
        if callback is not None:
            callback(i, u)
        rn = float(np.linalg.norm(r))
        hist.append(rn)
        if rn <= r_max:
            r_true = f - h.apply(L, u)
            if float(np.linalg.norm(r_true)) <= r_max:
                return SolveResult(u, i, hist, True)
            r = r_true
        z = M(r)
        beta = float(z @ (r - r_old)) / delta
        p = z + beta * p
        delta = float(z @ r)
        r_old = r.copy()
    return SolveResult(u, i_max, hist, False)


def mg_solve(h: Hierarchy, f: np.ndarray, u0: np.ndarray, tol: float = 1e-10,
             i_max: int = 200) -> SolveResult:
    """Multigrid alone: u <- MultigridCycle(u, f) until ||f - A u|| <= tol ||r_0||."""
    u = u0.copy()
    L = h.L
    r0 = float(np.linalg.norm(f - h.apply(L, u)))
    hist = [r0]
    for i in range(1, i_max + 1):
        u = h.vcycle(u, f)
        rn = float(np.linalg.norm(f - h.apply(L, u)))
        hist.append(rn)
        if rn <= tol * r0:
            return SolveResult(u, i, hist, True)
    return SolveResult(u, i_max, hist, False)
