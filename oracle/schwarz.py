"""Overlapping Schwarz smoothers of Sec. 3.1 (oracle; test infrastructure).

Subdomains (per direction d, in the 1D global index I = m (P+1) + i):
* element-centred (EC) for element m: the element's P+1 nodes plus N_O node
  layers of each neighbour: I in [m(P+1) - N_O, (m+1)(P+1) + N_O);
* face-centred (FC) normal to d, for the face f between elements f-1 and f:
  the two adjoining elements without their far nodes: I in
  [(f-1)(P+1) + 1, f(P+1) + P), i.e. 2P nodes; laterally the EC range.
Nodes outside the domain are dropped (Dirichlet) or wrapped (periodic).

Local problems: A_ss = R_s A R_s^T, solved either densely (Cholesky of the
restricted matrix: the definition) or by fast diagonalisation with the 1D
generalised eigenpairs L_{s,d} S = M_{s,d} S Lambda (Sec. 3.1).

Weights (eq. (weight function:ec), eq. (weight function:fc)):
  w_H(xi_H) = 1/2 [phi((1 + xi_H)/dxi_O) + phi((1 - xi_H)/dxi_O)],
  dxi_O = eta_{N_O} + 1, xi_H = xi in the core element, xi -/+ 2 in its
  left/right neighbour; phi = the smoothed sign function (quintic, cubic),
  phi = 1 (unweighted) or phi~ = 0 (arithmetic averaging).
Readings: N_O = 0 gives weight 1 on the core; on a Dirichlet side the missing
term is replaced by 1; the face-centred normal weight is read as
  w_F(xi_F) = 1/2 [1 + phi(1 - |xi_F|)]
(1 at the face, 1/2 at the element mid-plane, 0 at the excluded far node), the
form for which the face patches of one orientation sum to one: the printed
phi(|xi_F|) does not.

Sweeps: EA = one additive sweep over all EC patches; FA = one additive sweep
per orientation d = 1..D in sequence, the residual recomputed before each.

Multiplicative Schwarz (EM, FM; Sec. 3.1): the subproblems of a partition are
solved one after another, each on the residual left by the previous ones, and
the correction added unweighted: u <- u + R_s^T A_ss^-1 R_s (g - A u).  EM: one
sweep over the element-centred subdomains per iteration; FM: one sweep per
orientation d = 1..D.  Within a partition the subdomains are taken in
lexicographic order (direction 1 fastest, as the elements are numbered).  Within
one smoothing call every second iteration runs backwards: reversed subdomain
order and, face-centred, reversed orientation order, so that a call with an
even number of iterations is symmetric (Sec. 3.1); with one iteration per call,
as in V(1,1), pre- and post-smoothing both sweep forwards (the reading under
which Table 2's MG rows with EM_0 and FM_0 are reproduced; running the
post-smoothing backwards gives r = 0.42 instead of the printed 0.63 for EM_0 at
P = 4).  order = "colour" takes the same steps in another order:
subdomains grouped in colour classes whose members share no node and no matrix
entry (so the members of one class could be solved at once), the classes in
lexicographic order of their colours, a class's members lexicographically.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np
import scipy.linalg as sla

from .gll import gll


# --------------------------------------------------------------------------- weights

def phi_tilde(x, kind: str):
    """Smoothed sign functions: cubic (3x - x^3)/2, quintic (15x - 10x^3 + 3x^5)/8."""
    x = np.asarray(x, dtype=np.float64)
    if kind == "cubic":
        return (3.0 * x - x ** 3) / 2.0
    if kind == "quintic":
        return (15.0 * x - 10.0 * x ** 3 + 3.0 * x ** 5) / 8.0
    if kind == "arith":
        return np.zeros_like(x)
    raise ValueError(kind)


def phi(x, kind: str):
    """phi(x) = phi~(x) inside (-1, 1), sgn(x) outside; phi = 1 when unweighted."""
    x = np.asarray(x, dtype=np.float64)
    if kind == "none":
        return np.ones_like(x)
    inside = np.abs(x) < 1.0
    return np.where(inside, phi_tilde(np.clip(x, -1.0, 1.0), kind), np.sign(x))


def w_hat(xi_h, dxi_o, kind, left_boundary=False, right_boundary=False):
    """Hat-shaped EC / lateral weight w_H (eq. (weight function:ec))."""
    a = np.ones_like(np.asarray(xi_h, dtype=np.float64)) if left_boundary else phi((1.0 + xi_h) / dxi_o, kind)
    b = np.ones_like(np.asarray(xi_h, dtype=np.float64)) if right_boundary else phi((1.0 - xi_h) / dxi_o, kind)
    return 0.5 * (a + b)


def w_face(xi_f, kind):
    """Face-centred normal weight w_F (eq. (weight function:fc), read as phi(1 - |xi_F|))."""
    return 0.5 * (1.0 + phi(1.0 - np.abs(xi_f), kind))


def w_face_theta(xi_f, theta, kind):
    """w_F with transition width theta: 1/2 [1 + phi((1 - |xi_F|) / theta)] (theta = 1: w_F).

    Not in the paper: the learned-weight variant scales the transition of the
    face weight; the resulting weights are renormalised per node (fc_patches_1d).
    """
    return 0.5 * (1.0 + phi((1.0 - np.abs(xi_f)) / theta, kind))


# --------------------------------------------------------------------------- 1D patch sets

@dataclass
class Patch1D:
    idx: np.ndarray        # global 1D indices (patch-local order)
    w: np.ndarray          # 1D weights on those indices


def ec_patches_1d(P: int, N: int, periodic: bool, n_o: int, kind: str) -> List[Patch1D]:
    eta, _ = gll(P)
    NP = P + 1
    out = []
    for m in range(N):
        g = np.arange(m * NP - n_o, (m + 1) * NP + n_o)
        if periodic:
            keep = np.ones(len(g), bool)
            gw = g % (N * NP)
        else:
            keep = (g >= 0) & (g < N * NP)
            gw = g
        g_raw = g[keep]
        idx = gw[keep]
        mm = np.floor_divide(g_raw, NP)          # element index before wrapping
        i = g_raw - mm * NP
        xi_h = eta[i] + 2.0 * (mm - m)
        if n_o == 0:
            w = np.ones(len(idx))
        else:
            dxi_o = eta[n_o] + 1.0
            lb = (not periodic) and m == 0
            rb = (not periodic) and m == N - 1
            w = w_hat(xi_h, dxi_o, kind, lb, rb)
        out.append(Patch1D(idx.astype(np.int64), w))
    return out


def fc_patches_1d(P: int, N: int, periodic: bool, kind: str, theta=None, omega=None) -> List[Patch1D]:
    """Face-centred patches normal to one direction, one per face.

    With theta / omega (one value per face) the normal weights are
    w_f = omega_f * w_F(xi; theta_f) / sum_{f' covering the node} w_F(xi'; theta_f'),
    so that for omega = 1 the patches of one orientation still sum to one at
    every node (a partition of unity) whatever the per-face widths are.
    """
    eta, _ = gll(P)
    NP = P + 1
    out = []
    nf = N if periodic else N + 1
    for f in range(nf):
        g = np.arange((f - 1) * NP + 1, f * NP + P)
        if periodic:
            keep = np.ones(len(g), bool)
            gw = g % (N * NP)
        else:
            keep = (g >= 0) & (g < N * NP)
            gw = g
        g_raw = g[keep]
        idx = gw[keep]
        mm = np.floor_divide(g_raw, NP)
        i = g_raw - mm * NP
        xi = eta[i]
        xi_f = np.where(mm == f - 1, xi - 1.0, xi + 1.0)
        w = w_face(xi_f, kind) if theta is None else w_face_theta(xi_f, float(theta[f]), kind)
        out.append(Patch1D(idx.astype(np.int64), w))
    if theta is not None:
        total = np.zeros(N * NP)
        for p in out:
            np.add.at(total, p.idx, p.w)
        om = np.ones(nf) if omega is None else np.asarray(omega, dtype=np.float64)
        out = [Patch1D(p.idx, om[f] * p.w / total[p.idx]) for f, p in enumerate(out)]
    elif omega is not None:
        out = [Patch1D(p.idx, float(omega[f]) * p.w) for f, p in enumerate(out)]
    return out


# --------------------------------------------------------------------------- multiplicative order

def colour_modulus(n_o: int, normal: bool) -> int:
    """Colours per direction of the multiplicative colour classes: two subdomains
    of one colour must lie k apart.  Face-centred normal direction: faces f and
    f + 2 share neither a node nor a matrix entry (the near half of an element
    couples to its neighbour only through that neighbour's first node), k = 2;
    element-centred / lateral extent without overlap: elements two apart are not
    coupled, k = 2; with overlap a subdomain reaches N_O <= P nodes into both
    neighbours, so three apart, k = 3."""
    if normal or n_o == 0:
        return 2
    return 3


def colour_digit(c: int, N: int, k: int, periodic: bool) -> int:
    """Colour of subdomain index c (0 <= c < N) along one direction: c mod k; on a
    periodic direction whose count N is not a multiple of k, the last N mod k
    indices get colours of their own (k, k + 1, ...), so that two subdomains of
    one colour stay k apart across the wrap as well."""
    r = N % k if periodic else 0
    return c % k if c < N - r else k + (c - (N - r))


# --------------------------------------------------------------------------- level context

def overlap_for(P_l: int, overlap) -> int:
    """N_O on level l.

    'level': 1 + P_l/8 rounded to the nearest integer, halves up (Sec. 4.3
    prints a floor; with the floor N_O = 1 for P_l <= 4, where every weighting
    gives the same weights, yet Table 2 lists different rates for cubic and
    quintic weighting at P = 4; rounding reproduces Tables 2 and 3 and agrees
    with the floor for P_l >= 8).  'level_floor': 1 + floor(P_l/8) as printed.
    'zero': 0.  An int: that value on every level.
    """
    if overlap == "level":
        return 1 + (2 * P_l + 8) // 16
    if overlap == "level_floor":
        return 1 + P_l // 8
    if overlap == "zero":
        return 0
    return int(overlap)


@dataclass
class SmootherLevel:
    grid: object
    P: int
    n_o: int
    kind: str
    smoother: str            # "EA", "FA" (weighted additive) or "EM", "FM" (multiplicative)
    apply_A: object          # callable u_lex -> A u_lex
    A: object                # sparse matrix (lex) or None
    ops: list                # per direction (Mvec, Ldense)
    mode: str = "fdm"        # "fdm" or "dense"
    ec: list = field(default_factory=list)     # per direction list[Patch1D]
    fc: list = field(default_factory=list)
    face_params: Optional[list] = None        # per direction (theta[nf], omega[nf]) or None
    order: str = "lex"                        # multiplicative subdomain order: "lex" or "colour"
    _eig: Dict = field(default_factory=dict)
    _chol: Dict = field(default_factory=dict)

    def __post_init__(self):
        g = self.grid
        for d in range(g.dim):
            self.ec.append(ec_patches_1d(self.P, g.n[d], g.periodic[d], self.n_o, self.kind))
            th, om = (None, None) if self.face_params is None else self.face_params[d]
            self.fc.append(fc_patches_1d(self.P, g.n[d], g.periodic[d], self.kind, th, om))

    @property
    def shape(self):
        return tuple(nd * (self.P + 1) for nd in reversed(self.grid.n))

    # ---- 1D generalised eigenpairs  L_{s,d} S = M_{s,d} S Lambda
    def eig1d(self, d: int, kind: str, k: int):
        key = (d, kind, k)
        if key not in self._eig:
            p = (self.fc if kind == "fc" else self.ec)[d][k]
            Mv, L = self.ops[d]
            Ls = L[np.ix_(p.idx, p.idx)]
            Ms = np.diag(Mv[p.idx])
            lam, S = sla.eigh(0.5 * (Ls + Ls.T), Ms)
            self._eig[key] = (S, lam)
        return self._eig[key]

    def patch_sets(self, normal: int):
        """List of tuples (per-direction (kind, k)) of the partition used in one sweep."""
        dim = self.grid.dim
        choices = []
        for d in range(dim):
            if d == normal:
                choices.append([("fc", k) for k in range(len(self.fc[d]))])
            else:
                choices.append([("ec", k) for k in range(len(self.ec[d]))])
        out = []
        for combo in np.ndindex(*[len(c) for c in choices]):
            out.append(tuple(choices[d][combo[d]] for d in range(dim)))
        return out

    def patch_1d(self, d, kk):
        kind, k = kk
        return (self.fc if kind == "fc" else self.ec)[d][k]

    def solve_patch(self, sig, r_patch: np.ndarray, glob_idx: np.ndarray) -> np.ndarray:
        """Delta u_s = A_ss^{-1} r_s on the tensor patch (array axes: slowest direction first)."""
        dim = self.grid.dim
        if self.mode == "dense":
            key = sig
            if key not in self._chol:
                Ass = self.A[glob_idx][:, glob_idx].toarray()
                self._chol[key] = sla.cho_factor(Ass)
            return sla.cho_solve(self._chol[key], r_patch.reshape(-1)).reshape(r_patch.shape)
        # fast diagonalisation: (x)S (sum Lambda)^-1 (x)S^T
        Ss, lams = [], []
        for d in range(dim):
            S, lam = self.eig1d(d, sig[d][0], sig[d][1])
            Ss.append(S)
            lams.append(lam)
        t = r_patch
        for d in range(dim):
            ax = dim - 1 - d
            t = np.moveaxis(np.tensordot(Ss[d].T, np.moveaxis(t, ax, 0), axes=(1, 0)), 0, ax)
        denom = np.zeros(t.shape)
        for d in range(dim):
            ax = dim - 1 - d
            sh = [1] * dim
            sh[ax] = -1
            denom = denom + lams[d].reshape(sh)
        t = t / denom
        for d in range(dim):
            ax = dim - 1 - d
            t = np.moveaxis(np.tensordot(Ss[d], np.moveaxis(t, ax, 0), axes=(1, 0)), 0, ax)
        return t

    def sweep(self, u: np.ndarray, f: np.ndarray, normal: int) -> np.ndarray:
        """One additive sweep over a partition: u + sum_s R_s^T (w_s Delta u_s)."""
        dim = self.grid.dim
        shape = self.shape
        r = (f - self.apply_A(u)).reshape(shape)
        corr = np.zeros(shape)
        strides = [1]
        for d in range(dim - 1):
            strides.append(strides[-1] * shape[dim - 1 - d])
        for sig in self.patch_sets(normal):
            p1 = [self.patch_1d(d, sig[d]) for d in range(dim)]
            ix = np.ix_(*[p1[d].idx for d in reversed(range(dim))])
            rs = r[ix]
            gidx = None
            if self.mode == "dense":
                gidx = np.zeros([len(p1[d].idx) for d in reversed(range(dim))], dtype=np.int64)
                for d in range(dim):
                    ax = dim - 1 - d
                    sh = [1] * dim
                    sh[ax] = -1
                    gidx = gidx + (p1[d].idx * strides[d]).reshape(sh)
                gidx = gidx.reshape(-1)
            du = self.solve_patch(sig, rs, gidx)
            w = np.ones(du.shape)
            for d in range(dim):
                ax = dim - 1 - d
                sh = [1] * dim
                sh[ax] = -1
                w = w * p1[d].w.reshape(sh)
            corr[ix] += w * du          # indices are distinct within one patch
        return u + corr.reshape(-1)

    def sweep_at(self, u: np.ndarray, f: np.ndarray, normal: int, nodes, r: np.ndarray = None) -> np.ndarray:
        """Values at the lexicographic indices `nodes` after one sweep (as `sweep`),
        computed from the patches that cover each node only: for grids too large
        for a full sweep in numpy.  r: the residual f - A u if already known."""
        dim = self.grid.dim
        shape = self.shape
        if r is None:
            r = f - self.apply_A(u)
        r = np.asarray(r).reshape(shape)
        out = []
        for node in nodes:
            coords = np.unravel_index(int(node), shape)          # slowest direction first
            g = [int(coords[dim - 1 - d]) for d in range(dim)]
            cover = []
            for d in range(dim):
                kind = "fc" if d == normal else "ec"
                pts = self.fc[d] if kind == "fc" else self.ec[d]
                cover.append([(kind, k, int(np.nonzero(p.idx == g[d])[0][0]))
                              for k, p in enumerate(pts) if np.any(p.idx == g[d])])
            val = float(np.asarray(u).reshape(-1)[int(node)])
            for combo in itertools.product(*cover):
                sig = tuple((c[0], c[1]) for c in combo)
                p1 = [self.patch_1d(d, sig[d]) for d in range(dim)]
                ix = np.ix_(*[p1[d].idx for d in reversed(range(dim))])
                du = self.solve_patch(sig, r[ix], None)
                pos = tuple(combo[d][2] for d in reversed(range(dim)))
                w = 1.0
                for d in range(dim):
                    w *= p1[d].w[combo[d][2]]
                val += w * du[pos]
            out.append(val)
        return np.asarray(out)

    # ---- multiplicative Schwarz
    def mult_order(self, normal: int):
        """Subdomains of one partition in the order of a forward multiplicative sweep."""
        dim = self.grid.dim
        counts = [len(self.fc[d]) if d == normal else len(self.ec[d]) for d in range(dim)]
        lex = []
        for combo in np.ndindex(*reversed(counts)):          # direction dim-1 slowest, 0 fastest
            lex.append(tuple(reversed(combo)))
        if self.order == "colour":
            def key(c):
                col = tuple(colour_digit(c[d], counts[d], colour_modulus(self.n_o, d == normal),
                                         self.grid.periodic[d]) for d in reversed(range(dim)))
                return col
            lex = sorted(lex, key=key)                        # stable: lexicographic within a class
        elif self.order != "lex":
            raise ValueError(self.order)
        return [tuple(("fc", c[d]) if d == normal else ("ec", c[d]) for d in range(dim)) for c in lex]

    def msweep(self, u: np.ndarray, f: np.ndarray, normal: int, reverse: bool) -> np.ndarray:
        """One multiplicative sweep over a partition (reverse: backwards)."""
        dim = self.grid.dim
        shape = self.shape
        strides = [1]
        for d in range(dim - 1):
            strides.append(strides[-1] * shape[dim - 1 - d])
        u = np.array(u, dtype=np.float64, copy=True)
        order = self.mult_order(normal)
        if reverse:
            order = order[::-1]
        for sig in order:
            p1 = [self.patch_1d(d, sig[d]) for d in range(dim)]
            gidx = np.zeros([len(p1[d].idx) for d in reversed(range(dim))], dtype=np.int64)
            for d in range(dim):
                ax = dim - 1 - d
                sh = [1] * dim
                sh[ax] = -1
                gidx = gidx + (p1[d].idx * strides[d]).reshape(sh)
            pshape = gidx.shape
            gidx = gidx.reshape(-1)
            if self.A is not None:
                rs = f[gidx] - self.A[gidx] @ u
            else:
                rs = (f - self.apply_A(u))[gidx]
            du = self.solve_patch(sig, rs.reshape(pshape), gidx)
            u[gidx] += du.reshape(-1)               # indices are distinct within one patch
        return u

    def smooth(self, u: np.ndarray, f: np.ndarray, steps: int, start: int = 0) -> np.ndarray:
        """`steps` Schwarz iterations (EA, EM: one sweep each; FA, FM: one sweep per
        direction).  Multiplicative: iteration t = start, start + 1, ... runs
        forwards for even t, backwards for odd t."""
        if self.smoother in ("EM", "FM"):
            dim = self.grid.dim
            for i in range(steps):
                rev = (start + i) % 2 == 1
                if self.smoother == "EM":
                    u = self.msweep(u, f, -1, rev)
                else:
                    dirs = list(range(dim))
                    for d in (dirs[::-1] if rev else dirs):
                        u = self.msweep(u, f, d, rev)
            return u
        for _ in range(steps):
            if self.smoother == "EA":
                u = self.sweep(u, f, normal=-1)
            elif self.smoother == "FA":
                for d in range(self.grid.dim):
                    u = self.sweep(u, f, normal=d)
            else:
                raise ValueError(self.smoother)
        return u
