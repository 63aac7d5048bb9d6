"""The DG system matrix A of eq. (discrete problem), three independent ways (oracle).

Orderings.  Internally the oracle uses the lexicographic global ordering of
eq. (IJ): per direction the 1D index I_d = m_d (P+1) + i_d, flattened with
direction 1 fastest.  ``lex_to_elem`` converts to the library's element-major
order (element e = m1 + N1 (m2 + N2 m3), local node (k (P+1) + j)(P+1) + i).

Assemblies (must agree to rounding; pinned by tests/test_oracle_operator.py):

(i)   ``assemble_sipg_textbook``: the symmetric interior penalty bilinear form
      a(u,v) = sum_e int grad u . grad v - sum_F int ({du/dn}[v] + {dv/dn}[u])
               + sum_F int mu [u][v]
      evaluated element by element and face by face with GLL quadrature in
      D dimensions (IP fluxes of Sec. 2.3, beta = 0).
(ii)  ``assemble_ldg_mixed``: A = sum_d G_d^T Mass G_d + J, with G_d the
      discrete gradient including the face lifts of eq. (sigma) and J the
      mu_LDG = mu - mu_0 jump penalty (Sec. 2.4, LDG fluxes).
(iii) ``assemble_kron``: A = sum_d (x)_{d' != d} M_{d'} (x) L_d with the global
      1D operators M_d of eq. (M:generic) and L_d of eq. (L:generic), whose
      blocks L^0, L^-, L^+ are taken from eq. (primal form).

Readings (each stated where it is used):
* the printed L^- and L^+ blocks carry Delta x^{m-1} / Delta x^{m+1} in their
  first term; eq. (primal form) gives Delta x^m there, which is what is used
  (the printed form is not symmetric on non-uniform grids);
* homogeneous Dirichlet faces (not treated by the paper, which is periodic):
  u_hat = 0, sigma_hat = grad u^- - mu_b u^- n; the lift on a boundary face has
  the full factor (2 instead of 1 -/+ 2 beta); beta plays no role there;
  mu_0^b = 2 / (Delta x rho_end) and mu^b = (1 + mu_star) mu_0^b;
* the penalty on a face joining unequal elements is
  mu = (1 + mu_star)(1/(2 Dx_m rho_P) + 1/(2 Dx_{m+1} rho_0)).
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np
import scipy.sparse as sp

from .gll import diff_matrix, gll, stiffness_std


# --------------------------------------------------------------------------- indexing

def lex_shape(n: Sequence[int], P: int) -> Tuple[int, ...]:
    """Shape of the lexicographic nodal array, slowest direction first."""
    return tuple(int(nd) * (P + 1) for nd in reversed(list(n)))


def lex_to_elem(n: Sequence[int], P: int) -> np.ndarray:
    """Index array idx with u_elem = u_lex_flat[idx]."""
    dim = len(n)
    NP = P + 1
    shape = lex_shape(n, P)
    lex = np.arange(int(np.prod(shape))).reshape(shape)
    if dim == 1:
        return lex.reshape(-1).copy()
    if dim == 2:
        n1, n2 = n
        # lex[m2*NP + j, m1*NP + i] -> [m2, m1, j, i]
        a = lex.reshape(n2, NP, n1, NP).transpose(0, 2, 1, 3)
        return a.reshape(-1).copy()
    n1, n2, n3 = n
    a = lex.reshape(n3, NP, n2, NP, n1, NP).transpose(0, 2, 4, 1, 3, 5)
    return a.reshape(-1).copy()


def to_elem(u_lex: np.ndarray, n, P) -> np.ndarray:
    return np.asarray(u_lex).reshape(-1)[lex_to_elem(n, P)]


def to_lex(u_elem: np.ndarray, n, P) -> np.ndarray:
    idx = lex_to_elem(n, P)
    out = np.empty(len(idx), dtype=np.asarray(u_elem).dtype)
    out[idx] = np.asarray(u_elem).reshape(-1)
    return out


def node_coords_1d(dx: np.ndarray, P: int) -> np.ndarray:
    """Physical coordinates of the 1D global nodes (element map of Sec. 2.2)."""
    eta, _ = gll(P)
    left = np.concatenate(([0.0], np.cumsum(dx)[:-1]))
    return (left[:, None] + 0.5 * (1.0 + eta[None, :]) * dx[:, None]).reshape(-1)


# --------------------------------------------------------------------------- penalties

def _mu_interior(P, dxl, dxr, mu_star):
    _, rho = gll(P)
    mu0 = 1.0 / (2.0 * dxl * rho[P]) + 1.0 / (2.0 * dxr * rho[0])
    return mu0, (1.0 + mu_star) * mu0


def _mu_boundary(P, dx, mu_star):
    _, rho = gll(P)
    mu0 = 2.0 / (dx * rho[0])
    return mu0, (1.0 + mu_star) * mu0


# --------------------------------------------------------------------------- (iii) 1D primal blocks

def operators_1d(P: int, dx: np.ndarray, periodic: bool, beta: float, mu_star: float):
    """Global 1D mass (diagonal, as a vector) and stiffness L_d (dense) of eq. (L:generic).

    Blocks from eq. (primal form), with B_{m+1/2} = 2(b^2+b)/(Dx_m rho_P)
    + 2(b^2-b)/(Dx_{m+1} rho_0) + mu_{m+1/2}:
      L0_m = 2/Dx_m L^s + [left]  (1-2b)/Dx_m (D_0i d_k0 + d_i0 D_0k) + B_{m-1/2} d_i0 d_k0
                        + [right] -(1+2b)/Dx_m (D_Pi d_kP + d_iP D_Pk) + B_{m+1/2} d_iP d_kP
      L-_m = -(1-2b)/Dx_m D_0i d_kP + (1+2b)/Dx_{m-1} d_i0 D_Pk - B_{m-1/2} d_i0 d_kP
      L+_m =  (1+2b)/Dx_m D_Pi d_k0 - (1-2b)/Dx_{m+1} d_iP D_0k - B_{m+1/2} d_iP d_k0
    """
    eta, rho = gll(P)
    D = diff_matrix(P)
    Ls = stiffness_std(P)
    NP = P + 1
    N = len(dx)
    b = float(beta)
    Mvec = np.concatenate([0.5 * dx[m] * rho for m in range(N)])
    L = np.zeros((N * NP, N * NP))
    e0 = np.zeros(NP); e0[0] = 1.0
    eP = np.zeros(NP); eP[P] = 1.0
    D0 = D[0, :]
    DP = D[P, :]

    def B(ml, mr):
        _, mu = _mu_interior(P, dx[ml], dx[mr], mu_star)
        return 2 * (b * b + b) / (dx[ml] * rho[P]) + 2 * (b * b - b) / (dx[mr] * rho[0]) + mu

    for m in range(N):
        h = dx[m]
        blk = (2.0 / h) * Ls.copy()
        has_left = periodic or m > 0
        has_right = periodic or m < N - 1
        ml = (m - 1) % N
        mr = (m + 1) % N
        if has_left:
            blk += (1 - 2 * b) / h * (np.outer(D0, e0) + np.outer(e0, D0))
            blk += B(ml, m) * np.outer(e0, e0)
        else:
            _, mub = _mu_boundary(P, h, mu_star)
            blk += (2.0 / h) * (np.outer(D0, e0) + np.outer(e0, D0)) + mub * np.outer(e0, e0)
        if has_right:
            blk += -(1 + 2 * b) / h * (np.outer(DP, eP) + np.outer(eP, DP))
            blk += B(m, mr) * np.outer(eP, eP)
        else:
            _, mub = _mu_boundary(P, h, mu_star)
            blk += -(2.0 / h) * (np.outer(DP, eP) + np.outer(eP, DP)) + mub * np.outer(eP, eP)
        r0 = m * NP
        L[r0:r0 + NP, r0:r0 + NP] += blk
        if has_left:
            Lm = (-(1 - 2 * b) / h * np.outer(D0, eP)
                  + (1 + 2 * b) / dx[ml] * np.outer(e0, DP)
                  - B(ml, m) * np.outer(e0, eP))
            c0 = ml * NP
            L[r0:r0 + NP, c0:c0 + NP] += Lm
        if has_right:
            Lp = ((1 + 2 * b) / h * np.outer(DP, e0)
                  - (1 - 2 * b) / dx[mr] * np.outer(eP, D0)
                  - B(m, mr) * np.outer(eP, e0))
            c0 = mr * NP
            L[r0:r0 + NP, c0:c0 + NP] += Lp
    return Mvec, L


def _kron_list(mats):
    out = mats[0]
    for m in mats[1:]:
        out = sp.kron(out, m, format="csr")
    return sp.csr_matrix(out)


def _betas(beta, dim):
    if np.isscalar(beta):
        return (float(beta),) * dim
    return tuple(float(b) for b in beta)[:dim]


def assemble_kron(grid, P: int, beta=0.0, mu_star: float = 1.0) -> sp.csr_matrix:
    """(iii) A = sum_d (x)_{d'!=d} M_{d'} (x) L_d in lexicographic order (eq. (discrete problem))."""
    dim = grid.dim
    betas = _betas(beta, dim)
    ops = [operators_1d(P, np.asarray(grid.dx[d]), grid.periodic[d], betas[d], mu_star)
           for d in range(dim)]
    A = None
    for d in range(dim):
        # kron order: slowest direction first
        mats = []
        for dd in reversed(range(dim)):
            if dd == d:
                mats.append(sp.csr_matrix(ops[dd][1]))
            else:
                mats.append(sp.diags(ops[dd][0]))
        term = _kron_list(mats)
        A = term if A is None else A + term
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    return A


def mass_vector(grid, P: int) -> np.ndarray:
    """Diagonal of the global mass matrix (tensor product of eq. (1D mass matrix)), lex order."""
    _, rho = gll(P)
    vecs = [np.concatenate([0.5 * h * rho for h in np.asarray(grid.dx[d])]) for d in range(grid.dim)]
    out = vecs[grid.dim - 1]
    for d in reversed(range(grid.dim - 1)):
        out = np.kron(out, vecs[d])
    return out


def apply_kron(grid, P: int, u_lex: np.ndarray, beta=0.0, mu_star: float = 1.0,
               ops=None) -> np.ndarray:
    """A u via the Kronecker-product identity (each term applied axis by axis).

    The same operator as ``assemble_kron``; used where the assembled matrix
    would be too large.  (M3 (x) M2 (x) L1) u is L1 applied along axis x and the
    diagonal masses along the other axes.
    """
    dim = grid.dim
    betas = _betas(beta, dim)
    if ops is None:
        ops = [operators_1d(P, np.asarray(grid.dx[d]), grid.periodic[d], betas[d], mu_star)
               for d in range(dim)]
    shape = lex_shape(grid.n, P)
    u = np.asarray(u_lex, dtype=np.float64).reshape(shape)
    y = np.zeros(shape)
    for d in range(dim):
        ax = dim - 1 - d            # axis of direction d in the lex array
        t = np.moveaxis(u, ax, -1) @ ops[d][1].T
        t = np.moveaxis(t, -1, ax)
        for dd in range(dim):
            if dd == d:
                continue
            axx = dim - 1 - dd
            sh = [1] * dim
            sh[axx] = -1
            t = t * ops[dd][0].reshape(sh)
        y += t
    return y.reshape(-1)


# --------------------------------------------------------------------------- (i) textbook SIPG

def _local_index_arrays(dim, NP):
    """Local multi-indices a[d] for the lex-local ordering (direction 1 fastest)."""
    grids = np.meshgrid(*[np.arange(NP)] * dim, indexing="ij")  # axis order d = 0..dim-1
    # flatten with direction 1 fastest: transpose so that the last axis is d=0
    return [g.transpose(tuple(reversed(range(dim)))).reshape(-1) for g in grids]


def assemble_sipg_textbook(grid, P: int, mu_star: float = 1.0) -> sp.csr_matrix:
    """(i) Symmetric interior penalty bilinear form with GLL quadrature, face by face."""
    dim = grid.dim
    eta, rho = gll(P)
    D = diff_matrix(P)
    NP = P + 1
    n = grid.n
    strides = [1]
    for d in range(dim - 1):
        strides.append(strides[-1] * n[d] * NP)
    Ntot = int(np.prod([nd * NP for nd in n]))
    loc = _local_index_arrays(dim, NP)
    nloc = NP ** dim
    rows, cols, vals = [], [], []

    def gidx(m, a_list):
        g = 0
        for d in range(dim):
            g = g + (m[d] * NP + a_list[d]) * strides[d]
        return g

    elem_iter = np.ndindex(*n)
    for m in elem_iter:
        hs = [float(grid.dx[d][m[d]]) for d in range(dim)]
        W = np.ones(nloc)
        for d in range(dim):
            W *= 0.5 * hs[d] * rho[loc[d]]
        K = np.zeros((nloc, nloc))
        for d in range(dim):
            # (grad_d phi_b)(q) = 2/h_d D[q_d, b_d] prod_{d'!=d} delta(q_d', b_d')
            G = np.zeros((nloc, nloc))
            for q in range(nloc):
                for bb in range(nloc):
                    ok = all(loc[dd][q] == loc[dd][bb] for dd in range(dim) if dd != d)
                    if ok:
                        G[q, bb] = 2.0 / hs[d] * D[loc[d][q], loc[d][bb]]
            K += G.T @ (W[:, None] * G)
        g = gidx(m, loc)
        rr, cc = np.meshgrid(g, g, indexing="ij")
        rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(K.ravel())

    # faces
    for d in range(dim):
        others = [dd for dd in range(dim) if dd != d]
        tl = np.meshgrid(*[np.arange(NP)] * len(others), indexing="ij")
        tl = [t.reshape(-1) for t in tl] if others else []
        nface_pts = NP ** len(others)
        for m in np.ndindex(*n):
            # face on the right side of element m in direction d, plus the left
            # boundary face when m_d == 0 and the direction is not periodic
            faces = []
            if m[d] < n[d] - 1 or grid.periodic[d]:
                mr = list(m); mr[d] = (m[d] + 1) % n[d]
                faces.append(("int", tuple(m), tuple(mr)))
            else:
                faces.append(("bnd_right", tuple(m), None))
            if m[d] == 0 and not grid.periodic[d]:
                faces.append(("bnd_left", None, tuple(m)))
            for kind, mL, mR in faces:
                Wf = np.ones(nface_pts)
                ref = mL if mL is not None else mR
                for j, dd in enumerate(others):
                    Wf *= 0.5 * float(grid.dx[dd][ref[dd]]) * rho[tl[j]]
                # sparse operators on the union of DoFs touched by this face
                cols_map = {}
                def col(gi):
                    if gi not in cols_map:
                        cols_map[gi] = len(cols_map)
                    return cols_map[gi]
                entries_tr_L, entries_tr_R, entries_dn_L, entries_dn_R = [], [], [], []
                for t in range(nface_pts):
                    a_tan = {dd: tl[j][t] for j, dd in enumerate(others)}
                    if mL is not None:
                        hL = float(grid.dx[d][mL[d]])
                        al = [a_tan.get(dd, P) for dd in range(dim)]
                        entries_tr_L.append((t, col(gidx(mL, al)), 1.0))
                        for k in range(NP):
                            ak = [a_tan.get(dd, k) for dd in range(dim)]
                            entries_dn_L.append((t, col(gidx(mL, ak)), 2.0 / hL * D[P, k]))
                    if mR is not None:
                        hR = float(grid.dx[d][mR[d]])
                        ar = [a_tan.get(dd, 0) for dd in range(dim)]
                        entries_tr_R.append((t, col(gidx(mR, ar)), 1.0))
                        for k in range(NP):
                            ak = [a_tan.get(dd, k) for dd in range(dim)]
                            entries_dn_R.append((t, col(gidx(mR, ak)), 2.0 / hR * D[0, k]))
                nc = len(cols_map)
                def mat(entries):
                    Mx = np.zeros((nface_pts, nc))
                    for (t, c, v) in entries:
                        Mx[t, c] += v
                    return Mx
                TrL, TrR, DnL, DnR = map(mat, (entries_tr_L, entries_tr_R, entries_dn_L, entries_dn_R))
                Jmp = TrL - TrR
                if kind == "int":
                    Avg = 0.5 * (DnL + DnR)
                    _, mu = _mu_interior(P, float(grid.dx[d][mL[d]]), float(grid.dx[d][mR[d]]), mu_star)
                else:
                    Avg = DnL + DnR
                    _, mu = _mu_boundary(P, float(grid.dx[d][ref[d]]), mu_star)
                Kf = (-Avg.T @ (Wf[:, None] * Jmp) - Jmp.T @ (Wf[:, None] * Avg)
                      + mu * Jmp.T @ (Wf[:, None] * Jmp))
                g = np.empty(nc, dtype=np.int64)
                for gi, c in cols_map.items():
                    g[c] = gi
                rr, cc = np.meshgrid(g, g, indexing="ij")
                rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(Kf.ravel())

    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(Ntot, Ntot)).tocsr()
    A.sum_duplicates()
    return A


# --------------------------------------------------------------------------- (ii) mixed LDG

def gradient_1d(P: int, dx: np.ndarray, periodic: bool, beta: float) -> np.ndarray:
    """1D discrete flux sigma = G u of eq. (sigma): 2/Dx D u plus the face lifts.

    Left face of element m:  + (1-2b)/(Dx_m rho_0) (u_0^m - u_P^{m-1}) at node 0;
    right face:              + (1+2b)/(Dx_m rho_P) (u_0^{m+1} - u_P^m) at node P.
    On a Dirichlet face u_hat = 0 and the lift factor is 2 (neighbour value 0).
    """
    _, rho = gll(P)
    D = diff_matrix(P)
    NP = P + 1
    N = len(dx)
    b = float(beta)
    G = np.zeros((N * NP, N * NP))
    for m in range(N):
        h = dx[m]
        r0 = m * NP
        G[r0:r0 + NP, r0:r0 + NP] += 2.0 / h * D
        if periodic or m > 0:
            c = (1 - 2 * b) / (h * rho[0])
            ml = (m - 1) % N
            G[r0, r0] += c
            G[r0, ml * NP + P] -= c
        else:
            G[r0, r0] += 2.0 / (h * rho[0])
        if periodic or m < N - 1:
            c = (1 + 2 * b) / (h * rho[P])
            mr = (m + 1) % N
            G[r0 + P, mr * NP] += c
            G[r0 + P, r0 + P] -= c
        else:
            G[r0 + P, r0 + P] -= 2.0 / (h * rho[P])
    return G


def jump_penalty_1d(P: int, dx: np.ndarray, periodic: bool, mu_star: float) -> np.ndarray:
    """1D face penalty sum_F mu_LDG [u][v] with mu_LDG = mu - mu_0 (Sec. 2.4)."""
    NP = P + 1
    N = len(dx)
    J = np.zeros((N * NP, N * NP))
    for f in range(N + 1):
        if 0 < f < N or (periodic and f < N):
            ml = (f - 1) % N
            mr = f % N
            mu0, mu = _mu_interior(P, dx[ml], dx[mr], mu_star)
            v = np.zeros(N * NP)
            v[ml * NP + P] += 1.0
            v[mr * NP] -= 1.0
            J += (mu - mu0) * np.outer(v, v)
        elif not periodic:
            m = 0 if f == 0 else N - 1
            mu0, mu = _mu_boundary(P, dx[m], mu_star)
            v = np.zeros(N * NP)
            v[m * NP + (0 if f == 0 else P)] = 1.0
            J += (mu - mu0) * np.outer(v, v)
    return J


def assemble_ldg_mixed(grid, P: int, beta=0.0, mu_star: float = 1.0) -> sp.csr_matrix:
    """(ii) A = sum_d G_d^T Mass G_d + sum_d J_d (mixed form of the LDG method)."""
    dim = grid.dim
    betas = _betas(beta, dim)
    _, rho = gll(P)
    Mv = [np.concatenate([0.5 * h * rho for h in np.asarray(grid.dx[d])]) for d in range(dim)]
    eye = [sp.identity(len(Mv[d]), format="csr") for d in range(dim)]
    Mass = sp.diags(mass_vector(grid, P))
    A = None
    for d in range(dim):
        G1 = sp.csr_matrix(gradient_1d(P, np.asarray(grid.dx[d]), grid.periodic[d], betas[d]))
        J1 = sp.csr_matrix(jump_penalty_1d(P, np.asarray(grid.dx[d]), grid.periodic[d], mu_star))
        Gm, Jm = [], []
        for dd in reversed(range(dim)):
            Gm.append(G1 if dd == d else eye[dd])
            Jm.append(J1 if dd == d else sp.diags(Mv[dd]))
        Gd = _kron_list(Gm)
        term = Gd.T @ Mass @ Gd + _kron_list(Jm)
        A = term if A is None else A + term
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    return A
