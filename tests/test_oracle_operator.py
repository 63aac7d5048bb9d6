"""Pins of the oracle's DG operator: three independent assemblies, a hand-derived
closed form, symmetry/definiteness and manufactured-solution convergence."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import operator as op


def _grid(dim, n, periodic, seed=0, nonuniform=True):
    rng = np.random.default_rng(seed)
    if nonuniform:
        dx = tuple(rng.uniform(0.3, 1.5, size=n) for _ in range(dim))
    else:
        dx = tuple(np.full(n, 1.0 / n) for _ in range(dim))
    return synth.Grid(dim, dx, (periodic,) * dim)


def _rel(a, b):
    return abs(a - b).max() / abs(b).max()


@pytest.mark.parametrize("dim,n,P", [(1, 4, 1), (1, 5, 4), (2, 3, 2), (2, 4, 3), (3, 2, 2), (3, 3, 1)])
@pytest.mark.parametrize("periodic", [False, True])
def test_three_assemblies_agree(dim, n, P, periodic):
    if periodic and n < 3:
        n = 3
    g = _grid(dim, n, periodic, seed=dim * 10 + P)
    A3 = op.assemble_kron(g, P, 0.0, 1.0)
    A1 = op.assemble_sipg_textbook(g, P, 1.0)
    A2 = op.assemble_ldg_mixed(g, P, 0.0, 1.0)
    assert _rel(A1, A3) < 1e-13       # textbook SIPG == eq. (discrete problem)
    assert _rel(A2, A3) < 1e-13       # IP == LDG(beta=0) with mu_LDG = mu - mu_0
    for beta in (0.5, 0.3, -0.5):
        mu_star = 0.7
        A3b = op.assemble_kron(g, P, beta, mu_star)
        A2b = op.assemble_ldg_mixed(g, P, beta, mu_star)
        assert _rel(A2b, A3b) < 1e-13


def test_printed_offdiagonal_blocks_are_not_symmetric():
    """The printed L-/L+ use Dx^{m-1}/Dx^{m+1} in their first term; the primal form
    gives Dx^m.  With the printed version the operator is not symmetric on a
    non-uniform grid, which is why the primal-form blocks are used."""
    from oracle.gll import diff_matrix
    P = 3
    dx = np.array([0.5, 1.0, 2.0])
    D = diff_matrix(P)
    NP = P + 1
    _, L = op.operators_1d(P, dx, False, 0.0, 1.0)
    assert np.allclose(L, L.T, atol=1e-13)
    # printed L- first term with Dx^{m-1} differs from the used one on row block m=1
    e0 = np.zeros(NP); e0[0] = 1
    eP = np.zeros(NP); eP[P] = 1
    used = -1.0 / dx[1] * np.outer(D[0], eP)
    printed = -1.0 / dx[0] * np.outer(D[0], eP)
    Lp = L.copy()
    Lp[NP:2 * NP, 0:NP] += printed - used
    assert abs(Lp - Lp.T).max() > 0.1


@pytest.mark.parametrize("h,mu_star", [(1.0, 1.0), (0.25, 1.0), (0.5, 2.5)])
def test_closed_form_single_element_p1(h, mu_star):
    """Hand-derived SIPG matrix for one linear element with Dirichlet ends:
    a = (1/h) [[1 + 2 mu*, 1], [1, 1 + 2 mu*]]."""
    g = synth.Grid(1, (np.array([h]),), (False,))
    A = op.assemble_kron(g, 1, 0.0, mu_star).toarray()
    ref = np.array([[1 + 2 * mu_star, 1.0], [1.0, 1 + 2 * mu_star]]) / h
    assert np.allclose(A, ref, rtol=1e-14)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_symmetric_definite(dim):
    for periodic in (False, True):
        g = _grid(dim, 3, periodic, seed=7)
        for beta in (0.0, 0.5):
            A = op.assemble_kron(g, 2, beta, 1.0)
            assert abs(A - A.T).max() < 1e-12 * abs(A).max()
            w = np.linalg.eigvalsh(A.toarray())
            if periodic:
                assert abs(w[0]) < 1e-10 * w[-1]
                assert w[1] > 1e-8 * w[-1]
                assert np.allclose(A @ np.ones(A.shape[0]), 0.0, atol=1e-11 * abs(A).max())
            else:
                assert w[0] > 1e-8 * w[-1]


def test_apply_kron_matches_assembled():
    g = _grid(3, 3, False, seed=3)
    A = op.assemble_kron(g, 3, (0.5, 0.0, 0.3), 1.0)
    u = np.random.default_rng(0).standard_normal(A.shape[0])
    y = op.apply_kron(g, 3, u, beta=(0.5, 0.0, 0.3), mu_star=1.0)
    assert np.allclose(y, A @ u, rtol=1e-13, atol=1e-12 * abs(A @ u).max())


def test_lex_elem_permutation_roundtrip():
    n, P = (3, 2, 4), 2
    idx = op.lex_to_elem(n, P)
    assert sorted(idx.tolist()) == list(range(len(idx)))
    u = np.arange(len(idx), dtype=float)
    assert np.array_equal(op.to_lex(op.to_elem(u, n, P), n, P), u)
    # element 1 (m1 = 1), node (i, j, k) = (0, 0, 0) sits at lex (0, 0, P+1)
    NP = P + 1
    shape = op.lex_shape(n, P)
    lex = np.arange(np.prod(shape)).reshape(shape)
    assert op.to_elem(lex.reshape(-1), n, P)[1 * NP ** 3] == lex[0, 0, NP]


def _l2_error(dim, n, P):
    """True L2 error of the discrete solution (Gauss rule with P+3 points per element)."""
    from oracle.gll import gll, lagrange_eval
    g = synth.uniform_grid(dim, n, 1.0, False)
    A = op.assemble_kron(g, P, 0.0, 1.0)
    xs = [op.node_coords_1d(np.asarray(g.dx[d]), P) for d in range(dim)]
    grids = np.meshgrid(*reversed(xs), indexing="ij")  # lex: slowest first
    f = dim * np.pi ** 2 * np.prod([np.sin(np.pi * G) for G in grids], axis=0)
    M = op.mass_vector(g, P)
    u = spla.spsolve(A.tocsc(), M * f.reshape(-1)).reshape(grids[0].shape)
    eta, _ = gll(P)
    xg, wg = np.polynomial.legendre.leggauss(P + 3)
    B = lagrange_eval(eta, xg)
    uq = u
    qx, qw = [], []
    for d in range(dim):
        h = np.asarray(g.dx[d])
        left = np.concatenate(([0.0], np.cumsum(h)[:-1]))
        qx.append((left[:, None] + 0.5 * (1 + xg[None, :]) * h[:, None]).reshape(-1))
        qw.append((0.5 * h[:, None] * wg[None, :]).reshape(-1))
        ax = dim - 1 - d
        t = np.moveaxis(uq, ax, -1)
        t = t.reshape(t.shape[:-1] + (n, P + 1)) @ B.T
        uq = np.moveaxis(t.reshape(t.shape[:-2] + (-1,)), -1, ax)
    Q = np.meshgrid(*reversed(qx), indexing="ij")
    W = np.meshgrid(*reversed(qw), indexing="ij")
    u_ex = np.prod([np.sin(np.pi * G) for G in Q], axis=0)
    w = np.prod(W, axis=0)
    return np.sqrt(np.sum(w * (uq - u_ex) ** 2))


@pytest.mark.parametrize("dim,P,ns", [(1, 2, (4, 8, 16)), (1, 4, (2, 4, 8)), (2, 2, (4, 8, 16)),
                                      (2, 3, (2, 4, 8)), (3, 2, (2, 4, 6))])
def test_manufactured_convergence_order(dim, P, ns):
    """L2 error of the SIPG solution against sin(pi x)...: order P + 1."""
    errs = [_l2_error(dim, n, P) for n in ns]
    rates = [np.log(errs[i] / errs[i + 1]) / np.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)]
    assert rates[-1] == pytest.approx(P + 1, abs=0.35), rates
