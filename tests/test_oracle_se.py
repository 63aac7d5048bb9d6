"""Pins of the continuous spectral-element (SE) oracle: matrices against closed
forms and an independent Kronecker assembly, exact energies, the order of
convergence, the transfers, the Schwarz weights and local solves, and the
convergence rates Sec. 4.3 quotes for the SE counterpart."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import metrics as me
from oracle import multigrid as mg
from oracle import se

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def _grid(dim, n, periodic, seed=0):
    rng = np.random.default_rng(seed)
    if isinstance(periodic, bool):
        periodic = (periodic,) * dim
    if isinstance(n, int):
        n = (n,) * dim
    return synth.Grid(dim, tuple(rng.uniform(0.3, 1.2, n[d]) for d in range(dim)), tuple(periodic))


@pytest.mark.parametrize("periodic", [False, True])
def test_p1_matrices_closed_form(periodic):
    """P = 1: the lumped mass is (h_left + h_right)/2 and the stiffness the
    three-point difference -1/h_left, 1/h_left + 1/h_right, -1/h_right."""
    dx = np.array([0.5, 0.25, 1.0, 0.75, 0.4])
    N = len(dx)
    M, L = se.assemble_1d(1, dx, periodic)
    n = se.lattice_size(1, N, periodic)
    Mx = np.zeros(n)
    Lx = np.zeros((n, n))
    for s in range(n):
        g = s if periodic else s + 1                 # lattice position = node between elements g-1, g
        hl, hr = dx[(g - 1) % N], dx[g % N]
        Mx[s] = 0.5 * (hl + hr)
        Lx[s, s] = 1 / hl + 1 / hr
        for g2, h in ((g - 1, hl), (g + 1, hr)):
            s2 = se.stored_index(g2, 1, N, periodic)
            if s2 >= 0:
                Lx[s, s2] -= 1 / h
    assert np.allclose(M, Mx, rtol=0, atol=1e-15)
    assert np.allclose(L, Lx, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dim,periodic,P", [(2, False, 3), (2, (True, False), 4), (3, (False, True, False), 2),
                                            (3, True, 3)])
def test_assembly_matches_kronecker_form(dim, periodic, P):
    """Direct stiffness summation of the element matrices equals the Kronecker
    sum of the separately assembled 1D matrices (Cartesian tensor cells), and the
    matrix-free element loop equals the assembled matrix."""
    g = _grid(dim, 3, periodic, seed=dim + P)
    A = se.assemble(g, P)
    ops = [se.assemble_1d(P, g.dx[d], g.periodic[d]) for d in range(dim)]
    K = None
    for d in range(dim):
        t = sp.identity(1, format="csr")
        for dd in reversed(range(dim)):
            B = sp.csr_matrix(ops[dd][1]) if dd == d else sp.diags(ops[dd][0])
            t = sp.kron(t, B, format="csr")
        K = t if K is None else K + t
    assert abs(A - K).max() < 1e-12 * abs(K).max()
    assert abs(A - se.assemble_kron(g, P)).max() < 1e-12 * abs(K).max()
    u = np.random.default_rng(1).standard_normal(A.shape[0])
    assert np.allclose(se.apply(g, P, u), A @ u, rtol=0, atol=1e-12 * np.abs(A @ u).max())
    assert np.allclose(se.apply_kron(g, P, u), A @ u, rtol=0, atol=1e-12 * np.abs(A @ u).max())
    assert abs(A - A.T).max() < 1e-13 * abs(A).max()


@pytest.mark.parametrize("P", [3, 4, 6])
def test_energy_of_a_polynomial_is_exact(P):
    """q = x(1-x) y(1-y) on the unit square (Dirichlet) lies in the discrete space
    and GLL quadrature integrates |grad q|^2 exactly for P >= 3:
    u^T A u = 2 (1/3)(1/30) = 1/45 on any element sizes."""
    dx = (np.array([0.2, 0.5, 0.3]), np.array([0.6, 0.4]))
    g = synth.Grid(2, dx, (False, False))
    x = se.node_coords_1d(dx[0], P, False)
    y = se.node_coords_1d(dx[1], P, False)
    Y, X = np.meshgrid(y, x, indexing="ij")
    u = (X * (1 - X) * Y * (1 - Y)).reshape(-1)
    A = se.assemble(g, P)
    assert u @ (A @ u) == pytest.approx(1.0 / 45.0, rel=1e-12)
    # the lumped mass integrates q (degree 2 per direction) exactly: 1/36
    assert se.mass_vector(g, P) @ u == pytest.approx(1.0 / 36.0, rel=1e-12)


def test_constants_span_the_periodic_null_space():
    g = _grid(2, (3, 4), True, seed=3)
    A = se.assemble(g, 4)
    assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-12
    ev = np.linalg.eigvalsh(A.toarray())
    assert abs(ev[0]) < 1e-10 and ev[1] > 1e-6


def test_manufactured_solution_converges_at_high_order():
    """-Lap u = 2 pi^2 sin(pi x) sin(pi y) on the unit square: the nodal error
    falls by at least 2^P when the elements are halved (P = 4)."""
    errs = []
    for n in (2, 4):
        g = synth.uniform_grid(2, n, 1.0, False)
        P = 4
        x = se.node_coords_1d(g.dx[0], P, False)
        Y, X = np.meshgrid(x, x, indexing="ij")
        ue = (np.sin(np.pi * X) * np.sin(np.pi * Y)).reshape(-1)
        f = 2 * np.pi ** 2 * ue
        u = spla.spsolve(sp.csc_matrix(se.assemble(g, P)), se.mass_vector(g, P) * f)
        errs.append(np.abs(u - ue).max())
    assert errs[1] < 1e-4
    assert errs[0] / errs[1] > 2 ** 4


def test_prolongation_reproduces_coarse_polynomials():
    dx = (np.array([0.3, 0.7, 0.5]), np.array([0.4, 0.6]), np.array([1.0, 0.5]))
    g = synth.Grid(3, dx, (False, False, False))
    def q(P):
        xs = [se.node_coords_1d(dx[d], P, False) for d in range(3)]
        Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
        return (X * (1.5 - X) * Y * (1 - Y) * Z * (1.5 - Z)).reshape(-1)
    I = se.interp(g, 4, 2)
    assert np.allclose(I @ q(2), q(4), rtol=0, atol=1e-13)


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("Pf,Pc", [(2, 1), (4, 2), (8, 4), (6, 3)])
def test_transfers_are_galerkin_in_1d(periodic, Pf, Pc):
    """In 1D the GLL stiffness is exact for the coarse functions, so the
    rediscretised coarse matrix equals I^T L_f I."""
    dx = np.array([0.3, 0.9, 0.5, 0.6])
    I = se.interp_1d(Pf, Pc, len(dx), periodic)
    Lf = se.assemble_1d(Pf, dx, periodic)[1]
    Lc = se.assemble_1d(Pc, dx, periodic)[1]
    assert np.allclose(I.T @ Lf @ I, Lc, rtol=0, atol=1e-11 * np.abs(Lc).max())


@pytest.mark.parametrize("kind", ["quintic", "cubic", "arith"])
@pytest.mark.parametrize("P,overlap", [(2, "level"), (4, "level"), (8, "level"), (16, "level"), (4, 3), (8, 4)])
@pytest.mark.parametrize("periodic", [False, True])
def test_weights_are_a_partition_of_unity(kind, P, overlap, periodic):
    g = _grid(2, (4, 3), periodic, seed=P)
    sm = se.SESmoother(g, P, se.se_overlap(P, overlap), kind, None)
    assert np.allclose(sm.weight_sum(), 1.0, rtol=0, atol=1e-13)


def test_unweighted_sum_counts_the_covering_subdomains():
    P, n_o = 4, 1
    sm = se.SESmoother(_grid(1, 4, False), P, n_o, "none", None)
    tot = sm.weight_sum()
    # lattice g = 1 .. 15: g within n_o of an interior element boundary lies in 2 subdomains,
    # the boundary node itself too; the others in one
    g = np.arange(1, 16)
    near = np.min(np.abs(g[:, None] - np.array([4, 8, 12])[None, :]), axis=1) <= n_o
    assert np.array_equal(tot, np.where(near, 2.0, 1.0))


def test_overlap_zero_has_no_continuous_counterpart():
    with pytest.raises(ValueError):
        se.se_overlap(4, "zero")


@pytest.mark.parametrize("dim,periodic,P", [(2, (True, False), 4), (3, (False, False, True), 2), (2, False, 8)])
def test_fast_diagonalisation_equals_dense_patch_solves(dim, periodic, P):
    g = _grid(dim, 3, periodic, seed=7)
    m = synth.Method(P=P, smoother="EA")
    hd = se.SEHierarchy(g, m, patch_mode="dense")
    hf = se.SEHierarchy(g, m, patch_mode="fdm")
    rng = np.random.default_rng(2)
    L = hd.L
    f = rng.standard_normal(se.n_dof(g, P))
    u = rng.standard_normal(len(f))
    a = hd.smooth(L, u, f, 1)
    b = hf.smooth(L, u, f, 1)
    assert np.allclose(a, b, rtol=0, atol=1e-11 * np.abs(a).max())


def test_one_element_sweep_is_an_exact_solve():
    """A single Dirichlet element: its subdomain is the whole domain with weight 1."""
    g = synth.Grid(2, (np.array([0.7]), np.array([1.3])), (False, False))
    h = se.SEHierarchy(g, synth.Method(P=6, smoother="EA"))
    f = np.random.default_rng(0).standard_normal(se.n_dof(g, 6))
    u = h.smooth(h.L, np.zeros_like(f), f, 1)
    assert np.allclose(h.apply(h.L, u), f, rtol=0, atol=1e-11)


def test_unweighted_additive_correction_is_symmetric_positive_definite():
    """sum_s R_s^T A_ss^-1 R_s (weights 1) is symmetric positive definite; a
    transposed restriction or a wrong local matrix breaks one of the two."""
    g = _grid(2, 3, (False, True), seed=4)
    h = se.SEHierarchy(g, synth.Method(P=4, smoother="EA", weighting="none"))
    L = h.L
    n = se.n_dof(g, 4)
    B = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        B[:, j] = h.smooth(L, np.zeros(n), e, 1)
    assert np.allclose(B, B.T, rtol=0, atol=1e-12 * np.abs(B).max())
    assert np.linalg.eigvalsh(B).min() > 0


def _paper_run_se(P, n, seed=1):
    w = synth.paper_periodic_2d(P, n=n, smoother="EA")
    g, m = w.grid, w.method
    h = se.SEHierarchy(g, m)
    xs = [se.node_coords_1d(g.dx[d], P, True) for d in range(2)]
    Y, X = np.meshgrid(xs[1], xs[0], indexing="ij")
    f = (2 * np.pi ** 2 * np.sin(np.pi * X) * np.sin(np.pi * Y)).reshape(-1)
    gv = se.mass_vector(g, P) * f
    gv -= gv.mean()
    u0 = np.random.default_rng(seed).uniform(0, 1, size=len(gv))
    return mg.mgcg(h, gv, u0, tol=1e-10, i_max=100)


def test_rates_follow_section_4_3():
    """Sec. 4.3: the continuous counterpart of EA_l converges with nearly the
    rates of the DG method (Table 3's EA_l column: within 20 % in r_bar), rates
    improving with P from about 0.02 (P = 4) to about 0.003 (P = 32) (within a
    factor two: the text gives one digit read from a logarithmic figure).
    Element counts (256/P)^2 as in Fig. 6, except 16^2 at P = 4 (the rates do not
    depend on the element count)."""
    with open(GOLD) as fh:
        rows = {(r["P"], r["smoother"], r["overlap"]): r for r in json.load(fh)["rows"]
                if r["cite"].startswith("Table 3")}
    rates = {}
    for P, n in ((4, 16), (8, 32), (16, 16), (32, 8)):
        res = _paper_run_se(P, n)
        assert res.converged
        n10 = me.n10(res.history)
        rb = me.r_bar(res.history, n10)
        rates[P] = 10 ** -rb
        assert rb == pytest.approx(rows[(P, "EA", "level")]["r_bar"], rel=0.2), (P, rb)
    assert rates[4] > rates[8] > rates[16] > rates[32]
    assert 0.01 <= rates[4] <= 0.04
    assert 0.0015 <= rates[32] <= 0.006
