"""Pins of the oracle's Schwarz smoothers: weight closed forms, partition of unity,
fast diagonalisation against the dense patch solve, block-Jacobi special case."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import operator as op
from oracle import schwarz as sw
from oracle.gll import gll


def test_phi_closed_forms_and_endpoint_conditions():
    x = np.linspace(-1, 1, 41)
    assert np.allclose(sw.phi_tilde(x, "cubic"), (3 * x - x ** 3) / 2)
    assert np.allclose(sw.phi_tilde(x, "quintic"), (15 * x - 10 * x ** 3 + 3 * x ** 5) / 8)
    for kind, nder in (("cubic", 1), ("quintic", 2)):
        c = {"cubic": [0, 1.5, 0, -0.5], "quintic": [0, 15 / 8, 0, -10 / 8, 0, 3 / 8]}[kind]
        p = np.polynomial.Polynomial(c)
        assert p(1) == pytest.approx(1) and p(-1) == pytest.approx(-1)
        for k in range(1, nder + 1):
            assert p.deriv(k)(1) == pytest.approx(0, abs=1e-14)
            assert p.deriv(k)(-1) == pytest.approx(0, abs=1e-14)
        assert np.all(np.diff(sw.phi_tilde(x, kind)) > 0)       # strictly monotonic
    # phi = sgn outside [-1, 1]
    assert sw.phi(np.array([-3.0, 2.0]), "quintic").tolist() == [-1.0, 1.0]


@pytest.mark.parametrize("kind", ["quintic", "cubic"])
def test_hat_weight_values(kind):
    eta, _ = gll(16)
    dxi = eta[3] + 1
    assert sw.w_hat(np.array([0.0]), dxi, kind)[0] == pytest.approx(1.0)
    assert sw.w_hat(np.array([1.0, -1.0]), dxi, kind) == pytest.approx([0.5, 0.5])
    assert sw.w_hat(np.array([1 + dxi, -1 - dxi]), dxi, kind) == pytest.approx([0.0, 0.0])
    # face weight: 1 at the face, 1/2 at the mid-plane, 0 at the far node
    assert sw.w_face(np.array([0.0, 1.0, -1.0, 2.0, -2.0]), kind) == pytest.approx([1, .5, .5, 0, 0])


def _cover(patches, n_glob):
    c = np.zeros(n_glob)
    for p in patches:
        np.add.at(c, p.idx, p.w)
    return c


@pytest.mark.parametrize("P", [1, 2, 4, 6, 8, 16])
@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("kind", ["quintic", "cubic", "arith", "none"])
def test_partition_of_unity_1d(P, periodic, kind):
    N = 5
    for n_o in range(0, min(P, (P + 1) // 2) + 1):
        ec = sw.ec_patches_1d(P, N, periodic, n_o, kind)
        if kind != "none":
            assert np.allclose(_cover(ec, N * (P + 1)), 1.0), (n_o,)
        else:
            assert np.all(_cover(ec, N * (P + 1)) >= 1.0)
    fc = sw.fc_patches_1d(P, N, periodic, kind)
    if kind != "none":
        assert np.allclose(_cover(fc, N * (P + 1)), 1.0)
    assert all(len(p.idx) == 2 * P for p in fc[1:-1])
    assert len(fc) == (N if periodic else N + 1)


def test_patch_sizes_match_paper():
    """EC: N_P + 2 N_O nodes; FC normal: 2 N_P - 2 (Sec. 3.1)."""
    P, N, n_o = 8, 6, 2
    ec = sw.ec_patches_1d(P, N, True, n_o, "quintic")
    assert {len(p.idx) for p in ec} == {P + 1 + 2 * n_o}
    fc = sw.fc_patches_1d(P, N, True, "quintic")
    assert {len(p.idx) for p in fc} == {2 * (P + 1) - 2}
    ecd = sw.ec_patches_1d(P, N, False, n_o, "quintic")
    assert len(ecd[0].idx) == P + 1 + n_o and len(ecd[-1].idx) == P + 1 + n_o


def _level(dim, n, P, periodic, smoother, n_o, beta=0.0, mode="fdm", seed=0):
    rng = np.random.default_rng(seed)
    dx = tuple(rng.uniform(0.4, 1.6, size=n) for _ in range(dim))
    g = synth.Grid(dim, dx, (periodic,) * dim)
    betas = (beta,) * dim
    A = op.assemble_kron(g, P, betas, 1.0)
    ops = [op.operators_1d(P, np.asarray(g.dx[d]), periodic, beta, 1.0) for d in range(dim)]
    return g, A, sw.SmootherLevel(g, P, n_o, "quintic", smoother, lambda u: A @ u, A, ops, mode=mode)


@pytest.mark.parametrize("dim,n,P,n_o", [(2, 3, 3, 1), (2, 4, 4, 2), (3, 3, 2, 1), (3, 2, 3, 2)])
@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("smoother", ["EA", "FA"])
def test_fdm_equals_dense_patch_solve(dim, n, P, n_o, periodic, smoother):
    if periodic and n < 3:
        n = 3
    g, A, lev_fdm = _level(dim, n, P, periodic, smoother, n_o, beta=0.5 if dim == 2 else 0.0)
    _, _, lev_dense = _level(dim, n, P, periodic, smoother, n_o, beta=0.5 if dim == 2 else 0.0,
                             mode="dense")
    rng = np.random.default_rng(1)
    u = rng.standard_normal(A.shape[0])
    f = rng.standard_normal(A.shape[0])
    a = lev_fdm.smooth(u, f, 1)
    b = lev_dense.smooth(u, f, 1)
    assert np.allclose(a, b, rtol=1e-10, atol=1e-10 * np.abs(b).max())


def test_local_1d_operators_spd():
    g, A, lev = _level(3, 3, 4, False, "FA", 2)
    for d in range(3):
        for kind in ("ec", "fc"):
            for k in range(len((lev.fc if kind == "fc" else lev.ec)[d])):
                S, lam = lev.eig1d(d, kind, k)
                assert np.all(lam > 0)
                p = (lev.fc if kind == "fc" else lev.ec)[d][k]
                Mv = lev.ops[d][0][p.idx]
                assert np.allclose(S.T @ (Mv[:, None] * S), np.eye(len(lam)), atol=1e-11)


def test_ea0_is_element_block_jacobi():
    """N_O = 0: element-centred subdomains are the elements, weights are 1 and the
    additive Schwarz step is block Jacobi with exact element blocks."""
    dim, n, P = 2, 3, 3
    g, A, lev = _level(dim, n, P, False, "EA", 0)
    rng = np.random.default_rng(2)
    u = rng.standard_normal(A.shape[0])
    f = rng.standard_normal(A.shape[0])
    got = lev.smooth(u, f, 1)
    # element-major block Jacobi written independently
    perm = op.lex_to_elem(g.n, P)
    Ae = A[perm][:, perm].toarray()
    r = (f - A @ u)[perm]
    nb = (P + 1) ** dim
    du = np.zeros_like(r)
    for e in range(g.n_elem):
        s = slice(e * nb, (e + 1) * nb)
        du[s] = np.linalg.solve(Ae[s, s], r[s])
    ref = u.copy()
    ref[perm] += du
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-12)


def test_zero_residual_gives_zero_correction():
    g, A, lev = _level(2, 3, 4, False, "FA", 1)
    u = np.random.default_rng(3).standard_normal(A.shape[0])
    assert np.allclose(lev.smooth(u, A @ u, 2), u, atol=1e-12)


@pytest.mark.parametrize("dim,periodic,smoother,P", [(2, True, "EA", 3), (3, False, "FA", 4), (3, True, "FA", 2),
                                                     (2, False, "FA", 6)])
def test_sampled_sweep_equals_full_sweep(dim, periodic, smoother, P):
    """sweep_at (covering patches only) reproduces the full sweep at sampled nodes."""
    from oracle.multigrid import Hierarchy
    rng = np.random.default_rng(dim * 10 + P)
    n = (3, 4, 3)[:dim]
    g = synth.Grid(dim, tuple(rng.uniform(0.5, 1.5, n[d]) for d in range(dim)), (periodic,) * dim)
    m = synth.Method(P=P, smoother=smoother)
    H = Hierarchy(g, m, assemble=False, coarse=False)
    sm = H.levels[H.L].smoother
    N = g.n_dof(P)
    u = rng.standard_normal(N)
    f = rng.standard_normal(N)
    nodes = np.concatenate([[0, N - 1], rng.choice(N, 25, replace=False)])
    for normal in ([-1] if smoother == "EA" else list(range(dim))):
        full = sm.sweep(u, f, normal)
        part = sm.sweep_at(u, f, normal, nodes)
        assert np.allclose(part, full[nodes], rtol=0, atol=1e-12 * np.abs(full).max()), normal
