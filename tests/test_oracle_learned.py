"""Pins of the learned face-weight variant of the oracle (weights, features, output map)."""
import numpy as np
import pytest

import synth
from synth.workloads import Grid, Method
from oracle import learned
from oracle import schwarz as sw
from oracle.gll import gll
from oracle.multigrid import Hierarchy


def _node_sums(patches, G):
    tot = np.zeros(G)
    for p in patches:
        np.add.at(tot, p.idx, p.w)
    return tot


def test_theta_one_is_the_fixed_face_weight():
    xi = np.linspace(-2, 2, 41)
    for kind in ("quintic", "cubic"):
        assert np.array_equal(sw.w_face_theta(xi, 1.0, kind), sw.w_face(xi, kind))


@pytest.mark.parametrize("P,periodic", [(2, False), (4, True), (5, False), (8, True)])
def test_random_widths_keep_partition_of_unity(P, periodic):
    rng = np.random.default_rng(P)
    N = 5
    nf = learned.n_faces(N, periodic)
    theta = rng.uniform(0.25, 2.0, nf)
    pts = sw.fc_patches_1d(P, N, periodic, "quintic", theta, np.ones(nf))
    assert np.allclose(_node_sums(pts, N * (P + 1)), 1.0, atol=1e-14)
    # without the renormalisation the raw width-scaled weights do not sum to one
    eta, _ = gll(P)
    raw_sum = np.zeros(N * (P + 1))
    for f, p in enumerate(pts):
        for g in p.idx:
            m, i = divmod(int(g), P + 1)
            xi_f = eta[i] - 1.0 if m == (f - 1) % N else eta[i] + 1.0
            raw_sum[g] += sw.w_face_theta(xi_f, theta[f], "quintic")
    assert not np.allclose(raw_sum, 1.0, atol=1e-3)


def test_damping_gives_omega_weighted_sums():
    P, N = 4, 4
    rng = np.random.default_rng(1)
    nf = N + 1
    om = rng.uniform(0.5, 1.5, nf)
    pts = sw.fc_patches_1d(P, N, False, "quintic", np.ones(nf), om)
    tot = _node_sums(pts, N * (P + 1))
    # each node is covered by the two faces of its element: the sum lies between their dampings
    for m in range(N):
        lo, hi = min(om[m], om[m + 1]), max(om[m], om[m + 1])
        seg = tot[m * (P + 1):(m + 1) * (P + 1)]
        assert np.all(seg >= lo - 1e-14) and np.all(seg <= hi + 1e-14)
    # a uniform damping scales the fixed weights
    pts_c = sw.fc_patches_1d(P, N, False, "quintic", np.ones(nf), np.full(nf, 1.3))
    fixed = sw.fc_patches_1d(P, N, False, "quintic")
    for a, b in zip(pts_c, fixed):
        assert np.allclose(a.w, 1.3 * b.w, atol=1e-14)


def test_narrow_width_limit_is_a_step():
    """theta -> 0: weight 1 on the near half of each element, 1/2 on the mid-plane, 0 beyond."""
    P, N = 4, 3
    pts = sw.fc_patches_1d(P, N, True, "quintic", np.full(N, 1e-6), np.ones(N))
    eta, _ = gll(P)
    for f, p in enumerate(pts):
        m_left = (f - 1) % N
        for g, w in zip(p.idx, p.w):
            m, i = divmod(int(g), P + 1)
            xi_f = eta[i] - 1.0 if m == m_left else eta[i] + 1.0
            expect = 1.0 if abs(xi_f) < 1 - 1e-12 else (0.5 if abs(abs(xi_f) - 1) < 1e-12 else 0.0)
            assert w == pytest.approx(expect, abs=1e-12)


def test_features_of_a_hand_computed_grid():
    g = Grid(2, (np.array([0.5, 0.5]), np.array([0.25, 0.5, 0.25])), (False, False))
    m = Method(P=4, smoother="FA")
    X = learned.face_features(g, m)
    assert X.shape == (2 * (3 + 4), 6)
    a = (-1 + 5 / 3) / 5           # log2(0.5) against the lateral mean of log2 (-2, -1, -2)
    lvl1 = [[2 / 32, a, a, 1, 0, 1 / 3], [2 / 32, a, a, 0, 0, 1 / 3], [2 / 32, a, a, 1, 0, 1 / 3],
            [2 / 32, -0.2, -0.2, 1, 0, 1 / 3], [2 / 32, -0.2, 0.0, 0, 0, 1 / 3],
            [2 / 32, 0.0, -0.2, 0, 0, 1 / 3], [2 / 32, -0.2, -0.2, 1, 0, 1 / 3]]
    assert np.allclose(X[:7], lvl1)
    # level 2 (P = 4, N_O = 2)
    assert np.allclose(X[7:, 0], 4 / 32) and np.allclose(X[7:, 5], 2 / 5)
    assert np.allclose(X[7:, 1:5], X[:7, 1:5])


def test_output_map_neutral_point_and_inverse():
    th, om = learned.outputs_to_params(np.zeros((1, 2)))
    assert th[0] == pytest.approx(1.125) and om[0] == pytest.approx(1.0)
    rng = np.random.default_rng(2)
    t = rng.uniform(0.3, 1.9, 10)
    o = rng.uniform(0.6, 1.4, 10)
    th, om = learned.outputs_to_params(learned.params_to_outputs(t, o))
    assert np.allclose(th, t) and np.allclose(om, o)


def test_unit_face_params_reproduce_the_fixed_vcycle():
    w = synth.c1_poisson2d_p4()
    g, m = w.grid, synth.with_method(w, smoother="FA").method
    nface = len(learned.face_index(g, m))
    fp = learned.face_params_dict(g, m, np.ones(nface), np.ones(nface))
    h0 = Hierarchy(g, m)
    h1 = Hierarchy(g, m, face_params=fp)
    r = synth.rhs_uniform(7, g.n_dof(m.P))
    z0 = h0.vcycle(np.zeros_like(r), r)
    z1 = h1.vcycle(np.zeros_like(r), r)
    assert np.allclose(z1, z0, rtol=0, atol=1e-13 * np.abs(z0).max())


def test_uniform_damping_scales_one_sweep():
    w = synth.c1_poisson2d_p4()
    g, m = w.grid, synth.with_method(w, smoother="FA").method
    nface = len(learned.face_index(g, m))
    h1 = Hierarchy(g, m, face_params=learned.face_params_dict(g, m, np.ones(nface), np.full(nface, 0.7)))
    h0 = Hierarchy(g, m)
    L = h0.L
    f = synth.rhs_uniform(3, g.n_dof(m.P))
    u = synth.rhs_uniform(4, g.n_dof(m.P))
    d0 = h0.levels[L].smoother.sweep(u, f, normal=0) - u
    d1 = h1.levels[L].smoother.sweep(u, f, normal=0) - u
    assert np.allclose(d1, 0.7 * d0, atol=1e-13 * np.abs(d0).max())
