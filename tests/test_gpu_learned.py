"""GPU checks of the learned face-weight path: the MLP kernels against the FP64
oracle, per-face weights in the smoother against the oracle, the probe
fallback, and the gain of the shipped network over the fixed weights.

Tolerances: the MLP runs in FP32; the oracle evaluates the same FP32-rounded
parameters and inputs in FP64, so differences are float rounding of sums of
at most 64 products of O(1) terms (bounded by ~1e-5 relative here)."""
import os
from dataclasses import replace

import numpy as np
import pytest

import synth
from gpu_util import case, check_solve_parity, residual_bound, to_elem, to_lex
from oracle import learned
from oracle import mlp as omlp
from oracle import multigrid as mg

torch = pytest.importorskip("torch")
from paper_1603_02524_amd import dgmg as D  # noqa: E402
from paper_1603_02524_amd import learn  # noqa: E402

pytestmark = pytest.mark.gpu


def _f32(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda").contiguous()


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _rounded(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _net(seed, B):
    rng = np.random.default_rng(seed)
    p = _rounded(omlp.init(seed) + 0.05 * rng.standard_normal(omlp.N_PARAMS))
    X = _rounded(rng.standard_normal((B, omlp.D_IN)))
    T = _rounded(rng.standard_normal((B, omlp.D_OUT)))
    return p, X, T


@pytest.mark.parametrize("B", [1, 37, 300])
def test_mlp_forward_matches_oracle(B):
    p, X, _ = _net(1, B)
    Y, work = D.mlp_forward(_f32(p), _f32(X))
    ref, (_, h1, h2) = omlp.forward(p, X)
    assert np.allclose(_host(Y), ref, rtol=1e-5, atol=1e-5)
    w = _host(work)
    assert np.allclose(w[:, :64], h1, atol=1e-6) and np.allclose(w[:, 64:], h2, atol=1e-6)


@pytest.mark.parametrize("B", [1, 37, 300])
def test_mlp_backward_matches_oracle(B):
    p, X, T = _net(2, B)
    pd, Xd, Td = _f32(p), _f32(X), _f32(T)
    Y, work = D.mlp_forward(pd, Xd)
    g = _host(D.mlp_backward(pd, Xd, Td, Y, work))
    ref = omlp.grad(p, X, T)
    scale = np.abs(ref).max()
    assert np.abs(g - ref).max() <= 2e-5 * scale + 1e-7
    # deterministic: a second call gives the same bits
    g2 = _host(D.mlp_backward(pd, Xd, Td, Y, work))
    assert np.array_equal(g, g2)


def test_mlp_adam_matches_oracle():
    rng = np.random.default_rng(3)
    p = _rounded(rng.standard_normal(omlp.N_PARAMS))
    pd = _f32(p)
    m = torch.zeros_like(pd)
    v = torch.zeros_like(pd)
    pm, mm, vm = p.copy(), np.zeros_like(p), np.zeros_like(p)
    # the kernel takes its hyper-parameters as floats: the oracle gets the same rounded values
    lr, b1, b2, eps = (float(np.float32(c)) for c in (1e-2, 0.9, 0.999, 1e-8))
    for t in range(1, 4):
        g = _rounded(rng.standard_normal(omlp.N_PARAMS))
        D.mlp_adam(pd, _f32(g), m, v, t, lr=1e-2)
        pm, mm, vm = omlp.adam_step(pm, g, mm, vm, t, lr=lr, b1=b1, b2=b2, eps=eps)
    assert np.allclose(_host(pd), pm, rtol=1e-5, atol=1e-6)
    assert np.allclose(_host(m), mm, rtol=1e-5, atol=1e-7)
    assert np.allclose(_host(v), vm, rtol=1e-5, atol=1e-9)


def test_training_with_the_kernels_fits_a_teacher():
    """Adam on the GPU kernels fits a teacher network's outputs (loss measured by the oracle)."""
    rng = np.random.default_rng(4)
    teacher = omlp.init(9) * 1.5
    X = _rounded(rng.uniform(-1, 1, (256, omlp.D_IN)))
    T = _rounded(omlp.forward(teacher, X)[0])
    p0 = learn.init_params(0).astype(np.float64)
    l0 = omlp.loss(p0, X, T)
    params, hist = learn.train(X, T, steps=1500, lr=3e-3)
    l1 = omlp.loss(params.astype(np.float64), X, T)
    assert l1 < 0.05 * l0, (l0, l1, hist)


# ------------------------------------------------------------------ weights in the smoother
def _random_face_params(g, m, seed):
    n = len(learned.face_index(g, m))
    rng = np.random.default_rng(seed)
    return rng.uniform(0.4, 1.8, n), rng.uniform(0.7, 1.3, n)


@pytest.mark.parametrize("cid", ["2d_per_ldg_p3_fa", "3d_dir_ip_p8_fa", "2d_dir_ip_p8_fa_cubic"])
def test_face_params_vcycle_and_solve_match_oracle(cid):
    g, m = case(cid)
    print(f"[case {cid}]", flush=True)
    th, om = _random_face_params(g, m, 5)
    S = D.Solver(g, m, max_iter=200)
    try:
        assert S.face_count() == len(th)
        S.set_face_params(th, om)
        th2, om2, learned_on = S.face_params()
        assert learned_on and np.array_equal(th2, th) and np.array_equal(om2, om)
        H = mg.Hierarchy(g, m, face_params=learned.face_params_dict(g, m, th, om))
        rng = np.random.default_rng(6)
        n = H.levels[-1].A.shape[0]
        r = rng.standard_normal(n)
        if all(g.periodic):
            r -= r.mean()
        ref = H.vcycle(np.zeros_like(r), r)
        z = _host(S.vcycle(torch.tensor(to_elem(r, g, m.P), device="cuda")))
        assert np.abs(to_lex(z, g, m.P) - ref).max() < 1e-10 * np.abs(ref).max()
        f = rng.uniform(-1, 1, n)
        if all(g.periodic):
            f -= f.mean()
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        st = S.solve(torch.tensor(to_elem(f, g, m.P), device="cuda"), x, tol=1e-10)
        assert st["converged"]
        z_gap = np.linalg.norm(to_lex(z, g, m.P) - ref) / np.linalg.norm(ref)
        check_solve_parity(H, f, st, to_lex(_host(x), g, m.P), z_gap=z_gap, label=cid)
        # back to the fixed weights
        S.set_face_params(None)
        H0 = mg.Hierarchy(g, m)
        z0 = _host(S.vcycle(torch.tensor(to_elem(r, g, m.P), device="cuda")))
        ref0 = H0.vcycle(np.zeros_like(r), r)
        assert np.abs(to_lex(z0, g, m.P) - ref0).max() < 1e-10 * np.abs(ref0).max()
    finally:
        S.close()


def test_face_params_mixed_precision_converges():
    g, m = case("3d_dir_ip_p8_fa")
    m = replace(m, precision="mixed")
    th, om = _random_face_params(g, m, 7)
    S = D.Solver(g, m, max_iter=200)
    try:
        S.set_face_params(th, om)
        n = S.n_dof()
        f = torch.tensor(np.random.default_rng(8).uniform(-1, 1, n), device="cuda")
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        st = S.solve(f, x, tol=1e-10)
        assert st["converged"] and st["r_true"] <= 1e-10 * st["r0"]
        A = mg.Hierarchy(g, replace(m, precision="fp64")).levels[-1].A
        fl, xl = to_lex(_host(f), g, m.P), to_lex(_host(x), g, m.P)
        assert np.linalg.norm(fl - A @ xl) <= residual_bound(A, fl, xl)
    finally:
        S.close()


def test_face_param_errors():
    g, m = case("3d_dir_ldg_p4_ea")
    S = D.Solver(g, m)
    try:
        with pytest.raises(D.DgmgError) as e:
            S.set_face_params(np.ones(S.face_count()), np.ones(S.face_count()))
        assert e.value.code == -4
    finally:
        S.close()
    g, m = case("3d_dir_ip_p8_fa")
    S = D.Solver(g, m)
    try:
        n = S.face_count()
        bad = np.ones(n)
        bad[3] = -1.0
        with pytest.raises(D.DgmgError) as e:
            S.set_face_params(bad, np.ones(n))
        assert e.value.code == -1
        bad[3] = np.nan
        with pytest.raises(D.DgmgError):
            S.set_face_params(np.ones(n), bad)
        assert S.face_params()[2] is False
    finally:
        S.close()


# ------------------------------------------------------------------ MLP application + fallback
def _c5_like(seed, n, P):
    rng = np.random.default_rng(seed)
    dx = tuple(synth.random_spacing(rng, n, 5.0, 1.0) for _ in range(3))
    return synth.Grid(3, dx, (False,) * 3), synth.Method(P=P, smoother="FA", overlap="level")


def test_nonfinite_network_falls_back():
    g, m = _c5_like(51, 3, 4)
    S = D.Solver(g, m, max_iter=100)
    try:
        p = torch.full((D.mlp_param_count(),), float("nan"), dtype=torch.float32, device="cuda")
        kept, rl, rf = S.apply_mlp(p, probe_iters=3)
        assert not kept and np.isinf(rl) and 0 < rf < 1
        assert S.face_params()[2] is False
    finally:
        S.close()


def test_neutral_network_equals_fixed_weights():
    """W = 0 and b3 at the neutral point give theta = omega = 1: both probes agree."""
    g, m = _c5_like(52, 3, 8)
    S = D.Solver(g, m, max_iter=100)
    try:
        p = np.zeros(D.mlp_param_count(), dtype=np.float32)
        p[-2] = np.log((1.0 - 0.25) / 1.75 / (1 - (1.0 - 0.25) / 1.75))
        kept, rl, rf = S.apply_mlp(_f32(p), probe_iters=4)
        assert abs(rl - rf) <= 1e-4 * rf
        th, om, on = S.face_params()
        if on:
            assert np.allclose(th, 1.0, atol=1e-6) and np.allclose(om, 1.0, atol=1e-6)
    finally:
        S.close()


@pytest.mark.skipif(not os.path.exists(learn.DEFAULT_PARAMS), reason="no trained network shipped")
def test_shipped_network_gains_on_held_out_problems():
    """The shipped network against the fixed weights of Sec. 3.1 on 12 held-out
    problems (P in {4, 8, 16}, aspect ratios 1 to 32, none trained on), each an
    MGCG solve to 1e-10 from x = 0: never more iterations, fewer in total, and
    the mean residual reduction per iteration (geometric mean of
    rho_learned / rho_fixed) at least 5 % better; the probe keeps the network on
    some problems and falls back on others."""
    rows = learn.evaluate(learn.load_params(), learn.held_out_problems())
    for r in rows:
        print(f"  P={r[0]} AR={r[1]:.1f}: iterations {r[2]} -> {r[3]}, rho {r[4]:.4f} -> {r[5]:.4f}, kept {r[6]}")
    assert all(r[3] <= r[2] for r in rows)
    assert sum(r[3] for r in rows) < sum(r[2] for r in rows)
    gm = float(np.exp(np.mean([np.log(r[5] / r[4]) for r in rows])))
    print(f"  geometric mean rho ratio {gm:.3f}")
    assert gm <= 0.95
    kept = sum(r[6] for r in rows)
    assert 0 < kept < len(rows)
    # a rejected network leaves the fixed weights: the same solve exactly
    assert all(r[5] == r[4] for r in rows if not r[6])


@pytest.mark.skipif(not os.path.exists(learn.DEFAULT_PARAMS), reason="no trained network shipped")
@pytest.mark.parametrize("seed,n,P", [(55, 8, 8), (56, 5, 16), (57, 8, 4)])
def test_shipped_network_is_no_worse_than_fixed(seed, n, P):
    """Learned weights (after the probe) never take more MGCG iterations than the fixed ones."""
    g, m = _c5_like(seed, n, P)
    print(f"[learned seed={seed} n={n} P={P} AR={g.aspect_ratio():.1f}]", flush=True)
    S = D.Solver(g, m, max_iter=200)
    try:
        nd = S.n_dof()
        f = torch.tensor(np.random.default_rng(seed).uniform(-1, 1, nd), device="cuda")
        x = torch.zeros(nd, dtype=torch.float64, device="cuda")
        fixed = S.solve(f, x, tol=1e-10)
        kept, rl, rf = S.apply_mlp(_f32(learn.load_params()), probe_iters=4)
        x.zero_()
        st = S.solve(f, x, tol=1e-10)
        assert st["converged"] and st["r_true"] <= 1e-10 * st["r0"]
        print(f"  kept={kept} probe {rl:.3e} vs {rf:.3e}; iterations {st['iterations']} vs "
              f"{fixed['iterations']}; rho {st['rho']:.4f} vs {fixed['rho']:.4f}", flush=True)
        assert st["iterations"] <= fixed["iterations"]
    finally:
        S.close()
