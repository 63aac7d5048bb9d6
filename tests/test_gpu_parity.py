"""GPU parity: every kernel of the HIP path against the FP64 oracle, element by
element, on seeded grids whose element counts leave ragged final blocks.

Tolerances: FP64 results within 1e-12 relative (operator, transfers) and the
solver within the 1e-10 relative bound of the FP64 path; FP32 kernels within a
bound derived from float rounding (see the individual tests)."""
from dataclasses import replace

import numpy as np
import pytest

import synth
from gpu_util import CASES, case, check_solve_parity, hierarchy, rand_grid, residual_bound, to_elem, to_lex
from oracle import operator as op

torch = pytest.importorskip("torch")
from paper_1603_02524_amd import dgmg as D  # noqa: E402

pytestmark = pytest.mark.gpu
IDS = [c[0] for c in CASES]


def _dev(a, dtype=None):
    return torch.tensor(np.asarray(a), dtype=dtype or torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module", params=IDS)
def pair(request):
    g, m = case(request.param)
    print(f"[case {request.param}]", flush=True)
    S = D.Solver(g, m, max_iter=200)
    H = hierarchy(g, m)
    yield request.param, g, m, S, H
    S.close()


def test_apply_all_levels_fp64(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(11)
    for l, P in enumerate(H.orders):
        x = rng.standard_normal(H.levels[l].A.shape[0])
        ref = H.levels[l].A @ x
        y = _host(S.apply(l, _dev(to_elem(x, g, P))))
        assert _rel(to_lex(y, g, P), ref) < 1e-12, (cid, l)


def test_apply_fp32(pair):
    """FP32: error bounded by float rounding of |A||x| (a few ulps of the row sums)."""
    cid, g, m, S, H = pair
    rng = np.random.default_rng(12)
    l = H.L
    P = H.orders[l]
    A = H.levels[l].A
    x = rng.standard_normal(A.shape[0]).astype(np.float32).astype(np.float64)
    ref = A @ x
    y = to_lex(_host(S.apply(l, _dev(to_elem(x, g, P), torch.float32))), g, P)
    bound = 64 * np.finfo(np.float32).eps * (abs(A) @ np.abs(x))
    assert np.all(np.abs(y - ref) <= bound + 1e-30), cid


def test_residual_fp64(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(13)
    l = H.L
    P = H.orders[l]
    A = H.levels[l].A
    x, f = rng.standard_normal((2, A.shape[0]))
    r = _host(S.residual(l, _dev(to_elem(f, g, P)), _dev(to_elem(x, g, P))))
    assert _rel(to_lex(r, g, P), f - A @ x) < 1e-12


def test_smooth_one_step_fp64(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(14)
    for l in range(1, H.L + 1):
        P = H.orders[l]
        n = H.levels[l].A.shape[0]
        u, f = rng.standard_normal((2, n))
        ref = H.smooth(l, u, f, 1)
        ud = _dev(to_elem(u, g, P))
        S.smooth(l, ud, _dev(to_elem(f, g, P)), 1)
        assert _rel(to_lex(_host(ud), g, P), ref) < 1e-11, (cid, l)


def test_smooth_two_steps_fp32(pair):
    cid, g, m, S, H = pair
    if H.L == 0:
        pytest.skip("single level: no smoother")
    rng = np.random.default_rng(15)
    l = H.L
    P = H.orders[l]
    n = H.levels[l].A.shape[0]
    u, f = rng.standard_normal((2, n))
    ref = H.smooth(l, u, f, 2)
    ud = _dev(to_elem(u, g, P), torch.float32)
    S.smooth(l, ud, _dev(to_elem(f, g, P), torch.float32), 2)
    assert _rel(to_lex(_host(ud), g, P), ref) < 5e-4, cid


def test_transfers(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(16)
    for l in range(1, H.L + 1):
        Pf, Pc = H.orders[l], H.orders[l - 1]
        rf = rng.standard_normal(H.levels[l].A.shape[0])
        uc = rng.standard_normal(H.levels[l - 1].A.shape[0])
        uf = rng.standard_normal(H.levels[l].A.shape[0])
        fc = _host(S.restrict(l, _dev(to_elem(rf, g, Pf))))
        assert _rel(to_lex(fc, g, Pc), H.restrict(l, rf)) < 1e-13
        ufd = _dev(to_elem(uf, g, Pf))
        S.prolong(l, _dev(to_elem(uc, g, Pc)), ufd)
        assert _rel(to_lex(_host(ufd), g, Pf), uf + H.prolong(l, uc)) < 1e-13


def test_coarse_solve_exact(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(17)
    A0 = H.levels[0].A
    f = rng.standard_normal(A0.shape[0])
    if all(g.periodic):
        f -= f.mean()
    ref = H.coarse_solve(f)
    u = _host(S.coarse_solve(_dev(to_elem(f, g, 1))))
    assert _rel(to_lex(u, g, 1), ref) < 1e-11, cid
    u32 = _host(S.coarse_solve(_dev(to_elem(f, g, 1), torch.float32)))
    assert _rel(to_lex(u32, g, 1), ref) < 1e-5


def test_vcycle_fp64(pair):
    cid, g, m, S, H = pair
    if m.precision != "fp64":
        pytest.skip("FP64 handle only")
    rng = np.random.default_rng(18)
    r = rng.standard_normal(H.levels[-1].A.shape[0])
    if all(g.periodic):
        r -= r.mean()
    ref = H.vcycle(np.zeros_like(r), r)
    z = _host(S.vcycle(_dev(to_elem(r, g, m.P))))
    assert _rel(to_lex(z, g, m.P), ref) < 1e-10, cid


def test_solve_matches_oracle_fp64(pair):
    """Alg. 2 against the oracle from x0 = 0: x within 1e-10 of the oracle's iterate
    after the same number of iterations, the iteration count and the residual
    history as rounding allows (check_solve_parity), and the true residual within
    1e-10 ||f|| up to the rounding of evaluating it."""
    cid, g, m, S, H = pair
    rng = np.random.default_rng(19)
    A = H.levels[-1].A
    f = rng.uniform(-1, 1, A.shape[0])
    if all(g.periodic):
        f -= f.mean()
    r = rng.standard_normal(A.shape[0])
    if all(g.periodic):
        r -= r.mean()
    z_ref = H.vcycle(np.zeros_like(r), r)
    z_gap = np.linalg.norm(to_lex(_host(S.vcycle(_dev(to_elem(r, g, m.P)))), g, m.P) - z_ref) / np.linalg.norm(z_ref)
    x = _dev(np.zeros(A.shape[0]))
    st = S.solve(_dev(to_elem(f, g, m.P)), x, tol=1e-10)
    assert st["converged"]
    xs = to_lex(_host(x), g, m.P)
    check_solve_parity(H, f, st, xs, z_gap=z_gap, label=cid)
    assert np.linalg.norm(f - A @ xs) <= residual_bound(A, f, xs)
    assert st["r_true"] <= 1e-10 * st["r0"]


def test_solve_is_deterministic(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(20)
    f = rng.uniform(-1, 1, S.n_dof())
    if all(g.periodic):
        f -= f.mean()
    f = _dev(f)
    x1 = _dev(np.zeros(S.n_dof()))
    x2 = _dev(np.zeros(S.n_dof()))
    S.solve(f, x1)
    S.solve(f, x2)
    assert torch.equal(x1, x2)


@pytest.mark.parametrize("cid", ["3d_dir_ldg_p4_ea", "3d_dir_ip_p8_fa", "2d_per_ldg_p3_fa", "3d_dir_ip_p32_fa",
                                 "2d_per_ip_p32_ea"])
def test_mixed_precision_solve(cid):
    """FP32 V-cycle inside FP64 PCG reaches the same 1e-10 true residual."""
    from oracle import multigrid as mg
    g, m = case(cid)
    m.precision = "mixed"
    S = D.Solver(g, m, max_iter=60)
    H = hierarchy(g, m)
    A = H.levels[-1].A
    rng = np.random.default_rng(21)
    f = rng.uniform(-1, 1, A.shape[0])
    if all(g.periodic):
        f -= f.mean()
    ref = mg.mgcg(H, f, np.zeros_like(f), tol=1e-10, i_max=60)
    x = _dev(np.zeros(A.shape[0]))
    st = S.solve(_dev(to_elem(f, g, m.P)), x, tol=1e-10)
    xs = to_lex(_host(x), g, m.P)
    assert st["converged"]
    assert st["iterations"] <= ref.iterations + 2
    assert np.linalg.norm(f - A @ xs) <= residual_bound(A, f, xs)
    assert st["r_true"] <= 1e-10 * st["r0"]
    if all(g.periodic):
        xs, rx = xs - xs.mean(), ref.x - ref.x.mean()
    else:
        rx = ref.x
    print(cid, "mixed vs oracle rel err", _rel(xs, rx), "iters", st["iterations"], ref.iterations)
    # the mixed preconditioner changes the iterates; both solutions lie within the
    # residual bound of the exact one, so they agree to cond(A)-scaled 1e-10
    assert _rel(xs, rx) < 1e-6
    S.close()


def test_mass_and_manufactured_c1():
    """2D Poisson on [0,1]^2, 4x4 elements, P = 4, SIPG, manufactured RHS: the
    GPU solution equals the oracle's and approximates sin(pi x) sin(pi y)."""
    from oracle import multigrid as mg
    w = synth.c1_poisson2d_p4()
    g, m = w.grid, w.method
    S = D.Solver(g, m)
    H = hierarchy(g, m)
    x1 = S.node_coords(S.num_levels - 1, 0)
    x2 = S.node_coords(S.num_levels - 1, 1)
    X, Y = np.meshgrid(x1, x2)
    f_lex = (2 * np.pi ** 2 * np.sin(np.pi * X) * np.sin(np.pi * Y)).reshape(-1)
    gv = _host(S.mass(_dev(to_elem(f_lex, g, m.P))))
    ref_g = op.mass_vector(g, m.P) * f_lex
    assert _rel(to_lex(gv, g, m.P), ref_g) < 1e-14
    x = _dev(np.zeros(len(gv)))
    st = S.solve(_dev(gv), x, tol=1e-10)
    ref = mg.mgcg(H, ref_g, np.zeros_like(ref_g), tol=1e-10)
    xs = to_lex(_host(x), g, m.P)
    assert st["iterations"] == ref.iterations
    assert _rel(xs, ref.x) < 1e-10
    err = np.abs(xs - (np.sin(np.pi * X) * np.sin(np.pi * Y)).reshape(-1)).max()
    assert err < 2e-4
    S.close()


@pytest.mark.parametrize("cid", ["3d_dir_ip_p8_fa", "2d_dir_ip_p4_ea", "3d_dir_ldg_p4_ea", "3d_per_ip_p6_fa"])
def test_fused_residual_restriction_is_bitwise_two_step(cid, monkeypatch):
    """The V-cycle's residual + restriction in one launch gives the same bits as
    the residual followed by the separate transfer (selected at setup by
    DGMG_NO_FUSED_RESTRICTION), in FP64 and in the FP32 V-cycle."""
    g, m = case(cid)
    rng = np.random.default_rng(23)
    for prec in ("fp64", "mixed"):
        mm = replace(m, precision=prec)
        S1 = D.Solver(g, mm)
        monkeypatch.setenv("DGMG_NO_FUSED_RESTRICTION", "1")
        S2 = D.Solver(g, mm)
        monkeypatch.delenv("DGMG_NO_FUSED_RESTRICTION")
        try:
            n = S1.n_dof()
            r = rng.standard_normal(n)
            if all(g.periodic):
                r -= r.mean()
            dt = torch.float64 if prec == "fp64" else torch.float32
            z1 = S1.vcycle(_dev(r, dt))
            z2 = S2.vcycle(_dev(r, dt))
            assert torch.equal(z1, z2), (cid, prec)
            x1, x2 = _dev(np.zeros(n)), _dev(np.zeros(n))
            st1 = S1.solve(_dev(r), x1)
            st2 = S2.solve(_dev(r), x2)
            assert st1["iterations"] == st2["iterations"] and torch.equal(x1, x2), (cid, prec)
        finally:
            S1.close()
            S2.close()


def test_kernel_timing_of_top_level_patch_solves():
    """dgmg_kernel_timing / dgmg_kernel_time: one event pair per top-level patch
    solve (FA: 3 sweeps before and 3 after the coarse correction of each of the
    k V-cycles of a k-iteration solve), algorithmic flops from the tile sizes;
    a second enable reuses the event pool and starts the counts afresh."""
    g, m = case("3d_dir_ip_p8_fa")
    S = D.Solver(g, m)
    try:
        n = S.n_dof()
        f = _dev(np.random.default_rng(24).uniform(-1, 1, n))
        NA, NL = 2 * m.P, (m.P + 1) + 2 * 2  # face-centred tile 2P x (N_P + 2 N_O), N_O = 2 at P = 8
        ts = NA * NL * NL
        per_launch = 4.0 * ts * (NA + 2 * NL) + 2.0 * ts
        patches = sum(np.prod([g.n[d] + (1 if d == nd else 0) for d in range(3)]) for nd in range(3))
        for _ in range(2):
            S.kernel_timing(True)
            st = S.solve(f, _dev(np.zeros(n)))
            kt = S.kernel_time()
            S.kernel_timing(False)
            k = st["iterations"]
            assert kt["launches"] == 6 * k
            assert kt["ms"] > 0
            assert kt["flops"] == pytest.approx(2 * k * patches * per_launch, rel=1e-12)
        S.kernel_timing(True, stride=5)  # every fifth launch, the first included
        st = S.solve(f, _dev(np.zeros(n)))
        kt = S.kernel_time()
        S.kernel_timing(False)
        assert kt["launches"] == -(-6 * st["iterations"] // 5)
        assert kt["ms"] > 0
        S.solve(f, _dev(np.zeros(n)))  # timing off: nothing recorded
        assert S.kernel_time()["launches"] == 0
    finally:
        S.close()


def test_zero_rhs_and_exact_guess():
    """g = 0 returns at once with x untouched at 0; an initial guess that already
    solves the system to round-off also takes no iteration."""
    g, m = case("3d_dir_ip_p8_fa")
    S = D.Solver(g, m)
    try:
        x = _dev(np.zeros(S.n_dof()))
        st = S.solve(_dev(np.zeros(S.n_dof())), x, tol=1e-10)
        assert st["iterations"] == 0 and st["converged"] and st["r0"] == 0.0
        assert not torch.any(x != 0)
        f = _dev(synth.rhs_uniform(5, S.n_dof()))
        S.solve(f, x, tol=1e-12)
        st = S.solve(f, x, tol=1e-1)
        assert st["iterations"] == 0 or st["r0"] < 1e-10 * float(torch.linalg.norm(f))
    finally:
        S.close()


def test_periodic_rhs_must_sum_to_zero():
    """Fully periodic: a right-hand side with a non-zero sum makes the singular
    system inconsistent and is rejected; its mean-free part is solved."""
    g, m = case("2d_per_ldg_p3_fa")
    S = D.Solver(g, m)
    try:
        f = synth.rhs_uniform(9, S.n_dof()) + 0.1
        x = _dev(np.zeros(S.n_dof()))
        with pytest.raises(D.DgmgError) as ei:
            S.solve(_dev(f), x)
        assert ei.value.code == -1
        st = S.solve(_dev(f - f.mean()), x, tol=1e-10)
        assert st["converged"]
    finally:
        S.close()


def test_error_paths_on_device():
    g = rand_grid(3, (2, 2, 2), seed=3)
    S = D.Solver(g, synth.Method(P=4))
    x = _dev(np.zeros(S.n_dof()))
    with pytest.raises(D.DgmgError):
        S.apply(S.num_levels - 1, x, x)                 # aliasing is rejected
    with pytest.raises(D.DgmgError):
        S.smooth(0, x, x, 1)                            # level 0 has no smoother
    nan = _dev(np.full(S.n_dof(), np.nan))
    with pytest.raises(D.DgmgError) as ei:
        S.solve(nan, x)
    assert ei.value.code == -5
    S.close()
