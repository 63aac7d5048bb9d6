"""GPU parity of the continuous spectral-element counterpart (Sec. 4.3) against
the oracle's SE hierarchy: operator at every level, mass, transfers, exact coarse
solve, smoother, V-cycle and MGCG, FP64 and mixed precision.  Library and oracle
share the lattice layout (direction 1 fastest), so vectors compare as they are.

Tolerances as for the DG path: FP64 kernels within 1e-12 (operator, transfers)
or 1e-11 (smoother, coarse solve) relative, the V-cycle within 1e-10; MGCG by
check_solve_parity (same iterations as rounding allows, x within 1e-10) and the
true residual within tol ||f|| plus its evaluation rounding; FP32 kernels within
a bound derived from float rounding."""
import numpy as np
import pytest

import synth
from gpu_util import check_solve_parity, rand_grid, residual_bound
from oracle import se

torch = pytest.importorskip("torch")
from paper_1603_02524_amd import dgmg as D  # noqa: E402

pytestmark = pytest.mark.gpu

# (id, grid kwargs, method kwargs): ragged element counts, every dimension and
# boundary kind, orders through the 2D-only P = 32 tile
SE_CASES = [
    ("se_2d_dir_p4", dict(dim=2, n=(5, 3), seed=31), dict(P=4)),
    ("se_2d_per_p8", dict(dim=2, n=(4, 3), periodic=True, seed=32), dict(P=8)),
    ("se_2d_dir_p12_cubic", dict(dim=2, n=(2, 3), seed=38), dict(P=12, weighting="cubic")),
    ("se_2d_per_p32", dict(dim=2, n=(3, 3), periodic=True, seed=36), dict(P=32)),
    ("se_3d_dir_p8", dict(dim=3, n=(3, 2, 3), seed=33), dict(P=8)),
    ("se_3d_mixed_p6", dict(dim=3, n=(3, 2, 3), periodic=(True, False, False), seed=34), dict(P=6)),
    ("se_3d_dir_p16", dict(dim=3, n=(2, 2, 2), seed=35), dict(P=16)),
    ("se_3d_per_p2", dict(dim=3, n=(3, 4, 3), periodic=True, seed=37), dict(P=2)),
    ("se_3d_dir_p4_overlap2", dict(dim=3, n=(2, 3, 2), seed=39), dict(P=4, overlap=2)),
]
IDS = [c[0] for c in SE_CASES]


def se_case(cid):
    for c in SE_CASES:
        if c[0] == cid:
            return rand_grid(**c[1]), synth.Method(smoother="EA", disc="se", **c[2])
    raise KeyError(cid)


def _dev(a, dtype=None):
    return torch.tensor(np.asarray(a), dtype=dtype or torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module", params=IDS)
def pair(request):
    g, m = se_case(request.param)
    print(f"[case {request.param}]", flush=True)
    S = D.Solver(g, m, max_iter=200)
    H = se.SEHierarchy(g, m)
    yield request.param, g, m, S, H
    S.close()


def test_level_sizes_and_coordinates(pair):
    cid, g, m, S, H = pair
    assert S.num_levels == len(H.orders)
    for l, P in enumerate(H.orders):
        assert S.n_dof(l) == se.n_dof(g, P)
        for d in range(g.dim):
            assert np.allclose(S.node_coords(l, d), se.node_coords_1d(g.dx[d], P, g.periodic[d]), atol=1e-14)


def test_apply_all_levels_fp64(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(41)
    for l in range(H.L + 1):
        A = H.levels[l].A
        x = rng.standard_normal(A.shape[0])
        y = _host(S.apply(l, _dev(x)))
        assert _rel(y, A @ x) < 1e-12, (cid, l)


def test_apply_fp32(pair):
    """FP32: error bounded by float rounding of |A||x| (a few ulps of the row sums)."""
    cid, g, m, S, H = pair
    rng = np.random.default_rng(42)
    A = H.levels[-1].A
    x = rng.standard_normal(A.shape[0]).astype(np.float32).astype(np.float64)
    y = _host(S.apply(H.L, _dev(x, torch.float32)))
    bound = 64 * np.finfo(np.float32).eps * (abs(A) @ np.abs(x))
    assert np.all(np.abs(y - A @ x) <= bound + 1e-30), cid


def test_residual_and_mass_fp64(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(43)
    A = H.levels[-1].A
    x, f = rng.standard_normal((2, A.shape[0]))
    r = _host(S.residual(H.L, _dev(f), _dev(x)))
    assert _rel(r, f - A @ x) < 1e-12
    gm = _host(S.mass(_dev(f)))
    assert _rel(gm, se.mass_vector(g, m.P) * f) < 1e-14


def test_transfers(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(44)
    for l in range(1, H.L + 1):
        nf, nc = H.levels[l].A.shape[0], H.levels[l - 1].A.shape[0]
        rf, uf = rng.standard_normal((2, nf))
        uc = rng.standard_normal(nc)
        fc = _host(S.restrict(l, _dev(rf)))
        assert _rel(fc, H.restrict(l, rf)) < 1e-13, (cid, l)
        ufd = _dev(uf)
        S.prolong(l, _dev(uc), ufd)
        assert _rel(_host(ufd), uf + H.prolong(l, uc)) < 1e-13, (cid, l)


def test_coarse_solve_exact(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(45)
    f = rng.standard_normal(H.levels[0].A.shape[0])
    if all(g.periodic):
        f -= f.mean()
    ref = H.coarse_solve(f)
    assert _rel(_host(S.coarse_solve(_dev(f))), ref) < 1e-11, cid
    assert _rel(_host(S.coarse_solve(_dev(f, torch.float32))), ref) < 1e-5


def test_smooth_one_step_fp64(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(46)
    for l in range(1, H.L + 1):
        n = H.levels[l].A.shape[0]
        u, f = rng.standard_normal((2, n))
        ref = H.smooth(l, u, f, 1)
        ud = _dev(u)
        S.smooth(l, ud, _dev(f), 1)
        assert _rel(_host(ud), ref) < 1e-11, (cid, l)
        ud = _dev(u)
        S.sweep(l, ud, _dev(f), -1)
        assert _rel(_host(ud), ref) < 1e-11, (cid, l)


def test_smooth_two_steps_fp32(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(47)
    n = H.levels[-1].A.shape[0]
    u, f = rng.standard_normal((2, n))
    ref = H.smooth(H.L, u, f, 2)
    ud = _dev(u, torch.float32)
    S.smooth(H.L, ud, _dev(f, torch.float32), 2)
    assert _rel(_host(ud), ref) < 5e-4, cid


def test_face_centred_sweep_rejected(pair):
    cid, g, m, S, H = pair
    with pytest.raises(D.DgmgError):
        S.sweep(H.L, _dev(np.zeros(S.n_dof())), _dev(np.zeros(S.n_dof())), 0)


def test_vcycle_fp64(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(48)
    r = rng.standard_normal(H.levels[-1].A.shape[0])
    if all(g.periodic):
        r -= r.mean()
    ref = H.vcycle(np.zeros_like(r), r)
    assert _rel(_host(S.vcycle(_dev(r))), ref) < 1e-10, cid


def test_solve_matches_oracle_fp64(pair):
    cid, g, m, S, H = pair
    rng = np.random.default_rng(49)
    A = H.levels[-1].A
    f = rng.uniform(-1, 1, A.shape[0])
    r = rng.standard_normal(A.shape[0])
    if all(g.periodic):
        f -= f.mean()
        r -= r.mean()
    z_ref = H.vcycle(np.zeros_like(r), r)
    z_gap = np.linalg.norm(_host(S.vcycle(_dev(r))) - z_ref) / np.linalg.norm(z_ref)
    x = _dev(np.zeros(A.shape[0]))
    st = S.solve(_dev(f), x, tol=1e-10)
    assert st["converged"]
    xs = _host(x)
    check_solve_parity(H, f, st, xs, z_gap=z_gap, label=cid)
    assert np.linalg.norm(f - A @ xs) <= residual_bound(A, f, xs)
    assert st["r_true"] <= 1e-10 * st["r0"]


@pytest.mark.parametrize("cid", ["se_3d_dir_p8", "se_2d_per_p8", "se_3d_mixed_p6"])
def test_mixed_precision_solve(cid):
    """FP32 V-cycle inside FP64 PCG reaches the same 1e-10 true residual."""
    from oracle import multigrid as mg
    g, m = se_case(cid)
    m.precision = "mixed"
    S = D.Solver(g, m, max_iter=60)
    H = se.SEHierarchy(g, m)
    A = H.levels[-1].A
    rng = np.random.default_rng(50)
    f = rng.uniform(-1, 1, A.shape[0])
    if all(g.periodic):
        f -= f.mean()
    ref = mg.mgcg(H, f, np.zeros_like(f), tol=1e-10, i_max=60)
    x = _dev(np.zeros(A.shape[0]))
    st = S.solve(_dev(f), x, tol=1e-10)
    xs = _host(x)
    assert st["converged"]
    assert st["iterations"] <= ref.iterations + 2
    assert np.linalg.norm(f - A @ xs) <= residual_bound(A, f, xs)
    assert st["r_true"] <= 1e-10 * st["r0"]
    S.close()


def _kron_residual_se(grid, P, f, x, tol=1e-10):
    """(||f - A x||, bound) with the oracle's matrix-free Kronecker operator; bound =
    tol ||f|| + 2 gamma_m || |f| + |A| |x| ||, m = D (2P + 1) terms in a row."""
    ops = [se.assemble_1d(P, grid.dx[d], grid.periodic[d]) for d in range(grid.dim)]
    r = f - se.apply_kron(grid, P, x, ops=ops)
    aops = [(M, np.abs(L)) for M, L in ops]
    ax = se.apply_kron(grid, P, np.abs(x), ops=aops)
    m = grid.dim * (2 * P + 1)
    u = np.finfo(np.float64).eps / 2
    gam = m * u / (1 - m * u)
    return np.linalg.norm(r), tol * np.linalg.norm(f) + 2 * gam * np.linalg.norm(np.abs(f) + ax)


def test_fullsize_fp64_solve_matches_oracle_mgcg():
    """The continuous 16^3 P = 8 workload (2,048,383 unknowns): the library's MGCG
    against the oracle's full solve recorded by tests/golden/make_se_reference.py —
    the same iteration count, the residual history within 1e-6, the final iterate
    at 4096 sampled positions and its 2-norm within 1e-10, and the true residual
    (oracle operator) within 1e-10 ||f|| up to its evaluation rounding."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "se_oracle_mgcg.json")
    with open(path) as fh:
        ref = json.load(fh)
    w = synth.se_poisson3d_p8()
    g, m = w.grid, w.method
    n = w.n_dof
    assert ref["n_dof"] == n and ref["workload"] == w.name
    print("[case se 16^3 p8 fp64 full size]", flush=True)
    S = D.Solver(g, m, max_iter=200)
    try:
        f_np = synth.rhs_uniform(w.seed, n)
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        st = S.solve(_dev(f_np), x, tol=ref["tol"])
        k = st["iterations"]
        print(f"  se 16^3 fp64: {k} iterations (oracle {ref['iterations']})", flush=True)
        assert st["converged"] and k == ref["iterations"]
        assert np.allclose(st["history"][: k + 1], ref["history"], rtol=1e-6, atol=0)
        it = ref["iterates"][str(k)]
        idx = np.asarray(ref["sample_index"])
        xs = _host(x)
        xr = np.asarray(it["x"])
        err = np.abs(xs[idx] - xr).max() / np.abs(xr).max()
        nerr = abs(np.linalg.norm(xs) - it["norm"]) / it["norm"]
        print(f"  se 16^3 fp64 iterate: sampled rel err {err:.2e}, norm rel err {nerr:.2e}", flush=True)
        assert err <= 1e-10 and nerr <= 1e-10
        rn, bound = _kron_residual_se(g, m.P, f_np, xs)
        assert rn <= bound, (rn, bound)
    finally:
        S.close()


def test_fullsize_mixed_solve_reaches_the_true_residual():
    w = synth.with_method(synth.se_poisson3d_p8(), precision="mixed")
    g, m = w.grid, w.method
    n = w.n_dof
    print("[case se 16^3 p8 mixed full size]", flush=True)
    S = D.Solver(g, m, max_iter=200)
    try:
        f_np = synth.rhs_uniform(w.seed, n)
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        st = S.solve(_dev(f_np), x, tol=w.tol)
        assert st["converged"] and st["r_true"] <= w.tol * st["r0"]
        rn, bound = _kron_residual_se(g, m.P, f_np, _host(x))
        assert rn <= bound, (rn, bound)
    finally:
        S.close()


@pytest.mark.parametrize("dim,n,periodic,P", [(3, (12, 11, 10), (False, True, False), 8),
                                              (2, (64, 64), (True, False), 16),
                                              (3, (17, 16, 16), True, 4),
                                              (3, (8, 8, 8), False, 12),
                                              (3, (8, 6, 6), (False, False, True), 16)])
def test_owner_computes_operator_on_large_levels(dim, n, periodic, P):
    """Levels with at least 64k element lines take the one-launch owner-computes
    operator (the parity grids above are smaller and take the two-launch form):
    y = A x and r = f - A x against the oracle's matrix-free operator, FP64 within
    1e-12 and FP32 within its rounding bound, on every level."""
    g = rand_grid(dim, n, periodic=periodic, seed=60 + P)
    m = synth.Method(P=P, smoother="EA", disc="se")
    print(f"[case owned {dim}d {n} P={P}]", flush=True)
    S = D.Solver(g, m)
    try:
        rng = np.random.default_rng(61)
        from oracle.multigrid import level_orders
        for l, Pl in enumerate(level_orders(P)):
            nl = se.n_dof(g, Pl)
            x, f = rng.standard_normal((2, nl))
            ref = se.apply_kron(g, Pl, x)
            assert _rel(_host(S.apply(l, _dev(x))), ref) < 1e-12, l
            assert _rel(_host(S.residual(l, _dev(f), _dev(x))), f - ref) < 1e-12, l
            x32 = x.astype(np.float32).astype(np.float64)
            ops = [se.assemble_1d(Pl, g.dx[d], g.periodic[d]) for d in range(dim)]
            ax = se.apply_kron(g, Pl, np.abs(x32), ops=[(M, np.abs(Lm)) for M, Lm in ops])
            y32 = _host(S.apply(l, _dev(x32, torch.float32)))
            assert np.all(np.abs(y32 - se.apply_kron(g, Pl, x32)) <= 64 * np.finfo(np.float32).eps * ax + 1e-30), l
    finally:
        S.close()
