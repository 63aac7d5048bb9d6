"""GPU parity of the multiplicative Schwarz smoothers (EM, FM; Sec. 3.1) against
the oracle, in both subdomain orders: the lexicographic order of the paper (one
patch solve per launch) and the coloured order (one launch per colour class of
subdomains that share no node and no matrix entry: the same steps, reordered).

Per case: one forward sweep, one and two smoothing steps (two: forwards then
backwards) in FP64 within 1e-11 of the oracle relative to the largest value,
two steps in FP32 within 5e-4; the V-cycle within 1e-10; the MGCG solve by the
rules of the FP64 parity tests (x within 1e-10 of the oracle's iterate at the
library's iteration count); the mixed-precision solve to the 1e-10 true
residual.  Grids leave ragged patch counts per colour class (counts that are
and are not multiples of the colour modulus, periodic and Dirichlet)."""
from dataclasses import replace

import numpy as np
import pytest

import synth
from gpu_util import check_solve_parity, hierarchy, rand_grid, residual_bound, to_elem, to_lex

torch = pytest.importorskip("torch")
from paper_1603_02524_amd import dgmg as D  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = {
    "2d_dir_ip_p4_em0_lex": (dict(dim=2, n=(5, 3), seed=61), dict(P=4, smoother="EM", overlap="zero", order="lex")),
    "2d_dir_ip_p4_em0_colour": (dict(dim=2, n=(5, 3), seed=61), dict(P=4, smoother="EM", overlap="zero",
                                                                     order="colour")),
    "2d_per_ldg_p3_fml_colour": (dict(dim=2, n=(4, 5), periodic=True, seed=62),
                                 dict(P=3, smoother="FM", flux="ldg", beta=(0.5, 0.3), order="colour")),
    "2d_dir_ip_p8_fml_lex": (dict(dim=2, n=(3, 2), seed=63), dict(P=8, smoother="FM", order="lex")),
    "3d_dir_ip_p4_fm0_colour": (dict(dim=3, n=(3, 2, 4), seed=64), dict(P=4, smoother="FM", overlap="zero",
                                                                        order="colour")),
    "3d_dir_ip_p8_eml_colour": (dict(dim=3, n=(4, 3, 2), seed=65), dict(P=8, smoother="EM", order="colour")),
    "3d_per_ip_p6_fml_colour": (dict(dim=3, n=(3, 4, 3), periodic=True, seed=66), dict(P=6, smoother="FM",
                                                                                       order="colour")),
    "3d_mixed_ldg_p4_em0_lex": (dict(dim=3, n=(3, 3, 2), periodic=(True, False, False), seed=67),
                                dict(P=4, smoother="EM", overlap="zero", flux="ldg", beta=(0.5, 0.5, 0.5),
                                     order="lex")),
    # a run-time order (P = 5: no compiled kernels) with colour-class patch lattices
    "3d_dir_ip_p5_fml_colour": (dict(dim=3, n=(3, 2, 3), seed=68), dict(P=5, smoother="FM", order="colour")),
}


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module", params=list(CASES))
def mcase(request):
    gk, mk = CASES[request.param]
    g, m = rand_grid(**gk), synth.Method(**mk)
    print(f"[case {request.param}]", flush=True)
    S = D.Solver(g, m, max_iter=300)
    H = hierarchy(g, m)
    yield request.param, g, m, S, H
    S.close()


def test_sweep_and_smoothing_steps_fp64(mcase):
    cid, g, m, S, H = mcase
    rng = np.random.default_rng(71)
    for l in range(1, H.L + 1):
        P = H.orders[l]
        sm = H.levels[l].smoother
        n = H.levels[l].A.shape[0]
        u, f = rng.standard_normal((2, n))
        normal = -1 if m.smoother == "EM" else g.dim - 1
        ud = _dev(to_elem(u, g, P))
        S.sweep(l, ud, _dev(to_elem(f, g, P)), normal=normal)
        assert _rel(to_lex(_host(ud), g, P), sm.msweep(u, f, normal, False)) < 1e-11, (cid, l, "sweep")
        for steps in (1, 2):
            ud = _dev(to_elem(u, g, P))
            S.smooth(l, ud, _dev(to_elem(f, g, P)), steps)
            assert _rel(to_lex(_host(ud), g, P), H.smooth(l, u, f, steps)) < 1e-11, (cid, l, steps)


def test_two_steps_fp32(mcase):
    cid, g, m, S, H = mcase
    rng = np.random.default_rng(72)
    l = H.L
    P = H.orders[l]
    n = H.levels[l].A.shape[0]
    u, f = rng.standard_normal((2, n))
    ud = _dev(to_elem(u, g, P), torch.float32)
    S.smooth(l, ud, _dev(to_elem(f, g, P), torch.float32), 2)
    assert _rel(to_lex(_host(ud), g, P), H.smooth(l, u, f, 2)) < 5e-4, cid


def test_vcycle_and_solve_fp64(mcase):
    cid, g, m, S, H = mcase
    rng = np.random.default_rng(73)
    A = H.levels[-1].A
    r = rng.standard_normal(A.shape[0])
    if all(g.periodic):
        r -= r.mean()
    ref = H.vcycle(np.zeros_like(r), r)
    z = to_lex(_host(S.vcycle(_dev(to_elem(r, g, m.P)))), g, m.P)
    assert _rel(z, ref) < 1e-10, cid
    z_gap = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    f = rng.uniform(-1, 1, A.shape[0])
    if all(g.periodic):
        f -= f.mean()
    x = _dev(np.zeros(A.shape[0]))
    st = S.solve(_dev(to_elem(f, g, m.P)), x, tol=1e-10)
    assert st["converged"] and st["r_true"] <= 1e-10 * st["r0"]
    xs = to_lex(_host(x), g, m.P)
    check_solve_parity(H, f, st, xs, z_gap=z_gap, label=cid)
    assert np.linalg.norm(f - A @ xs) <= residual_bound(A, f, xs)


@pytest.mark.parametrize("cid", ["2d_dir_ip_p4_em0_colour", "3d_dir_ip_p8_eml_colour", "3d_per_ip_p6_fml_colour"])
def test_mixed_precision_solve(cid):
    gk, mk = CASES[cid]
    g, m = rand_grid(**gk), replace(synth.Method(**mk), precision="mixed")
    S = D.Solver(g, m, max_iter=300)
    try:
        A = hierarchy(g, replace(m, precision="fp64")).levels[-1].A
        f = np.random.default_rng(74).uniform(-1, 1, A.shape[0])
        if all(g.periodic):
            f -= f.mean()
        x = _dev(np.zeros(A.shape[0]))
        st = S.solve(_dev(to_elem(f, g, m.P)), x, tol=1e-10)
        assert st["converged"] and st["r_true"] <= 1e-10 * st["r0"]
        xs = to_lex(_host(x), g, m.P)
        assert np.linalg.norm(f - A @ xs) <= residual_bound(A, f, xs)
    finally:
        S.close()


def test_multiplicative_rejections():
    """A multiplicative handle sweeps its own kind of partition only; 3D P = 32 tiles
    (beyond LDS) are not built for subsets of a partition."""
    g = rand_grid(3, (2, 2, 2), seed=68)
    S = D.Solver(g, synth.Method(P=4, smoother="EM", order="colour"))
    try:
        x = _dev(np.zeros(S.n_dof()))
        with pytest.raises(D.DgmgError):
            S.sweep(S.num_levels - 1, x, x.clone(), normal=0)
    finally:
        S.close()
    with pytest.raises(D.DgmgError) as ei:
        D.Solver(rand_grid(3, (1, 1, 1), seed=69), synth.Method(P=32, smoother="FM"))
    assert ei.value.code == -4
