"""GPU tests of the batched solver, hipGraph replay and the autotuner.

* graph replay gives bitwise the eager result, on every replay, with eager
  work of the program in between;
* autotuning changes only the block shapes: results stay bitwise identical;
* a batch of grids of uneven order and size reproduces the single-grid solver
  bitwise and the oracle to 1e-10, with its phases run as work-list plans
  (launches shared by the grids) and, when the grids cannot share launches,
  per grid;
* the 64-grid batched workload (elements 4^3..16^3, P in {4,6,8,12,16}, aspect
  ratios up to 8, FP32 multigrid in FP64 MGCG) converges every grid to the
  1e-10 true residual."""
import numpy as np
import pytest

import synth
from gpu_util import hierarchy, kron_residual, rand_grid, residual_bound, to_elem, to_lex

torch = pytest.importorskip("torch")
from paper_1603_02524_amd import dgmg as D  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def test_graph_replay_matches_eager():
    g = rand_grid(3, (3, 2, 2), seed=31)
    m = synth.Method(P=4, smoother="FA")
    S = D.Solver(g, m)
    n = S.n_dof()
    rng = np.random.default_rng(1)
    f = _dev(rng.uniform(-1, 1, n))
    x_ref = _dev(np.zeros(n))
    st_ref = S.solve(f, x_ref)
    S.use_graphs(True)
    for rep in range(3):
        x = _dev(np.zeros(n))
        st = S.solve(f, x)                      # first solve captures, later ones replay
        junk = S.apply(S.num_levels - 1, x)     # eager work of the program between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk).all()
        assert st["iterations"] == st_ref["iterations"], rep
        assert torch.equal(x, x_ref), rep
    # a different x pointer forces a new capture
    x2 = _dev(np.zeros(n))
    S.solve(f, x2)
    assert torch.equal(x2, x_ref)
    S.close()


def test_autotune_is_bitwise_neutral():
    g = rand_grid(3, (4, 3, 2), seed=32)
    m = synth.Method(P=8, smoother="FA")
    S = D.Solver(g, m)
    n = S.n_dof()
    f = _dev(np.random.default_rng(2).uniform(-1, 1, n))
    x1 = _dev(np.zeros(n))
    S.solve(f, x1)
    tune = S.autotune()
    assert len(tune) == 3 * (S.num_levels - 1)   # FA: three sweep kinds per smoothing level
    assert all(w in (1, 2, 4, 8) and ms > 0 for (w, ms) in tune.values())
    x2 = _dev(np.zeros(n))
    S.solve(f, x2)
    assert torch.equal(x1, x2)
    for w2 in (1, 2, 4, 8):                          # every forced shape gives the same result
        for (l, kind) in tune:
            S.set_tuning(l, kind, w2)
        x3 = _dev(np.zeros(n))
        S.solve(f, x3)
        assert torch.equal(x1, x3), w2
    S.close()


def _small_batch(precision="fp64"):
    rng = np.random.default_rng(7)
    probs = []
    for b, P in enumerate([4, 6, 8, 2, 12, 3]):
        n = tuple(int(v) for v in rng.integers(1, 4, size=3))
        g = rand_grid(3, n, seed=100 + b)
        m = synth.Method(P=P, smoother="FA" if b % 2 == 0 else "EA", precision=precision)
        probs.append((g, m))
    return probs


@pytest.mark.parametrize("graphs", [True, False])
def test_batch_matches_single_and_oracle(graphs):
    from oracle import multigrid as mg
    probs = _small_batch()
    B = D.BatchSolver(probs)
    B.use_graphs(graphs)
    rng = np.random.default_rng(3)
    f_all = rng.uniform(-1, 1, B.n_dof)
    x_all = _dev(np.zeros(B.n_dof))
    stats = B.solve(_dev(f_all), x_all)
    xb = x_all.cpu().numpy()
    for i, (g, m) in enumerate(probs):
        sl = slice(B.offsets[i], B.offsets[i + 1])
        S = D.Solver(g, m)
        xs = _dev(np.zeros(sl.stop - sl.start))
        st = S.solve(_dev(f_all[sl]), xs)
        assert st["iterations"] == stats[i]["iterations"], i
        assert np.array_equal(xs.cpu().numpy(), xb[sl]), i          # bitwise: same kernels, same order
        H = hierarchy(g, m)
        f_lex = to_lex(f_all[sl], g, m.P)
        ref = mg.mgcg(H, f_lex, np.zeros_like(f_lex), tol=1e-10)
        assert ref.iterations == stats[i]["iterations"]
        xl = to_lex(xb[sl], g, m.P)
        assert np.abs(xl - ref.x).max() <= 1e-10 * np.abs(ref.x).max()
        S.close()
    B.close()


def test_batch_with_periodic_grids():
    """Fully periodic and mixed-boundary grids in one batch: each solved as by a
    single handle, bit for bit; a periodic part of rhs that does not sum to zero
    is rejected."""
    probs = [(rand_grid(3, (2, 2, 1), seed=41), synth.Method(P=4, smoother="FA")),
             (rand_grid(3, (3, 3, 3), periodic=True, seed=42), synth.Method(P=4, smoother="FA")),
             (rand_grid(3, (3, 2, 3), periodic=(True, False, True), seed=43), synth.Method(P=3, smoother="EA"))]
    B = D.BatchSolver(probs)
    try:
        f_all = np.random.default_rng(5).uniform(-1, 1, B.n_dof)
        sp = slice(B.offsets[1], B.offsets[2])
        f_all[sp] += 0.5
        with pytest.raises(D.DgmgError) as ei:
            B.solve(_dev(f_all), _dev(np.zeros(B.n_dof)))
        assert ei.value.code == -1
        f_all[sp] -= f_all[sp].mean()
        x_all = _dev(np.zeros(B.n_dof))
        stats = B.solve(_dev(f_all), x_all)
        xb = x_all.cpu().numpy()
        for i, (g, m) in enumerate(probs):
            sl = slice(B.offsets[i], B.offsets[i + 1])
            S = D.Solver(g, m)
            xs = _dev(np.zeros(sl.stop - sl.start))
            st = S.solve(_dev(f_all[sl]), xs)
            assert stats[i]["converged"] and st["iterations"] == stats[i]["iterations"], i
            assert np.array_equal(xs.cpu().numpy(), xb[sl]), i
            S.close()
    finally:
        B.close()


def test_batch_mixed_autotuned_converges():
    probs = _small_batch("mixed")
    B = D.BatchSolver(probs)
    B.autotune()
    rng = np.random.default_rng(4)
    f_all = rng.uniform(-1, 1, B.n_dof)
    x_all = _dev(np.zeros(B.n_dof))
    stats = B.solve(_dev(f_all), x_all)
    for i, (g, m) in enumerate(probs):
        sl = slice(B.offsets[i], B.offsets[i + 1])
        H = hierarchy(g, m)
        A = H.levels[-1].A
        f = to_lex(f_all[sl], g, m.P)
        x = to_lex(x_all[sl].cpu().numpy(), g, m.P)
        assert stats[i]["converged"] and stats[i]["r_true"] <= 1e-10 * stats[i]["r0"]
        assert np.linalg.norm(f - A @ x) <= residual_bound(A, f, x), i
    B.close()


@pytest.mark.timeout(900)
def test_batched_64_grid_workload():
    """64 grids (4^3..16^3 elements, P in {4,6,8,12,16}, AR 1..8), FP32 MG in FP64
    MGCG, one graph per phase: every grid reaches the 1e-10 true residual."""
    ws = synth.c4_batched()
    probs = [(w.grid, w.method) for w in ws]
    print(f"[c4] total dof {sum(w.n_dof for w in ws)}", flush=True)
    B = D.BatchSolver(probs, max_iter=60)
    planned, kernels, grid_ops = B.plan_info()
    print(f"[c4] plan: {kernels} batched launches and {grid_ops} per-grid operations per iteration", flush=True)
    assert planned
    rhs = np.concatenate([synth.rhs_uniform(w.seed, w.n_dof) for w in ws])
    f = _dev(rhs)
    x = _dev(np.zeros(B.n_dof))
    stats = B.solve(f, x)
    assert all(s["converged"] for s in stats), [s["iterations"] for s in stats]
    # true residual per grid with the oracle's matrix-free operator of each grid
    xh, fh = x.cpu().numpy(), rhs
    for i, w in enumerate(ws):
        sl = slice(B.offsets[i], B.offsets[i + 1])
        g, m = w.grid, w.method
        res, bound = kron_residual(g, m, to_lex(fh[sl], g, m.P), to_lex(xh[sl], g, m.P))
        assert res <= bound, (i, res / np.linalg.norm(fh[sl]), bound / np.linalg.norm(fh[sl]))
        assert stats[i]["r_true"] <= 1e-10 * stats[i]["r0"], i
    B.close()


@pytest.mark.parametrize("graphs", [True, False])
def test_unplanned_batch_matches_single(graphs):
    """A batch whose grids cannot share launches (here a multiplicative grid next
    to an additive one) issues each grid's chain on its own and still equals the
    single-grid solves bit for bit."""
    probs = [(rand_grid(3, (2, 2, 2), seed=44), synth.Method(P=4, smoother="FA")),
             (rand_grid(3, (3, 2, 2), seed=45), synth.Method(P=4, smoother="FM", order="colour"))]
    B = D.BatchSolver(probs)
    try:
        assert B.plan_info()[0] is False
        B.use_graphs(graphs)
        f_all = np.random.default_rng(6).uniform(-1, 1, B.n_dof)
        x_all = _dev(np.zeros(B.n_dof))
        stats = B.solve(_dev(f_all), x_all)
        xb = x_all.cpu().numpy()
        for i, (g, m) in enumerate(probs):
            sl = slice(B.offsets[i], B.offsets[i + 1])
            S = D.Solver(g, m)
            xs = _dev(np.zeros(sl.stop - sl.start))
            st = S.solve(_dev(f_all[sl]), xs)
            assert stats[i]["converged"] and st["iterations"] == stats[i]["iterations"], i
            assert np.array_equal(xs.cpu().numpy(), xb[sl]), i
            S.close()
    finally:
        B.close()


@pytest.mark.parametrize("graphs", [False, True])
def test_batch_with_large_grids_matches_single(graphs):
    """Two grids whose top level fills the GPU alone (>= 2^20 unknowns: their
    large-level steps run as per-grid steps on the side streams, overlapping the
    small grids' work-list launches) next to three small grids: every grid's
    solution equals its single-grid solve bit for bit, eager and replayed."""
    probs = [(rand_grid(3, (12, 12, 12), seed=47), synth.Method(P=8, smoother="FA")),
             (rand_grid(3, (2, 3, 2), seed=48), synth.Method(P=4, smoother="FA")),
             (rand_grid(3, (11, 12, 12), seed=49), synth.Method(P=8, smoother="EA")),
             (rand_grid(3, (3, 2, 2), seed=50), synth.Method(P=6, smoother="EA")),
             (rand_grid(3, (2, 2, 3), seed=51), synth.Method(P=8, smoother="FA"))]
    B = D.BatchSolver(probs)
    try:
        assert B.plan_info()[0] is True
        big = [B.offsets[i + 1] - B.offsets[i] >= 1 << 20 for i in range(len(probs))]
        assert big == [True, False, True, False, False]
        B.use_graphs(graphs)
        f_all = np.random.default_rng(7).uniform(-1, 1, B.n_dof)
        x_all = _dev(np.zeros(B.n_dof))
        for _ in range(2):  # a second solve replays the recorded phases
            x_all.zero_()
            stats = B.solve(_dev(f_all), x_all)
        xb = x_all.cpu().numpy()
        for i, (g, m) in enumerate(probs):
            sl = slice(B.offsets[i], B.offsets[i + 1])
            S = D.Solver(g, m)
            xs = _dev(np.zeros(sl.stop - sl.start))
            st = S.solve(_dev(f_all[sl]), xs)
            assert stats[i]["converged"] and st["iterations"] == stats[i]["iterations"], i
            assert np.array_equal(xs.cpu().numpy(), xb[sl]), i
            S.close()
    finally:
        B.close()
