"""The paper's printed convergence rates (Tables 2-4) reproduced by the GPU solver.

The same golden rows as the oracle's test (tests/golden/paper_tables.json):
2D periodic (0, 2 AR) x (0, 2), N x N elements, right-hand side g = M f with
f = 2 pi^2 sin(pi x) sin(pi y) at the GLL nodes (mean removed), random initial
guess in [0, 1].  MGCG rows run dgmg_solve; multigrid-alone rows iterate
u <- u + V(f - A u) with the library's residual and V-cycle.  Tolerances as for
the oracle: mean convergence rate r_bar within 7 % and n10 within one cycle.
Multiplicative rows (EM_0, FM_0) run the paper's lexicographic order: one
patch per launch."""
import json
import os

import numpy as np
import pytest

import synth
from gpu_util import to_elem
from oracle import metrics as me
from oracle import multigrid as mg
from oracle import operator as op

torch = pytest.importorskip("torch")
from paper_1603_02524_amd import dgmg as D  # noqa: E402

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def _rows():
    with open(GOLD) as fh:
        return json.load(fh)["rows"]


def _run(row, seed=1, i_max=400):
    w = synth.paper_periodic_2d(row["P"], n=row["n"], ar=row["ar"], smoother=row["smoother"],
                                overlap=row["overlap"], beta=row["beta"], krylov=row["krylov"],
                                weighting=row["weighting"], vcycle=row["vcycle"], order=row.get("order", "lex"))
    g, m = w.grid, w.method
    S = D.Solver(g, m, max_iter=i_max)
    try:
        L = S.num_levels - 1
        P = m.P
        # the oracle test's data: f at the GLL nodes in lexicographic order, then element order
        xs = [S.node_coords(L, d) for d in range(2)]
        X, Y = np.meshgrid(xs[0], xs[1])
        f = (2 * np.pi ** 2 * np.sin(np.pi * X) * np.sin(np.pi * Y)).reshape(-1)
        gv = S.mass(torch.tensor(to_elem(f, g, P), device="cuda"))
        gv -= gv.mean()
        u0 = np.random.default_rng(seed).uniform(0, 1, size=len(f))
        u = torch.tensor(to_elem(u0, g, P), device="cuda")
        if m.krylov:
            st = S.solve(gv, u, tol=1e-10)
            return st["history"]
        hist = []
        r = S.residual(L, gv, u)
        r0 = float(torch.linalg.norm(r))
        hist.append(r0)
        for _ in range(i_max):
            u += S.vcycle(r)
            r = S.residual(L, gv, u)
            hist.append(float(torch.linalg.norm(r)))
            if hist[-1] <= 1e-10 * r0:
                break
        return hist
    finally:
        S.close()


@pytest.mark.parametrize("row", _rows(), ids=lambda r: r["cite"][:60])
def test_gpu_reproduces_paper_rates(row):
    print(f"[{row['cite']}]", flush=True)
    hist = _run(row)
    n10 = me.n10(hist)
    assert n10 is not None
    rb = me.r_bar(hist, n10)
    tol = 0.07
    print(f"  r_bar {rb:.3f} (printed {row['r_bar']}), n10 {n10} (printed {row['n10']})")
    assert rb == pytest.approx(row["r_bar"], rel=tol), (rb, row["r_bar"])
    if row["n10"] is not None:
        assert abs(n10 - row["n10"]) <= 1


def _oracle_history(row, seed=1, i_max=400):
    """The oracle's run on the same data (CPU, FP64)."""
    w = synth.paper_periodic_2d(row["P"], n=row["n"], ar=row["ar"], smoother=row["smoother"],
                                overlap=row["overlap"], beta=row["beta"], krylov=row["krylov"],
                                weighting=row["weighting"], vcycle=row["vcycle"], order=row.get("order", "lex"))
    g, m = w.grid, w.method
    h = mg.Hierarchy(g, m, patch_mode="fdm")
    xs = [op.node_coords_1d(np.asarray(g.dx[d]), m.P) for d in range(2)]
    X, Y = np.meshgrid(xs[0], xs[1])
    f = (2 * np.pi ** 2 * np.sin(np.pi * X) * np.sin(np.pi * Y)).reshape(-1)
    gvec = op.mass_vector(g, m.P) * f
    gvec -= gvec.mean()
    u0 = np.random.default_rng(seed).uniform(0, 1, size=len(gvec))
    solver = mg.mgcg if m.krylov else mg.mg_solve
    return solver(h, gvec, u0, tol=1e-10, i_max=i_max).history


def _variant(base, **kw):
    row = dict(_rows()[base])
    row.update(kw)
    return row


# (row, iteration cap): unit weights (conventional additive Schwarz without
# damping) over-correct, so those two runs are compared over a few iterations
HISTORY_CASES = {
    "EA_l_mgcg_p4": (_variant(0), 400),
    "EA_l_mg_cubic_p4": (_variant(8), 400),
    "FA_l_variable_ar8_p4": (_variant(15), 400),
    "EA_l_mgcg_arith_p4": (_variant(0, weighting="arith"), 400),
    "EA_floor_mgcg_p4": (_variant(0, overlap="level_floor"), 400),
    "FA_l_ldg_mg_p4": (_variant(5, beta=0.5, krylov=False), 400),
    "EA_l_mgcg_none_p4": (_variant(0, weighting="none"), 12),
    "FA_0_mg_none_diverges_p4": (_variant(3, weighting="none", krylov=False), 6),
}


@pytest.mark.parametrize("name", list(HISTORY_CASES))
def test_gpu_history_matches_oracle(name):
    """Residual history of the GPU solve against the oracle's, iteration by iteration,
    on the same data (printed rows, the weightings no printed row uses, the printed
    floor overlap rule and multigrid alone with LDG)."""
    row, i_max = HISTORY_CASES[name]
    print(f"[{name}]", flush=True)
    hg = np.asarray(_run(row, i_max=i_max))
    ho = np.asarray(_oracle_history(row, i_max=i_max))
    assert len(hg) == len(ho), (len(hg), len(ho))
    # relative early on; near convergence rounding of the recursively updated residual dominates
    err = np.abs(hg - ho) / (ho + 1e-6 * ho[0])
    print(f"  {len(hg) - 1} iterations, max rel history diff {err.max():.2e}")
    assert err.max() < 1e-6
