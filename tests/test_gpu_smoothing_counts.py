"""V-cycle and MGCG against the oracle for other smoothing counts (N_S1, N_S2)
of Alg. 1: without pre-smoothing the library starts each level from u = 0,
with it the first pre-smoothing sweep assigns u; two steps exercise the
accumulating sweeps after the first.  Both smoothers, FP64 and the variable
V-cycle.  Tolerances as in the main parity tests (1e-10 relative for the
V-cycle; the solve by check_solve_parity: x within 1e-10 of the oracle's iterate
after the same number of iterations)."""
from dataclasses import replace

import numpy as np
import pytest

from gpu_util import case, check_solve_parity, to_elem, to_lex
from oracle import multigrid as mg

torch = pytest.importorskip("torch")
from paper_1603_02524_amd import dgmg as D  # noqa: E402

pytestmark = pytest.mark.gpu


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("cid", ["3d_dir_ip_p8_fa", "2d_dir_ip_p4_ea", "3d_dir_ldg_p4_ea"])
@pytest.mark.parametrize("ns,vcycle", [((0, 1), "classical"), ((1, 0), "classical"), ((2, 1), "classical"),
                                       ((0, 2), "classical"), ((1, 1), "variable")])
def test_smoothing_counts_match_oracle(cid, ns, vcycle):
    g, m = case(cid)
    m = replace(m, ns=ns, vcycle=vcycle)
    print(f"[{cid} ns={ns} {vcycle}]", flush=True)
    H = mg.Hierarchy(g, m, patch_mode="fdm")
    S = D.Solver(g, m, max_iter=300)
    try:
        rng = np.random.default_rng(31)
        n = H.levels[-1].A.shape[0]
        r = rng.standard_normal(n)
        if all(g.periodic):
            r -= r.mean()
        ref = H.vcycle(np.zeros_like(r), r)
        z = _host(S.vcycle(torch.tensor(to_elem(r, g, m.P), device="cuda")))
        assert np.abs(to_lex(z, g, m.P) - ref).max() <= 1e-10 * np.abs(ref).max()
        # a second V-cycle on the same handle: no state from the first may leak in
        z2 = _host(S.vcycle(torch.tensor(to_elem(r, g, m.P), device="cuda")))
        assert np.array_equal(z, z2)
        f = rng.uniform(-1, 1, n)
        z_gap = np.linalg.norm(to_lex(z, g, m.P) - ref) / np.linalg.norm(ref)
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        st = S.solve(torch.tensor(to_elem(f, g, m.P), device="cuda"), x, tol=1e-10)
        assert st["converged"]
        check_solve_parity(H, f, st, to_lex(_host(x), g, m.P), z_gap=z_gap, label=f"{cid} {ns} {vcycle}")
    finally:
        S.close()
