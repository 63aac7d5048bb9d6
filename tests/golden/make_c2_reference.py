"""Writes c2_oracle_mgcg.json: the oracle's MGCG (Alg. 2) on the 3D 16^3, P = 8,
SIPG, face-centred Schwarz, FP64 workload (2,985,984 DoF, U[-1,1] right-hand
side of seed 2, x0 = 0, tol 1e-10), recorded so that a GPU test can compare a
full-size solve without running the oracle for minutes:

* the iteration count and the residual history ||r_k||, k = 0..n;
* for the iterations k = n - 1, n, n + 1 around the oracle's exit n, ||x_k||_2
  and x_k at 4096 seeded sample positions (indices in the element-major order
  of the library's vectors), so that an iterate the library stops at (the
  oracle's count or one off it) can be checked.

Calls only the oracle and the seeded input generator.  Run from the repository
root:  python tests/golden/make_c2_reference.py   (about 3 minutes)."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import multigrid as mg  # noqa: E402
from oracle import operator as op  # noqa: E402

N_SAMPLES = 4096


def main():
    w = synth.c2_poisson3d_p8()
    g, m = w.grid, w.method
    n = g.n_dof(m.P)
    t0 = time.time()
    H = mg.Hierarchy(g, m, patch_mode="fdm", assemble=False)
    print(f"hierarchy {time.time() - t0:.0f} s", flush=True)
    f_elem = synth.rhs_uniform(w.seed, n)
    f = op.to_lex(f_elem, g.n, m.P)
    idx = np.sort(np.random.default_rng(2024).choice(n, N_SAMPLES, replace=False))
    # element-major index e -> lexicographic position: map a vector of positions
    pos_lex = op.to_lex(np.arange(n, dtype=np.float64), g.n, m.P)
    lex_of_elem = np.empty(n, dtype=np.int64)
    lex_of_elem[pos_lex.astype(np.int64)] = np.arange(n)
    iters = {}

    def keep(i, u):
        iters[i] = {"norm": float(np.linalg.norm(u)), "x": u[lex_of_elem[idx]].tolist()}
        print(f"iteration {i}  {time.time() - t0:.0f} s", flush=True)

    ref = mg.mgcg(H, f, np.zeros_like(f), tol=w.tol, i_max=20, callback=keep)
    # one iteration past the exit, for a library that stops one later
    extra = mg.mgcg(H, f, np.zeros_like(f), tol=0.0, i_max=ref.iterations + 1,
                    callback=lambda i, u: keep(i, u) if i == ref.iterations + 1 else None)
    out = {"_source": "oracle MGCG (oracle/multigrid.py) on the 16^3 P = 8 SIPG FA_l FP64 workload, seed 2; "
                      "written by tests/golden/make_c2_reference.py",
           "workload": w.name, "n_dof": n, "tol": w.tol, "iterations": ref.iterations,
           "converged": ref.converged, "history": ref.history,
           "history_one_more": extra.history,
           "sample_index_elem": idx.tolist(),
           "iterates": {str(k): v for k, v in sorted(iters.items()) if abs(k - ref.iterations) <= 1}}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_oracle_mgcg.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"wrote {path}: {ref.iterations} iterations, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
