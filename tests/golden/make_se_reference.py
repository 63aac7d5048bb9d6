"""Writes se_oracle_mgcg.json: the oracle's MGCG (Alg. 2) on the continuous
spectral-element counterpart of EA_l on the 16^3, P = 8 grid (2,048,383
unknowns, U[-1,1] right-hand side of seed 6, x0 = 0, tol 1e-10, FP64),
recorded so that a GPU test can compare a full-size solve without running the
oracle for minutes:

* the iteration count and the residual history ||r_k||, k = 0..n;
* for the iterations k = n - 1, n, n + 1 around the oracle's exit n, ||x_k||_2
  and x_k at 4096 seeded sample positions of the lattice vector.

Calls only the oracle and the seeded input generator.  Run from the repository
root:  python tests/golden/make_se_reference.py   (a few minutes)."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import multigrid as mg  # noqa: E402
from oracle import se  # noqa: E402

N_SAMPLES = 4096


def main():
    w = synth.se_poisson3d_p8()
    g, m = w.grid, w.method
    n = w.n_dof
    t0 = time.time()
    H = se.SEHierarchy(g, m, patch_mode="fdm", assemble_all=False)
    print(f"hierarchy {time.time() - t0:.0f} s", flush=True)
    f = synth.rhs_uniform(w.seed, n)
    idx = np.sort(np.random.default_rng(2025).choice(n, N_SAMPLES, replace=False))
    iters = {}

    def keep(i, u):
        iters[i] = {"norm": float(np.linalg.norm(u)), "x": u[idx].tolist()}
        print(f"iteration {i}  {time.time() - t0:.0f} s", flush=True)

    ref = mg.mgcg(H, f, np.zeros_like(f), tol=w.tol, i_max=20, callback=keep)
    extra = mg.mgcg(H, f, np.zeros_like(f), tol=0.0, i_max=ref.iterations + 1,
                    callback=lambda i, u: keep(i, u) if i == ref.iterations + 1 else None)
    out = {"_source": "oracle MGCG (oracle/multigrid.py with oracle/se.py) on the continuous 16^3 P = 8 "
                      "EA_l FP64 workload, seed 6; written by tests/golden/make_se_reference.py",
           "workload": w.name, "n_dof": n, "tol": w.tol, "iterations": ref.iterations,
           "converged": ref.converged, "history": ref.history,
           "history_one_more": extra.history,
           "sample_index": idx.tolist(),
           "iterates": {str(k): v for k, v in sorted(iters.items()) if abs(k - ref.iterations) <= 1}}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "se_oracle_mgcg.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"wrote {path}: {ref.iterations} iterations, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
