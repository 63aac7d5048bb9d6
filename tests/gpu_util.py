"""Shared helpers of the GPU parity tests: seeded problems, the oracle twin of a
library handle, and layout conversion (oracle: lexicographic; library:
element-major)."""
import numpy as np

import synth
from oracle import multigrid as mg
from oracle import operator as op


def rand_grid(dim, n, periodic=False, seed=0, lo=0.4, hi=1.6):
    rng = np.random.default_rng(seed)
    if isinstance(n, int):
        n = (n,) * dim
    dx = tuple(rng.uniform(lo, hi, size=n[d]) for d in range(dim))
    per = tuple(periodic) if isinstance(periodic, (tuple, list)) else (periodic,) * dim
    return synth.Grid(dim, dx, per)


# (id, grid kwargs, method kwargs) -- element counts chosen so that blocks end ragged
CASES = [
    ("2d_dir_ip_p4_ea", dict(dim=2, n=(5, 3), seed=1), dict(P=4, smoother="EA", beta=(0, 0))),
    ("2d_per_ldg_p3_fa", dict(dim=2, n=(4, 3), periodic=True, seed=2),
     dict(P=3, smoother="FA", flux="ldg", beta=(0.5, 0.3))),
    ("2d_dir_ip_p8_fa_cubic", dict(dim=2, n=(3, 4), seed=3), dict(P=8, smoother="FA", weighting="cubic",
                                                                  beta=(0, 0))),
    ("3d_dir_ip_p2_fa", dict(dim=3, n=(3, 2, 4), seed=4), dict(P=2, smoother="FA")),
    ("3d_dir_ldg_p4_ea", dict(dim=3, n=(3, 3, 2), seed=5), dict(P=4, smoother="EA", flux="ldg",
                                                                beta=(0.5, 0.5, 0.5))),
    ("3d_dir_ip_p8_fa", dict(dim=3, n=(2, 3, 2), seed=6), dict(P=8, smoother="FA")),
    ("3d_per_ip_p6_fa", dict(dim=3, n=(3, 3, 3), periodic=True, seed=7), dict(P=6, smoother="FA")),
    ("3d_dir_ip_p8_ea0", dict(dim=3, n=(3, 2, 2), seed=8), dict(P=8, smoother="EA", overlap="zero")),
    ("3d_dir_ip_p8_ea", dict(dim=3, n=(2, 3, 2), seed=28), dict(P=8, smoother="EA")),
    ("3d_dir_ip_p12_fa", dict(dim=3, n=(2, 2, 1), seed=9), dict(P=12, smoother="FA")),
    ("3d_dir_ip_p16_ea", dict(dim=3, n=(2, 1, 2), seed=10), dict(P=16, smoother="EA")),
    ("3d_dir_ip_p16_fa", dict(dim=3, n=(1, 2, 2), seed=13), dict(P=16, smoother="FA")),
    # 2D at high order: long rows of the element apply and the patch solves in 2D tiles
    ("2d_dir_ip_p16_fa", dict(dim=2, n=(3, 2), seed=14), dict(P=16, smoother="FA")),
    ("2d_per_ip_p32_ea", dict(dim=2, n=(3, 3), periodic=True, seed=15), dict(P=32, smoother="EA")),
    # degenerate shapes: a single level (P = 1: the V-cycle is the exact coarse
    # solve), a single element, and mixed periodic / Dirichlet directions
    ("3d_dir_ip_p1_ea", dict(dim=3, n=(3, 2, 2), seed=21), dict(P=1, smoother="EA")),
    ("2d_per_ip_p1_fa", dict(dim=2, n=(3, 4), periodic=True, seed=22), dict(P=1, smoother="FA")),
    ("3d_dir_ip_1x1x1_p4_fa", dict(dim=3, n=(1, 1, 1), seed=23), dict(P=4, smoother="FA")),
    ("3d_mixed_ip_p4_fa", dict(dim=3, n=(3, 2, 3), periodic=(True, False, True), seed=26), dict(P=4, smoother="FA")),
    ("3d_mixed_ldg_p6_ea", dict(dim=3, n=(2, 3, 2), periodic=(False, True, False), seed=27),
     dict(P=6, smoother="EA", flux="ldg", beta=(0.5, 0.5, 0.5))),
    # P = 32: 3D elements and patch tiles beyond LDS (two-stage transfers, three-stage patch solves)
    ("3d_dir_ip_p32_fa", dict(dim=3, n=(2, 1, 2), seed=11), dict(P=32, smoother="FA")),
    ("3d_dir_ip_p32_ea", dict(dim=3, n=(1, 2, 2), seed=12), dict(P=32, smoother="EA")),
    # orders without compiled kernels (run-time order and tile forms), alone and
    # next to compiled levels of the same series
    ("2d_dir_ip_p5_ea", dict(dim=2, n=(4, 3), seed=41), dict(P=5, smoother="EA")),
    ("3d_dir_ip_p7_fa", dict(dim=3, n=(2, 3, 2), seed=42), dict(P=7, smoother="FA")),
    ("3d_per_ldg_p10_fa", dict(dim=3, n=(3, 3, 3), periodic=True, seed=43),
     dict(P=10, smoother="FA", flux="ldg", beta=(0.5, 0.5, 0.5))),
    ("2d_per_ip_p24_ea", dict(dim=2, n=(3, 3), periodic=True, seed=44), dict(P=24, smoother="EA")),
    ("3d_dir_ip_p17_fa", dict(dim=3, n=(2, 1, 2), seed=45), dict(P=17, smoother="FA")),
    ("3d_mixed_ip_p9_ea0", dict(dim=3, n=(2, 3, 2), periodic=(False, True, False), seed=46),
     dict(P=9, smoother="EA", overlap="zero")),
]


def case(cid):
    for c in CASES:
        if c[0] == cid:
            g = rand_grid(**c[1])
            return g, synth.Method(**c[2])
    raise KeyError(cid)


def to_elem(v_lex, grid, P):
    return op.to_elem(v_lex, grid.n, P)


def to_lex(v_elem, grid, P):
    return op.to_lex(v_elem, grid.n, P)


def hierarchy(grid, method, assemble=True):
    return mg.Hierarchy(grid, method, patch_mode="fdm", assemble=assemble)


# ------------------------------------------------------------------ solve parity (Alg. 2)
def rounding_envelope(H, f, n_iter, eps, runs=3, seed=0):
    """Per-iteration spread of the oracle's own residual history under rounding-level
    changes: MGCG runs of n_iter iterations whose preconditioned residual z carries a
    relative perturbation of size eps (seeded), compared with the unperturbed run.
    Returns, for k = 0..n_iter, the running maximum over j <= k of
    max_run |h_run[j] / h[j] - 1|: once orthogonality is lost the rounding
    differences between two runs do not die out again, while a single run's
    deviation at one k fluctuates (it can pass near zero by chance).

    Finite-precision CG loses orthogonality, after which ||r_k|| reacts to the last
    bits of every step: two FP64 runs of the same algorithm that differ only in
    rounding keep x within ~1e-11 of each other, yet their recursive residual norms
    part by per cent after a few dozen iterations (pinned on the CPU by
    test_oracle_multigrid.test_cg_history_is_rounding_sensitive)."""
    base = mg.mgcg(H, f, np.zeros_like(f), tol=0.0, i_max=n_iter)
    env = np.zeros(n_iter + 1)
    for k in range(runs):
        rs = np.random.default_rng(seed + k)

        def M(r, rs=rs):
            z = H.vcycle(np.zeros_like(r), r)
            return z * (1.0 + eps * rs.standard_normal(z.shape))

        pert = mg.mgcg(H, f, np.zeros_like(f), tol=0.0, i_max=n_iter, precond=M)
        env = np.maximum(env, np.abs(np.asarray(pert.history) / np.asarray(base.history) - 1.0))
    return np.maximum.accumulate(env)


def check_solve_parity(H, f, st, x_gpu, tol=1e-10, z_gap=None, label=""):
    """FP64 library solve against the oracle's MGCG started from the same x0 = 0.

    * x: the oracle is run for exactly the library's iteration count (tol = 0) and
      ||x - x_oracle||_2 <= 1e-10 ||x_oracle||_2 (after removing the mean on a fully
      periodic grid).
    * iteration count: equal to the oracle's; one more or one fewer only when the
      residual history sits within the band that rounding alone moves it by at the
      exit iteration (the oracle's rounding envelope at the measured library/oracle
      V-cycle gap z_gap, times 4), the generalisation of "within 1 % of the
      threshold" to long solves.
    * history: every ||r_k|| within rtol max(1e-6, 4 * envelope_k) of the oracle's
      (near the 1e-10 exit the residual carries rounding of order the V-cycle gap
      times ||r_0|| / ||r_k||, so even short solves need the envelope there).
    Returns the oracle result at the library's iteration count."""
    periodic = all(H.grid.periodic)
    n_gpu = st["iterations"]
    ref = mg.mgcg(H, f, np.zeros_like(f), tol=tol, i_max=max(200, n_gpu + 5))
    assert ref.converged, label
    n_ref = ref.iterations
    fixed = ref if n_gpu == n_ref else mg.mgcg(H, f, np.zeros_like(f), tol=0.0, i_max=n_gpu)
    h_gpu = np.asarray(st["history"][: n_gpu + 1])
    h_ref = np.asarray(fixed.history[: n_gpu + 1])
    eps = max(float(z_gap or 0.0), 1e-16)
    env = rounding_envelope(H, f, max(n_gpu, n_ref), eps)
    band = np.maximum(1e-6, 4.0 * env)
    thr = tol * h_ref[0]
    if n_gpu != n_ref:
        assert abs(n_gpu - n_ref) == 1, (label, n_gpu, n_ref)
        k = min(n_gpu, n_ref)        # the iteration where one stopped and the other did not
        assert abs(np.asarray(ref.history)[k] / thr - 1.0) <= band[k], (label, n_gpu, n_ref,
                                                                          ref.history[k] / thr, band[k])
    dev = np.abs(h_gpu / h_ref - 1.0)
    assert np.all(dev <= band[: n_gpu + 1]), (label, int(np.argmax(dev / band[: n_gpu + 1])),
                                              float(dev.max()))
    xs, rx = np.asarray(x_gpu), fixed.x
    if periodic:
        xs, rx = xs - xs.mean(), rx - rx.mean()
    err = np.linalg.norm(xs - rx) / np.linalg.norm(rx)
    assert err <= 1e-10, (label, err)
    return fixed


def residual_bound(A, f, x, tol=1e-10):
    """tol ||f|| plus the rounding of evaluating f - A x in FP64 twice (the library's
    exit check and the test's own): 2 gamma_m || |f| + |A| |x| ||, gamma_m = m u / (1 - m u),
    m the largest number of terms of a row (Higham, inner-product error bound)."""
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    m = int(np.diff(A.indptr).max()) + 1
    u = np.finfo(np.float64).eps / 2
    gam = m * u / (1 - m * u)
    return tol * np.linalg.norm(f) + 2 * gam * np.linalg.norm(np.abs(f) + abs(A) @ np.abs(x))


def kron_residual(grid, method, f_lex, x_lex, tol=1e-10):
    """(||f - A x||, bound) with the oracle's matrix-free Kronecker-sum operator of the
    top level; bound = tol ||f|| + 2 gamma_m || |f| + |A| |x| ||, |A| |x| bounded by the
    Kronecker sum of the element-wise absolute 1D operators (the masses are positive),
    m the most terms in a row (the sum over directions of the most non-zeros in a row
    of the 1D operator)."""
    ops = [op.operators_1d(method.P, np.asarray(grid.dx[d]), grid.periodic[d], b, method.mu_star)
           for d, b in enumerate(op._betas(method.beta, grid.dim))]
    res = np.linalg.norm(f_lex - op.apply_kron(grid, method.P, x_lex, ops=ops))
    aops = [(M, np.abs(Ld)) for (M, Ld) in ops]
    ax = op.apply_kron(grid, method.P, np.abs(x_lex), ops=aops)
    nterms = sum(int((np.asarray(Ld) != 0).sum(axis=1).max()) for (_, Ld) in aops)
    u = np.finfo(np.float64).eps / 2
    gam = nterms * u / (1 - nterms * u)
    return res, tol * np.linalg.norm(f_lex) + 2 * gam * np.linalg.norm(np.abs(f_lex) + ax)
