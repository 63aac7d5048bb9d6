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
