"""Learned face-weight variant: features, output map, face enumeration (oracle; test infrastructure).

Not part of the paper.  The face-centred smoother of Sec. 3.1 may use, per
face f of each smoothing level and normal direction, a transition width
theta_f and a damping omega_f in its normal weights (schwarz.fc_patches_1d).
A small MLP (oracle.mlp) predicts them from per-face features.

Faces are enumerated level by level (l = 1 .. L), then by direction d, then
face f = 0 .. nf_d - 1 (nf_d = N_d periodic, N_d + 1 Dirichlet; face f lies
between elements f-1 and f).

Features per face:
  P_l / 32,
  log2(dx_left / h_lat) / 5,  log2(dx_right / h_lat) / 5,
  1 on a Dirichlet boundary face else 0,
  D - 2,
  N_O,l / (P_l + 1),
where dx_left, dx_right are the sizes (in direction d) of the elements on
either side (the existing one at a boundary face) and h_lat is the geometric
mean of all element sizes of the other directions.

Output map: theta = 0.25 + 1.75 sigmoid(y0), omega = 0.5 + sigmoid(y1).

Pins (tests/test_oracle_learned.py): features of a hand-computed grid, the
output map at its neutral point, and theta = omega = 1 reproducing the fixed
smoother.
"""
from __future__ import annotations

import numpy as np

from .multigrid import level_orders
from .schwarz import overlap_for

THETA_MIN, THETA_MAX = 0.25, 2.0
OMEGA_MIN, OMEGA_MAX = 0.5, 1.5


def n_faces(n: int, periodic: bool) -> int:
    return n if periodic else n + 1


def face_index(grid, method):
    """List of (level, d, f) in the enumeration order."""
    out = []
    for l in range(1, len(level_orders(method.P))):
        for d in range(grid.dim):
            for f in range(n_faces(grid.n[d], grid.periodic[d])):
                out.append((l, d, f))
    return out


def face_features(grid, method) -> np.ndarray:
    orders = level_orders(method.P)
    logs = [np.log2(np.asarray(grid.dx[d], dtype=np.float64)) for d in range(grid.dim)]
    rows = []
    for l in range(1, len(orders)):
        P = orders[l]
        n_o = overlap_for(P, method.overlap)
        for d in range(grid.dim):
            others = [logs[e].mean() for e in range(grid.dim) if e != d]
            lat = float(np.mean(others))
            N = grid.n[d]
            for f in range(n_faces(N, grid.periodic[d])):
                if grid.periodic[d]:
                    left, right, bnd = (f - 1) % N, f % N, 0.0
                else:
                    left, right = max(f - 1, 0), min(f, N - 1)
                    bnd = 1.0 if f in (0, N) else 0.0
                rows.append([P / 32.0, (logs[d][left] - lat) / 5.0, (logs[d][right] - lat) / 5.0, bnd,
                             grid.dim - 2.0, n_o / (P + 1.0)])
    return np.asarray(rows, dtype=np.float64)


def outputs_to_params(Y):
    """MLP outputs y [n][2] -> (theta [n], omega [n])."""
    Y = np.asarray(Y, dtype=np.float64)
    sig = 1.0 / (1.0 + np.exp(-Y))
    return THETA_MIN + (THETA_MAX - THETA_MIN) * sig[:, 0], OMEGA_MIN + (OMEGA_MAX - OMEGA_MIN) * sig[:, 1]


def params_to_outputs(theta, omega):
    """Inverse of outputs_to_params (targets for training)."""
    a = (np.asarray(theta, dtype=np.float64) - THETA_MIN) / (THETA_MAX - THETA_MIN)
    b = (np.asarray(omega, dtype=np.float64) - OMEGA_MIN) / (OMEGA_MAX - OMEGA_MIN)
    return np.stack([np.log(a / (1 - a)), np.log(b / (1 - b))], axis=1)


def face_params_dict(grid, method, theta, omega):
    """Flat per-face arrays -> {level: [(theta_d, omega_d) per direction]} for Hierarchy."""
    out = {}
    k = 0
    for l in range(1, len(level_orders(method.P))):
        per_d = []
        for d in range(grid.dim):
            nf = n_faces(grid.n[d], grid.periodic[d])
            per_d.append((np.asarray(theta[k:k + nf], dtype=np.float64), np.asarray(omega[k:k + nf], dtype=np.float64)))
            k += nf
        out[l] = per_d
    assert k == len(theta)
    return out
