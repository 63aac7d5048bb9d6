"""Training driver of the face-weight MLP (learned overlap weights and damping).

Extension beyond the paper: the face-centred smoother's normal weights get a
transition width theta and a damping omega per face (include/dgmg.h), predicted
by a 2 x 64 tanh MLP from per-face features.  Everything numerical runs in the
library: the solves that generate the data and the MLP forward, backward and
Adam kernels.  This module only organises them.

Data.  For each training problem (3D, random per-direction element sizes, FA
smoother) and each smoothing level, a coordinate search over a candidate grid
of uniform (theta, omega) on that level (other levels held at their current
best) measures the mean MGCG convergence factor
rho = (||r_n|| / ||r_0||)^(1/n) of a solve to 1e-10.  The best pair of a level
becomes the target of every face of that level (through the inverse of the
output map).  Training: full-batch Adam on the mean squared error.

File format (little-endian): 8-byte magic b"DGMGMLP1", uint32 version (1),
uint32 IN, HIDDEN, OUT, PARAMS, then PARAMS float32 values in the layout of
include/dgmg.h.

Usage: python -m paper_1603_02524_amd.learn --out <file.bin> [--problems K]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import struct
import sys
import time

import numpy as np

from . import dgmg

MAGIC = b"DGMGMLP1"
VERSION = 1
DEFAULT_PARAMS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "face_mlp_v1.bin")
THETA_MIN, THETA_MAX, OMEGA_MIN, OMEGA_MAX = 0.25, 2.0, 0.5, 1.5
THETAS = (0.5, 0.75, 1.0, 1.25, 1.5, 1.75)
OMEGAS = (0.8, 0.9, 1.0, 1.1, 1.2, 1.3)


# ---------------------------------------------------------------------- params file
def save_params(path, params):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
    if p.size != dgmg.mlp_param_count():
        raise ValueError("wrong parameter count")
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "wb") as fh:
        fh.write(MAGIC)
        fh.write(struct.pack("<5I", VERSION, dgmg.MLP_IN, dgmg.MLP_HIDDEN, dgmg.MLP_OUT, p.size))
        fh.write(p.astype("<f4").tobytes())


def load_params(path=DEFAULT_PARAMS):
    """Parameter vector (float32 numpy) of a saved network; raises on a foreign file."""
    with open(path, "rb") as fh:
        head = fh.read(8 + 20)
        if len(head) != 28 or head[:8] != MAGIC:
            raise ValueError(f"{path}: not a face-MLP parameter file")
        ver, n_in, n_hid, n_out, n_par = struct.unpack("<5I", head[8:])
        if ver != VERSION or (n_in, n_hid, n_out) != (dgmg.MLP_IN, dgmg.MLP_HIDDEN, dgmg.MLP_OUT):
            raise ValueError(f"{path}: version {ver} / shape {(n_in, n_hid, n_out)} not supported")
        data = np.frombuffer(fh.read(4 * n_par), dtype="<f4")
        if data.size != n_par or n_par != dgmg.mlp_param_count():
            raise ValueError(f"{path}: truncated")
    return data.astype(np.float32)


def init_params(seed=0):
    """U(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases (float32)."""
    rng = np.random.default_rng(seed)
    I, H, O = dgmg.MLP_IN, dgmg.MLP_HIDDEN, dgmg.MLP_OUT
    parts = [rng.uniform(-1, 1, H * I) / math.sqrt(I), np.zeros(H), rng.uniform(-1, 1, H * H) / math.sqrt(H),
             np.zeros(H), rng.uniform(-1, 1, O * H) / math.sqrt(H), np.zeros(O)]
    return np.concatenate(parts).astype(np.float32)


def params_to_outputs(theta, omega):
    a = (np.asarray(theta, dtype=np.float64) - THETA_MIN) / (THETA_MAX - THETA_MIN)
    b = (np.asarray(omega, dtype=np.float64) - OMEGA_MIN) / (OMEGA_MAX - OMEGA_MIN)
    return np.stack([np.log(a / (1 - a)), np.log(b / (1 - b))], axis=1)


# ---------------------------------------------------------------------- data
def training_problems(seed=11, count=24):
    """3D Dirichlet FA problems, P in {4, 8, 16, 32} on 8^3 / 8^3 / 6^3 / 4^3 elements,
    aspect ratios 1 .. 32 (per-direction sizes 2^U(0, a), a in {0, 2, 3.5, 5})."""
    import synth
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        P = (4, 8, 16, 32)[k % 4]
        n = {4: 8, 8: 8, 16: 6, 32: 4}[P]
        max_log2 = (0.0, 2.0, 3.5, 5.0)[(k // 4) % 4]
        dx = tuple(synth.random_spacing(rng, n, max_log2, 1.0) for _ in range(3))
        g = synth.Grid(3, dx, (False, False, False))
        m = synth.Method(P=P, smoother="FA", overlap="level")
        out.append((g, m))
    return out


def _rate(S, rhs, x):
    x.zero_()
    st = S.solve(rhs, x, tol=1e-10)
    return st["rho"] if st["iterations"] > 0 else 0.0


def search_problem(g, m, log=None):
    """Coordinate search of per-level uniform (theta, omega); returns per-level best and rates."""
    import torch
    S = dgmg.Solver(g, m, max_iter=60)
    try:
        n = S.n_dof()
        rng = np.random.default_rng(1)
        rhs = torch.tensor(rng.uniform(-1, 1, n), dtype=torch.float64, device="cuda")
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        nface = S.face_count()
        L = S.num_levels - 1
        per = nface // L
        theta = np.ones(nface)
        omega = np.ones(nface)
        S.set_face_params(None)
        base = _rate(S, rhs, x)
        best_rate = base
        for l in range(L, 0, -1):           # top level first
            sl = slice((l - 1) * per, l * per)
            bt, bo = theta[sl][0], omega[sl][0]
            for t in THETAS:
                for o in OMEGAS:
                    theta[sl], omega[sl] = t, o
                    S.set_face_params(theta, omega)
                    r = _rate(S, rhs, x)
                    if r < best_rate - 1e-12:
                        best_rate, bt, bo = r, t, o
            theta[sl], omega[sl] = bt, bo
        X = S.face_features()
        levels = [(S.level_info(l)[0], float(theta[(l - 1) * per]), float(omega[(l - 1) * per]))
                  for l in range(1, L + 1)]
        if log:
            log(f"  P={m.P} AR={g.aspect_ratio():.1f}: rho fixed {base:.4f} -> {best_rate:.4f}, "
                f"(P_l, theta, omega) {levels}")
        return X, theta, omega, base, best_rate, levels
    finally:
        S.close()


# ---------------------------------------------------------------------- training
def train(X, Y, steps=3000, lr=3e-3, seed=0, log=None):
    """Full-batch Adam on (1/B) sum (MLP(X) - Y)^2 with the library kernels."""
    import torch
    dev = "cuda"
    p = torch.tensor(init_params(seed), device=dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    Xd = torch.tensor(np.asarray(X, dtype=np.float32), device=dev).contiguous()
    Td = torch.tensor(np.asarray(Y, dtype=np.float32), device=dev).contiguous()
    hist = []
    for t in range(1, steps + 1):
        out, work = dgmg.mlp_forward(p, Xd)
        g = dgmg.mlp_backward(p, Xd, Td, out, work)
        dgmg.mlp_adam(p, g, m, v, t, lr=lr)
        if t == 1 or t % 500 == 0 or t == steps:
            loss = float(((out - Td) ** 2).sum() / Xd.shape[0])
            hist.append((t, loss))
            if log:
                log(f"  step {t}: loss {loss:.5f}")
    return p.cpu().numpy(), hist


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=DEFAULT_PARAMS)
    ap.add_argument("--problems", type=int, default=32)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--report", default=None, help="JSON summary path")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    t0 = time.time()
    Xs, Ys, summary = [], [], []
    for k, (g, m) in enumerate(training_problems(count=a.problems)):
        log(f"problem {k}")
        X, th, om, base, best, levels = search_problem(g, m, log)
        Xs.append(X)
        Ys.append(params_to_outputs(th, om))
        summary.append({"P": m.P, "aspect_ratio": g.aspect_ratio(), "rho_fixed": base, "rho_best": best,
                        "levels": levels})
    X = np.concatenate(Xs)
    Y = np.concatenate(Ys)
    log(f"training on {len(X)} faces")
    params, hist = train(X, Y, steps=a.steps, log=log)
    save_params(a.out, params)
    rep = {"samples": int(len(X)), "loss": hist, "problems": summary, "seconds": time.time() - t0}
    if a.report:
        with open(a.report, "w") as fh:
            json.dump(rep, fh, indent=1)
    log(f"saved {a.out} ({time.time() - t0:.0f} s)")
    return 0


if __name__ == "__main__":
    sys.exit(main())
