"""1D spectral toolkit on Gauss-Lobatto-Legendre (GLL) points (oracle; test infrastructure).

Sec. 2.4: nodal Lagrange basis on the GLL points eta_i, GLL quadrature weights
rho_i (diagonal mass M^s = diag(rho)), differentiation D^s_{ik} = phi_k'(eta_i)
and the standard stiffness L^s_{ik} = sum_j rho_j D^s_{ji} D^s_{jk}.
Sec. 3.2: embedded interpolation between GLL bases of two orders.

Pins (tests/test_oracle_gll.py): end weights 2/(P(P+1)); weights sum to 2;
quadrature exact to degree 2P-1; D exact on degree <= P; L^s symmetric PSD
with null space = constants and equal to the exact integral of phi_i' phi_k';
interpolation exact on polynomials of the coarse degree; closed forms at P = 1, 2.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
from numpy.polynomial import legendre as npleg


@lru_cache(maxsize=None)
def gll(P: int):
    """GLL nodes eta (ascending) and weights rho for polynomial degree P >= 1.

    Nodes: -1, 1 and the roots of the derivative of the Legendre polynomial L_P.
    Weights: 2 / (P (P+1) L_P(eta_i)^2).
    """
    if P < 1:
        raise ValueError("P >= 1 required")
    cP = np.zeros(P + 1)
    cP[P] = 1.0
    inner = npleg.legroots(npleg.legder(cP)) if P >= 2 else np.zeros(0)
    eta = np.concatenate(([-1.0], np.sort(inner.real), [1.0]))
    # polish interior roots by Newton on L_P'
    d1 = npleg.legder(cP)
    d2 = npleg.legder(cP, 2)
    for _ in range(3):
        if P >= 2:
            x = eta[1:-1]
            eta[1:-1] = x - npleg.legval(x, d1) / npleg.legval(x, d2)
    LP = npleg.legval(eta, cP)
    rho = 2.0 / (P * (P + 1) * LP ** 2)
    eta.setflags(write=False)
    rho.setflags(write=False)
    return eta, rho


def lagrange_eval(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Matrix B[q, k] = phi_k(x_q) of the Lagrange basis on ``nodes`` (product formula)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = len(nodes)
    B = np.ones((len(x), n))
    for k in range(n):
        for j in range(n):
            if j != k:
                B[:, k] *= (x - nodes[j]) / (nodes[k] - nodes[j])
    return B


@lru_cache(maxsize=None)
def diff_matrix(P: int) -> np.ndarray:
    """D^s_{ik} = phi_k'(eta_i) via barycentric weights w_k = 1/prod_{j!=k}(eta_k - eta_j)."""
    eta, _ = gll(P)
    n = P + 1
    w = np.array([1.0 / np.prod([eta[k] - eta[j] for j in range(n) if j != k]) for k in range(n)])
    D = np.zeros((n, n))
    for i in range(n):
        for k in range(n):
            if i != k:
                D[i, k] = (w[k] / w[i]) / (eta[i] - eta[k])
        D[i, i] = -np.sum(D[i, :])
    D.setflags(write=False)
    return D


@lru_cache(maxsize=None)
def stiffness_std(P: int) -> np.ndarray:
    """L^s_{ik} = sum_j rho_j D^s_{ji} D^s_{jk} (Sec. 2.4)."""
    _, rho = gll(P)
    D = diff_matrix(P)
    L = D.T @ np.diag(rho) @ D
    L = 0.5 * (L + L.T)
    L.setflags(write=False)
    return L


@lru_cache(maxsize=None)
def interp_matrix(P_fine: int, P_coarse: int) -> np.ndarray:
    """Embedded interpolation J[i, k] = phi^{coarse}_k(eta^{fine}_i) (Sec. 3.2)."""
    ef, _ = gll(P_fine)
    ec, _ = gll(P_coarse)
    J = lagrange_eval(ec, ef)
    J.setflags(write=False)
    return J
