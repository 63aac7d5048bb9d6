"""Convergence and cost measures of Sec. 4.1 (oracle).

rho   = (r_n / r_0)^(1/n)            eq. (rho)
r_bar = -log10(rho)                   eq. (r)
n_10  = cycles to reduce the residual by 10^10
W_op  = 2 N_P^3 N_E (2D, sum factorisation)
W_cyc = [C_S N_S (C_D M_D / 2 + 1) + C_CG] W_op      eq. (W_cyc)
omega = W_cyc / (r_bar W_op)          eq. (omega), read as the number of
        operator applications per decade: the printed product r_bar W_cyc/W_op
        does not reproduce the table values, the quotient does.
w_10  = 20/r_bar [C_S N_S (C_D M_D / 2 + 1) + C_CG] N_P       eq. (w_10)
C_D   = 4 (1 + 2 C_O)^3 (element-centred), 12 (1 + 2 C_O)(1 + 2 C_O/3)
        (face-centred), C_O = N_O / N_P (Sec. 3.1).
"""
from __future__ import annotations

import math
from typing import Sequence


def rho_rate(history: Sequence[float], n: int | None = None) -> float:
    if n is None:
        n = len(history) - 1
    return (history[n] / history[0]) ** (1.0 / n)


def r_bar(history: Sequence[float], n: int | None = None) -> float:
    return -math.log10(rho_rate(history, n))


def n10(history: Sequence[float]) -> int | None:
    for i, h in enumerate(history):
        if h <= 1e-10 * history[0]:
            return i
    return None


def c_d(kind: str, n_o: int, n_p: int) -> float:
    co = n_o / n_p
    if kind == "EC":
        return 4.0 * (1.0 + 2.0 * co) ** 3
    if kind == "FC":
        return 12.0 * (1.0 + 2.0 * co) * (1.0 + 2.0 * co / 3.0)
    raise ValueError(kind)


def w_cyc_over_w_op(kind: str, n_o: int, n_p: int, c_s: float = 4.0 / 3.0, n_s: int = 2,
                    c_cg: float = 1.0) -> float:
    m_d = 1 if kind == "EC" else 2
    return c_s * n_s * (0.5 * c_d(kind, n_o, n_p) * m_d + 1.0) + c_cg


def omega_bar(rbar: float, kind: str, n_o: int, n_p: int, **kw) -> float:
    return w_cyc_over_w_op(kind, n_o, n_p, **kw) / rbar


def w10(rbar: float, kind: str, n_o: int, n_p: int, **kw) -> float:
    return 10.0 / rbar * w_cyc_over_w_op(kind, n_o, n_p, **kw) * 2.0 * n_p
