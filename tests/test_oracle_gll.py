"""Pins of the oracle's 1D spectral toolkit against closed forms and exact integrals."""
import numpy as np
import pytest

from oracle.gll import diff_matrix, gll, interp_matrix, lagrange_eval, stiffness_std


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 8, 12, 16, 32])
def test_gll_weights_and_exactness(P):
    eta, rho = gll(P)
    assert len(eta) == P + 1
    assert eta[0] == -1.0 and eta[-1] == 1.0
    assert np.all(np.diff(eta) > 0)
    # end weights 2/(P(P+1)) (the value behind mu_0 = {1/dx} P(P+1)/2)
    assert rho[0] == pytest.approx(2.0 / (P * (P + 1)), rel=1e-13)
    assert rho[-1] == pytest.approx(2.0 / (P * (P + 1)), rel=1e-13)
    assert rho.sum() == pytest.approx(2.0, rel=1e-14)
    # exact for degree <= 2P - 1
    for k in range(2 * P):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert np.dot(rho, eta ** k) == pytest.approx(exact, abs=1e-13)
    # and not for degree 2P: GLL gives 2/P for the integral 2/(2P+1) of L_P^2
    LP = np.polynomial.legendre.legval(eta, [0] * P + [1])
    assert np.dot(rho, LP ** 2) == pytest.approx(2.0 / P, rel=1e-12)
    assert np.allclose(eta, -eta[::-1], atol=1e-15)


def test_gll_closed_forms():
    eta, rho = gll(1)
    assert np.allclose(eta, [-1, 1]) and np.allclose(rho, [1, 1])
    eta, rho = gll(2)
    assert np.allclose(eta, [-1, 0, 1]) and np.allclose(rho, [1 / 3, 4 / 3, 1 / 3])
    eta, rho = gll(3)
    assert np.allclose(eta, [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1])
    assert np.allclose(rho, [1 / 6, 5 / 6, 5 / 6, 1 / 6])
    assert np.allclose(diff_matrix(1), [[-0.5, 0.5], [-0.5, 0.5]])
    assert np.allclose(stiffness_std(1), [[0.5, -0.5], [-0.5, 0.5]])


@pytest.mark.parametrize("P", [1, 2, 4, 7, 8, 16, 32])
def test_diff_matrix_exact_on_polynomials(P):
    eta, _ = gll(P)
    D = diff_matrix(P)
    for k in range(P + 1):
        ref = k * eta ** (k - 1) if k > 0 else np.zeros_like(eta)
        assert np.allclose(D @ eta ** k, ref, atol=1e-10 * max(1, P ** 2))
    # end-point entries of the GLL differentiation matrix
    assert D[0, 0] == pytest.approx(-P * (P + 1) / 4.0, rel=1e-12)
    assert D[P, P] == pytest.approx(P * (P + 1) / 4.0, rel=1e-12)


@pytest.mark.parametrize("P", [1, 2, 3, 6, 8, 16])
def test_stiffness_equals_exact_integral(P):
    """L^s_{ik} = int phi_i' phi_k' (GLL is exact for the degree 2P-2 product)."""
    eta, _ = gll(P)
    L = stiffness_std(P)
    xg, wg = np.polynomial.legendre.leggauss(2 * P + 2)
    # derivative of Lagrange basis at Gauss points by finite differences of the
    # product formula would be inaccurate; use the exact polynomial instead
    coeffs = []
    for k in range(P + 1):
        y = np.zeros(P + 1); y[k] = 1.0
        c = np.polynomial.polynomial.polyfit(eta, y, P)
        coeffs.append(np.polynomial.polynomial.polyder(c))
    dphi = np.array([np.polynomial.polynomial.polyval(xg, c) for c in coeffs])
    Lex = (dphi * wg) @ dphi.T
    assert np.allclose(L, Lex, atol=1e-8 * np.abs(Lex).max())
    assert np.allclose(L, L.T)
    w = np.linalg.eigvalsh(L)
    assert w[0] == pytest.approx(0.0, abs=1e-10 * w[-1])
    assert np.all(w[1:] > 1e-8)
    assert np.allclose(L @ np.ones(P + 1), 0.0, atol=1e-11 * max(1, P ** 3))


@pytest.mark.parametrize("pf,pc", [(2, 1), (4, 2), (8, 4), (6, 3), (3, 1), (12, 6), (32, 16)])
def test_interpolation_exact(pf, pc):
    ef, _ = gll(pf)
    ec, _ = gll(pc)
    J = interp_matrix(pf, pc)
    for k in range(pc + 1):
        assert np.allclose(J @ ec ** k, ef ** k, atol=1e-12)
    assert np.allclose(J.sum(axis=1), 1.0)
    B = lagrange_eval(ec, ec)
    assert np.allclose(B, np.eye(pc + 1))
