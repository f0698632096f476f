"""Pins of the oracle's 1-D basis against closed forms and exact polynomial
arithmetic (numpy.polynomial), independent of the oracle's own formulas.

Basis: Lagrange polynomials on Gauss-Legendre points, same order in time
(paper Sec. 2.1); inter-grid transfer for 3-partitioning (Sec. 2.3)."""
import numpy as np
import pytest
from numpy.polynomial import Polynomial as Poly

import oracle


def integrate01(f):
    """int_0^1 f by numpy's own 30-point Gauss-Legendre rule (exact for the
    polynomial degrees used here)."""
    x, w = np.polynomial.legendre.leggauss(30)
    return 0.5 * (w * f(0.5 * (x + 1.0))).sum()


def lagrange_polys(xi):
    """Exact Lagrange polynomials (numpy Polynomial objects) on nodes xi."""
    out = []
    for e in range(len(xi)):
        others = np.delete(xi, e)
        p = Poly.fromroots(others) if len(others) else Poly([1.0])
        out.append(p / p(xi[e]))
    return out


@pytest.mark.parametrize("N", range(1, 10))
def test_quadrature_exactness(N):
    xi, w = oracle.gauss_legendre(N)
    assert np.all(np.diff(xi) > 0) and xi[0] > 0 and xi[-1] < 1
    for k in range(2 * N):
        assert abs((w * xi ** k).sum() - 1.0 / (k + 1)) < 1e-14
    # degree 2N is not integrated exactly: the Gauss remainder on [0,1] for
    # x^(2N) is -(N!)^4 / ((2N+1) ((2N)!)^2)
    import math
    rem = -math.factorial(N) ** 4 / ((2 * N + 1) * math.factorial(2 * N) ** 2)
    err = (w * xi ** (2 * N)).sum() - 1.0 / (2 * N + 1)
    assert abs(err - rem) < 1e-3 * abs(rem)


def test_gl4_closed_form():
    # nodes of P_4 on [-1,1]: +-sqrt(3/7 -+ (2/7) sqrt(6/5))
    a = np.sqrt(3 / 7 - 2 / 7 * np.sqrt(6 / 5))
    b = np.sqrt(3 / 7 + 2 / 7 * np.sqrt(6 / 5))
    x = np.array([-b, -a, a, b])
    xi, w = oracle.gauss_legendre(4)
    # ascending on [0,1]: xi = (1 + x)/2
    assert np.allclose(xi, (1 + x) / 2, atol=1e-15, rtol=0)


def test_gl4_weights_closed_form():
    # weights on [-1,1] are (18 +- sqrt 30)/36; halved on [0,1]
    xi, w = oracle.gauss_legendre(4)
    wx = np.array([18 - np.sqrt(30), 18 + np.sqrt(30), 18 + np.sqrt(30), 18 - np.sqrt(30)]) / 72
    assert np.allclose(w, wx, atol=1e-15, rtol=0)


@pytest.mark.parametrize("N", range(1, 9))
def test_operators_against_exact_polynomials(N):
    b = oracle.basis(N)
    xi, w = b["xi"], b["w"]
    phi = lagrange_polys(xi)
    dphi = [p.deriv() for p in phi]
    # D[a][e] = phi_e'(xi_a)
    D = np.array([[dphi[e](xi[a]) for e in range(N)] for a in range(N)])
    assert np.allclose(b["D"], D, atol=1e-11 * max(1, np.abs(D).max()), rtol=0)
    # L, R: values at 0 and 1
    assert np.allclose(b["L"], [p(0.0) for p in phi], atol=1e-12)
    assert np.allclose(b["R"], [p(1.0) for p in phi], atol=1e-12)
    # Kw[a][e] = int_0^1 phi_a' phi_e (exact polynomial integration)
    Kw = np.array([[integrate01(lambda x: dphi[a](x) * phi[e](x)) for e in range(N)] for a in range(N)])
    assert np.allclose(b["Kw"], Kw, atol=1e-11 * max(1, np.abs(Kw).max()), rtol=0)
    # K1[k][l] = phi_k(1) phi_l(1) - int phi_k' phi_l, Kinv its inverse
    K1 = np.array([[phi[k](1.0) * phi[l](1.0) - integrate01(lambda x: dphi[k](x) * phi[l](x))
                    for l in range(N)] for k in range(N)])
    assert np.allclose(b["Kinv"] @ K1, np.eye(N), atol=1e-10)
    # K1 * 1 = L: a state without flux stays constant in time
    assert np.allclose(K1 @ np.ones(N), b["L"], atol=1e-11)


@pytest.mark.parametrize("N", range(1, 9))
def test_derivative_exact_on_monomials(N):
    b = oracle.basis(N)
    xi = b["xi"]
    for k in range(N):
        ref = k * xi ** (k - 1) if k > 0 else np.zeros(N)
        assert np.allclose(b["D"] @ xi ** k, ref, atol=1e-10)
    assert np.allclose(b["D"].sum(axis=1), 0.0, atol=1e-11)


@pytest.mark.parametrize("N", [1, 2, 4, 5, 7])
@pytest.mark.parametrize("r", [3, 9])
def test_transfer(N, r):
    xi, w = oracle.gauss_legendre(N)
    acc = np.zeros((N, N))
    for s in range(r):
        P, Rm = oracle.transfer(N, r, s)
        # P is exact on polynomials of degree <= p
        for k in range(N):
            assert np.allclose(P @ xi ** k, ((s + xi) / r) ** k, atol=1e-12)
        acc += Rm @ P
        # conservation identity: sum_k w_k (Rm F)_k = (1/r) sum_e w_e F_e
        F = np.cos(np.arange(N) + 0.3 * s)
        assert abs(w @ (Rm @ F) - (w @ F) / r) < 1e-14
    assert np.allclose(acc, np.eye(N), atol=5e-14)


def test_invalid_orders():
    with pytest.raises(AssertionError):
        oracle.gauss_legendre(0)
    with pytest.raises(AssertionError):
        oracle.gauss_legendre(11)
