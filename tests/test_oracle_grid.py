"""Pins for the oracle's imaginary-time grid and propagator weights.

The weights are pinned to things other than the oracle's own quadrature:
the textbook two-stage Gauss collocation (Gauss-Legendre Runge-Kutta) matrix at
Delta = 0, the exact variation-of-constants result for a constant source, and
independent arbitrary-precision quadrature (mpmath).
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import grid as G


def test_gauss_legendre_nodes_two_point():
    c, b = G.panel_nodes(2)
    r = math.sqrt(3.0) / 6.0
    assert np.allclose(c, [0.5 - r, 0.5 + r], atol=1e-15, rtol=0)
    assert np.allclose(b, [0.5, 0.5], atol=1e-15, rtol=0)


@pytest.mark.parametrize("kind", ["etd", "lawson"])
def test_zero_delta_is_gauss_collocation(kind):
    """At Delta = 0 both schemes reduce to the Gauss-Legendre RK tableau (A, b)."""
    gr = G.Grid(beta=1.0, n_panels=1, m=2, kind=kind)
    E, Ee, W, We = gr.weights(np.array([0.0]))
    r = math.sqrt(3.0) / 6.0
    A = np.array([[0.25, 0.25 - r], [0.25 + r, 0.25]])
    assert np.allclose(W[:, :, 0], A, atol=1e-15, rtol=0)
    assert np.allclose(We[:, 0], [0.5, 0.5], atol=1e-15, rtol=0)
    assert np.allclose(E[:, 0], 1.0) and Ee[0] == 1.0


@pytest.mark.parametrize("m", [2, 4, 5])
@pytest.mark.parametrize("dh", [-9.0, -1.0, -1e-3, 0.0, 0.7, 4.0, 25.0])
def test_constant_source_exact(m, dh):
    """For constant S the variation-of-constants integral is exact:
    sum_x' W_xx' = (1 - exp(-Delta h c_x)) / Delta, sum_x' We_x' = (1 - exp(-Delta h)) / Delta."""
    h = 0.5
    gr = G.Grid(beta=h, n_panels=1, m=m)
    d = dh / h
    E, Ee, W, We = gr.weights(np.array([d]))
    if d == 0.0:
        expect = h * gr.c
        expect_e = h
    else:
        expect = -np.expm1(-d * h * gr.c) / d
        expect_e = -math.expm1(-d * h) / d
    assert np.allclose(W[:, :, 0].sum(1), expect, rtol=1e-13, atol=1e-16)
    assert math.isclose(We[:, 0].sum(), expect_e, rel_tol=1e-13)


@pytest.mark.parametrize("kind", ["etd", "lawson"])
@pytest.mark.parametrize("dh", [-12.0, 3.0, 30.0])
def test_weights_against_mpmath(kind, dh):
    mpmath.mp.dps = 40
    m, h = 4, 0.75
    gr = G.Grid(beta=h * 3, n_panels=3, m=m, kind=kind)
    d = dh / h
    E, Ee, W, We = gr.weights(np.array([d]))
    c = [mpmath.mpf(x) for x in gr.c]
    # For Delta < 0 the integrand reaches exp(|Delta h|) while the Lagrange basis
    # changes sign, so the FP64 sum cancels: allow eps * exp(|Delta h|) * 1e3.
    tol = max(1e-13, 2.2e-16 * math.exp(max(0.0, -dh)) * 1e3)

    def ell(k, u):
        out = mpmath.mpf(1)
        for j in range(m):
            if j != k:
                out *= (u - c[j]) / (c[k] - c[j])
        return out

    for x in range(m):
        for y in range(m):
            if kind == "etd":
                ref = h * mpmath.quad(lambda u: mpmath.exp(d * h * (u - c[x])) * ell(y, u), [0, c[x]])
            else:
                ref = h * mpmath.quad(lambda u: ell(y, u), [0, c[x]]) * mpmath.exp(d * h * (c[y] - c[x]))
            assert abs(W[x, y, 0] - float(ref)) <= tol * max(1.0, abs(float(ref)))
    for y in range(m):
        if kind == "etd":
            ref = h * mpmath.quad(lambda u: mpmath.exp(d * h * (u - 1)) * ell(y, u), [0, 1])
        else:
            ref = h * float(gr.b[y]) * mpmath.exp(d * h * (c[y] - 1))
        assert abs(We[y, 0] - float(ref)) <= tol * max(1.0, abs(float(ref)))


def test_h_derivative_matches_difference():
    gr = G.Grid(beta=2.0, n_panels=2, m=4)
    d = np.array([-3.0, 0.0, 0.4, 7.0])
    h, eps = gr.h, 1e-6
    w = gr.weights(d, deriv=True)
    wp = gr.weights(d, h=h + eps)
    wm = gr.weights(d, h=h - eps)
    for k in range(4):
        fd = (wp[k] - wm[k]) / (2 * eps)
        assert np.allclose(w[4 + k], fd, rtol=1e-7, atol=1e-9)


def test_grid_quadrature_weights():
    gr = G.Grid(beta=3.0, n_panels=5, m=4)
    assert gr.n_g == 20
    assert math.isclose(gr.g.sum(), 3.0, rel_tol=1e-14)
    # composite GL integrates exp(-tau) to near roundoff
    # 4-point GL on panels of width 0.6: error ~ h^9 f^(8) / 10^5 ~ 1e-11
    assert abs(gr.g @ np.exp(-gr.tau) - (1 - math.exp(-3.0))) < 2e-11
