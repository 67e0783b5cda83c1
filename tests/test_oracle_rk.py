"""Pins of the differential-form oracle (Algorithm alg:diff with explicit
Runge-Kutta and Simpson's rule, Table tab:numerr).

* the tableaus: one step of each method on dy/dt = -y multiplies y by the
  Taylor polynomial of exp(-h) truncated at the method's order (the defining
  property of an explicit RK method of order <= 4 with that many stages), and
  the step error on a nonlinear scalar problem with a closed-form solution
  falls at the method's order;
* Simpson's rule integrates cubics exactly and its weights sum to beta;
* the FT-CCSD march converges to the independently pinned exponential
  collocation limit at the orders the paper's table states (RK1 h, RK2 h^2,
  RK4 h^4; the Simpson quadrature adds h^4);
* the reverse-mode derivatives equal Richardson-extrapolated central
  differences of the same discretised Omega (mu, beta, U, h_pq).
"""
import math

import numpy as np
import pytest

import ftcc_inputs as fi
from oracle import grid as G, restricted as R, rk as K, solver as S


def _r_model(h, eri, eps, mu, beta):
    return R.RestrictedModel(R.RestrictedIntegrals(h, eri, eps, mu, beta))


def _richardson(f, x0, d=1e-4):
    fd1 = (f(x0 + d) - f(x0 - d)) / (2 * d)
    fd2 = (f(x0 + d / 2) - f(x0 - d / 2)) / d
    return (4 * fd2 - fd1) / 3


@pytest.mark.parametrize("method,order", [("rk1", 1), ("rk2", 2), ("rk4", 4)])
def test_tableau_stability_polynomial(method, order):
    h = 0.3
    st, _, _ = K.rk_march(lambda y: (-y[0],), (np.array([1.0]),), h, 1, method)
    taylor = sum((-h) ** k / math.factorial(k) for k in range(order + 1))
    assert abs(st[1][0][0] - taylor) < 1e-15


@pytest.mark.parametrize("method,order", [("rk1", 1), ("rk2", 2), ("rk4", 4)])
def test_global_order_on_logistic_equation(method, order):
    """y' = y (1 - y), y(0) = 0.2: y(t) = 1 / (1 + 4 e^{-t})."""
    exact = 1.0 / (1.0 + 4.0 * math.exp(-2.0))
    errs = []
    for n in (20, 40, 80):
        st, _, _ = K.rk_march(lambda y: (y[0] * (1.0 - y[0]),), (np.array([0.2]),), 2.0 / n, n, method)
        errs.append(abs(st[-1][0][0] - exact))
    p = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert all(abs(x - order) < 0.15 for x in p), p


def test_simpson_weights():
    beta, n = 1.7, 10
    g = K.simpson_weights(n, beta / n)
    tau = np.linspace(0.0, beta, n + 1)
    assert abs(g.sum() - beta) < 1e-15
    for k in range(4):
        assert abs(g @ tau ** k - beta ** (k + 1) / (k + 1)) < 1e-13
    with pytest.raises(ValueError):
        K.simpson_weights(7, 0.1)


@pytest.fixture(scope="module")
def hub():
    s = fi.hubbard_config(L=4, U=2.0, T=1.0)
    model = _r_model(s.h, s.eri, s.eps, s.mu, s.beta)
    ref = S.solve(model, G.Grid(s.beta, 8, 6), tol=1e-14).omega_cc   # collocation limit
    return s, model, ref


@pytest.mark.parametrize("method,grids,lo,hi", [("rk1", (32, 64, 128), 0.8, 1.2),
                                                ("rk2", (16, 32, 64), 1.85, 2.15),
                                                ("rk4", (16, 32, 64), 3.8, 4.2)])
def test_ftccsd_order_matches_table(hub, method, grids, lo, hi):
    s, model, ref = hub
    errs = [abs(K.solve(model, s.beta, n, method).omega_cc - ref) for n in grids]
    p = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert p[0] < p[1] + 0.05 and lo < p[1] < hi, p      # approaching the order from below


def test_rk4_extrapolates_to_collocation_limit(hub):
    s, model, ref = hub
    a = K.solve(model, s.beta, 64, "rk4").omega_cc
    b = K.solve(model, s.beta, 128, "rk4").omega_cc
    assert abs(b - ref) > 1e-9                              # not converged by itself
    assert abs((16 * b - a) / 15 - ref) < 3e-10 * max(1.0, abs(ref))


def test_zero_step_count_rejected(hub):
    s, model, _ = hub
    with pytest.raises(ValueError):
        K.solve(model, s.beta, 5, "rk4")


@pytest.fixture(scope="module")
def grad_case():
    s = fi.hubbard_config(L=3, U=2.0, T=1.0)
    rng = np.random.default_rng(3)
    dh = rng.standard_normal((3, 3)) * 0.05
    h = s.h + dh + dh.T

    def run(mu=s.mu, beta=s.beta, h=h, eri=s.eri, method="rk4", n_g=6):
        m = _r_model(h, eri, s.eps, mu, beta)
        return m, K.solve(m, beta, n_g, method)

    return s, h, run


@pytest.mark.parametrize("method", ["rk1", "rk2", "rk4"])
def test_gradients_against_finite_differences(grad_case, method):
    s, h, run = grad_case
    model, sol = run(method=method)
    adj = K.adjoint(model, sol)
    for theta, f, x0 in (("mu", lambda x: run(mu=x, method=method)[1].omega, s.mu),
                         ("beta", lambda x: run(beta=x, method=method)[1].omega, s.beta)):
        an = K.d_omega(model, sol, adj, theta)
        assert abs(an - _richardson(f, x0)) < 1e-8 * max(1.0, abs(an)), theta
    U = s.meta["U"]
    an = K.d_omega(model, sol, adj, "h", deri=s.eri / U)
    fd = _richardson(lambda x: run(eri=s.eri * x / U, method=method)[1].omega, U)
    assert abs(an - fd) < 1e-8 * max(1.0, abs(an))
    gh = K.d_omega_dh(model, sol, adj)
    for p, q in ((0, 1), (1, 1), (2, 0)):
        e = np.zeros((3, 3))
        e[p, q] = 1.0
        fd = _richardson(lambda x: run(h=h + x * e, method=method)[1].omega, 0.0)
        assert abs(gh[p, q] - fd) < 1e-8


def test_electron_number_matches_collocation(grad_case):
    """-dOmega/dmu of the two discretisations agree as both grids are refined."""
    s, h, run = grad_case
    model, sol = run(n_g=32)
    n_rk = -K.d_omega(model, sol, K.adjoint(model, sol), "mu")
    gr = G.Grid(s.beta, 4, 4)
    sc = S.solve(model, gr, tol=1e-14)
    n_col = -S.d_omega(model, gr, sc, S.adjoint(model, gr, sc, tol=1e-14), "mu")
    assert abs(n_rk - n_col) < 1e-6
