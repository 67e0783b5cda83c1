"""Pins of the orbital-energy response dOmega/deps_q (Section II.D, type 2;
Appendix B): the derivative at frozen h, <pq|rs>, mu, beta and orbitals.

  * Richardson-extrapolated central differences of the re-solved Omega in each
    eps_q, for the exponential-collocation and integrating-factor integral
    forms and the RK4 differential form, restricted and in spin orbitals, with a
    reference that is not Hartree-Fock (so that the occupation, Fock and
    explicit u = f - diag(eps) parts all contribute);
  * the shift identity: moving every eps_q and every h_qq by c equals moving mu
    by -c (occupations, Delta, u and the mean-field parts are unchanged), so
    sum_q (dOmega/deps_q + dOmega/dh_qq) = -dOmega/dmu: the trace of the
    paper's relaxed density p^cc equals the electron number.
"""
import numpy as np
import pytest

import ftcc_inputs as fi
from oracle import grid as G, restricted as R, rk as K, solver as S, spinorb as so


def _richardson(f, x0, d=1e-4):
    fd1 = (f(x0 + d) - f(x0 - d)) / (2 * d)
    fd2 = (f(x0 + d / 2) - f(x0 - d / 2)) / d
    return (4 * fd2 - fd1) / 3


def _ring_case():
    s = fi.hubbard_config(L=3, U=2.0, T=1.0)
    rng = np.random.default_rng(7)
    dh = rng.standard_normal((3, 3)) * 0.05
    h = s.h + dh + dh.T
    eps = s.eps + rng.uniform(-0.1, 0.1, 3)          # not the Fock diagonal
    return h, s.eri, eps, s.mu, s.beta


def _restricted(h, eri, eps, mu, beta):
    return R.RestrictedModel(R.RestrictedIntegrals(h, eri, eps, mu, beta))


@pytest.mark.parametrize("form", ["etd", "lawson", "rk4"])
def test_deps_against_finite_differences(form):
    h, eri, eps, mu, beta = _ring_case()

    def omega(e):
        m = _restricted(h, eri, e, mu, beta)
        if form == "rk4":
            return K.solve(m, beta, 8, "rk4").omega
        return S.solve(m, G.Grid(beta, 2, 4, form), tol=1e-14).omega

    model = _restricted(h, eri, eps, mu, beta)
    if form == "rk4":
        sol = K.solve(model, beta, 8, "rk4")
        d = K.d_omega_deps(model, sol, K.adjoint(model, sol))
    else:
        gr = G.Grid(beta, 2, 4, form)
        sol = S.solve(model, gr, tol=1e-14)
        d = S.d_omega_deps(model, gr, sol, S.adjoint(model, gr, sol, tol=1e-14))
    for q in range(3):
        def f(x, q=q):
            e = eps.copy()
            e[q] = x
            return omega(e)
        fd = _richardson(f, eps[q])
        assert abs(d[q] - fd) < 1e-8 * max(1.0, abs(fd)), (q, d[q], fd)


@pytest.mark.parametrize("form,case", [("etd", "ring"), ("rk4", "ring"), ("etd", "random")])
def test_trace_of_relaxed_density_is_electron_number(form, case):
    if case == "ring":
        h, eri, eps, mu, beta = _ring_case()
    else:
        h, eri, eps = fi.random_hamiltonian(5, seed=8, scale=0.04)
        mu, beta = 0.05, 1.5
    model = _restricted(h, eri, eps, mu, beta)
    if form == "rk4":
        sol = K.solve(model, beta, 6, "rk4")
        adj = K.adjoint(model, sol)
        deps = K.d_omega_deps(model, sol, adj)
        dh = K.d_omega_dh(model, sol, adj)
        dmu = K.d_omega(model, sol, adj, "mu")
    else:
        gr = G.Grid(beta, 2, 4)
        sol = S.solve(model, gr, tol=1e-13)
        adj = S.adjoint(model, gr, sol, tol=1e-13)
        deps = S.d_omega_deps(model, gr, sol, adj)
        dh = S.d_omega_dh(model, gr, sol, adj)
        dmu = S.d_omega(model, gr, sol, adj, "mu")
    trace = float(np.sum(deps + np.diag(dh)))
    assert abs(trace + dmu) < 1e-10 * abs(dmu)
    # the Delta part is not seen by the trace: it must still be there
    assert np.abs(deps + np.diag(dh) - 2.0 * model.ints.n_occ).max() > 1e-6


def test_deps_spin_orbital_against_finite_differences():
    h, eri, eps, mu, beta = _ring_case()
    H, ERI, EPS = so.spin_orbital_from_spatial(h, eri, eps)
    gr = G.Grid(beta, 2, 4)

    def model(e):
        return so.SpinOrbitalModel(so.ThermalIntegrals(H, ERI, e, mu, beta))
    m0 = model(EPS)
    sol = S.solve(m0, gr, tol=1e-14)
    d = S.d_omega_deps(m0, gr, sol, S.adjoint(m0, gr, sol, tol=1e-14))
    for q in (0, 3):            # an alpha and a beta spin orbital
        def f(x, q=q):
            e = EPS.copy()
            e[q] = x
            return S.solve(model(e), gr, tol=1e-14).omega
        fd = _richardson(f, EPS[q])
        assert abs(d[q] - fd) < 1e-8 * max(1.0, abs(fd)), (q, d[q], fd)
