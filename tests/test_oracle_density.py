"""The two-body response density of the oracle (Gamma = dOmega/d<pq|rs> within
the integrals keeping <pq|rs> = <qp|sr>) against central differences of the
re-solved Omega (Richardson), for single elements and a random direction, on
the integral form and on the differential form."""
import math

import numpy as np
import pytest

import ftcc_inputs as fi
from oracle import grid as G, restricted as R, rk as K, solver as S, spinorb as so


def _richardson(f, d=1e-4):
    fd1 = (f(d) - f(-d)) / (2 * d)
    fd2 = (f(d / 2) - f(-d / 2)) / d
    return (4 * fd2 - fd1) / 3


@pytest.fixture(scope="module")
def case():
    s = fi.hubbard_config(L=3, U=2.0, T=1.0)
    rng = np.random.default_rng(5)
    c = rng.standard_normal((3,) * 4) * 0.05
    eri = s.eri + c + c.transpose(1, 0, 3, 2)          # generic, keeps <pq|rs> = <qp|sr>
    return s, eri


def _model(s, eri):
    return R.RestrictedModel(R.RestrictedIntegrals(s.h, eri, s.eps, s.mu, s.beta))


@pytest.mark.parametrize("form", ["collocation", "rk4"])
def test_two_body_density_against_finite_differences(case, form):
    s, eri = case
    gr = G.Grid(s.beta, 2, 4)

    def solve(e):
        m = _model(s, e)
        if form == "rk4":
            sol = K.solve(m, s.beta, 6, "rk4")
            return m, sol, None
        return m, S.solve(m, gr, tol=1e-14), None

    m, sol, _ = solve(eri)
    if form == "rk4":
        adj = K.adjoint(m, sol)
        along = lambda d: K.d_omega(m, sol, adj, "h", deri=d)
    else:
        adj = S.adjoint(m, gr, sol, tol=1e-14)
        along = lambda d: S.d_omega(m, gr, sol, adj, "h", deri=d)
    gam = S.two_body_density(along, 3)
    assert np.abs(gam - gam.transpose(1, 0, 3, 2)).max() < 1e-14
    rng = np.random.default_rng(9)
    dirs = []
    for (p, q, r, t) in ((0, 0, 0, 0), (0, 1, 0, 1), (0, 1, 1, 0), (2, 0, 1, 1)):
        d = np.zeros((3,) * 4)
        d[p, q, r, t] += 0.5
        d[q, p, t, r] += 0.5
        dirs.append(d)
    x = rng.standard_normal((3,) * 4)
    dirs.append(x + x.transpose(1, 0, 3, 2))
    for d in dirs:
        fd = _richardson(lambda h: solve(eri + h * d)[1].omega)
        assert abs(np.sum(gam * d) - fd) < 1e-8 * max(1.0, abs(fd))


@pytest.mark.parametrize("U,beta", [(4.0, 1.0), (2.0, 3.0)])
def test_atomic_limit_density_is_double_occupancy(U, beta):
    """One orbital (two spin orbitals), where FT-CCSD is exact: the grand
    potential is -(1/beta) ln(1 + 2 e^{beta mu} + e^{beta(2 mu - U)}) for every U
    at fixed mu and reference, so the density element dOmega/d<00|00> =
    dOmega/dU is the thermal double occupancy <n_up n_down> =
    e^{beta(2 mu - U)} / Z, a closed form independent of the method.  Restricted
    model (the single element) and spin-orbital model (every integral scales
    with U, so sum Gamma <pq|rs> / U is the same number)."""
    mu = U / 2
    h = np.zeros((1, 1))
    eri = np.full((1, 1, 1, 1), U)
    eps = np.array([U / 2])
    z = 1 + 2 * math.exp(beta * mu) + math.exp(beta * (2 * mu - U))
    docc = math.exp(beta * (2 * mu - U)) / z
    gr = G.Grid(beta, 8, 4)
    m = R.RestrictedModel(R.RestrictedIntegrals(h, eri, eps, mu, beta))
    sol = S.solve(m, gr, tol=1e-14)
    adj = S.adjoint(m, gr, sol, tol=1e-14)
    gam = S.two_body_density(lambda d: S.d_omega(m, gr, sol, adj, "h", deri=d), 1)
    assert abs(gam[0, 0, 0, 0] - docc) < 1e-8 * max(1.0, docc)
    hs, es, epss = so.spin_orbital_from_spatial(h, eri, eps)
    ms = so.SpinOrbitalModel(so.ThermalIntegrals(hs, es, epss, mu, beta))
    sols = S.solve(ms, gr, tol=1e-14)
    adjs = S.adjoint(ms, gr, sols, tol=1e-14)
    gams = S.two_body_density(lambda d: S.d_omega(ms, gr, sols, adjs, "h", deri=d), 2)
    assert abs(np.sum(gams * es) / U - docc) < 1e-8 * max(1.0, docc)


@pytest.mark.parametrize("U,beta", [(4.0, 1.0), (2.0, 3.0)])
def test_atomic_limit_density_differential_form_converges_at_fourth_order(U, beta):
    """The same closed form for the differential form: the RK4 march, its
    reverse pass and the density approach <n_up n_down> with the method's
    order (the error falls by about 2^4 when the grid is doubled)."""
    mu = U / 2
    h = np.zeros((1, 1))
    eri = np.full((1, 1, 1, 1), U)
    eps = np.array([U / 2])
    z = 1 + 2 * math.exp(beta * mu) + math.exp(beta * (2 * mu - U))
    docc = math.exp(beta * (2 * mu - U)) / z
    m = R.RestrictedModel(R.RestrictedIntegrals(h, eri, eps, mu, beta))
    errs = []
    for n_g in (32, 64):
        sol = K.solve(m, beta, n_g, "rk4")
        adj = K.adjoint(m, sol)
        gam = S.two_body_density(lambda d: K.d_omega(m, sol, adj, "h", deri=d), 1)
        errs.append(abs(gam[0, 0, 0, 0] - docc))
    assert errs[1] < 1e-8
    assert 3.5 < math.log2(errs[0] / errs[1]) < 4.5
