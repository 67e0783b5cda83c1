"""Pins of the FT-CCSD oracle against what the theory fixes.

Each test pins the oracle to something other than itself:
  P1  two spin orbitals (one-site Hubbard): FT-CCSD is exact, closed form
  P2  spinless two-site model in a rotated basis with a non-HF reference:
      exact closed form, singles with Delta != 0 and a nonzero diagonal u
  P3  O(U^2) term = finite-temperature MP2 closed form
  P4  free fermions in a rotated basis with wrong orbital energies: exact
  P5  grand-canonical exact diagonalisation: error vanishes as U^4
  P6  grid convergence order (the paper's Table tab:numerr style check)
  P8  restricted (spin-summed) kernels = spin-orbital kernels; t2 symmetry;
      invariance under rotations inside degenerate plane-wave shells
  P9  the vector-Jacobian product equals the transpose of a complex-step JVP
  P10 adjoint derivatives agree with Richardson-extrapolated central FD;
"""
import math

import numpy as np
import pytest

import ftcc_inputs as fi
from oracle import ed, grid as G, restricted as R, solver as S, spinorb as so


def _so_model(h, eri, eps, mu, beta, thr=0.0):
    return so.SpinOrbitalModel(so.ThermalIntegrals(h, eri, eps, mu, beta, thr))


def _r_model(h, eri, eps, mu, beta, thr=0.0):
    return R.RestrictedModel(R.RestrictedIntegrals(h, eri, eps, mu, beta, thr))


# ------------------------------------------------------------------ P1
@pytest.mark.parametrize("U,beta", [(4.0, 1.0), (8.0, 0.5), (2.0, 3.0)])
def test_p1_atomic_limit_exact(U, beta):
    mu = U / 2
    h = np.zeros((1, 1))
    eri = np.full((1, 1, 1, 1), U)
    eps = np.array([U / 2])                       # thermal HF at half filling
    exact = -math.log(1 + 2 * math.exp(beta * mu) + math.exp(-beta * (U - 2 * mu))) / beta
    for model in (_so_model(*so.spin_orbital_from_spatial(h, eri, eps), mu, beta),
                  _r_model(h, eri, eps, mu, beta)):
        sol = S.solve(model, G.Grid(beta, 8, 4))
        assert abs(sol.omega - exact) < 1e-11 * abs(exact)


# ------------------------------------------------------------------ P2
def _dimer(theta=0.35, t=1.0, V=1.5):
    hs = np.array([[0.0, -t], [-t, 0.0]])
    es = np.zeros((2,) * 4)
    es[0, 1, 0, 1] = V
    es[1, 0, 1, 0] = V
    C = np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]])
    h = C.T @ hs @ C
    eri = np.einsum("ijkl,ip,jq,kr,ls->pqrs", es, C, C, C, C)
    return h, eri


@pytest.mark.parametrize("kind", ["etd", "lawson"])
def test_p2_spinless_dimer_exact(kind):
    t, V, beta, mu = 1.0, 1.5, 2.0, 0.3
    h, eri = _dimer(t=t, V=V)
    eps = np.diag(h) + np.array([-0.2, 0.4])      # deliberately not Hartree-Fock
    exact = -math.log(1 + math.exp(beta * (mu + t)) + math.exp(beta * (mu - t))
                      + math.exp(-beta * (V - 2 * mu))) / beta
    model = _so_model(h, eri, eps, mu, beta)
    errs = []
    for P in (2, 4, 8):
        errs.append(abs(S.solve(model, G.Grid(beta, P, 4, kind)).omega - exact))
    assert errs[-1] < 1e-9
    assert errs[0] > errs[1] > errs[2]


# ------------------------------------------------------------------ P3
def _mp2_closed_form(model):
    """-(1/4 beta) sum n n (1-n)(1-n) |<ij||ab>|^2 Phi - (1/beta) sum n (1-n) |u_ai|^2 Phi,
    Phi(D) = beta/D - (1 - exp(-beta D)) / D^2, Phi(0) = beta^2 / 2."""
    b = model.ints
    beta = b.beta

    def phi(d):
        out = np.empty_like(d)
        small = np.abs(beta * d) < 1e-6
        ds = np.where(small, 1.0, d)
        out[~small] = (beta / ds - (-np.expm1(-beta * ds)) / ds ** 2)[~small]
        out[small] = (beta ** 2 / 2 - beta ** 3 * d / 6)[small]
        return out

    n, v = b.n_occ, b.n_vir
    w2 = n[:, None, None, None] * n[None, :, None, None] * v[None, None, :, None] * v[None, None, None, :]
    om = -np.sum(w2 * b.vas ** 2 * phi(model.delta2)) / (4 * beta)
    w1 = n[:, None] * v[None, :]
    om -= np.sum(w1 * b.u.T ** 2 * phi(model.delta1)) / beta
    return om


def test_p3_second_order_is_mp2():
    """Half-filled ring at mu = U/2 with eps = -2t cos k + U/2: occupations and
    Delta do not depend on U, so Omega_CC(U) / U^2 -> the MP2 closed form."""
    L, beta = 4, 1.0
    vals = {}
    for U in (0.01, 0.02):
        sysm = fi.hubbard_config(L=L, U=U, T=1.0 / beta)
        hs, es, ps = so.spin_orbital_from_spatial(sysm.h, sysm.eri, sysm.eps)
        model = _so_model(hs, es, ps, sysm.mu, beta)
        vals[U] = S.solve(model, G.Grid(beta, 5, 4)).omega_cc / U ** 2
        if U == 0.01:
            c_exact = _mp2_closed_form(model) / U ** 2
    c_rich = 2 * vals[0.01] - vals[0.02]          # removes the O(U) correction
    assert abs(c_rich - c_exact) < 1e-6 * abs(c_exact)


def test_p3_single_site_coefficient():
    """One site: the closed form gives -beta U^2 / 32 (Taylor series of the exact Omega)."""
    beta, U = 1.0, 1e-3
    h = np.zeros((1, 1))
    model = _so_model(*so.spin_orbital_from_spatial(h, np.full((1, 1, 1, 1), U), np.array([U / 2])), U / 2, beta)
    assert abs(_mp2_closed_form(model) / U ** 2 + beta / 32) < 1e-12


# ------------------------------------------------------------------ P4
def test_p4_free_fermions_rotated_basis_exact():
    rng = np.random.default_rng(7)
    L, beta, mu = 3, 1.0, 0.2
    h0, _ = fi.hubbard_ring(L, 1.0, 0.0)
    Q, _ = np.linalg.qr(rng.standard_normal((L, L)))
    h = Q.T @ h0 @ Q
    eri = np.zeros((L,) * 4)
    eps = np.diag(h) + np.array([0.3, -0.25, 0.1])     # wrong reference energies
    exact = -2.0 * np.sum(np.logaddexp(0.0, -beta * (np.linalg.eigvalsh(h) - mu))) / beta
    model = _r_model(h, eri, eps, mu, beta)
    sol = S.solve(model, G.Grid(beta, 8, 4))
    assert abs(sol.omega - exact) < 1e-10 * abs(exact)


# ------------------------------------------------------------------ P5
@pytest.mark.parametrize("L", [2, 3])
def test_p5_exact_diagonalisation_u4(L):
    errs = []
    Us = (0.25, 0.5)
    for U in Us:
        sysm = fi.hubbard_config(L=L, U=U, T=1.0)
        hs, es, ps = so.spin_orbital_from_spatial(sysm.h, sysm.eri, sysm.eps)
        exact = ed.grand_potential(hs, es, sysm.mu, sysm.beta)
        sol = S.solve(_r_model(sysm.h, sysm.eri, sysm.eps, sysm.mu, sysm.beta), G.Grid(sysm.beta, 5, 4))
        errs.append(abs(sol.omega - exact))
    order = math.log(errs[1] / errs[0]) / math.log(Us[1] / Us[0])
    assert 3.6 < order < 4.4
    assert errs[0] < 2e-6


def test_p5_ed_free_fermions():
    """ED itself against the free-fermion formula (pins the ED code)."""
    sysm = fi.hubbard_config(L=3, U=0.0, T=0.7)
    hs, es, _ = so.spin_orbital_from_spatial(sysm.h, sysm.eri, sysm.eps)
    exact = -np.sum(np.logaddexp(0.0, -sysm.beta * (np.linalg.eigvalsh(hs) - sysm.mu))) / sysm.beta
    assert abs(ed.grand_potential(hs, es, sysm.mu, sysm.beta) - exact) < 1e-12


# ------------------------------------------------------------------ P6
def test_p6_grid_convergence_order():
    sysm = fi.hubbard_config(L=3, U=1.5, T=1.0)
    model = _r_model(sysm.h, sysm.eri, sysm.eps, sysm.mu, sysm.beta)
    ref = S.solve(model, G.Grid(sysm.beta, 16, 4)).omega_cc
    errs = [abs(S.solve(model, G.Grid(sysm.beta, P, 4)).omega_cc - ref) for P in (1, 2, 4)]
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(orders) > 4.0          # at least the order of the paper's Simpson rule


# ------------------------------------------------------------------ P8
def _so_amplitudes(t1, t2):
    n = t1.shape[0]
    N = 2 * n
    s1 = np.zeros((N, N))
    s2 = np.zeros((N,) * 4)
    for a in range(2):
        s1[a * n:(a + 1) * n, a * n:(a + 1) * n] = t1
        for b in range(2):
            A, B = slice(a * n, (a + 1) * n), slice(b * n, (b + 1) * n)
            s2[A, B, A, B] += t2
            s2[A, B, B, A] -= t2.transpose(0, 1, 3, 2)
    return s1, s2


@pytest.mark.parametrize("case", ["random", "ueg"])
def test_p8_restricted_equals_spin_orbital(case):
    if case == "random":
        n = 5
        h, eri, eps = fi.random_hamiltonian(n, seed=3)
        mu, beta = 0.1, 1.3
    else:
        s = fi.ueg_config(19, 14, 1.0, 0.5)
        n, h, eri, mu, beta = s.n, s.h, s.eri, s.mu, s.beta
        eps = s.eps + 0.01 * np.arange(n)
    t1, t2 = fi.random_amplitudes(n, seed=4, scale=0.2)
    rm = _r_model(h, eri, eps, mu, beta)
    sm = _so_model(*so.spin_orbital_from_spatial(h, eri, eps), mu, beta)
    s1, s2 = _so_amplitudes(t1, t2)
    R1, R2 = rm.residual((t1, t2))
    S1, S2 = sm.residual((s1, s2))
    assert abs(rm.energy((t1, t2)) - sm.energy((s1, s2))) < 1e-13
    assert np.abs(R1 - S1[:n, :n]).max() < 1e-13
    assert np.abs(R2 - S2[:n, n:, :n, n:]).max() < 1e-13
    assert np.abs(R2 - R2.transpose(0, 1, 3, 2) - S2[:n, :n, :n, :n]).max() < 1e-13
    assert np.abs(R2 - R2.transpose(1, 0, 3, 2)).max() < 1e-13


def test_p8_solution_symmetry_and_shell_rotation():
    s = fi.ueg_config(7, 2, 1.0, 1.0)
    gr = G.Grid(s.beta, 1, 4)
    sol = S.solve(_r_model(s.h, s.eri, s.eps, s.mu, s.beta), gr)
    for t1, t2 in sol.nodes:
        assert np.abs(t2 - t2.transpose(1, 0, 3, 2)).max() < 1e-14
    # rotate orbitals inside the degenerate |n|^2 = 1 shell (indices 1..6)
    rng = np.random.default_rng(2)
    Q = np.eye(s.n)
    q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    Q[1:7, 1:7] = q
    h2 = Q.T @ s.h @ Q
    eri2 = np.einsum("pqrs,pi,qj,rk,sl->ijkl", s.eri, Q, Q, Q, Q, optimize=True)
    sol2 = S.solve(_r_model(h2, eri2, s.eps, s.mu, s.beta), gr)
    assert abs(sol2.omega - sol.omega) < 1e-11 * abs(sol.omega)


# ------------------------------------------------------------------ P9
@pytest.mark.parametrize("model_kind", ["so", "r"])
def test_p9_vjp_is_transpose_of_jvp(model_kind):
    rng = np.random.default_rng(11)
    if model_kind == "so":
        h, eri, eps = fi.random_hamiltonian(3, seed=1)
        h, eri, eps = so.spin_orbital_from_spatial(h, eri, eps)
        model = _so_model(h, eri, eps, 0.05, 1.1)
    else:
        h, eri, eps = fi.random_hamiltonian(4, seed=1)
        model = _r_model(h, eri, eps, 0.05, 1.1)
    n = model.n
    s = (rng.standard_normal((n, n)) * 0.3, rng.standard_normal((n,) * 4) * 0.3)
    v = (rng.standard_normal((n, n)), rng.standard_normal((n,) * 4))
    lt = (rng.standard_normal((n, n)), rng.standard_normal((n,) * 4))
    eb = 0.37
    hstep = 1e-30
    sc = (s[0] + 1j * hstep * v[0], s[1] + 1j * hstep * v[1])
    J1, J2 = model.residual(sc)
    jv = (J1.imag / hstep, J2.imag / hstep)
    e_c = model._kernel("E", sc, model.ints)
    lhs = np.sum(lt[0] * jv[0]) + np.sum(lt[1] * jv[1]) + eb * (e_c.imag / hstep)
    g = model.vjp(s, eb, lt)
    rhs = np.sum(g[0] * v[0]) + np.sum(g[1] * v[1])
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


# ------------------------------------------------------------------ P10
@pytest.fixture(scope="module")
def p10_case():
    sysm = fi.hubbard_config(L=3, U=2.0, T=1.0)
    rng = np.random.default_rng(1)
    dh = rng.standard_normal((3, 3)) * 0.05
    h = sysm.h + dh + dh.T
    gr = G.Grid(sysm.beta, 3, 4)

    def run(mu=sysm.mu, beta=sysm.beta, h=h, eri=sysm.eri):
        g = G.Grid(beta, 3, 4)
        m = _r_model(h, eri, sysm.eps, mu, beta)
        return m, g, S.solve(m, g, tol=1e-14)

    model, _, sol = run()
    adj = S.adjoint(model, gr, sol)
    return dict(sysm=sysm, h=h, gr=gr, run=run, model=model, sol=sol, adj=adj)


def _richardson(f, x0, d=1e-4):
    fd1 = (f(x0 + d) - f(x0 - d)) / (2 * d)
    fd2 = (f(x0 + d / 2) - f(x0 - d / 2)) / d
    return (4 * fd2 - fd1) / 3


def test_p10_dmu_dbeta(p10_case):
    c = p10_case
    s = c["sysm"]
    for theta, f, x0 in (("mu", lambda x: c["run"](mu=x)[2].omega, s.mu),
                         ("beta", lambda x: c["run"](beta=x)[2].omega, s.beta)):
        an = S.d_omega(c["model"], c["gr"], c["sol"], c["adj"], theta)
        assert abs(an - _richardson(f, x0)) < 1e-8 * max(1.0, abs(an))


def test_p10_du_and_dh(p10_case):
    c = p10_case
    s = c["sysm"]
    U = s.meta["U"]
    an = S.d_omega(c["model"], c["gr"], c["sol"], c["adj"], "h", deri=s.eri / U)
    fd = _richardson(lambda x: c["run"](eri=s.eri * x / U)[2].omega, U)
    assert abs(an - fd) < 1e-8 * max(1.0, abs(an))
    gh = S.d_omega_dh(c["model"], c["gr"], c["sol"], c["adj"])
    for p, q in ((0, 1), (1, 1), (2, 0)):
        e = np.zeros((3, 3))
        e[p, q] = 1.0
        fd = _richardson(lambda x: c["run"](h=c["h"] + x * e)[2].omega, 0.0)
        assert abs(gh[p, q] - fd) < 1e-8


def test_p10_electron_number(p10_case):
    """<N> = -dOmega/dmu lies strictly between 0 and 2n and is close to the
    reference count 2 sum_p n_p (the correlation correction is small at U = 2)."""
    c = p10_case
    n_el = -S.d_omega(c["model"], c["gr"], c["sol"], c["adj"], "mu")
    n_ref = 2.0 * float(np.sum(c["model"].ints.n_occ))
    assert 0.0 < n_el < 2 * c["model"].n
    assert abs(n_el - n_ref) < 0.2


def test_find_mu_free_fermions_closed_form():
    """U = 0 with the exact reference: N(mu) = 2 sum_k f(eps_k - mu), so the
    fixed-<N> search must land on the root of the closed form."""
    from scipy.optimize import brentq
    s = fi.hubbard_config(L=6, U=0.0, T=1.0)
    gr = G.Grid(s.beta, 2, 4)

    def make(mu):
        return R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, mu, s.beta))
    mu, n, _ = S.find_mu(make, gr, 5.0, mu0=0.0, tol=1e-12)

    def n_exact(m):
        return 2.0 * np.sum(1.0 / (1.0 + np.exp(s.beta * (s.eps - m)))) - 5.0
    mu_exact = brentq(n_exact, -5.0, 5.0, xtol=1e-15)
    assert abs(mu - mu_exact) < 1e-10
    assert abs(n - 5.0) < 1e-11


def test_find_mu_interacting_against_finite_differences():
    """U != 0: at the returned mu, -dOmega/dmu from central differences of Omega
    itself (no adjoint) equals the target electron number."""
    s = fi.hubbard_config(L=4, U=2.0, T=1.0)
    gr = G.Grid(s.beta, 2, 4)

    def make(mu):
        return R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, mu, s.beta))
    mu, n, _ = S.find_mu(make, gr, 3.5, mu0=s.mu, tol=1e-12)
    assert abs(n - 3.5) < 1e-11

    def om(m):
        return S.solve(make(m), gr, tol=1e-14).omega
    d = 1e-3
    d1 = (om(mu + d) - om(mu - d)) / (2 * d)
    d2 = (om(mu + d / 2) - om(mu - d / 2)) / d
    n_fd = -(4 * d2 - d1) / 3
    assert abs(n_fd - 3.5) < 1e-8


def test_adjoint_diis_same_solution(p10_case):
    """Extrapolating the adjoint sweeps (DIIS) leaves the solution of the linear
    panel equations unchanged: lambda, lambda-tilde and dOmega/dmu agree with the
    plain sweeps (whose derivatives the central differences above pin)."""
    c = p10_case
    plain = c["adj"]
    fast = S.adjoint(c["model"], c["gr"], c["sol"], diis=5)
    for a, b in zip(plain.lam + plain.lamt, fast.lam + fast.lamt):
        scale = max(1.0, np.abs(a[1]).max())
        assert np.abs(a[0] - b[0]).max() < 1e-11 * scale and np.abs(a[1] - b[1]).max() < 1e-11 * scale
    d0 = S.d_omega(c["model"], c["gr"], c["sol"], plain, "mu")
    d1 = S.d_omega(c["model"], c["gr"], c["sol"], fast, "mu")
    assert abs(d0 - d1) < 1e-11 * max(1.0, abs(d0))
    assert sum(fast.iters) < sum(plain.iters)
