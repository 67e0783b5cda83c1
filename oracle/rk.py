"""Differential form of the amplitude equations (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm alg:diff: the amplitudes obey ds/dtau = -(Delta s + S[s])
(eqn:smud) from s(0) = 0 and are stepped across a uniform grid
tau_i = i h, h = beta / n_g, i = 0..n_g, by an explicit Runge-Kutta method;
Omega_CC = (1/beta) sum_i g_i E[s(tau_i)] uses Simpson's rule on the same
grid (Section III, numerical integration and propagation schemes; the
paper's Table tab:numerr lists RK1, RK2 and RK4 with a Simpson quadrature).

Readings where the paper is silent:
  * n_g counts grid intervals and must be even (composite Simpson);
  * RK1 is forward Euler, RK2 the explicit trapezoidal rule (Heun), RK4 the
    classical fourth-order method;
  * the same grid carries the quadrature and the integrator (as the paper
    states for its own runs).

Adjoint: reverse-mode differentiation of the explicit march (the discrete
counterpart of eqn:lmud).  With the stage states Y_j = s_n + h sum_l a_jl k_l,
k_j = f(Y_j), s_{n+1} = s_n + h sum_j b_j k_j and the cotangent sbar_{n+1} of
s_{n+1}:
  kbar_j = h b_j sbar_{n+1} + h sum_{i>j} a_ij Ybar_i
  Ybar_j = J_f(Y_j)^T kbar_j = -(Delta kbar_j + J_S(Y_j)^T kbar_j)
  sbar_n = sbar_{n+1} + sum_j Ybar_j + (g_n / beta) dE/ds(s_n)
Derivatives: dOmega/dtheta = d(Omega_0 + Omega_1)/dtheta
  + sum_i (g_i/beta) E(s_i; dI) - sum_n sum_j <kbar_j, S(Y_j; dI)>
  + for beta: (1/n_g) sum_n [<sbar_{n+1}, sum_j b_j k_j> + sum_j <Ybar_j, sum_l a_jl k_l>]
((1/beta) g_i = w_i / (3 n_g) with the Simpson pattern w does not depend on beta).
"""
from __future__ import annotations

import dataclasses

import numpy as np

# Butcher tableaus (a strictly lower triangular, b); c is not needed because
# the right-hand side does not depend on tau explicitly.
TABLEAUS = {
    "rk1": (np.zeros((1, 1)), np.array([1.0])),
    "rk2": (np.array([[0.0, 0.0], [1.0, 0.0]]), np.array([0.5, 0.5])),
    "rk4": (np.array([[0.0, 0.0, 0.0, 0.0],
                      [0.5, 0.0, 0.0, 0.0],
                      [0.0, 0.5, 0.0, 0.0],
                      [0.0, 0.0, 1.0, 0.0]]), np.array([1.0, 2.0, 2.0, 1.0]) / 6.0),
}


def simpson_weights(n_g: int, h: float) -> np.ndarray:
    """Composite Simpson weights g_0..g_{n_g} on a uniform grid of n_g (even) intervals."""
    if n_g < 2 or n_g % 2:
        raise ValueError("Simpson's rule needs an even number of intervals")
    w = np.ones(n_g + 1)
    w[1:-1:2] = 4.0
    w[2:-1:2] = 2.0
    return w * (h / 3.0)


def _axpy(y, a, x):
    return tuple(yi + a * xi for yi, xi in zip(y, x))


def _inner(a, b):
    return float(sum(np.sum(x * y) for x, y in zip(a, b)))


def rk_march(f, y0, h, n_steps, method):
    """Generic explicit Runge-Kutta march of dy/dt = f(y) over tuples of arrays.
    Returns the states y_0..y_n and, per step, the stage states and slopes."""
    A, b = TABLEAUS[method]
    y = y0
    states, stages, slopes = [y0], [], []
    for _ in range(n_steps):
        Y, K = [], []
        for j in range(len(b)):
            yj = y
            for l in range(j):
                if A[j, l] != 0.0:
                    yj = _axpy(yj, h * A[j, l], K[l])
            Y.append(yj)
            K.append(f(yj))
        for j in range(len(b)):
            y = _axpy(y, h * b[j], K[j])
        states.append(y)
        stages.append(Y)
        slopes.append(K)
    return states, stages, slopes


@dataclasses.dataclass
class RKSolution:
    method: str
    n_g: int
    beta: float
    states: list       # s_0 .. s_{n_g}
    stages: list       # per step: stage states Y_j
    slopes: list       # per step: k_j
    energies: np.ndarray
    omega_cc: float
    omega0: float
    omega1: float

    @property
    def omega(self):
        return self.omega0 + self.omega1 + self.omega_cc

    @property
    def h(self):
        return self.beta / self.n_g


def _rhs(model, s):
    S = model.residual(s)
    return (-(model.delta1 * s[0] + S[0]), -(model.delta2 * s[1] + S[1]))


def solve(model, beta, n_g, method="rk4"):
    """Forward march of Algorithm alg:diff with Simpson's rule for Omega_CC."""
    h = beta / n_g
    g = simpson_weights(n_g, h)
    states, stages, slopes = rk_march(lambda s: _rhs(model, s), model.zeros(), h, n_g, method)
    for s in states:
        if not all(np.all(np.isfinite(x)) for x in s):
            raise FloatingPointError("non-finite amplitudes")
    energies = np.array([model.energy(s) for s in states])
    return RKSolution(method, n_g, float(beta), states, stages, slopes, energies,
                      float(g @ energies) / beta, float(model.omega0()), float(model.omega1()))


@dataclasses.dataclass
class RKAdjoint:
    kbar: list         # per step: cotangents of the slopes k_j
    hbar: float        # d Omega_CC / d h at fixed thermal integrals
    sbar: list         # per grid point: d Omega_CC / d s_i (total, through every later step)


def adjoint(model, sol: RKSolution):
    A, b = TABLEAUS[sol.method]
    h, n_g = sol.h, sol.n_g
    wts = simpson_weights(n_g, h) / sol.beta
    sbar = model.vjp(sol.states[n_g], wts[n_g], (None, None))
    sbar_all = [None] * (n_g + 1)
    sbar_all[n_g] = sbar
    kbar_all = [None] * n_g
    hbar = 0.0
    for n in reversed(range(n_g)):
        Y, K = sol.stages[n], sol.slopes[n]
        ns = len(b)
        Ybar, Kbar = [None] * ns, [None] * ns
        for j in reversed(range(ns)):
            kb = tuple(h * b[j] * x for x in sbar)
            for i in range(j + 1, ns):
                if A[i, j] != 0.0:
                    kb = _axpy(kb, h * A[i, j], Ybar[i])
            Kbar[j] = kb
            g = model.vjp(Y[j], None, kb)
            Ybar[j] = (-(model.delta1 * kb[0] + g[0]), -(model.delta2 * kb[1] + g[1]))
        # explicit dependence on the step h
        step = model.zeros()
        for j in range(ns):
            step = _axpy(step, b[j], K[j])
        hbar += _inner(sbar, step)
        for j in range(ns):
            inc = model.zeros()
            for l in range(j):
                if A[j, l] != 0.0:
                    inc = _axpy(inc, A[j, l], K[l])
            hbar += _inner(Ybar[j], inc)
        new = sbar
        for j in range(ns):
            new = _axpy(new, 1.0, Ybar[j])
        new = _axpy(new, 1.0, model.vjp(sol.states[n], wts[n], (None, None)))
        sbar = new
        sbar_all[n] = sbar
        kbar_all[n] = Kbar
    return RKAdjoint(kbar_all, hbar, sbar_all)


def _integral_term(model, sol, adj, dints):
    """sum_i (g_i/beta) E(s_i; dI) - sum_n sum_j <kbar_j, S(Y_j; dI)>."""
    wts = simpson_weights(sol.n_g, sol.h) / sol.beta
    tot = 0.0
    for i, s in enumerate(sol.states):
        tot += wts[i] * model.energy(s, dints)
    for n in range(sol.n_g):
        for Y, kb in zip(sol.stages[n], adj.kbar[n]):
            tot -= _inner(kb, model.residual(Y, dints))
    return tot


def d_omega(model, sol, adj, theta, dh=None, deri=None):
    """dOmega/dtheta for theta in {'mu', 'beta', 'h'} at a frozen reference
    (orbitals, eps and the dropped slots fixed); 'h' takes a direction
    (dh, deri) of the one-body matrix and the two-electron integrals."""
    ints = model.ints
    dn_mu, dn_beta = model.occ_derivs()
    if theta == "mu":
        return (model.domega0("mu") + model.domega_mf(dn_mu)
                + _integral_term(model, sol, adj, ints.derivative(dn=dn_mu)))
    if theta == "h":
        return (model.domega_mf(np.zeros_like(dn_mu), dh=dh, deri=deri)
                + _integral_term(model, sol, adj, ints.derivative(dh=dh, deri=deri)))
    if theta == "beta":
        return (model.domega0("beta") + model.domega_mf(dn_beta)
                + _integral_term(model, sol, adj, ints.derivative(dn=dn_beta))
                + adj.hbar / sol.n_g)
    raise ValueError(theta)


def d_omega_dh(model, sol, adj):
    """dOmega/dh_pq (matrix) at a frozen reference."""
    wts = simpson_weights(sol.n_g, sol.h) / sol.beta
    out = model.dmf_dh()
    for i, s in enumerate(sol.states):
        out = out + model.vjp_fock(s, wts[i], (None, None))
    for n in range(sol.n_g):
        for Y, kb in zip(sol.stages[n], adj.kbar[n]):
            out = out + model.vjp_fock(Y, None, tuple(-x for x in kb))
    return out


def d_omega_deps(model, sol, adj):
    """dOmega/deps_q at a frozen reference for the differential form: the
    occupation and explicit-u parts as in solver.d_omega_deps, and the slopes'
    dependence on Delta, d k_j / d Delta = -Y_j, weighted by the slope
    cotangents kbar_j."""
    from .solver import _eps_from_delta
    ints = model.ints
    n = model.n
    dn_mu, _ = model.occ_derivs()
    d0 = model.domega0_deps()
    out = np.zeros(n)
    for q in range(n):
        dn = np.zeros(n)
        dn[q] = -dn_mu[q]
        du = np.zeros((n, n))
        du[q, q] = -1.0
        out[q] = (d0[q] + model.domega_mf(dn, dh=du)
                  + _integral_term(model, sol, adj, ints.derivative(dn=dn, dh=du)))
    D1, D2 = model.zeros()
    for n_step in range(sol.n_g):
        for Y, kb in zip(sol.stages[n_step], adj.kbar[n_step]):
            D1 = D1 - kb[0] * Y[0]
            D2 = D2 - kb[1] * Y[1]
    return out + _eps_from_delta(model, D1, D2)
