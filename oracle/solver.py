"""Imaginary-time march, Lambda adjoint and response derivatives (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Works with any model object that provides delta1/delta2, zeros(), energy(),
residual(), vjp(), vjp_fock(), occ_derivs(), domega_mf(), omega0(), omega1()
and `ints.derivative()` (spin-orbital or restricted).

Forward (Algorithm alg:int in panels, with the grid of grid.py):
  s(0) = 0; for each panel, from the initial guess s_x = E_x s_b iterate
      s_x <- E_x s_b - sum_x' W_xx' S[s_x']
  (Picard) until max|change| <= tol * max(1, max|s|), then
      s_b <- E_e s_b - sum_x' We_x' S[s_x'].
  Omega_CC = (1/beta) sum_x g_x E[s_x]            (eqn:Ecc with eqn:g)

Adjoint (the stationarity conditions of the discrete form of eqn:Lagrangian):
  L = Omega_CC + sum_x <lam_x, F_x> + sum_p <a_{p+1}, F_e,p>
  F_x   = s_x - E_x s_b + sum_x' W_xx' S_x',  F_e = s_b' - E_e s_b + sum We_x' S_x'
  lam_x = -(g_x/beta) dE/ds(s_x) - J_x^T lamt_x,   J_x = dS/ds at s_x
  lamt_x = sum_x'' W_x''x lam_x'' + We_x a_{p+1}   (the discrete eqn:ltilde)
  a_p    = sum_x E_x lam_x + E_e a_{p+1},  a_P = 0
which is the discrete counterpart of eqn:lmu / eqn:ltilde (lam_x = -L_x).

Derivatives dOmega/dtheta = dL/dtheta at fixed (s, lam, a):
  d(Omega_0 + Omega_1)/dtheta
  + sum_x [(g_x/beta) E(s_x; dI) + <lamt_x, S(s_x; dI)>]     (E, S linear in I)
  + for beta: sum_x <lam_x, -dE_x/dbeta s_b + sum dW_xx'/dbeta S_x'>
              + sum_p <a_{p+1}, -dE_e/dbeta s_b + sum dWe_x'/dbeta S_x'>
(the paper's response types 1, 2, 4, 5 and 6 for this discretisation;
(1/beta) g_x = b_x / P does not depend on beta).
"""
from __future__ import annotations

import dataclasses

import numpy as np


def _inner(a, b):
    return float(np.sum(a[0] * b[0]) + np.sum(a[1] * b[1]))


def _maxabs(s):
    return max(float(np.max(np.abs(s[0]), initial=0.0)), float(np.max(np.abs(s[1]), initial=0.0)))


@dataclasses.dataclass
class Solution:
    nodes: list          # per node (s1, s2)
    resid: list          # per node (S1, S2) at the converged amplitudes
    sb: list             # per panel: state at the panel start
    energies: np.ndarray
    omega_cc: float
    omega0: float
    omega1: float
    iters: list

    @property
    def omega(self):
        return self.omega0 + self.omega1 + self.omega_cc


def _panel_weights(model, grid, deriv=False):
    w1 = grid.weights(model.delta1, deriv=deriv)
    w2 = grid.weights(model.delta2, deriv=deriv)
    return w1, w2


def _diis_next(hist_s, hist_r):
    """Anderson/DIIS extrapolation: minimise |sum c_j r_j| with sum c_j = 1."""
    k = len(hist_r)
    G = np.array([[float(np.dot(a, b)) for b in hist_r] for a in hist_r])
    A = np.zeros((k + 1, k + 1))
    A[:k, :k] = G / max(np.max(np.abs(np.diag(G))), 1e-300)
    A[:k, k] = A[k, :k] = -1.0
    rhs = np.zeros(k + 1)
    rhs[k] = -1.0
    c = np.linalg.lstsq(A, rhs, rcond=None)[0][:k]
    return sum(cj * (sj + rj) for cj, sj, rj in zip(c, hist_s, hist_r))


def _flat(vs):
    return np.concatenate([np.concatenate([v[0].ravel(), v[1].ravel()]) for v in vs])


def _unflat(vec, like):
    out, off = [], 0
    for v in like:
        a = vec[off:off + v[0].size].reshape(v[0].shape)
        off += v[0].size
        b = vec[off:off + v[1].size].reshape(v[1].shape)
        off += v[1].size
        out.append((a, b))
    return out


def solve(model, grid, tol=1e-13, max_iter=400, mix=1.0, diis=0):
    """Forward march.  `mix` < 1 applies linear damping to the Picard update;
    diis > 1 extrapolates over that many sweeps (the fixed point is unchanged)."""
    (E1, Ee1, W1, We1), (E2, Ee2, W2, We2) = _panel_weights(model, grid)
    m = grid.m
    sb = model.zeros()
    nodes, resid, starts, iters = [], [], [], []
    for p in range(grid.P):
        starts.append(sb)
        s = [(E1[x] * sb[0], E2[x] * sb[1]) for x in range(m)]
        hist_s, hist_r = [], []
        for it in range(1, max_iter + 1):
            S = [model.residual(s[x]) for x in range(m)]
            new = []
            for x in range(m):
                n1 = E1[x] * sb[0] - sum(W1[x, y] * S[y][0] for y in range(m))
                n2 = E2[x] * sb[1] - sum(W2[x, y] * S[y][1] for y in range(m))
                if mix != 1.0:
                    n1 = mix * n1 + (1.0 - mix) * s[x][0]
                    n2 = mix * n2 + (1.0 - mix) * s[x][1]
                new.append((n1, n2))
            change = max(_maxabs((new[x][0] - s[x][0], new[x][1] - s[x][1])) for x in range(m))
            scale = max(1.0, max(_maxabs(v) for v in new))
            if not np.isfinite(change):
                raise FloatingPointError(f"panel {p}: non-finite amplitudes")
            if change <= tol * scale:
                s = new
                break
            if diis > 1:
                hist_s.append(_flat(s))
                hist_r.append(_flat(new) - hist_s[-1])
                hist_s, hist_r = hist_s[-diis:], hist_r[-diis:]
                new = _unflat(_diis_next(hist_s, hist_r), new) if len(hist_r) > 1 else new
            s = new
        else:
            raise RuntimeError(f"panel {p}: Picard iteration did not converge (last change {change:.3e})")
        iters.append(it)
        S = [model.residual(s[x]) for x in range(m)]
        nodes.extend(s)
        resid.extend(S)
        sb = (Ee1 * sb[0] - sum(We1[y] * S[y][0] for y in range(m)),
              Ee2 * sb[1] - sum(We2[y] * S[y][1] for y in range(m)))
    wts = np.tile(grid.b / grid.P, grid.P)            # (1/beta) g_x
    energies = np.array([model.energy(s) for s in nodes])
    return Solution(nodes, resid, starts, energies, float(wts @ energies),
                    float(model.omega0()), float(model.omega1()), iters)


@dataclasses.dataclass
class Adjoint:
    lam: list        # per node
    lamt: list       # per node (lambda tilde)
    a: list          # per panel boundary p = 1..P (a[p] multiplies F_e of panel p-1); a[P] = 0
    iters: list


def adjoint(model, grid, sol: Solution, tol=1e-13, max_iter=400, diis=0):
    """Backward sweep over the panels.  The panel equations for lam are linear
    and solved by fixed-point sweeps; diis > 1 extrapolates over that many
    sweeps as in the forward march (the solution is unchanged)."""
    (E1, Ee1, W1, We1), (E2, Ee2, W2, We2) = _panel_weights(model, grid)
    m, P = grid.m, grid.P
    z = model.zeros()
    lam = [None] * (m * P)
    lamt = [None] * (m * P)
    a = [None] * (P + 1)
    a[P] = z
    iters = [0] * P
    for p in reversed(range(P)):
        idx = [p * m + x for x in range(m)]
        dE = []
        for x, k in enumerate(idx):
            g = model.vjp(sol.nodes[k], grid.b[x] / P, (None, None))
            dE.append(g)
        l = [(-g[0], -g[1]) for g in dE]
        an = a[p + 1]
        hist_s, hist_r = [], []
        for it in range(1, max_iter + 1):
            lt = []
            for x in range(m):
                t1 = We1[x] * an[0] + sum(W1[y, x] * l[y][0] for y in range(m))
                t2 = We2[x] * an[1] + sum(W2[y, x] * l[y][1] for y in range(m))
                lt.append((t1, t2))
            new = []
            for x, k in enumerate(idx):
                j = model.vjp(sol.nodes[k], None, lt[x])
                new.append((-dE[x][0] - j[0], -dE[x][1] - j[1]))
            change = max(_maxabs((new[x][0] - l[x][0], new[x][1] - l[x][1])) for x in range(m))
            scale = max(1e-300, max(_maxabs(v) for v in new))
            if change <= tol * max(scale, 1e-30) or change == 0.0:
                l = new
                break
            if diis > 1:
                hist_s.append(_flat(l))
                hist_r.append(_flat(new) - hist_s[-1])
                hist_s, hist_r = hist_s[-diis:], hist_r[-diis:]
                new = _unflat(_diis_next(hist_s, hist_r), new) if len(hist_r) > 1 else new
            l = new
        else:
            raise RuntimeError(f"panel {p}: adjoint iteration did not converge")
        iters[p] = it
        lt = []
        for x in range(m):
            t1 = We1[x] * an[0] + sum(W1[y, x] * l[y][0] for y in range(m))
            t2 = We2[x] * an[1] + sum(W2[y, x] * l[y][1] for y in range(m))
            lt.append((t1, t2))
        for x, k in enumerate(idx):
            lam[k], lamt[k] = l[x], lt[x]
        a[p] = (Ee1 * an[0] + sum(E1[x] * l[x][0] for x in range(m)),
                Ee2 * an[1] + sum(E2[x] * l[x][1] for x in range(m)))
    return Adjoint(lam, lamt, a, iters)


def _integral_term(model, grid, sol, adj, dints):
    """sum_x [(g_x/beta) E(s_x; dI) + <lamt_x, S(s_x; dI)>]."""
    tot = 0.0
    m, P = grid.m, grid.P
    for k, s in enumerate(sol.nodes):
        x = k % m
        tot += grid.b[x] / P * model.energy(s, dints)
        tot += _inner(adj.lamt[k], model.residual(s, dints))
    return tot


def d_omega(model, grid, sol, adj, theta, dh=None, deri=None):
    """dOmega/dtheta for theta in {'mu', 'beta', 'h'} (frozen reference).

    theta='h' takes a direction (dh, deri) of the one-body matrix and the
    two-electron integrals (for example deri = eri/U for d/dU).
    """
    ints = model.ints
    dn_mu, dn_beta = model.occ_derivs()
    if theta == "mu":
        dn = dn_mu
        return (model.domega0("mu") + model.domega_mf(dn)
                + _integral_term(model, grid, sol, adj, ints.derivative(dn=dn)))
    if theta == "h":
        d = model.domega_mf(np.zeros_like(dn_mu), dh=dh, deri=deri)
        return d + _integral_term(model, grid, sol, adj, ints.derivative(dh=dh, deri=deri))
    if theta == "beta":
        dn = dn_beta
        tot = (model.domega0("beta") + model.domega_mf(dn)
               + _integral_term(model, grid, sol, adj, ints.derivative(dn=dn)))
        tot += _grid_beta_term(model, grid, sol, adj)
        return tot
    raise ValueError(theta)


def _grid_beta_term(model, grid, sol, adj):
    """Explicit beta dependence of E_x, E_e, W, We through h = beta / P."""
    w1, w2 = _panel_weights(model, grid, deriv=True)
    _, _, _, _, dE1, dEe1, dW1, dWe1 = w1
    _, _, _, _, dE2, dEe2, dW2, dWe2 = w2
    m, P = grid.m, grid.P
    tot = 0.0
    for p in range(P):
        sb = sol.sb[p]
        S = [sol.resid[p * m + y] for y in range(m)]
        for x in range(m):
            lam = adj.lam[p * m + x]
            f1 = -dE1[x] * sb[0] + sum(dW1[x, y] * S[y][0] for y in range(m))
            f2 = -dE2[x] * sb[1] + sum(dW2[x, y] * S[y][1] for y in range(m))
            tot += _inner(lam, (f1, f2))
        an = adj.a[p + 1]
        fe1 = -dEe1 * sb[0] + sum(dWe1[y] * S[y][0] for y in range(m))
        fe2 = -dEe2 * sb[1] + sum(dWe2[y] * S[y][1] for y in range(m))
        tot += _inner(an, (fe1, fe2))
    return tot / P


def d_omega_dh(model, grid, sol, adj):
    """dOmega/dh_pq (matrix) at frozen reference: n_p delta_pq + one-body response density."""
    m, P = grid.m, grid.P
    out = model.dmf_dh()
    for k, s in enumerate(sol.nodes):
        x = k % m
        out = out + model.vjp_fock(s, grid.b[x] / P, adj.lamt[k])
    return out


def _eps_from_delta(model, D1, D2):
    """Chain a cotangent of the orbital-energy differences to the orbital
    energies: Delta_i^a = eps_a - eps_i (t1[i, a]), Delta_ij^ab = eps_a + eps_b -
    eps_i - eps_j (t2[i, j, a, b])."""
    return (D1.sum(0) - D1.sum(1) + D2.sum((0, 1, 3)) + D2.sum((0, 1, 2))
            - D2.sum((1, 2, 3)) - D2.sum((0, 2, 3)))


def d_omega_deps(model, grid, sol, adj):
    """dOmega/deps_q (vector) at frozen h, <pq|rs>, mu, beta, orbitals and
    dropped slots: the response to the reference orbital energies of Section
    II.D (type 2; Appendix B).  eps_q enters
      * Omega_0 and Omega_1, and the occupation n_q (dn_q/deps_q = -beta n_q (1 - n_q)),
        which moves the thermal integrals (weights and Fock operator) -- one
        directional derivative per orbital, as for mu;
      * u = f - diag(eps) explicitly (du = -e_q e_q^T);
      * the propagator weights through Delta (dL/dDelta of the discrete
        Lagrangian, chained to eps by Delta's definition).
    The paper's relaxed diagonal is p^cc_qq = dOmega/deps_q + dOmega/dh_qq."""
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
                  + _integral_term(model, grid, sol, adj, ints.derivative(dn=dn, dh=du)))
    dE1, dEe1, dW1, dWe1 = grid.weights_ddelta(model.delta1)
    dE2, dEe2, dW2, dWe2 = grid.weights_ddelta(model.delta2)
    m, P = grid.m, grid.P
    D1, D2 = model.zeros()
    for p in range(P):
        sb = sol.sb[p]
        S = [sol.resid[p * m + y] for y in range(m)]
        for x in range(m):
            lam = adj.lam[p * m + x]
            D1 = D1 + lam[0] * (-dE1[x] * sb[0] + sum(dW1[x, y] * S[y][0] for y in range(m)))
            D2 = D2 + lam[1] * (-dE2[x] * sb[1] + sum(dW2[x, y] * S[y][1] for y in range(m)))
        an = adj.a[p + 1]
        D1 = D1 + an[0] * (-dEe1 * sb[0] + sum(dWe1[y] * S[y][0] for y in range(m)))
        D2 = D2 + an[1] * (-dEe2 * sb[1] + sum(dWe2[y] * S[y][1] for y in range(m)))
    return out + _eps_from_delta(model, D1, D2)


def two_body_density(d_omega_along, n):
    """Gamma_pqrs = dOmega/d<pq|rs> at a frozen reference, within the integrals
    that keep <pq|rs> = <qp|sr> (Section II.D: the response of Omega to the
    two-electron integrals), by its definition: for every element the derivative
    along the direction that moves <pq|rs> and <qp|sr> by 1/2 each.
    d_omega_along(deri) returns dOmega/dtheta for <pq|rs> + theta deri."""
    out = np.zeros((n,) * 4)
    seen = {}
    for p in range(n):
        for q in range(n):
            for r in range(n):
                for t in range(n):
                    key = min((p, q, r, t), (q, p, t, r))
                    if key not in seen:
                        d = np.zeros((n,) * 4)
                        d[p, q, r, t] += 0.5
                        d[q, p, t, r] += 0.5
                        seen[key] = d_omega_along(d)
                    out[p, q, r, t] = seen[key]
    return out


def find_mu(make_model, grid, n_target, mu0, tol=1e-10, max_iter=40, solve_tol=1e-13):
    """Chemical potential at which the FT-CCSD electron number N = -dOmega/dmu
    (Section II.D) equals n_target, as the paper fixes <N> for the electron gas
    (Section III; the appendix on the UEG basis-set error chooses mu_CC so that
    the coupled-cluster system holds N electrons).

    make_model(mu) builds the model at chemical potential mu (frozen reference:
    orbitals and eps fixed).  Regula falsi with the Illinois modification on
    N(mu) - n_target, after expanding a bracket from mu0 in steps set by the
    mean-field compressibility dN/dmu = 2 sum_p beta n_p (1 - n_p).  Returns
    (mu, N(mu), iterations)."""
    def n_of(mu):
        model = make_model(mu)
        sol = solve(model, grid, tol=solve_tol)
        adj = adjoint(model, grid, sol, tol=solve_tol)
        return -d_omega(model, grid, sol, adj, "mu")

    def mf_slope(mu):
        ints = make_model(mu).ints
        return 2.0 * grid.beta * float(np.sum(ints.n_occ * ints.n_vir))

    scale = max(1.0, abs(n_target))
    a, fa = mu0, n_of(mu0) - n_target
    its = 1
    if abs(fa) <= tol * scale:
        return a, fa + n_target, its
    step = -fa / max(mf_slope(mu0), 1e-12)
    b, fb = a + step, None
    while True:                      # expand until N - n_target changes sign
        fb = n_of(b) - n_target
        its += 1
        if abs(fb) <= tol * scale:
            return b, fb + n_target, its
        if fa * fb < 0:
            break
        a, fa = b, fb
        step *= 2.0
        b = a + step
        if its > max_iter:
            raise RuntimeError("find_mu: no bracket")
    side = 0
    while its < max_iter:
        c = (a * fb - b * fa) / (fb - fa)
        fc = n_of(c) - n_target
        its += 1
        if abs(fc) <= tol * scale:
            return c, fc + n_target, its
        if fc * fb < 0:
            a, fa = b, fb
            b, fb = c, fc
            side = 0
        else:
            b, fb = c, fc
            if side == -1:
                fa *= 0.5
            side = -1
    raise RuntimeError("find_mu: no convergence")
