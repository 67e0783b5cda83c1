"""GPU parity of the orbital-energy response dOmega/deps_q (Section II.D type 2,
Appendix B) through ftcc_response's dO_deps, against the oracle's
d_omega_deps (which Richardson differences of the re-solved Omega pin):

  * a 3-site ring with a perturbed h and orbital energies that are not the Fock
    diagonal, for the exponential-collocation and integrating-factor integral
    forms and the RK4 differential form;
  * a batch of two rings of different size (3 and 4 sites) in one context;
  * the same ring in spin orbitals (spin_orbital = 1);
  * the 19-plane-wave gas, momentum-blocked against dense, with the trace
    identity sum_q (dOmega/deps_q + dOmega/dh_qq) = -dOmega/dmu.
"""
import sys

import numpy as np
import pytest

import ftcc_inputs as fi
from oracle import grid as G, restricted as R, rk as K, solver as S, spinorb as so

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ftcc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_01729_amd import ftcc as F
    return F


def _ring(L, seed):
    s = fi.hubbard_config(L=L, U=2.0, T=1.0)
    rng = np.random.default_rng(seed)
    dh = rng.standard_normal((L, L)) * 0.05
    return s.h + dh + dh.T, s.eri, s.eps + rng.uniform(-0.1, 0.1, L), s.mu, s.beta


def _oracle_deps(h, eri, eps, mu, beta, form, n_tau):
    model = R.RestrictedModel(R.RestrictedIntegrals(h, eri, eps, mu, beta))
    if form == 4:
        sol = K.solve(model, beta, n_tau, "rk4")
        return K.d_omega_deps(model, sol, K.adjoint(model, sol))
    gr = G.Grid(beta, n_tau // 4, 4, "etd" if form == 0 else "lawson")
    sol = S.solve(model, gr, tol=1e-14)
    return S.d_omega_deps(model, gr, sol, S.adjoint(model, gr, sol, tol=1e-14))


@pytest.mark.parametrize("form", [0, 1, 4])
def test_deps_ring_against_oracle(ftcc, form):
    h, eri, eps, mu, beta = _ring(3, 7)
    _say(f"[deps] ring L=3 seed=7 propagator={form}")
    ctx = ftcc.Context(1, n_tau=8, nodes_per_panel=4, propagator=form, tol=1e-14)
    ctx.set_hamiltonian(0, h, eri, eps)
    ctx.solve(mu, beta)
    ctx.lam()
    r = ctx.response(want_eps=True)
    ctx.close()
    ref = _oracle_deps(h, eri, eps, mu, beta, form, 8)
    assert np.abs(r["eps"][0] - ref).max() < 1e-8 * max(1.0, np.abs(ref).max())
    # the relaxed density's trace is the electron number
    assert abs(np.sum(r["eps"][0] + np.diag(r["h"][0])) + r["mu"][0]) < 1e-9 * abs(r["mu"][0])


def test_deps_batch_of_two_sizes(ftcc):
    cases = [_ring(3, 7), _ring(4, 9)]
    _say("[deps] batch rings L=3 seed=7, L=4 seed=9")
    ctx = ftcc.Context(2, n_tau=8, nodes_per_panel=4, tol=1e-14)
    for i, (h, eri, eps, _, _) in enumerate(cases):
        ctx.set_hamiltonian(i, h, eri, eps)
    ctx.solve([c[3] for c in cases], [c[4] for c in cases])
    ctx.lam()
    r = ctx.response(want_eps=True, want_h=False)
    ctx.close()
    for i, (h, eri, eps, mu, beta) in enumerate(cases):
        ref = _oracle_deps(h, eri, eps, mu, beta, 0, 8)
        assert r["eps"][i].shape == ref.shape
        assert np.abs(r["eps"][i] - ref).max() < 1e-8 * max(1.0, np.abs(ref).max())


def test_deps_spin_orbital(ftcc):
    h, eri, eps, mu, beta = _ring(3, 7)
    H, ERI, EPS = so.spin_orbital_from_spatial(h, eri, eps)
    EPS = EPS + np.array([0.02, -0.03, 0.01, -0.01, 0.03, 0.0])   # spin-dependent reference energies
    _say("[deps] spin orbitals ring L=3 seed=7")
    ctx = ftcc.Context(1, n_tau=8, nodes_per_panel=4, tol=1e-14, spin_orbital=1)
    ctx.set_hamiltonian(0, H, ERI, EPS)
    ctx.solve(mu, beta)
    ctx.lam()
    r = ctx.response(want_eps=True, want_h=False)
    ctx.close()
    model = so.SpinOrbitalModel(so.ThermalIntegrals(H, ERI, EPS, mu, beta))
    gr = G.Grid(beta, 2, 4)
    sol = S.solve(model, gr, tol=1e-14)
    ref = S.d_omega_deps(model, gr, sol, S.adjoint(model, gr, sol, tol=1e-14))
    assert np.abs(r["eps"][0] - ref).max() < 1e-8 * max(1.0, np.abs(ref).max())


def test_deps_momentum_blocked_equals_dense(ftcc):
    s = fi.ueg_config(19, 14, 1.0, 0.5)
    out = []
    for blocked in (False, True):
        _say(f"[deps] ueg 19 PW n_tau=8 blocked={blocked}")
        ctx = ftcc.Context(1, n_tau=8, nodes_per_panel=4, tol=1e-13)
        if blocked:
            ctx.set_momentum(0, *s.momentum)
        ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
        ctx.solve(s.mu, s.beta)
        ctx.lam()
        out.append(ctx.response(want_eps=True))
        ctx.close()
    d, b = out
    assert np.abs(d["eps"][0] - b["eps"][0]).max() < 1e-10 * max(1.0, np.abs(d["eps"][0]).max())
    for r in out:
        assert abs(np.sum(r["eps"][0] + np.diag(r["h"][0])) + r["mu"][0]) < 1e-10 * abs(r["mu"][0])
