"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every case prints its name, shape and seed before touching the GPU.
Tolerances: kernels and Omega 1e-12 relative (both sides FP64, different
summation order); converged amplitudes and Omega_CC to 1e-10 relative and
1e-8 * max(1, |x|) as the workload specification requires.
"""
import sys

import numpy as np
import pytest

import ftcc_inputs as fi
from oracle import grid as G, restricted as R, solver as S

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


def _oracle(h, eri, eps, mu, beta, thr=0.0):
    return R.RestrictedModel(R.RestrictedIntegrals(h, eri, eps, mu, beta, thr))


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("case", ["random7", "random13", "ueg19"])
def test_residual_kernels(ftcc, case):
    if case.startswith("random"):
        n = int(case[6:])
        h, eri, eps = fi.random_hamiltonian(n, seed=3)
        mu, beta = 0.1, 1.3
    else:
        s = fi.ueg_config(19, 14, 1.0, 0.5)
        n, h, eri, eps, mu, beta = s.n, s.h, s.eri, s.eps, s.mu, s.beta
    t1, t2 = fi.random_amplitudes(n, seed=5, scale=0.2)
    _say(f"[residual] case={case} n={n} seed=5")
    ctx = ftcc.Context(1, n_tau=4, nodes_per_panel=4)
    ctx.set_hamiltonian(0, h, eri, eps)
    S1, S2, E = ctx.eval_residual(0, mu, beta, t1, t2)
    ctx.close()
    m = _oracle(h, eri, eps, mu, beta)
    R1, R2 = m.residual((t1, t2))
    Er = m.energy((t1, t2))
    assert _rel(S1, R1) < 1e-12
    assert _rel(S2, R2) < 1e-12
    assert abs(E - Er) < 1e-12 * max(1.0, abs(Er))


@pytest.mark.parametrize("kind", [0, 1])
def test_forward_hubbard6(ftcc, kind):
    """Config: 6-site ring, U = 4, mu = U/2, T = 1, 20 tau points (5 panels x 4)."""
    s = fi.hubbard_config(L=6, U=4.0, T=1.0)
    _say(f"[forward] hubbard L=6 U=4 T=1 n_tau=20 propagator={kind}")
    ctx = ftcc.Context(1, n_tau=20, nodes_per_panel=4, propagator=kind, tol=1e-13)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    its, st = ctx.solve(s.mu, s.beta)
    om, parts = ctx.grand_potential()
    nodes = [ctx.amplitudes(0, k) for k in range(20)]
    ctx.close()
    model = _oracle(s.h, s.eri, s.eps, s.mu, s.beta)
    sol = S.solve(model, G.Grid(s.beta, 5, 4, "etd" if kind == 0 else "lawson"), tol=1e-13)
    assert abs(parts[0, 0] - sol.omega0) < 1e-12 * abs(sol.omega0)
    assert abs(parts[0, 1] - sol.omega1) < 1e-12 * max(1.0, abs(sol.omega1))
    assert abs(parts[0, 2] - sol.omega_cc) < 1e-10 * abs(sol.omega_cc)
    assert abs(om[0] - sol.omega) < 1e-10 * abs(sol.omega)
    for k in range(20):                       # every node of every panel
        assert _rel(nodes[k][0], sol.nodes[k][0]) < 1e-8
        assert _rel(nodes[k][1], sol.nodes[k][1]) < 1e-8


def test_adjoint_and_response_small(ftcc):
    """3-site ring with a perturbed h: Lambda, dOmega/dmu, dbeta, dU, dh."""
    s = fi.hubbard_config(L=3, U=2.0, T=1.0)
    rng = np.random.default_rng(1)
    dh = rng.standard_normal((3, 3)) * 0.05
    h = s.h + dh + dh.T
    _say("[adjoint] hubbard L=3 U=2 T=1 n_tau=12 seed=1")
    ctx = ftcc.Context(1, n_tau=12, nodes_per_panel=4, tol=1e-14)
    ctx.set_hamiltonian(0, h, s.eri, s.eps)
    ctx.solve(s.mu, s.beta)
    ctx.lam()
    lam = ctx.get_lambda(0, 5)
    res = ctx.response(deri_dtheta=[s.eri / 2.0])
    ctx.close()
    model = _oracle(h, s.eri, s.eps, s.mu, s.beta)
    gr = G.Grid(s.beta, 3, 4)
    sol = S.solve(model, gr, tol=1e-14)
    adj = S.adjoint(model, gr, sol, tol=1e-14)

    def sym(x):
        return 0.5 * (x + x.transpose(1, 0, 3, 2))
    assert _rel(lam[0], adj.lam[5][0]) < 1e-8
    assert _rel(sym(lam[1]), sym(adj.lam[5][1])) < 1e-8
    for key, theta, kw in (("mu", "mu", {}), ("beta", "beta", {}), ("theta", "h", dict(deri=s.eri / 2.0))):
        ref = S.d_omega(model, gr, sol, adj, theta, **kw)
        assert abs(res[key][0] - ref) < 1e-8 * max(1.0, abs(ref)), key
    ref_h = S.d_omega_dh(model, gr, sol, adj)
    assert _rel(res["h"][0], ref_h) < 1e-8


def test_forward_and_adjoint_with_diis(ftcc):
    """DIIS changes the iteration, not the fixed point: Omega and dOmega/dmu as the
    plain oracle march."""
    s = fi.hubbard_config(L=4, U=4.0, T=1.0)
    _say("[diis] hubbard L=4 U=4 T=1 n_tau=8 diis_depth=6")
    ctx = ftcc.Context(1, n_tau=8, nodes_per_panel=4, tol=1e-13, diis_depth=6)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    ctx.solve(s.mu, s.beta)
    om, _ = ctx.grand_potential()
    ctx.lam()
    r = ctx.response(want_mu=True, want_beta=False, want_h=False)
    ctx.close()
    model = _oracle(s.h, s.eri, s.eps, s.mu, s.beta)
    gr = G.Grid(s.beta, 2, 4)
    sol = S.solve(model, gr, tol=1e-13)
    adj = S.adjoint(model, gr, sol, tol=1e-13)
    assert abs(om[0] - sol.omega) < 1e-10 * abs(sol.omega)
    ref = S.d_omega(model, gr, sol, adj, "mu")
    assert abs(r["mu"][0] - ref) < 1e-8 * max(1.0, abs(ref))
