"""Unrestricted references (spin_orbital = 1; Section IV.A's Neel-state and UHF
references of the Hubbard ring) on the GPU against the spin-orbital FP64
oracle: the residual kernels element by element, the march, Lambda and the
response derivatives, the staggered magnetisation of the one-particle response
density, and the restricted path on the same closed-shell system."""
import numpy as np
import pytest

import ftcc_inputs as fi
from oracle import grid as G, restricted as R, rk as K, solver as S, spinorb as so

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_01729_amd import ftcc
    return ftcc


def _so_model(s):
    return so.SpinOrbitalModel(so.ThermalIntegrals(s.h, s.eri, s.eps, s.mu, s.beta))


def _ctx(F, systems, spin_blocks=False, **opt):
    ctx = F.Context(len(systems), spin_orbital=1, **opt)
    for i, s in enumerate(systems):
        if spin_blocks:
            ctx.set_momentum(i, *s.momentum)
        ctx.set_hamiltonian(i, s.h, s.eri, s.eps)
    return ctx


def _staggered(dO_dh, s):
    """m_s = (1/L) sum_i (-1)^i (n_i,up - n_i,down) with n = diag(C gamma C^T),
    gamma = dOmega/dh in the reference orbitals (frozen orbitals, Section II.D)."""
    L, C = s.meta["L"], s.meta["C"]
    d = np.diag(C @ dO_dh @ C.T)
    sign = np.array([(-1.0) ** i for i in range(L)])
    return float(sign @ (d[:L] - d[L:])) / L


@pytest.mark.parametrize("ref,L", [("uhf", 4), ("neel", 6)])
def test_spin_orbital_residual_matches_oracle(F, ref, L):
    s = fi.hubbard_unrestricted(L=L, U=4.0, T=1.0, reference=ref)
    t1, t2 = fi.antisymmetric_amplitudes(s.n, seed=7, scale=0.1)
    print(f"[unrestricted] residual {ref} L={L} N={s.n} seed=7", flush=True)
    ctx = _ctx(F, [s], n_tau=4, nodes_per_panel=4)
    S1, S2, E = ctx.eval_residual(0, s.mu, s.beta, t1, t2)
    ctx.close()
    m = _so_model(s)
    R1, R2 = m.residual((t1, t2))
    Er = m.energy((t1, t2))
    assert np.abs(S1 - R1).max() < 1e-12 * max(1.0, np.abs(R1).max())
    assert np.abs(S2 - R2).max() < 1e-12 * max(1.0, np.abs(R2).max())
    assert abs(E - Er) < 1e-12 * max(1.0, abs(Er))


@pytest.mark.parametrize("spin_blocks", [False, True])
def test_neel_forward_adjoint_response(F, spin_blocks):
    s = fi.hubbard_unrestricted(L=4, U=4.0, T=1.0, reference="neel")
    print(f"[unrestricted] neel L=4 U=4 T=1 n_tau=8 spin_blocks={spin_blocks}", flush=True)
    ctx = _ctx(F, [s], spin_blocks=spin_blocks, n_tau=8, nodes_per_panel=4, tol=1e-14)
    ctx.solve(s.mu, s.beta)
    om, parts = ctx.grand_potential()
    t_node = ctx.amplitudes(0, 5)
    ctx.lam()
    U = s.meta["U"]
    r = ctx.response(want_mu=True, want_beta=True, want_h=True, deri_dtheta=[s.eri / U])
    ctx.close()
    model = _so_model(s)
    gr = G.Grid(s.beta, 2, 4)
    sol = S.solve(model, gr, tol=1e-14)
    adj = S.adjoint(model, gr, sol, tol=1e-14)
    assert abs(parts[0, 2] - sol.omega_cc) < 1e-10 * abs(sol.omega_cc)
    assert abs(om[0] - sol.omega) < 1e-10 * abs(sol.omega)
    for got, ref in zip(t_node, sol.nodes[5]):
        assert np.abs(got - ref).max() < 1e-8 * max(1.0, np.abs(ref).max())
    for key, theta, kw in (("mu", "mu", {}), ("beta", "beta", {}), ("theta", "h", dict(deri=s.eri / U))):
        ref = S.d_omega(model, gr, sol, adj, theta, **kw)
        assert abs(r[key][0] - ref) < 1e-8 * max(1.0, abs(ref)), key
    gh = S.d_omega_dh(model, gr, sol, adj)
    assert np.abs(r["h"][0] - gh).max() < 1e-8
    assert abs(_staggered(r["h"][0], s) - _staggered(gh, s)) < 1e-8


def test_uhf_staggered_magnetisation_against_field_derivative(F):
    """m_s from the response density equals the derivative of Omega with respect
    to a staggered field h_iσ += x (-1)^i (+1 up, -1 down) / L at frozen
    orbitals (Richardson central differences of the GPU's own Omega)."""
    s = fi.hubbard_unrestricted(L=6, U=4.0, T=0.5, reference="uhf")
    L, C = s.meta["L"], s.meta["C"]
    field = np.diag(np.concatenate([[(-1.0) ** i for i in range(L)], [-(-1.0) ** i for i in range(L)]])) / L
    dh = C.T @ field @ C
    print("[unrestricted] uhf L=6 U=4 T=0.5: staggered magnetisation", flush=True)
    ctx = _ctx(F, [s], spin_blocks=True, n_tau=12, nodes_per_panel=4, tol=1e-13)

    def omega(x):
        ctx.set_hamiltonian(0, s.h + x * dh, s.eri, s.eps)
        ctx.solve(s.mu, s.beta)
        return ctx.grand_potential()[0][0]

    d = 1e-4
    fd1 = (omega(d) - omega(-d)) / (2 * d)
    fd2 = (omega(d / 2) - omega(-d / 2)) / d
    fd = (4 * fd2 - fd1) / 3
    omega(0.0)
    ctx.lam()
    r = ctx.response(want_mu=False, want_beta=False, want_h=True)
    ctx.close()
    ms = _staggered(r["h"][0], s)
    assert abs(ms - fd) < 1e-7 * max(1.0, abs(fd))
    assert 0.05 < abs(ms) < 1.0      # broken spin symmetry survives (Section IV.A)


def test_spin_orbital_equals_restricted_on_closed_shell(F):
    """The restricted ring written in spin orbitals: the same Omega, dOmega/dmu
    and the spin-summed dOmega/dh as the restricted path."""
    s = fi.hubbard_config(L=4, U=2.0, T=1.0)
    h, eri, eps = so.spin_orbital_from_spatial(s.h, s.eri, s.eps)
    print("[unrestricted] restricted ring L=4 in spin orbitals vs restricted", flush=True)
    a = F.Context(1, n_tau=8, nodes_per_panel=4, tol=1e-14)
    a.set_hamiltonian(0, s.h, s.eri, s.eps)
    a.solve(s.mu, s.beta)
    oa, _ = a.grand_potential()
    a.lam()
    ra = a.response(want_mu=True, want_beta=True, want_h=True)
    a.close()
    b = F.Context(1, n_tau=8, nodes_per_panel=4, tol=1e-14, spin_orbital=1)
    b.set_hamiltonian(0, h, eri, eps)
    b.solve(s.mu, s.beta)
    ob, _ = b.grand_potential()
    b.lam()
    rb = b.response(want_mu=True, want_beta=True, want_h=True)
    b.close()
    n = s.n
    assert abs(oa[0] - ob[0]) < 1e-10 * abs(oa[0])
    for k in ("mu", "beta"):
        assert abs(ra[k][0] - rb[k][0]) < 1e-8 * max(1.0, abs(ra[k][0]))
    ghb = rb["h"][0]
    assert np.abs(ra["h"][0] - (ghb[:n, :n] + ghb[n:, n:])).max() < 1e-8


def test_spin_orbital_rk4_matches_oracle(F):
    s = fi.hubbard_unrestricted(L=4, U=2.0, T=1.0, reference="uhf")
    print("[unrestricted] uhf L=4 rk4 n_g=4", flush=True)
    ctx = _ctx(F, [s], spin_blocks=True, n_tau=4, propagator=4)
    ctx.solve(s.mu, s.beta)
    om, _ = ctx.grand_potential()
    ctx.lam()
    r = ctx.response(want_mu=True, want_beta=True, want_h=False)
    ctx.close()
    model = _so_model(s)
    sol = K.solve(model, s.beta, 4, "rk4")
    adj = K.adjoint(model, sol)
    assert abs(om[0] - sol.omega) < 1e-10 * abs(sol.omega)
    for key in ("mu", "beta"):
        ref = K.d_omega(model, sol, adj, key)
        assert abs(r[key][0] - ref) < 1e-8 * max(1.0, abs(ref)), key
