"""Two-body response density (ftcc_two_body_density: Gamma = dOmega/d<pq|rs>
within the integrals keeping <pq|rs> = <qp|sr>) on the GPU against the oracle's
element-by-element definition (integral and differential forms, restricted and
spin-orbital), against the directional response, and momentum-blocked against
dense."""
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


def _generic_ring():
    s = fi.hubbard_config(L=3, U=2.0, T=1.0)
    rng = np.random.default_rng(5)
    c = rng.standard_normal((3,) * 4) * 0.05
    return fi.System("ring3_generic", s.h, s.eri + c + c.transpose(1, 0, 3, 2), s.eps, s.mu, s.beta)


def _gpu_gamma(F, s, momentum=False, **opt):
    ctx = F.Context(1, **opt)
    if momentum:
        ctx.set_momentum(0, *s.momentum)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    ctx.solve(s.mu, s.beta)
    ctx.lam()
    gam = ctx.two_body_density()[0]
    ctx.close()
    return gam


@pytest.mark.parametrize("form", ["collocation", "rk4"])
def test_density_matches_oracle_restricted(F, form):
    s = _generic_ring()
    m = R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, s.mu, s.beta))
    print(f"[density] generic ring n=3 {form}", flush=True)
    if form == "rk4":
        gam = _gpu_gamma(F, s, n_tau=6, propagator=4)
        sol = K.solve(m, s.beta, 6, "rk4")
        adj = K.adjoint(m, sol)
        ref = S.two_body_density(lambda d: K.d_omega(m, sol, adj, "h", deri=d), 3)
    else:
        gam = _gpu_gamma(F, s, n_tau=8, nodes_per_panel=4, tol=1e-14)
        gr = G.Grid(s.beta, 2, 4)
        sol = S.solve(m, gr, tol=1e-14)
        adj = S.adjoint(m, gr, sol, tol=1e-14)
        ref = S.two_body_density(lambda d: S.d_omega(m, gr, sol, adj, "h", deri=d), 3)
    assert np.abs(gam - ref).max() < 1e-8 * max(1.0, np.abs(ref).max())


def test_density_matches_oracle_spin_orbital(F):
    s = fi.hubbard_unrestricted(L=2, U=3.0, T=1.0, reference="neel")
    print("[density] neel L=2 spin orbitals", flush=True)
    gam = _gpu_gamma(F, s, n_tau=8, nodes_per_panel=4, tol=1e-14, spin_orbital=1)
    m = so.SpinOrbitalModel(so.ThermalIntegrals(s.h, s.eri, s.eps, s.mu, s.beta))
    gr = G.Grid(s.beta, 2, 4)
    sol = S.solve(m, gr, tol=1e-14)
    adj = S.adjoint(m, gr, sol, tol=1e-14)
    ref = S.two_body_density(lambda d: S.d_omega(m, gr, sol, adj, "h", deri=d), s.n)
    assert np.abs(gam - ref).max() < 1e-8 * max(1.0, np.abs(ref).max())


def test_density_contracts_to_directional_response_ueg(F):
    """19-PW electron gas, momentum-blocked: sum Gamma * <pq|rs> equals
    dOmega/dlambda for <pq|rs> -> lambda <pq|rs> from ftcc_response."""
    s = fi.ueg_config(19, 14, 1.0, 0.5)
    print("[density] ueg19 momentum-blocked: <Gamma, eri> vs response", flush=True)
    ctx = F.Context(1, n_tau=8, nodes_per_panel=4, tol=1e-13)
    ctx.set_momentum(0, *s.momentum)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    ctx.solve(s.mu, s.beta)
    ctx.lam()
    r = ctx.response(want_mu=False, want_beta=False, want_h=False, deri_dtheta=[s.eri])
    gam = ctx.two_body_density()[0]
    ctx.close()
    ref = r["theta"][0]
    assert abs(np.sum(gam * s.eri) - ref) < 1e-9 * max(1.0, abs(ref))


def test_density_blocked_equals_dense(F):
    s = fi.hubbard_config(L=6, U=4.0, T=1.0)
    print("[density] hubbard L=6 blocked vs dense", flush=True)
    a = _gpu_gamma(F, s, momentum=False, n_tau=8, nodes_per_panel=4, tol=1e-14)
    b = _gpu_gamma(F, s, momentum=True, n_tau=8, nodes_per_panel=4, tol=1e-14)
    assert np.abs(a - b).max() < 1e-10 * max(1.0, np.abs(a).max())
    lab = np.arange(6)
    forbidden = (lab[:, None, None, None] + lab[None, :, None, None] - lab[None, None, :, None]
                 - lab[None, None, None, :]) % 6 != 0
    assert np.abs(b[forbidden]).max() < 1e-12
