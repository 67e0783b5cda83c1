"""Degenerate cases and error paths of the library on the GPU: one orbital
(every Delta = 0, the propagator's phi-functions at zero; the atomic limit of
the paper's two-spin-orbital exactness), wrong call orders, bad arguments, a
memory cap too small for the instance, and a cap that forces the lean schedule
(checkpointing, one executor slot) with unchanged results."""
import math

import numpy as np
import pytest

import ftcc_inputs as fi
from oracle import grid as G, restricted as R, rk as K, solver as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_01729_amd import ftcc
    return ftcc


def _model(s):
    return R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, s.mu, s.beta))


@pytest.mark.parametrize("prop", [0, 1, 4])
def test_one_orbital_atomic_limit(F, prop):
    """One site (n = 1): FT-CCSD is exact for two spin orbitals, so Omega tends
    to the closed form -(1/beta) ln(1 + 2 e^{beta mu} + e^{-beta (U - 2 mu)}) as
    the grid is refined; at each grid the GPU equals the oracle."""
    U, beta = 4.0, 1.0
    s = fi.hubbard_config(L=1, t=0.0, U=U, T=1.0 / beta)
    exact = -math.log(1.0 + 2.0 * math.exp(beta * s.mu) + math.exp(-beta * (U - 2.0 * s.mu))) / beta
    print(f"[edge] one orbital, propagator {prop}", flush=True)
    errs = []
    for n_tau in (4, 8):
        opt = dict(n_tau=n_tau, propagator=prop, tol=1e-14)
        if prop < 2:
            opt["nodes_per_panel"] = 4
        ctx = F.Context(1, **opt)
        ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
        ctx.solve(s.mu, s.beta)
        om, _ = ctx.grand_potential()
        ctx.close()
        m = _model(s)
        if prop == 4:
            ref = K.solve(m, s.beta, n_tau, "rk4").omega
        else:
            ref = S.solve(m, G.Grid(s.beta, n_tau // 4, 4, "lawson" if prop == 1 else "etd"), tol=1e-14).omega
        assert abs(om[0] - ref) < 1e-10 * abs(ref)
        errs.append(abs(om[0] - exact))
    assert errs[1] < errs[0] or errs[1] < 1e-12


def test_call_order_and_argument_errors(F):
    s = fi.hubbard_config(L=2, U=1.0, T=1.0)
    with pytest.raises(F.FTCCError):
        F.Context(0)
    for bad in (dict(n_tau=6, nodes_per_panel=4), dict(nodes_per_panel=7, n_tau=7), dict(tol=0.0),
                dict(diis_depth=1), dict(occ_thresh=-1.0), dict(spin_orbital=2)):
        with pytest.raises(F.FTCCError):
            F.Context(1, **bad)
    ctx = F.Context(2, n_tau=4, nodes_per_panel=4)
    with pytest.raises(F.FTCCError):      # no Hamiltonian yet
        ctx.solve([s.mu, s.mu], [s.beta, s.beta])
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    with pytest.raises(F.FTCCError):      # instance 1 still has none
        ctx.solve([s.mu, s.mu], [s.beta, s.beta])
    with pytest.raises(F.FTCCError):      # index out of range
        ctx.set_hamiltonian(2, s.h, s.eri, s.eps)
    h = s.h.copy()
    h[0, 0] = np.nan
    with pytest.raises(F.FTCCError):      # non-finite input
        ctx.set_hamiltonian(1, h, s.eri, s.eps)
    ctx.set_hamiltonian(1, s.h, s.eri, s.eps)
    with pytest.raises(F.FTCCError):      # adjoint before the march
        ctx.lam()
    with pytest.raises(F.FTCCError):      # non-positive beta
        ctx.solve([s.mu, s.mu], [s.beta, -1.0])
    ctx.solve([s.mu, s.mu], [s.beta, s.beta])
    with pytest.raises(F.FTCCError):      # response before the adjoint
        ctx.response()
    with pytest.raises(F.FTCCError):
        ctx.two_body_density()
    with pytest.raises(F.FTCCError):      # node out of range
        ctx.amplitudes(0, 4)
    ctx.lam()
    r = ctx.response(want_mu=True, want_beta=False, want_h=False)
    assert np.isfinite(r["mu"]).all()
    ctx.close()


def test_memory_cap(F):
    """A cap below the integral blocks fails cleanly with FTCC_ENOMEM; a cap that
    leaves room for the integrals but not for the stored tau grid (96 nodes of
    the 19-PW gas, 201 MB) switches on checkpointing and the one-slot schedule,
    with the same results."""
    s = fi.ueg_config(19, 14, 1.0, 0.5)
    print("[edge] ueg19 memory caps", flush=True)
    ctx = F.Context(1, n_tau=8, nodes_per_panel=4, mem_cap_bytes=4 << 20)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    with pytest.raises(F.FTCCError) as e:
        ctx.solve(s.mu, s.beta)
    assert e.value.code == F.ENOMEM
    ctx.close()
    out = []
    for cap in (0, 350 << 20):
        ctx = F.Context(1, n_tau=96, nodes_per_panel=4, tol=1e-13, mem_cap_bytes=cap)
        ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
        ctx.solve(s.mu, s.beta)
        om, _ = ctx.grand_potential()
        ctx.lam()
        r = ctx.response(want_mu=True, want_beta=True, want_h=False)
        out.append((om[0], r["mu"][0], r["beta"][0]))
        ctx.close()
    for a, b in zip(out[0], out[1]):
        assert abs(a - b) < 1e-11 * max(1.0, abs(a))
