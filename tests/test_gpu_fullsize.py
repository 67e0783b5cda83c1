"""Parity at the full 57-plane-wave UEG shape (n = 57, N = 14, r_s = 1, Theta = 0.5).

The oracle cannot march 16 nodes at this size in a test, so:
  * one residual evaluation (E, S1, S2) is compared element by element;
  * the GPU's converged amplitudes of the first panel must satisfy the oracle's
    own discrete equations s_x = -sum_y W_xy S(s_y) (s_b = 0) with the oracle's
    quadrature weights and the oracle's kernels;
  * dOmega/dmu from the adjoint agrees with central differences of the GPU Omega.
"""
import numpy as np
import pytest

import ftcc_inputs as fi
from oracle import grid as G, restricted as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_01729_amd import ftcc
    s = fi.ueg_config(57, 14, 1.0, 0.5)
    model = R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, s.mu, s.beta))
    return ftcc, s, model


def test_residual_n57(setup):
    F, s, model = setup
    print("[fullsize] residual n=57 seed=5", flush=True)
    t1, t2 = fi.random_amplitudes(s.n, seed=5, scale=0.02)
    ctx = F.Context(1, n_tau=16, nodes_per_panel=4)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    S1, S2, E = ctx.eval_residual(0, s.mu, s.beta, t1, t2)
    ctx.close()
    R1, R2 = model.residual((t1, t2))
    Er = model.energy((t1, t2))
    assert np.abs(S1 - R1).max() < 1e-12 * max(1.0, np.abs(R1).max())
    assert np.abs(S2 - R2).max() < 1e-12 * max(1.0, np.abs(R2).max())
    assert abs(E - Er) < 1e-12 * max(1.0, abs(Er))


def test_converged_first_panel_is_oracle_fixed_point(setup):
    F, s, model = setup
    print("[fullsize] forward n=57 n_tau=16, first panel against oracle equations", flush=True)
    ctx = F.Context(1, n_tau=16, nodes_per_panel=4, tol=1e-13)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    ctx.solve(s.mu, s.beta)
    nodes = [ctx.amplitudes(0, x) for x in range(4)]
    ctx.close()
    gr = G.Grid(s.beta, 4, 4)
    _, _, W1, _ = gr.weights(model.delta1)
    _, _, W2, _ = gr.weights(model.delta2)
    S = [model.residual(nd) for nd in nodes]
    scale = max(1.0, max(np.abs(nd[1]).max() for nd in nodes))
    for x in range(4):
        r1 = -sum(W1[x, y] * S[y][0] for y in range(4))
        r2 = -sum(W2[x, y] * S[y][1] for y in range(4))
        assert np.abs(r1 - nodes[x][0]).max() < 1e-10 * scale
        assert np.abs(r2 - nodes[x][1]).max() < 1e-10 * scale


def test_dmu_against_finite_difference_n57(setup):
    F, s, _ = setup
    print("[fullsize] dOmega/dmu adjoint vs central FD, n=57", flush=True)
    ctx = F.Context(1, n_tau=16, nodes_per_panel=4, tol=1e-13)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    ctx.solve(s.mu, s.beta)
    ctx.lam()
    d = ctx.response(want_mu=True, want_beta=False, want_h=False)["mu"][0]
    h = 1e-4
    vals = []
    for mu in (s.mu + h, s.mu - h, s.mu + h / 2, s.mu - h / 2):
        ctx.solve(mu, s.beta)
        vals.append(ctx.grand_potential()[0][0])
    ctx.close()
    fd1 = (vals[0] - vals[1]) / (2 * h)
    fd2 = (vals[2] - vals[3]) / h
    fd = (4 * fd2 - fd1) / 3
    assert abs(d - fd) < 1e-8 * max(1.0, abs(d))
