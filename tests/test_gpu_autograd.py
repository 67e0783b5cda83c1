"""The torch.autograd.Function over the C ABI: Omega and its gradients with
respect to mu, beta and h (a batch of two instances of different sizes) against
the oracle's discrete adjoint, with torch's caching allocator supplying the
device memory and torch's current stream carrying the work."""
import numpy as np
import pytest

import ftcc_inputs as fi
from oracle import grid as G, restricted as R, solver as S

pytestmark = pytest.mark.gpu


def _systems():
    a = fi.hubbard_config(L=4, U=2.0, T=1.0)
    b = fi.hubbard_config(L=3, U=1.5, T=0.8)
    rng = np.random.default_rng(7)
    d = rng.standard_normal((3, 3)) * 0.05
    return [(a.h, a.eri, a.eps, a.mu, a.beta), (b.h + d + d.T, b.eri, b.eps, b.mu, b.beta)]


def _oracle(h, eri, eps, mu, beta):
    model = R.RestrictedModel(R.RestrictedIntegrals(h, eri, eps, mu, beta))
    gr = G.Grid(beta, 2, 4)
    sol = S.solve(model, gr, tol=1e-14)
    adj = S.adjoint(model, gr, sol, tol=1e-14)
    return (sol.omega, S.d_omega(model, gr, sol, adj, "mu"), S.d_omega(model, gr, sol, adj, "beta"),
            S.d_omega_dh(model, gr, sol, adj))


def test_omega_function_gradients():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_01729_amd import autograd as A
    sys_ = _systems()
    print("[autograd] hubbard L=4 + L=3 (perturbed h), n_tau=8, torch allocator", flush=True)
    dev = torch.device("cuda", 0)
    solver = A.OmegaSolver([s[1] for s in sys_], [s[2] for s in sys_], device=dev, n_tau=8, nodes_per_panel=4,
                           tol=1e-14)
    nmax = 4
    h = torch.zeros(2, nmax, nmax, dtype=torch.float64)
    for i, s in enumerate(sys_):
        n = s[0].shape[0]
        h[i, :n, :n] = torch.from_numpy(s[0])
    h = h.to(dev).requires_grad_(True)
    mu = torch.tensor([s[3] for s in sys_], dtype=torch.float64, device=dev, requires_grad=True)
    beta = torch.tensor([s[4] for s in sys_], dtype=torch.float64, device=dev, requires_grad=True)
    w = torch.tensor([1.0, -0.5], dtype=torch.float64, device=dev)
    om = A.omega(mu, beta, h, solver)
    # a second forward at another mu before the backward: the backward restores its own state
    A.omega(mu.detach() + 0.1, beta.detach(), h.detach(), solver)
    (w * om).sum().backward()
    refs = [_oracle(*s) for s in sys_]
    for i, (o, dmu, dbeta, dh) in enumerate(refs):
        n = sys_[i][0].shape[0]
        assert abs(om[i].item() - o) < 1e-10 * abs(o)
        wi = w[i].item()
        assert abs(mu.grad[i].item() - wi * dmu) < 1e-8 * max(1.0, abs(dmu))
        assert abs(beta.grad[i].item() - wi * dbeta) < 1e-8 * max(1.0, abs(dbeta))
        gh = h.grad[i].cpu().numpy()
        assert np.abs(gh[:n, :n] - wi * dh).max() < 1e-8
        assert np.all(gh[n:, :] == 0) and np.all(gh[:, n:] == 0)
    solver.close()
