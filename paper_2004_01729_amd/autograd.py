"""Omega as a differentiable torch function of (mu, beta, h).

`FTCCOmega.apply(mu, beta, h, solver)` returns the FT-CCSD grand potential of
every instance (Section II.B: Omega = Omega_0 + Omega_1 + Omega_CC); its
backward runs the Lambda adjoint swept backward in tau and the response step
(Section II.D, Appendix B) and returns grad * dOmega/dmu, grad * dOmega/dbeta
and grad * dOmega/dh_pq at a frozen reference (orbitals, eps and the dropped
slots fixed).  -dOmega/dmu is the electron number, beta^2 dOmega/dbeta the
entropy, dOmega/dh_pq the one-particle response density.

All arithmetic runs in libftcc.so through the C ABI.  Torch supplies the HIP
stream (the current stream of the instances' device) and, optionally, the
device memory (its caching allocator, installed with ftcc_set_allocator).
There is no CPU path: CPU tensors are an error, as is a missing library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ftcc as _ftcc


class OmegaSolver:
    """One native context for a fixed batch of instances.

    eri[i] (n_i^4) and eps[i] (n_i) are fixed per instance; h (and mu, beta)
    are the differentiable inputs of FTCCOmega.  Options are those of
    ftcc_options (n_tau, nodes_per_panel, propagator, occ_thresh, tol,
    max_iter, checkpoint, diis_depth, mem_cap_bytes)."""

    def __init__(self, eri, eps, device=None, torch_memory=True, **options):
        if len(eri) != len(eps) or not eri:
            raise ValueError("eri and eps need one entry per instance")
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.type != "cuda":
            raise ValueError("FT-CCSD runs on a HIP device only")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.eri = [np.ascontiguousarray(np.asarray(e, dtype=np.float64)) for e in eri]
        self.eps = [np.ascontiguousarray(np.asarray(e, dtype=np.float64)) for e in eps]
        self.sizes = [e.shape[0] for e in self.eps]
        for n, e in zip(self.sizes, self.eri):
            if e.shape != (n,) * 4:
                raise ValueError("eri[i] must be n_i^4 with n_i = len(eps[i])")
        self.B = len(self.eps)
        self.ctx = _ftcc.Context(self.B, device=self.device.index, **options)
        if torch_memory:
            dev = self.device

            def alloc(nbytes):
                return torch.cuda.caching_allocator_alloc(nbytes, dev, torch.cuda.current_stream(dev))

            def free(ptr):
                torch.cuda.caching_allocator_delete(ptr)
            self.ctx.set_allocator(alloc, free)
        self._h = [None] * self.B
        self.generation = 0          # bumped by every solve: a backward checks it still owns the state

    def close(self):
        self.ctx.close()

    def _bind_stream(self):
        self.ctx.set_stream(torch.cuda.current_stream(self.device).cuda_stream)

    def _solve(self, mu, beta, h):
        """Set changed Hamiltonians, march forward, return Omega (numpy [B])."""
        self._bind_stream()
        for i in range(self.B):
            n = self.sizes[i]
            hi = h[i, :n, :n]
            if self._h[i] is None or not np.array_equal(self._h[i], hi):
                self.ctx.set_hamiltonian(i, hi, self.eri[i], self.eps[i])
                self._h[i] = hi.copy()
        self.ctx.solve(mu, beta)
        self.generation += 1
        return self.ctx.grand_potential()[0]


def _host(t, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} is on {t.device}: FT-CCSD has no CPU path, pass HIP (cuda) tensors")
    return t.detach().to(torch.float64).cpu().numpy()


class FTCCOmega(torch.autograd.Function):
    """Omega[B] = FTCCOmega.apply(mu[B], beta[B], h[B, n, n], solver).

    h is padded to the largest n of the batch; instance i uses h[i, :n_i, :n_i]
    and its gradient is zero outside that block."""

    @staticmethod
    def forward(ctx, mu, beta, h, solver):
        mu_h = _host(mu, "mu").reshape(solver.B)
        beta_h = _host(beta, "beta").reshape(solver.B)
        h_h = _host(h, "h")
        nmax = max(solver.sizes)
        if h_h.shape != (solver.B, nmax, nmax):
            raise ValueError(f"h must have shape ({solver.B}, {nmax}, {nmax})")
        om = solver._solve(mu_h, beta_h, h_h)
        ctx.solver = solver
        ctx.state = (mu_h, beta_h, h_h, solver.generation)
        ctx.dev = h.device
        return torch.as_tensor(om, dtype=torch.float64, device=h.device)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad):
        solver = ctx.solver
        mu_h, beta_h, h_h, gen = ctx.state
        if solver.generation != gen:          # another forward ran since: restore this one's amplitudes
            solver._solve(mu_h, beta_h, h_h)
        solver._bind_stream()
        want_mu, want_beta, want_h = ctx.needs_input_grad[:3]
        solver.ctx.lam()
        r = solver.ctx.response(want_mu=want_mu, want_beta=want_beta, want_h=want_h)
        g = grad.detach().to(torch.float64).cpu().numpy()
        dev = ctx.dev
        out_mu = torch.as_tensor(g * r["mu"], device=dev) if want_mu else None
        out_beta = torch.as_tensor(g * r["beta"], device=dev) if want_beta else None
        out_h = None
        if want_h:
            nmax = h_h.shape[1]
            gh = np.zeros((solver.B, nmax, nmax))
            for i, n in enumerate(solver.sizes):
                gh[i, :n, :n] = g[i] * r["h"][i]
            out_h = torch.as_tensor(gh, device=dev)
        return out_mu, out_beta, out_h, None


def omega(mu, beta, h, solver):
    """Differentiable grand potential of every instance of `solver`."""
    return FTCCOmega.apply(mu, beta, h, solver)
