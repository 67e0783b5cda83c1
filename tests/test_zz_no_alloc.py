"""The allocation-free entry point ftcc_response_noalloc against ftcc_response on
the same contexts: two calls in a row, the second with a smaller input (a
6-site ring with 12 tau nodes, then a 3-site ring with 8), and a
momentum-blocked checkpointed context, each compared to the allocating entry
point to the parity bar of the derivatives (1e-8 relative; the two share
kernels and summation order, so they agree to rounding)."""
import sys

import numpy as np
import pytest

import ftcc_inputs as fi

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


def _run(F, s, n_tau, momentum=False, **kw):
    ctx = F.Context(1, n_tau=n_tau, nodes_per_panel=4, tol=1e-13, **kw)
    if momentum:
        ctx.set_momentum(0, *s.momentum)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    ctx.solve(s.mu, s.beta)
    ctx.lam()
    ref = ctx.response(want_h=False)
    got = ctx.response_noalloc()
    again = ctx.response_noalloc(want_beta=False)
    ctx.close()
    return ref, got, again


def _close(a, b):
    return abs(a - b) <= 1e-8 * max(1.0, abs(b))


def test_noalloc_matches_response_two_calls(ftcc):
    for L, n_tau in ((6, 12), (3, 8)):
        s = fi.hubbard_config(L=L, U=4.0, T=1.0)
        _say(f"[noalloc] hubbard L={L} U=4 T=1 n_tau={n_tau}")
        ref, got, again = _run(ftcc, s, n_tau)
        assert _close(got["mu"][0], ref["mu"][0]) and _close(got["beta"][0], ref["beta"][0])
        assert _close(again["mu"][0], ref["mu"][0]) and again["beta"] is None


def test_noalloc_momentum_blocked_checkpointed(ftcc):
    s = fi.ueg_config(19, 14, 1.0, 0.5)
    _say("[noalloc] ueg 19 PW n_tau=8 momentum-blocked checkpoint=1")
    ref, got, _ = _run(ftcc, s, 8, momentum=True, checkpoint=1)
    assert _close(got["mu"][0], ref["mu"][0]) and _close(got["beta"][0], ref["beta"][0])


def test_noalloc_rejects_differential_form(ftcc):
    s = fi.hubbard_config(L=3, U=2.0, T=1.0)
    ctx = ftcc.Context(1, n_tau=4, propagator=4)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    ctx.solve(s.mu, s.beta)
    ctx.lam()
    with pytest.raises(ftcc.FTCCError):
        ctx.response_noalloc()
    ctx.close()
