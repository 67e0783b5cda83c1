"""Batching and checkpointing on the GPU: a mixed batch of instances of
different sizes gives the same results as single-instance runs and does not
depend on the batch order; panel checkpointing reproduces the stored-grid
adjoint."""
import sys

import numpy as np
import pytest

import ftcc_inputs as fi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_01729_amd import ftcc
    return ftcc


def _systems():
    return [fi.hubbard_config(L=4, U=2.0, T=1.0), fi.hubbard_config(L=5, U=3.0, T=0.8),
            fi.ueg_config(7, 2, 1.0, 1.0), fi.hubbard_config(L=6, U=1.5, T=1.2)]


def _run(F, systems, **opt):
    ctx = F.Context(len(systems), n_tau=8, nodes_per_panel=4, tol=1e-13, **opt)
    for i, s in enumerate(systems):
        ctx.set_hamiltonian(i, s.h, s.eri, s.eps)
    ctx.solve([s.mu for s in systems], [s.beta for s in systems])
    om, parts = ctx.grand_potential()
    ctx.lam()
    r = ctx.response(want_mu=True, want_beta=True, want_h=True)
    ctx.close()
    return om, r


def test_mixed_batch_equals_single(F):
    systems = _systems()
    print("[batch] mixed sizes", [s.n for s in systems], flush=True)
    om_b, r_b = _run(F, systems)
    for i, s in enumerate(systems):
        om_s, r_s = _run(F, [s])
        assert abs(om_b[i] - om_s[0]) < 1e-12 * abs(om_s[0])
        assert abs(r_b["mu"][i] - r_s["mu"][0]) < 1e-11 * max(1.0, abs(r_s["mu"][0]))
        assert abs(r_b["beta"][i] - r_s["beta"][0]) < 1e-11 * max(1.0, abs(r_s["beta"][0]))
        n = s.n
        assert np.abs(r_b["h"][i][:n, :n] - r_s["h"][0]).max() < 1e-11


def test_batch_order_independent(F):
    systems = _systems()
    print("[batch] order", flush=True)
    om_a, r_a = _run(F, systems)
    om_b, r_b = _run(F, systems[::-1])
    assert np.allclose(om_a, om_b[::-1], rtol=1e-12, atol=0)
    assert np.allclose(r_a["mu"], r_b["mu"][::-1], rtol=1e-11, atol=1e-12)


def test_checkpoint_reproduces_adjoint(F):
    systems = _systems()[:2]
    print("[checkpoint] recompute panels in the adjoint", flush=True)
    om0, r0 = _run(F, systems, checkpoint=0)
    om1, r1 = _run(F, systems, checkpoint=1)
    assert np.array_equal(om0, om1)
    assert np.allclose(r0["mu"], r1["mu"], rtol=1e-13, atol=1e-14)
    assert np.allclose(r0["beta"], r1["beta"], rtol=1e-13, atol=1e-14)


def test_one_slot_mode_matches(F, monkeypatch):
    """The memory-lean schedule (one executor slot per instance, nodes evaluated one
    after another) chosen automatically for large n gives the same Omega, gradients
    and Lambda as the all-nodes-at-once schedule."""
    systems = _systems()[:3]
    print("[slots] one executor slot vs m slots, checkpoint=1", flush=True)
    om0, r0 = _run(F, systems, checkpoint=1)
    monkeypatch.setenv("FTCC_NODE_SLOTS", "1")
    om1, r1 = _run(F, systems, checkpoint=1)
    assert np.allclose(om0, om1, rtol=1e-13, atol=0)
    for key in ("mu", "beta"):
        assert np.allclose(r0[key], r1[key], rtol=1e-12, atol=1e-13), key
    for a, b in zip(r0["h"], r1["h"]):
        assert np.abs(a - b).max() < 1e-12


def test_failed_instance_does_not_disturb_batch(F):
    """An instance whose march diverges (a low-temperature, strongly coupled ring
    with the restricted reference) is reported in its status slot and stops
    running; the other instance of the batch gets the single-instance results."""
    good = fi.hubbard_config(L=4, U=2.0, T=1.0)
    kind, kw = fi.batched_configs(0)[21]
    assert kind == "hubbard"
    bad = fi.hubbard_config(**kw)
    print(f"[batch] diverging instance {kw} next to hubbard L=4", flush=True)
    opt = dict(n_tau=20, nodes_per_panel=4, occ_thresh=1e-6, tol=1e-13, max_iter=100)

    def run(systems):
        ctx = F.Context(len(systems), **opt)
        for i, s in enumerate(systems):
            ctx.set_hamiltonian(i, s.h, s.eri, s.eps)
        _, st = ctx.solve([s.mu for s in systems], [s.beta for s in systems], raise_on_status=False)
        om, _ = ctx.grand_potential()
        _, lst = ctx.lam(raise_on_status=False)
        r = ctx.response(want_mu=True, want_beta=True, want_h=False)
        ctx.close()
        return st, lst, om, r

    st, lst, om, r = run([good, bad])
    assert st[0] == 0 and st[1] in (F.ENOCONV, F.ENONFINITE, F.EDIVERGE)
    assert lst[0] == 0 and lst[1] != 0
    st1, _, om1, r1 = run([good])
    assert st1[0] == 0
    assert abs(om[0] - om1[0]) < 1e-12 * abs(om1[0])
    assert abs(r["mu"][0] - r1["mu"][0]) < 1e-11 * max(1.0, abs(r1["mu"][0]))
    assert abs(r["beta"][0] - r1["beta"][0]) < 1e-11 * max(1.0, abs(r1["beta"][0]))


def test_kernel_profile_enabled_before_first_solve(F):
    """The plan is built (autotuned, graph-captured) inside the first solve; an
    enabled kernel profiler must not record inside that capture.  The
    57-plane-wave gas, whose O(n^6) GEMMs run in the profiled 128 x 128 tiles
    (the autotuner gives small systems 64 x 64 tiles)."""
    s = fi.ueg_config(57, 14, 1.0, 0.5)
    print("[profile] ueg 57 PW n_tau=16, profiler on before the first solve", flush=True)
    ctx = F.Context(1, n_tau=16, nodes_per_panel=4, tol=1e-12)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    ctx.kernel_profile(1)
    ctx.solve(s.mu, s.beta)
    kp = ctx.kernel_profile(0)
    om0 = ctx.grand_potential()[0][0]
    ctx.solve(s.mu, s.beta)
    om1 = ctx.grand_potential()[0][0]
    ctx.close()
    assert kp["launches"] > 0 and kp["seconds"] > 0.0 and kp["flops"] > 0.0
    assert om0 == om1
