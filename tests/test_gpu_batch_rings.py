"""The ring instances of the mixed 32-instance workload and the 6-site ring
against oracle values (tests/golden/rings.json, written by make_rings.py from
the oracle alone).

  * the 16 rings of the mixed batch (L = 6 + (i mod 9), U ~ U[1, 8],
    T ~ U[0.1, 2], mu = U/2; 20 tau nodes as 5 panels x 4; occupation threshold
    1e-6) in ONE batched context, dense and momentum-blocked: Omega and its
    parts to 1e-10 relative and dOmega/dmu, dOmega/dbeta to 1e-8 where the
    oracle's march converges; where the oracle's own march diverges (the
    low-temperature rings) the instance must report a failure status;
  * the 6-site ring (U = 4, T = 1, 20 tau nodes): Omega against the oracle, and
    its error against exact diagonalisation in the whole Fock space reported
    (the method's error, not a parity target).
"""
import json
import os

import numpy as np
import pytest

import ftcc_inputs as fi

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rings.json")


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_01729_amd import ftcc
    return ftcc


@pytest.mark.parametrize("blocked", [False, True])
def test_batch_rings_against_oracle(F, blocked):
    g = json.load(open(GOLDEN))["batch_rings"]
    rings = g["rings"]
    systems = [fi.hubbard_config(L=r["L"], U=r["U"], T=r["T"]) for r in rings]
    print(f"[batch rings] 16 rings in one context, 20 tau, thr 1e-6, blocked={blocked}", flush=True)
    ctx = F.Context(len(systems), n_tau=g["n_panels"] * g["m"], nodes_per_panel=g["m"], occ_thresh=g["thr"],
                    tol=1e-13, max_iter=300)
    for i, s in enumerate(systems):
        if blocked:
            ctx.set_momentum(i, *s.momentum)
        ctx.set_hamiltonian(i, s.h, s.eri, s.eps)
    _, st = ctx.solve([s.mu for s in systems], [s.beta for s in systems], raise_on_status=False)
    om, parts = ctx.grand_potential()
    _, lst = ctx.lam(raise_on_status=False)
    r = ctx.response(want_mu=True, want_beta=True, want_h=False)
    ctx.close()
    for i, ref in enumerate(rings):
        if not ref["converged"]:
            assert st[i] != 0, (i, ref)
            continue
        assert st[i] == 0, (i, int(st[i]))
        assert abs(om[i] - ref["omega"]) < 1e-10 * abs(ref["omega"]), i
        assert abs(parts[i, 2] - ref["omega_cc"]) < 1e-10 * max(1.0, abs(ref["omega_cc"])), i
        if ref.get("adjoint_converged"):
            assert lst[i] == 0, i
            assert abs(r["mu"][i] - ref["dOmega_dmu"]) < 1e-8 * max(1.0, abs(ref["dOmega_dmu"])), i
            assert abs(r["beta"][i] - ref["dOmega_dbeta"]) < 1e-8 * max(1.0, abs(ref["dOmega_dbeta"])), i


def test_hubbard6_against_oracle_and_exact(F):
    g = json.load(open(GOLDEN))["hubbard6"]
    s = fi.hubbard_config(L=g["L"], U=g["U"], T=g["T"])
    print("[batch rings] hubbard L=6 U=4 T=1 n_tau=20 against the oracle and exact diagonalisation", flush=True)
    ctx = F.Context(1, n_tau=g["n_panels"] * g["m"], nodes_per_panel=g["m"], tol=1e-13)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    ctx.solve(s.mu, s.beta)
    om, _ = ctx.grand_potential()
    ctx.close()
    assert abs(om[0] - g["omega"]) < 1e-10 * abs(g["omega"])
    err = om[0] - g["omega_exact"]
    print(f"[batch rings] FT-CCSD Omega {om[0]:.10f}, exact {g['omega_exact']:.10f}, error {err:.3e} "
          f"({100 * err / abs(g['omega_exact']):.3f}%)", flush=True)
    assert np.isfinite(err)
