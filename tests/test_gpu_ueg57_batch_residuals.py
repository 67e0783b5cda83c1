"""The 16 electron-gas instances of the mixed batch (57 plane waves, N = 14,
r_s in {0.5, 1, 2, 4} x Theta in {0.25, 0.5, 1, 2}, thermal HF reference,
occupation threshold 1e-6) in one context of the batch's configuration (20 tau
nodes as 5 panels x 4), each instance's residual against stored oracle values
(tests/golden/ueg57_batch_residuals.npz, written by make_ueg57_batch.py from
the oracle alone) at seeded momentum-allowed amplitudes: E (1e-10 relative),
S1 whole and S2 at 2200 sampled elements (1e-10 relative to max(1, max|S|)),
through the dense FP64-MFMA path and through the momentum-blocked path."""
import os

import numpy as np
import pytest

import ftcc_inputs as fi

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("blocked", [False, True])
def test_batch_gases_residuals_against_oracle(blocked):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_01729_amd import ftcc as F
    g = np.load(os.path.join(HERE, "ueg57_batch_residuals.npz"))
    n_pw, n_el, thr = int(g["n_pw"]), int(g["n_el"]), float(g["thr"])
    systems = [fi.ueg_config(n_pw, n_el, float(rs), float(th)) for rs, th in zip(g["rs"], g["theta"])]
    print(f"[ueg57 batch] 16 gases in one context, blocked={blocked}", flush=True)
    ctx = F.Context(len(systems), n_tau=20, nodes_per_panel=4, occ_thresh=thr, tol=1e-12)
    for i, s in enumerate(systems):
        assert abs(s.mu - g["mu"][i]) < 1e-14 and abs(s.beta - g["beta"][i]) < 1e-14
        if blocked:
            ctx.set_momentum(i, *s.momentum)
        ctx.set_hamiltonian(i, s.h, s.eri, s.eps)
    try:
        for i, s in enumerate(systems):
            t1, t2 = fi.momentum_allowed_amplitudes(s.momentum[0], seed=int(g["seed"][i]), scale=float(g["scale"]))
            S1, S2, E = ctx.eval_residual(i, s.mu, s.beta, t1, t2)
            E0, S10, S20 = float(g["E"][i]), g["S1"][i], g["S2"][i]
            s1 = max(1.0, np.abs(S10).max())
            s2 = max(1.0, np.abs(S20).max())
            err = (abs(E - E0) / max(1.0, abs(E0)), np.abs(S1 - S10).max() / s1,
                   np.abs(S2.ravel()[g["idx"][i]] - S20).max() / s2)
            print(f"  instance {i} rs={g['rs'][i]:g} theta={g['theta'][i]:g}: E {E:.15e} "
                  f"(oracle {E0:.15e}); errors E {err[0]:.1e} S1 {err[1]:.1e} S2 {err[2]:.1e}", flush=True)
            assert err[0] < 1e-10 and err[1] < 1e-10 and err[2] < 1e-10
    finally:
        ctx.close()
