"""Writes ueg57_batch_residuals.npz: one oracle evaluation of the kernels E, S1
and S2 (eqn:E, eqn:ccS1, eqn:ccS2) for each of the 16 electron-gas instances of
the mixed batch (57 plane waves, N = 14, r_s in {0.5, 1, 2, 4} x Theta in
{0.25, 0.5, 1, 2}, thermal HF reference at its own mu and beta, occupation
threshold 1e-6), at seeded random amplitudes restricted to the momentum-allowed
elements (t1: k_i = k_a; t2: k_i + k_j = k_a + k_b; scale 0.02, seed 5700 + k
for instance k), so that the dense and the momentum-blocked paths can both be
held against them.

Stored per instance: mu, beta, E, S1 whole, and S2 at a seeded sample of 2000
momentum-allowed elements and 200 forbidden ones (flat [i][j][a][b] indices;
the forbidden ones are zero by the momentum law).  About twenty minutes of
CPU.
Calls only the oracle.  Run from the repository root:
    python tests/golden/make_ueg57_batch.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import ftcc_inputs as fi  # noqa: E402
from oracle import restricted as R  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_PW, N_EL, THR, SCALE = 57, 14, 1e-6, 0.02
N_ALLOWED, N_FORBIDDEN = 2000, 200


def main():
    t0 = time.time()
    gases = [kw for kind, kw in fi.batched_configs(0) if kind == "ueg"]
    out = {k: [] for k in ("rs", "theta", "mu", "beta", "seed", "E", "S1", "idx", "S2")}
    for k, kw in enumerate(gases):
        s = fi.ueg_config(N_PW, N_EL, kw["rs"], kw["theta"])
        seed = 5700 + k
        t = fi.momentum_allowed_amplitudes(s.momentum[0], seed=seed, scale=SCALE)
        model = R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, s.mu, s.beta, THR))
        E = model.energy(t)
        S1, S2 = model.residual(t)
        model.ints._cache.clear()
        _, m2 = fi.momentum_masks(s.momentum[0])
        rng = np.random.default_rng(seed)
        allowed = np.flatnonzero(m2.ravel())
        forbidden = np.flatnonzero(~m2.ravel())
        idx = np.sort(np.concatenate([rng.choice(allowed, N_ALLOWED, replace=False),
                                      rng.choice(forbidden, N_FORBIDDEN, replace=False)]))
        for key, v in (("rs", kw["rs"]), ("theta", kw["theta"]), ("mu", s.mu), ("beta", s.beta), ("seed", seed),
                       ("E", E), ("S1", S1), ("idx", idx), ("S2", S2.ravel()[idx])):
            out[key].append(v)
        print(f"[{k + 1}/16] rs={kw['rs']:g} theta={kw['theta']:g} E={E:.15e} max|S2|={np.abs(S2).max():.3e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "ueg57_batch_residuals.npz"), n_pw=N_PW, n_el=N_EL, thr=THR,
                        scale=SCALE, **{k: np.asarray(v) for k, v in out.items()})


if __name__ == "__main__":
    main()
