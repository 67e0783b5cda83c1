"""Writes ueg123_residual.npz: one oracle evaluation of the kernels E, S1, S2
(eqn:E, eqn:ccS1, eqn:ccS2) for the 123-plane-wave electron gas of the largest
workload (N = 14, r_s = 4, Theta = 1, thermal HF reference, occupation
threshold 1e-6, which drops no slot here) at chemical potential and
temperature of that reference, with seeded dense random amplitudes
(ftcc_inputs.random_amplitudes(123, seed=123, scale=0.02): dense, so that
every element of S2 carries the contractions, not only the momentum-allowed
ones).

Stored: E, S1 whole, and S2 on the rows i in I = {0, 1, 122}, j in J = {4, 5,
122} (all a, b: 9 x 123^2 = 136161 elements; rows 4, 5, 122, 127, 128, 245,
15010, 15011 and 15128 of the (ij) x (ab) matrix: both sides of the 128-row
boundary and the last, ragged row).  S2 is too large for the oracle to form
whole (1.83 GB per tensor, one weighted integral block per slot pattern), so the
rows come from RestrictedModel.residual_rows.  About an hour of CPU time.
Calls only the oracle.  Run from the repository root:
    python tests/golden/make_ueg123.py
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
N_PW, N_EL, RS, THETA, THR = 123, 14, 4.0, 1.0, 1e-6
SEED, SCALE = 123, 0.02
ROWS_I, ROWS_J = [0, 1, 122], [4, 5, 122]


def main():
    t0 = time.time()
    s = fi.ueg_config(N_PW, N_EL, RS, THETA)
    model = R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, s.mu, s.beta, THR))
    t = fi.random_amplitudes(s.n, seed=SEED, scale=SCALE)
    print(f"set-up {time.time() - t0:.0f} s; dropped hole slots {int((~model.ints.keep_h).sum())}, "
          f"particle slots {int((~model.ints.keep_p).sum())}", flush=True)
    E = model.energy(t)
    model.ints._cache.clear()
    print(f"E = {E:.15e} ({time.time() - t0:.0f} s)", flush=True)
    S1, S2r = model.residual_rows(t, ROWS_I, ROWS_J)
    print(f"S1, S2 rows done ({time.time() - t0:.0f} s); max|S1| {np.abs(S1).max():.3e}, "
          f"max|S2 rows| {np.abs(S2r).max():.3e}", flush=True)
    np.savez_compressed(os.path.join(HERE, "ueg123_residual.npz"), n_pw=N_PW, n_el=N_EL, rs=RS, theta=THETA,
                        thr=THR, mu=s.mu, beta=s.beta, seed=SEED, scale=SCALE, rows_i=np.asarray(ROWS_I),
                        rows_j=np.asarray(ROWS_J), E=E, S1=S1, S2_rows=S2r)


if __name__ == "__main__":
    main()
