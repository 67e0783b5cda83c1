"""Writes the oracle values of the 57-plane-wave electron gas at its workload
configuration: N = 14, r_s = 1, Theta = 0.5, thermal HF reference, no
occupation threshold, 16 tau nodes as 4 panels of 4 Gauss-Legendre nodes,
exponential collocation, tolerance 1e-13.

  ueg57_forward.npz    Omega and its parts, E(tau_x) of every node, Picard
                       sweeps per panel; the amplitudes of every node of the
                       last panel (t1 whole, t2 at a seeded sample of its
                       momentum-allowed elements)
  ueg57_gradients.npz  dOmega/dmu, dOmega/dbeta, dOmega/dh (frozen reference),
                       and Lambda of nodes 0 and 15 at the same t2 sample
                       (Lambda2 symmetrised over [ijab] <-> [jiba])

Calls only the oracle.  The march and the adjoint extrapolate their sweeps by
DIIS, which leaves their fixed points unchanged.  Several hours of CPU time at
n = 57; `--state FILE` keeps the forward solution in FILE so that a second run
starts at the adjoint.  Run from the repository root:
    python tests/golden/make_ueg57.py [--state FILE]
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import ftcc_inputs as fi  # noqa: E402
from oracle import grid as G, restricted as R, solver as S  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_PW, N_EL, RS, THETA, P, M, TOL = 57, 14, 1.0, 0.5, 4, 4, 1e-13
N_SAMPLE, SEED = 20000, 2004


def allowed_t2_flat(labels):
    """Flat indices [i][j][a][b] of the t2 elements with k_i + k_j = k_a + k_b."""
    lab = np.asarray(labels, dtype=np.int64)
    base = 4 * int(np.abs(lab).max()) + 1
    code = (lab[:, 0] * base + lab[:, 1]) * base + lab[:, 2]
    pair = code[:, None] + code[None, :]
    return np.flatnonzero((pair[:, :, None, None] == pair[None, None, :, :]).ravel())


def _log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def _save_state(path, sol):
    arrs = dict(energies=sol.energies, omega_cc=sol.omega_cc, omega0=sol.omega0,
                omega1=sol.omega1, iters=np.asarray(sol.iters))
    for k, (a, b) in enumerate(sol.nodes):
        arrs[f"n1_{k}"], arrs[f"n2_{k}"] = a, b
    for k, (a, b) in enumerate(sol.resid):
        arrs[f"r1_{k}"], arrs[f"r2_{k}"] = a, b
    for k, (a, b) in enumerate(sol.sb):
        arrs[f"b1_{k}"], arrs[f"b2_{k}"] = a, b
    np.savez(path, **arrs)


def _load_state(path):
    z = np.load(path)
    n_nodes, n_panels = P * M, P
    return S.Solution([(z[f"n1_{k}"], z[f"n2_{k}"]) for k in range(n_nodes)],
                      [(z[f"r1_{k}"], z[f"r2_{k}"]) for k in range(n_nodes)],
                      [(z[f"b1_{k}"], z[f"b2_{k}"]) for k in range(n_panels)],
                      z["energies"], float(z["omega_cc"]), float(z["omega0"]), float(z["omega1"]),
                      list(z["iters"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--state", default=None)
    args = ap.parse_args()
    s = fi.ueg_config(N_PW, N_EL, RS, THETA)
    n = s.n
    model = R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, s.mu, s.beta))
    gr = G.Grid(s.beta, P, M)
    allowed = allowed_t2_flat(s.momentum[0])
    idx = np.sort(np.random.default_rng(SEED).choice(allowed, N_SAMPLE, replace=False))
    meta = dict(n_pw=N_PW, n_el=N_EL, rs=RS, theta=THETA, n_panels=P, m=M, tol=TOL,
                mu=s.mu, beta=s.beta, t2_index=idx)

    if args.state and os.path.exists(args.state):
        _log(f"forward solution from {args.state}")
        sol = _load_state(args.state)
    else:
        _log(f"forward march n={n} P={P} m={M} beta={s.beta:.6f} mu={s.mu:.6f}")
        sol = S.solve(model, gr, tol=TOL, diis=6)
        _log(f"forward done: sweeps {sol.iters}, Omega_CC {sol.omega_cc:.15f}")
        if args.state:
            _save_state(args.state, sol)
    last = range((P - 1) * M, P * M)
    np.savez_compressed(os.path.join(HERE, "ueg57_forward.npz"), **meta,
                        omega=sol.omega, omega0=sol.omega0, omega1=sol.omega1, omega_cc=sol.omega_cc,
                        energies=sol.energies, iters=np.asarray(sol.iters), nodes=np.asarray(list(last)),
                        t1=np.stack([sol.nodes[k][0] for k in last]),
                        t2=np.stack([sol.nodes[k][1].ravel()[idx] for k in last]))
    _log("wrote ueg57_forward.npz")

    adj = S.adjoint(model, gr, sol, tol=TOL, diis=6)
    _log(f"adjoint done: sweeps {adj.iters}")
    dmu = S.d_omega(model, gr, sol, adj, "mu")
    _log(f"dOmega/dmu {dmu:.15f}")
    dbeta = S.d_omega(model, gr, sol, adj, "beta")
    _log(f"dOmega/dbeta {dbeta:.15f}")
    dh = S.d_omega_dh(model, gr, sol, adj)
    lam_nodes = (0, P * M - 1)
    lam2 = []
    for k in lam_nodes:
        l2 = adj.lam[k][1]
        lam2.append((0.5 * (l2 + l2.transpose(1, 0, 3, 2))).ravel()[idx])
    np.savez_compressed(os.path.join(HERE, "ueg57_gradients.npz"), **meta,
                        dOmega_dmu=dmu, dOmega_dbeta=dbeta, dOmega_dh=dh,
                        adjoint_iters=np.asarray(adj.iters), lam_nodes=np.asarray(lam_nodes),
                        lam1=np.stack([adj.lam[k][0] for k in lam_nodes]), lam2_sym=np.stack(lam2))
    _log("wrote ueg57_gradients.npz")


if __name__ == "__main__":
    main()
