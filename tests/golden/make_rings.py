"""Writes rings.json: oracle values for the Hubbard rings of two workloads.

  * the 6-site ring, t = 1, U = 4, mu = U/2, T = 1, 20 tau nodes (5 panels x 4),
    exponential collocation: FT-CCSD Omega and its parts, and the exact
    grand-canonical Omega from diagonalising the Hamiltonian in the whole Fock
    space (4096 states; thermal FCI), whose difference from FT-CCSD is the
    method's error (reported, not a parity target);
  * the 16 rings of the mixed 32-instance batch (L = 6 + (i mod 9), U ~ U[1, 8],
    T ~ U[0.1, 2] from ftcc_inputs.batched_configs(0), mu = U/2), 20 tau nodes,
    occupation threshold 1e-6: Omega and its parts, dOmega/dmu and dOmega/dbeta
    where the oracle's march converges; where its fixed-point sweeps diverge or
    overflow, the panel at which that happened (the low-temperature growth of
    the restricted reference's inverted pairs).

Calls only the oracle.  Run from the repository root:
    python tests/golden/make_rings.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import ftcc_inputs as fi  # noqa: E402
from oracle import ed, grid as G, restricted as R, solver as S, spinorb as so  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _march(s, thr, P=5, m=4):
    model = R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, s.mu, s.beta, thr))
    gr = G.Grid(s.beta, P, m)
    try:
        sol = S.solve(model, gr, tol=1e-13, max_iter=300)
    except (FloatingPointError, RuntimeError) as e:
        return dict(converged=False, failure=str(e))
    out = dict(converged=True, omega=sol.omega, omega0=sol.omega0, omega1=sol.omega1, omega_cc=sol.omega_cc,
               sweeps=list(sol.iters))
    try:
        adj = S.adjoint(model, gr, sol, tol=1e-13, max_iter=300)
    except (FloatingPointError, RuntimeError) as e:
        out.update(adjoint_converged=False, adjoint_failure=str(e))
        return out
    out.update(adjoint_converged=True, dOmega_dmu=S.d_omega(model, gr, sol, adj, "mu"),
               dOmega_dbeta=S.d_omega(model, gr, sol, adj, "beta"))
    return out


def main():
    t0 = time.time()
    s = fi.hubbard_config(L=6, U=4.0, T=1.0)
    hs, es, _ = so.spin_orbital_from_spatial(s.h, s.eri, s.eps)
    h6 = dict(L=6, U=4.0, T=1.0, mu=s.mu, beta=s.beta, n_panels=5, m=4, **_march(s, 0.0),
              omega_exact=float(ed.grand_potential(hs, es, s.mu, s.beta)))
    h6["ftccsd_error"] = h6["omega"] - h6["omega_exact"]
    print(f"6-site ring: Omega {h6['omega']:.12f}, exact {h6['omega_exact']:.12f} ({time.time() - t0:.0f} s)",
          flush=True)
    rings = []
    for k, (kind, kw) in enumerate(fi.batched_configs(0)):
        if kind != "hubbard":
            continue
        s = fi.hubbard_config(**kw)
        r = dict(index=k, mu=s.mu, beta=s.beta, **kw, **_march(s, 1e-6))
        rings.append(r)
        print(f"batch instance {k}: L={kw['L']} U={kw['U']:.3f} T={kw['T']:.3f} converged={r['converged']} "
              f"({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, "rings.json"), "w") as f:
        json.dump(dict(hubbard6=h6, batch_rings=dict(n_panels=5, m=4, thr=1e-6, tol=1e-13, rings=rings)), f, indent=1)


if __name__ == "__main__":
    main()
