"""Writes hubbard10_u8.json: oracle values for the 10-site ring, U = 8,
mu = U/2, T in {1, 2}, 40 tau nodes (10 panels x 4 Gauss-Legendre), occupation
threshold 1e-6 (Section III.A's truncation), exponential collocation.

Calls only the oracle (Omega, its parts, and the discrete-adjoint dOmega/dmu and
dOmega/dU at a frozen reference).  Run from the repository root:
    python tests/golden/make_hubbard10.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import ftcc_inputs as fi  # noqa: E402
from oracle import grid as G, restricted as R, solver as S  # noqa: E402

U, L, THR, P, M = 8.0, 10, 1e-6, 10, 4


def main():
    out = dict(L=L, U=U, thr=THR, n_panels=P, m=M, propagator="exponential-collocation", tol=1e-12, cases=[])
    for T in (2.0, 1.0):
        s = fi.hubbard_config(L=L, U=U, T=T)
        model = R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, s.mu, s.beta, THR))
        gr = G.Grid(s.beta, P, M)
        sol = S.solve(model, gr, tol=1e-13)
        adj = S.adjoint(model, gr, sol, tol=1e-13)
        dmu = S.d_omega(model, gr, sol, adj, "mu")
        dU = S.d_omega(model, gr, sol, adj, "h", deri=s.eri / U)
        out["cases"].append(dict(T=T, mu=s.mu, beta=s.beta, omega=sol.omega, omega0=sol.omega0,
                                 omega1=sol.omega1, omega_cc=sol.omega_cc, dOmega_dmu=dmu, dOmega_dU=dU))
        print(out["cases"][-1], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "hubbard10_u8.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
