"""Wall time of the oracle (plain FP64 NumPy, test infrastructure) for the whole
forward march and the Lambda adjoint with its response derivatives, on the
host's cores, for the small workload configurations: the 6-site ring (U = 4,
T = 1, 20 tau nodes as 5 panels x 4), the 10-site ring (U = 8, T = 1, 40 nodes
as 10 x 4, occupation threshold 1e-6) and the first ring of the mixed batch
(20 nodes, threshold 1e-6).  Prints one JSON line.  Not a test: run from the
repository root as
    python tests/oracle_timing.py
"""
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import ftcc_inputs as fi  # noqa: E402
from oracle import grid as G, restricted as R, solver as S  # noqa: E402


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def time_one(name, s, panels, nodes, thr):
    model = R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, s.mu, s.beta, thr))
    gr = G.Grid(s.beta, panels, nodes)
    t0 = time.perf_counter()
    sol = S.solve(model, gr, tol=1e-12)
    t1 = time.perf_counter()
    adj = S.adjoint(model, gr, sol, tol=1e-12)
    d_mu = S.d_omega(model, gr, sol, adj, "mu")
    d_beta = S.d_omega(model, gr, sol, adj, "beta")
    S.d_omega_dh(model, gr, sol, adj)
    t2 = time.perf_counter()
    return dict(workload=name, n=int(s.n), n_tau=panels * nodes, forward_s=t1 - t0,
                adjoint_and_response_s=t2 - t1, omega=float(sol.omega), dOmega_dmu=float(d_mu),
                dOmega_dbeta=float(d_beta))


def main():
    ring0 = next(kw for kind, kw in fi.batched_configs(0) if kind == "hubbard")
    rows = [
        time_one("hubbard_L6_U4_T1", fi.hubbard_config(L=6, U=4.0, T=1.0), 5, 4, 0.0),
        time_one("hubbard_L10_U8_T1", fi.hubbard_config(L=10, U=8.0, T=1.0), 10, 4, 1e-6),
        time_one(f"batch_ring_L{ring0['L']}_U{ring0['U']:.3f}_T{ring0['T']:.3f}",
                 fi.hubbard_config(L=ring0["L"], U=ring0["U"], T=ring0["T"]), 5, 4, 1e-6),
    ]
    print(json.dumps(dict(kind="oracle", cpu_model=cpu_model(), cores=os.cpu_count(), rows=rows)), flush=True)


if __name__ == "__main__":
    main()
