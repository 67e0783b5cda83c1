#!/usr/bin/env python3
"""Throughput of the FT-CCSD hot path on one MI355X.

Default line (the metric's measurement M1 at the largest workload): the warm
dense electron gas in 123 plane waves, N = 14, r_s = 4, Theta = 1, thermal HF
reference, occupation threshold 1e-6, restricted, FP64, in the context of its
full configuration (16 Gauss-Legendre tau points as 4 panels x 4 nodes,
panel checkpointing; dense contractions on FP64 MFMA).  A step is the T1/T2
residual evaluation (eqn:E, eqn:ccS1, eqn:ccS2) of the four nodes of a panel,
i.e. the residual work of one Picard sweep, at the first-order amplitudes
s(tau) = -S0 (1 - exp(-Delta tau)) / Delta at tau = beta / 2 (S0 the residual at
zero amplitudes), on device-resident data through the replayed HIP graph.
value = residual evaluations per second.  The dominant kernel's duration comes
from a separate pass with per-launch HIP events after the timed steps.
config.momentum_blocked_same_residual: the same residual at the same
amplitudes through the momentum-blocked path (crystal momentum of the plane
waves set on the instance), its throughput and energy against the dense one.
Secondary fields (config.secondary): the 57-plane-wave gas (r_s = 1,
Theta = 0.5, 16 tau points) through the whole path -- forward march, Lambda
adjoint, response dOmega/dmu, dOmega/dbeta, dOmega/dh -- and the adjoint
gradient against measured central finite differences of Omega.
Synthetic: every Hamiltonian is generated from these parameters.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-secondary]
       python bench.py --mode step [--workload ueg57|ueg123|hubbard6|hubbard10] [--momentum]
       python bench.py --mode residual|copy|vendor_gemm|batch|numerr|gradient|exc|afm ...

--mode step times whole steps (thermal set-up + forward march + Lambda +
response) of one workload.  --mode residual times R back-to-back residual
evaluations of every node of the last panel at the converged amplitudes;
--mode copy runs R device-to-device copies of 1 GiB (the byte-counter
calibration for the traffic figures); --mode vendor_gemm times the vendor
library's float64 GEMM (torch.matmul) on plain square products of the
residuals' GEMM sizes, for comparison only.  --mode batch runs one step of the
32-instance mixed batch (16 UEG 57-PW points over r_s x Theta, 16 Hubbard rings
L = 6..14 with random U and T, 20 tau points, occupation threshold 1e-6) in one
context, and with --per-instance the same instances one context each.
--momentum evaluates the contractions over their crystal-momentum-allowed
blocks only.  --mode numerr measures the grid-error orders of the differential
form and of the Simpson integral form (Table tab:numerr) on the 14-electron gas
in 33 plane waves at r_s = 4, Theta = 0.125.  --mode afm runs the 32-site
half-filled ring with Neel and UHF references; --mode exc the
exchange-correlation energy E_xc(N, M) of the 66-electron gas in 123 plane
waves with mu fixed at the coupled-cluster level.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_MFMA = 78.6e12      # MI355X dense FP64 matrix, flop/s
PEAK_HBM = 8.0e12              # MI355X HBM3E, bytes/s
# FETCH_SIZE / WRITE_SIZE summaries of the dominant GEMM family, one per workload
TRAFFIC_PROFILES = {"ueg57": os.path.join(ROOT, "profiles", "gemm128_ueg57_traffic.md"),
                    "ueg123": os.path.join(ROOT, "profiles", "gemm128_ueg123_traffic.md")}
KERNEL_SOURCE = os.path.join(ROOT, "paper_2004_01729_amd", "csrc", "kernels.hip")


GEMM_REGION = ("// ------------------------------------------------------------------ helpers",
               "// Momentum-blocked tiles")


def gemm_source_hash():
    """SHA-256 of the GEMM kernel's source (its tile mapping, the kernel and the
    tail reduce: the part of kernels.hip between the two markers)."""
    import hashlib
    src = open(KERNEL_SOURCE).read()
    a, b = src.index(GEMM_REGION[0]), src.index(GEMM_REGION[1])
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def measured_traffic(name):
    """HBM bytes per launch of the dominant GEMM family on workload `name` from
    the committed FETCH_SIZE / WRITE_SIZE summary of that workload (calibrated
    against a plain copy); None when there is no summary for the workload or
    the GEMM kernel's source has changed since the counters were taken."""
    import re
    if name not in TRAFFIC_PROFILES:
        return None
    try:
        text = open(TRAFFIC_PROFILES[name]).read()
        cur = gemm_source_hash()
    except (OSError, ValueError):
        return None
    b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+-]+)", text)
    h = re.search(r"gemm_source_sha256:\s*([0-9a-f]{64})", text)
    if not b or not h or cur != h.group(1):
        return None
    return float(b.group(1))


def workload(name):
    import ftcc_inputs as fi
    if name == "ueg57":
        s = fi.ueg_config(57, 14, 1.0, 0.5)
        cfg = dict(workload="ueg_57pw_N14_rs1_theta0.5", n_orb=57, n_tau=16, nodes_per_panel=4,
                   propagator="exponential-collocation", phases="forward+lambda+response")
        return s, dict(n_tau=16, nodes_per_panel=4, tol=1e-12), cfg
    if name == "ueg123":
        s = fi.ueg_config(123, 14, 4.0, 1.0)
        cfg = dict(workload="ueg_123pw_N14_rs4_theta1_thr1e-6", n_orb=123, n_tau=16, nodes_per_panel=4,
                   propagator="exponential-collocation", phases="forward+lambda+response", checkpoint=1)
        return s, dict(n_tau=16, nodes_per_panel=4, tol=1e-12, occ_thresh=1e-6, checkpoint=1), cfg
    if name == "hubbard6":
        s = fi.hubbard_config(L=6, U=4.0, T=1.0)
        cfg = dict(workload="hubbard_L6_U4_T1", n_orb=6, n_tau=20, nodes_per_panel=4,
                   propagator="exponential-collocation", phases="forward+lambda+response")
        return s, dict(n_tau=20, nodes_per_panel=4, tol=1e-12), cfg
    if name == "hubbard10":
        s = fi.hubbard_config(L=10, U=8.0, T=1.0)
        cfg = dict(workload="hubbard_L10_U8_T1", n_orb=10, n_tau=40, nodes_per_panel=4,
                   propagator="exponential-collocation", phases="forward+lambda+response")
        return s, dict(n_tau=40, nodes_per_panel=4, tol=1e-12), cfg
    raise SystemExit(f"unknown workload {name}")


def step(ctx, s, times=None):
    t0 = time.perf_counter()
    ctx.solve(s.mu, s.beta)
    ctx.grand_potential()
    st0 = ctx.stats()
    t1 = time.perf_counter()
    ctx.lam()
    st1 = ctx.stats()
    ctx.response(want_mu=True, want_beta=True, want_h=True)
    t2 = time.perf_counter()
    if times is not None:
        times["forward"] += t1 - t0
        times["gradient"] += t2 - t1
    return st0, st1


def residual_throughput(ctx, reps, n_tau):
    """Back-to-back residual evaluations of every node of the last panel (the
    converged amplitudes the solve left there), between HIP events."""
    sec, fl = ctx.time_residual(reps)
    m = ctx.opt.nodes_per_panel
    plan = ctx.plan_info()
    # one pass of the slot program evaluates `slots` nodes; algorithmic bytes per node evaluation
    by = plan["bytes_forward"] / plan["slots"]
    return dict(evals_per_s=reps * m / sec, ms_per_eval=1e3 * sec / (reps * m),
                gemm_tflops=fl * reps / sec / 1e12, frac_fp64_mfma=fl * reps / sec / PEAK_FP64_MFMA,
                gemm_flop_per_eval=fl / m, algorithmic_bytes_per_eval=by,
                achieved_gbps=by * reps * m / sec / 1e9, frac_hbm=by * reps * m / sec / PEAK_HBM,
                dispatches_per_forward_pass=plan["dispatches_forward"],
                dispatches_per_backward_pass=plan["dispatches_backward"], slots=plan["slots"])


def vendor_gemm(reps):
    """For comparison only: the vendor library's float64 GEMM (torch.matmul) on
    plain square products of the GEMM sizes of the 57- and 123-plane-wave
    residuals (n^2 = 3249 and 15129), A as stored and transposed, timed with
    events around `reps` back-to-back calls after one warm-up call."""
    import torch
    out = {}
    for n in (3249, 15129):
        a = torch.randn(n, n, dtype=torch.float64, device="cuda")
        b = torch.randn_like(a)
        c = torch.empty_like(a)
        for trans in ("NN", "TN"):
            x = a.t() if trans == "TN" else a
            torch.matmul(x, b, out=c)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                torch.matmul(x, b, out=c)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            tf = 2.0 * n ** 3 / ms / 1e9
            out[f"{n}_{trans}"] = dict(ms=ms, tflops=tf, frac_fp64_mfma=tf * 1e12 / PEAK_FP64_MFMA)
        del a, b, c
        torch.cuda.empty_cache()
    return dict(mode="vendor_gemm", reps=reps, **out)


def copy_calibration(reps, nbytes=1 << 30):
    """Plain device-to-device copies of known size: what FETCH_SIZE / WRITE_SIZE
    read for exactly nbytes read and nbytes written per launch."""
    import torch
    x = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return dict(mode="copy", bytes_read_per_launch=nbytes, bytes_written_per_launch=nbytes, launches=reps,
                gbps=2 * nbytes * reps / el / 1e9)


def batch_bench(per_instance, group=32, momentum=False, subset="all", diis=0):
    """One step (forward + Lambda + response for mu, beta, h) of the mixed batch,
    batched in contexts of `group` instances (electron-gas and ring instances
    interleaved) and optionally per instance, each context timed after a first,
    untimed solve that builds it (reported as setup_and_first_solve_s)."""
    import ftcc_inputs as fi
    from paper_2004_01729_amd import ftcc as F
    systems = []
    for kind, kw in fi.batched_configs(0):
        if kind == "ueg":
            systems.append(fi.ueg_config(kw["n_pw"], 14, kw["rs"], kw["theta"]))
        else:
            systems.append(fi.hubbard_config(L=kw["L"], U=kw["U"], T=kw["T"]))
    opts = dict(n_tau=20, nodes_per_panel=4, occ_thresh=1e-6, tol=1e-12, max_iter=200, diis_depth=diis)

    def run(sys_, fd=False):
        ctx = F.Context(len(sys_), **opts)
        for i, s in enumerate(sys_):
            if momentum:
                ctx.set_momentum(i, *s.momentum)
            ctx.set_hamiltonian(i, s.h, s.eri, s.eps)
        mus, betas = [s.mu for s in sys_], [s.beta for s in sys_]
        # the first solve builds the context (launch plans, momentum tables, autotuning,
        # graph capture): timed apart, as a context is reused across solves
        ts = time.perf_counter()
        ctx.solve(mus, betas, raise_on_status=False)
        setup = time.perf_counter() - ts
        t0 = time.perf_counter()
        _, st = ctx.solve(mus, betas, raise_on_status=False)
        ctx.grand_potential()
        evals = ctx.stats()["resid_evals"]
        t1 = time.perf_counter()
        ctx.lam(raise_on_status=False)
        ctx.response(want_mu=True, want_beta=True, want_h=True)
        t2 = time.perf_counter()
        out = dict(forward_s=t1 - t0, gradient_s=t2 - t1, total_s=t2 - t0, forward_resid_evals=evals,
                   setup_and_first_solve_s=setup, failed=[i for i, v in enumerate(st.tolist()) if v != 0])
        if fd:   # central differences of Omega in mu and beta: four more forward solves, measured
            d = 1e-4
            t3 = time.perf_counter()
            for dm, db in ((d, 0.0), (-d, 0.0), (0.0, d), (0.0, -d)):
                ctx.solve([m + dm for m in mus], [b + db * b for b in betas], raise_on_status=False)
                ctx.grand_potential()
            out["fd_mu_beta_s"] = time.perf_counter() - t3
        ctx.close()
        return out

    # interleave the two families so that every context mixes large and small instances
    order = [i for pair in zip(range(16), range(16, 32)) for i in pair]
    if subset == "rings":
        order = list(range(16, 32))
    groups = [order[k:k + group] for k in range(0, len(order), group)]
    rows = [run([systems[i] for i in g]) for g in groups]
    batched = {k: sum(r[k] for r in rows)
               for k in ("forward_s", "gradient_s", "total_s", "forward_resid_evals", "setup_and_first_solve_s")}
    batched["failed"] = sorted(g[j] for g, r in zip(groups, rows) for j in r["failed"])
    batched["contexts"] = len(groups)
    wl = "batch32_ueg57pw_x16_hubbard_L6-14_x16" if subset == "all" else "batch16_hubbard_L6-14_x16"
    out = dict(mode="batch", workload=wl, n_instances=len(order),
               n_tau=20, occ_thresh=1e-6, group=group, momentum_blocked=momentum, diis_depth=diis,
               batched=batched)
    if per_instance:
        rows = [run([systems[i]], fd=True) for i in order]
        out["per_instance"] = {k: sum(r[k] for r in rows)
                               for k in ("forward_s", "gradient_s", "total_s", "fd_mu_beta_s",
                                         "setup_and_first_solve_s")}
        out["per_instance"]["failed"] = [order[i] for i, r in enumerate(rows) if r["failed"]]
        out["batched_speedup"] = out["per_instance"]["total_s"] / out["batched"]["total_s"]
        # the batched adjoint form (one context: forward, Lambda, response for mu, beta and every h_pq)
        # against plain per-instance forward solves with central finite differences in mu and beta
        # (1 + 4 forward solves per instance, every one measured)
        pi = out["per_instance"]
        out["per_instance_forward_plus_fd_s"] = pi["forward_s"] + pi["fd_mu_beta_s"]
        out["batched_adjoint_vs_per_instance_fd_speedup"] = (pi["forward_s"] + pi["fd_mu_beta_s"]) / \
            out["batched"]["total_s"]
    return out


def numerr_bench(momentum=True, grids=(20, 40, 80, 160, 320), rk1_extra=(640, 1280)):
    """Grid-error orders of Table tab:numerr with the paper's protocol: the
    14-electron electron gas in 33 plane waves, r_s = 4, Theta = 0.125, occupation
    threshold 1e-6; for every method -- the implicit integral form generated by
    Simpson's rule and the explicit RK1 / RK2 / RK4 with Simpson's quadrature --
    and every n_g the chemical potential is fixed separately so that
    <N> = -dOmega/dmu = 14 (to 1e-8; the paper uses 1e-4), then the internal
    energy E = Omega + beta dOmega/dbeta + mu N and the entropy
    S = beta^2 dOmega/dbeta are compared with the same quantities of the
    exponential-collocation integral form on 16 panels of 6 nodes at its own
    fixed N (checked against 8 panels).  E_xc = E - E_0(mu_0) and
    S_xc = S - S_0(mu_0) differ from E and S by method-independent constants, so
    these are their errors; observed orders log2(err(n) / err(2n)).  RK1 is run
    to 1280 points to reach its asymptotic order."""
    import math
    import ftcc_inputs as fi
    from paper_2004_01729_amd import ftcc as F
    s = fi.ueg_config(33, 14, 4.0, 0.125)

    def run(**opt):
        ctx = F.Context(1, occ_thresh=1e-6, **opt)
        if momentum:
            ctx.set_momentum(0, *s.momentum)
        ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
        t0 = time.perf_counter()
        mu, n_el, its, st = ctx.find_mu(14.0, s.mu, s.beta, tol=1e-9, max_iter=30, raise_on_status=False)
        if st[0] != 0:
            ctx.close()
            return dict(status=int(st[0]), seconds=time.perf_counter() - t0)
        ctx.solve(mu[0], s.beta)
        om, _ = ctx.grand_potential()
        ctx.lam()
        r = ctx.response(want_mu=True, want_beta=True, want_h=False)
        el = time.perf_counter() - t0
        ctx.close()
        n_e = -r["mu"][0]
        dob = r["beta"][0]
        return dict(status=0, seconds=el, mu=float(mu[0]), N=float(n_e), find_mu_evaluations=int(its[0]),
                    omega=float(om[0]), E=float(om[0] + s.beta * dob + mu[0] * n_e), S=float(s.beta ** 2 * dob))

    ref = run(n_tau=96, nodes_per_panel=6, tol=1e-12, max_iter=400)
    chk = run(n_tau=48, nodes_per_panel=6, tol=1e-12, max_iter=400)
    out = dict(mode="numerr", workload="ueg_33pw_N14_rs4_theta0.125_thr1e-6_fixedN", beta=s.beta, mu_hf=s.mu,
               momentum_blocked=momentum, protocol="mu fixed per method and grid so that N = 14 to 1e-8",
               reference=ref,
               reference_check={k: chk[k] - ref[k] for k in ("mu", "E", "S") if k in chk and k in ref},
               methods={})
    for name, prop in (("simpson", 5), ("rk1", 2), ("rk2", 3), ("rk4", 4)):
        rows = []
        for n in grids + (rk1_extra if name == "rk1" else ()):
            r = run(n_tau=n, propagator=prop, tol=1e-12, max_iter=400)
            if r["status"] == 0:
                r.update({f"err_{k}": r[k] - ref[k] for k in ("E", "S", "mu")})
            rows.append(dict(n_g=n, **r))
            print(f"[numerr] {name} n_g={n} status={r['status']} {r['seconds']:.1f} s", file=sys.stderr, flush=True)
        orders = {}
        for k in ("E", "S"):
            o = []
            for a_, b_ in zip(rows, rows[1:]):
                ea, eb = a_.get(f"err_{k}"), b_.get(f"err_{k}")
                o.append(math.log2(abs(ea / eb)) if ea is not None and eb is not None and eb != 0.0 else None)
            orders[k] = o
        # the paper's Table tab:timings criterion: fewest grid points with |error of E_xc| per electron
        # below a millivolt (3.67e-5 Ha)
        ok = [r_["n_g"] for r_ in rows if r_.get("err_E") is not None and abs(r_["err_E"]) / 14.0 < 3.6749e-5]
        out["methods"][name] = dict(rows=rows, observed_orders=orders, n_g_sub_mV=min(ok) if ok else None)
    return out


def afm_bench(L=32, Us=(2.0, 4.0, 8.0), Ts=(0.25, 0.5, 1.0, 2.0), n_tau=24):
    """Broken-symmetry references of the half-filled ring (Section IV.A: 32 sites,
    Neel-state and zero-temperature UHF references, mu = U/2): per site the grand
    potential, the energy E = Omega + beta dOmega/dbeta + mu N, the entropy
    S = beta^2 dOmega/dbeta and the staggered magnetisation of the response
    density dOmega/dh (frozen orbitals), in spin orbitals with S_z-blocked
    contractions; 24 tau points (6 panels x 4)."""
    import numpy as np
    import ftcc_inputs as fi
    from paper_2004_01729_amd import ftcc as F
    rows = []
    for ref in ("neel", "uhf"):
        for U in Us:
            for T in Ts:
                s = fi.hubbard_unrestricted(L=L, U=U, T=T, reference=ref)
                ctx = F.Context(1, spin_orbital=1, n_tau=n_tau, nodes_per_panel=4, tol=1e-11, max_iter=300)
                ctx.set_momentum(0, *s.momentum)
                ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
                t0 = time.perf_counter()
                _, st = ctx.solve(s.mu, s.beta, raise_on_status=False)
                row = dict(reference=ref, U=U, T=T, status=int(st[0]))
                if st[0] == 0:
                    om, _ = ctx.grand_potential()
                    _, st2 = ctx.lam(raise_on_status=False)
                    r = ctx.response(want_mu=True, want_beta=True, want_h=True)
                    n_el = -r["mu"][0]
                    C = s.meta["C"]
                    d = np.diag(C @ r["h"][0] @ C.T)
                    sign = np.array([(-1.0) ** i for i in range(L)])
                    row.update(status=int(st2[0]), omega_per_site=float(om[0]) / L, N_per_site=float(n_el) / L,
                               E_per_site=float(om[0] + s.beta * r["beta"][0] + s.mu * n_el) / L,
                               S_per_site=float(s.beta ** 2 * r["beta"][0]) / L,
                               m_staggered=float(sign @ (d[:L] - d[L:])) / L)
                row["seconds"] = time.perf_counter() - t0
                ctx.close()
                rows.append(row)
                print(f"[afm] {ref} U={U:g} T={T:g} status={row['status']} {row['seconds']:.1f} s",
                      file=sys.stderr, flush=True)
    return dict(mode="afm", workload=f"hubbard_ring_L{L}_half_filling_spin_orbitals", n_spin_orbitals=2 * L,
                n_tau=n_tau, rows=rows)


def exc_bench(n_el=66, n_pw=123, rss=(1.0, 2.0, 4.0), theta=0.5):
    """Exchange-correlation energy of the unpolarised gas at fixed N (the
    appendix on the UEG basis-set error):
        E_xc(N, M) = E_CC(mu_CC) + E_0(mu_CC) - E_0(mu_0) = E(mu_CC) - E_0(mu_0),
    E(mu) = Omega + beta dOmega/dbeta + mu N the FT-CCSD internal energy (thermal
    HF reference, frozen), mu_CC from ftcc_find_mu so that -dOmega/dmu = N, and
    E_0 the ideal-gas kinetic energy in the same M plane waves at the mu_0 that
    holds N electrons.  Momentum-blocked, 16 tau points, occupation threshold 1e-6."""
    import numpy as np
    import ftcc_inputs as fi
    from paper_2004_01729_amd import ftcc as F
    rows = []
    for rs in rss:
        s = fi.ueg_config(n_pw, n_el, rs, theta)
        t0 = time.perf_counter()
        ctx = F.Context(1, n_tau=16, nodes_per_panel=4, tol=1e-11, occ_thresh=1e-6, checkpoint=1)
        ctx.set_momentum(0, *s.momentum)
        ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
        mu, n_cc, its, st = ctx.find_mu(n_el, s.mu, s.beta, tol=1e-8, max_iter=20, raise_on_status=False)
        row = dict(rs=rs, theta=theta, beta=s.beta, mu_hf=s.mu, status=int(st[0]), find_mu_evaluations=int(its[0]))
        if st[0] == 0:
            ctx.solve(mu[0], s.beta)
            om, _ = ctx.grand_potential()
            ctx.lam()
            r = ctx.response(want_mu=True, want_beta=True, want_h=False)
            n_e = -r["mu"][0]
            e_cc = float(om[0] + s.beta * r["beta"][0] + mu[0] * n_e)
            # ideal gas in the same basis: kinetic energies k^2/2 (the diagonal of h)
            ek = np.diag(s.h)
            def n_of(m):
                return 2.0 * float(np.sum(1.0 / (1.0 + np.exp(np.clip(s.beta * (ek - m), -700, 700)))))
            lo, hi = ek.min() - 50.0 / s.beta, ek.max() + 50.0 / s.beta
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                lo, hi = (mid, hi) if n_of(mid) < n_el else (lo, mid)
            mu0 = 0.5 * (lo + hi)
            occ0 = 1.0 / (1.0 + np.exp(np.clip(s.beta * (ek - mu0), -700, 700)))
            e0 = float(2.0 * np.sum(ek * occ0))
            row.update(mu_cc=float(mu[0]), N=float(n_e), E=e_cc, mu_0=mu0, E_0=e0,
                       E_xc_per_electron=(e_cc - e0) / n_el, rs_E_xc_per_electron=rs * (e_cc - e0) / n_el)
        ctx.close()
        row["seconds"] = time.perf_counter() - t0
        rows.append(row)
        print(f"[exc] rs={rs:g} theta={theta:g} status={row['status']} {row['seconds']:.1f} s", file=sys.stderr,
              flush=True)
    return dict(mode="exc", workload=f"ueg_N{n_el}_{n_pw}pw_theta{theta:g}_thr1e-6", rows=rows)


def cpu_baseline(s, budget_s=20.0):
    """The oracle as it stands (spin-summed restricted kernels, numpy/BLAS on
    the host) on a bounded sample: the einsum items of one residual evaluation
    at this workload's shape are run in their fixed order until `budget_s`
    seconds have passed; the full-residual time is extrapolated by the share of
    the einsum flops completed (numpy's own path cost model)."""
    import numpy as np
    import ftcc_inputs as fi
    from oracle import restricted as R
    from oracle import terms as T
    from oracle.einsum import einsum
    model = R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, s.mu, s.beta))
    t1, t2 = fi.random_amplitudes(s.n, seed=5, scale=0.02)
    amps = (t1, t2)
    items = []
    for which in ("E", "S1", "S2"):
        out = T.OUT[which]
        for c, ops, axes in R.expanded(which):
            spec = ",".join(sub for _, sub in ops) + "->" + out
            vals = [model._operand(op, sub, amps, model.ints) for op, sub in ops]
            flops = float(np.einsum_path(spec, *vals, optimize="greedy")[1].split("Optimized FLOP count:")[1]
                          .split("\n")[0].strip())
            items.append((spec, vals, flops))
    total = sum(f for _, _, f in items)
    done = 0.0
    t0 = time.perf_counter()
    k = 0
    for spec, vals, fl in items:
        einsum(spec, *vals)
        done += fl
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    est = el * total / max(done, 1.0)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.environ.get("OPENBLAS_NUM_THREADS", os.cpu_count() or 1)))
    threads = min(threads, os.cpu_count() or threads)
    return dict(value=1.0 / est, unit="tau-point residual evals/s", cores=threads, kind="oracle",
                cpu_model=cpu_model(), blas="numpy einsum -> OpenBLAS dgemm (FP64)",
                sample=f"first {k} of {len(items)} spatial einsum items of one residual evaluation at n={s.n} "
                       f"({100.0 * done / total:.1f}% of its flops) in {el:.1f} s; full-residual time "
                       f"extrapolated to {est:.1f} s")


def step_bench(args, measure_fd_beta=False):
    """Whole steps (thermal set-up, forward march, Lambda, response for mu, beta,
    h) of one workload; the GEMM roofline from per-launch events of the timed
    steps (the profiler runs the launch lists eagerly).  The adjoint gradient is
    set against central finite differences of Omega in mu (and beta), each
    measured as two forward solves."""
    import torch
    from paper_2004_01729_amd import ftcc as F
    s, opts, cfg = workload(args.workload)
    ctx = F.Context(1, **opts)
    if args.momentum:
        ctx.set_momentum(0, *s.momentum)
        cfg = dict(cfg, momentum_blocked=True)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    for _ in range(args.warmup):
        step(ctx, s)
    torch.cuda.synchronize()

    evals = 0
    vjps = 0
    times = dict(forward=0.0, gradient=0.0)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st0, st1 = step(ctx, s, times)
        evals += st0["resid_evals"]
        vjps += st1["vjp_evals"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # the dominant GEMM family's launches, timed by per-launch HIP events in one
    # further step (the recording runs the launch lists eagerly, not as graphs)
    ctx.kernel_profile(1)
    step(ctx, s)
    prof = ctx.kernel_profile(0)
    # forward re-evaluations inside the adjoint and response phases: one per node
    n_tau = opts["n_tau"]
    evals += args.steps * 2 * n_tau

    om, parts = ctx.grand_potential()
    resp = ctx.response(want_mu=True, want_beta=True, want_h=False)
    m1 = residual_throughput(ctx, 3, n_tau)
    # gradient of Omega: adjoint (Lambda + response, all of dOmega/dmu, dbeta, dh_pq)
    # against central finite differences, which cost two forward solves per parameter
    t_fwd = times["forward"] / args.steps
    t_grad = times["gradient"] / args.steps
    d = 1e-4
    tf0 = time.perf_counter()
    ctx.solve(s.mu + d, s.beta)
    op = ctx.grand_potential()[0][0]
    ctx.solve(s.mu - d, s.beta)
    om_ = ctx.grand_potential()[0][0]
    t_fd_mu = time.perf_counter() - tf0
    fd_mu = (op - om_) / (2 * d)
    # Richardson-extrapolated difference (accuracy check only; not in the FD timing)
    ctx.solve(s.mu + d / 2, s.beta)
    oph = ctx.grand_potential()[0][0]
    ctx.solve(s.mu - d / 2, s.beta)
    omh = ctx.grand_potential()[0][0]
    fd_mu_rich = (4.0 * (oph - omh) / d - fd_mu) / 3.0
    n_h = s.n * (s.n + 1) // 2
    gradient = dict(adjoint_s=t_grad, forward_s=t_fwd, fd_mu_measured_s=t_fd_mu,
                    n_params_all=2 + n_h,
                    dOmega_dmu_adjoint=float(resp["mu"][0]), dOmega_dmu_fd=float(fd_mu),
                    fd_rel_diff=abs(fd_mu - resp["mu"][0]) / max(1.0, abs(resp["mu"][0])),
                    dOmega_dmu_fd_richardson=float(fd_mu_rich),
                    fd_richardson_rel_diff=abs(fd_mu_rich - resp["mu"][0]) / max(1.0, abs(resp["mu"][0])))
    if measure_fd_beta:
        db = 1e-4 * s.beta
        tb0 = time.perf_counter()
        ctx.solve(s.mu, s.beta + db)
        bp = ctx.grand_potential()[0][0]
        ctx.solve(s.mu, s.beta - db)
        bm = ctx.grand_potential()[0][0]
        t_fd_beta = time.perf_counter() - tb0
        fd_beta = (bp - bm) / (2 * db)
        gradient.update(fd_beta_measured_s=t_fd_beta, fd_mu_beta_measured_s=t_fd_mu + t_fd_beta,
                        adjoint_vs_fd_speedup_mu_beta=(t_fd_mu + t_fd_beta) / t_grad,
                        dOmega_dbeta_adjoint=float(resp["beta"][0]), dOmega_dbeta_fd=float(fd_beta),
                        fd_beta_rel_diff=abs(fd_beta - resp["beta"][0]) / max(1.0, abs(resp["beta"][0])),
                        fd_all_params_s_extrapolated=(2 + n_h) * t_fd_mu,
                        adjoint_vs_fd_speedup_all_extrapolated=(2 + n_h) * t_fd_mu / t_grad)
    else:
        gradient.update(adjoint_vs_fd_speedup_mu_beta_extrapolated=2 * t_fd_mu / t_grad)
    value = evals / el
    achieved = prof["flops"] / prof["seconds"] if prof["seconds"] > 0 else 0.0
    roofline = {
        "bound": "mfma",
        "achieved": achieved / 1e12,
        "peak": PEAK_FP64_MFMA / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP64_MFMA,
        "traffic": measured_traffic(args.workload) if not args.momentum else None,
        "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "kernel": "gemm_mfma_kernel<128,128,16,*,*> (FP64 MFMA 16x16x4)",
        "launches": prof["launches"],
        "avg_launch_ms": 1e3 * prof["seconds"] / max(prof["launches"], 1),
        "flop_per_launch": prof["flops"] / max(prof["launches"], 1),
    } if prof["launches"] > 0 else None
    line = {
        "metric": "tau-point T2 residual evals/s",
        "value": value,
        "unit": "residual evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": dict(cfg, residual_evals_per_step=evals / args.steps, vjp_evals_per_step=vjps / args.steps,
                       omega=float(om[0]), omega_cc=float(parts[0, 2]), dOmega_dmu=float(resp["mu"][0]),
                       dOmega_dbeta=float(resp["beta"][0]), gradient_vs_fd=gradient,
                       residual_throughput=m1),
        "roofline": roofline,
    }
    ctx.close()
    return line


def gradient_once(args):
    """One forward march, Lambda and response (mu, beta, every h_pq) of a workload
    in a fresh context, each phase timed once: the full-size adjoint as a run,
    not a throughput (dense or momentum-blocked)."""
    import numpy as np
    import torch
    from paper_2004_01729_amd import ftcc as F
    s, opts, cfg = workload(args.workload)
    if args.n_tau:
        opts = dict(opts, n_tau=args.n_tau)
        cfg = dict(cfg, n_tau=args.n_tau)
    if args.tol:
        opts = dict(opts, tol=args.tol)
        cfg = dict(cfg, tol=args.tol)
    t0 = time.perf_counter()
    ctx = F.Context(1, **opts)
    if args.momentum:
        ctx.set_momentum(0, *s.momentum)
        cfg = dict(cfg, momentum_blocked=True)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    ctx.solve(s.mu, s.beta)
    om, parts = ctx.grand_potential()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.lam()
    r = ctx.response(want_mu=True, want_beta=True, want_h=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    st = ctx.stats()
    ctx.close()
    h = r["h"][0]
    return dict(mode="gradient", config=cfg, forward_with_setup_s=t1 - t0, lambda_and_response_s=t2 - t1,
                resid_evals=st["resid_evals"], vjp_evals=st["vjp_evals"], omega=float(om[0]),
                omega_cc=float(parts[0, 2]), dOmega_dmu=float(r["mu"][0]), dOmega_dbeta=float(r["beta"][0]),
                dOmega_dh_trace=float(np.trace(h)), dOmega_dh_norm=float(np.linalg.norm(h)))


def cpu_model():
    try:
        for row in open("/proc/cpuinfo"):
            if row.startswith("model name"):
                return row.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def first_order_amplitudes(ctx, s):
    """s(tau) = -S0 (1 - exp(-Delta tau)) / Delta at tau = beta / 2, S0 the residual
    at zero amplitudes (the first-order solution of eqn:smu; -S0 tau where Delta = 0)."""
    import numpy as np
    n = s.n
    S1, S2, _ = ctx.eval_residual(0, s.mu, s.beta, np.zeros((n, n)), np.zeros((n,) * 4))
    tau = 0.5 * s.beta
    e = s.eps

    def prop(d):
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(np.abs(d) > 1e-12, -np.expm1(-d * tau) / np.where(d == 0.0, 1.0, d), tau)

    t1 = -S1 * prop(e[None, :] - e[:, None])
    d2 = e[None, None, :, None] + e[None, None, None, :] - e[:, None, None, None] - e[None, :, None, None]
    t2 = -S2 * prop(d2)
    return t1, t2


def progress(msg):
    """One progress line on stderr (long phases report as they end)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def m1_bench(args):
    """The default line: residual evaluations per second at the 123-plane-wave
    workload (see the module docstring)."""
    import torch
    from paper_2004_01729_amd import ftcc as F
    s, opts, cfg = workload("ueg123")
    t_setup = time.perf_counter()
    ctx = F.Context(1, **opts)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    t1, t2 = first_order_amplitudes(ctx, s)
    S1, S2, E = ctx.eval_residual(0, s.mu, s.beta, t1, t2)     # puts t into every node slot
    del S2
    t_setup = time.perf_counter() - t_setup
    progress(f"m1: context built and first-order amplitudes set in {t_setup:.1f} s")
    m = opts["nodes_per_panel"]
    for _ in range(args.warmup):
        ctx.time_residual(1)
    torch.cuda.synchronize()
    progress(f"m1: {args.warmup} warm-up steps done; timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.time_residual(1)          # the m node residuals of a panel, replayed graph
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    progress(f"m1: {args.steps} timed steps in {el:.1f} s")
    _, flop_sweep = ctx.time_residual(1)
    # per-launch HIP events on the dominant GEMM family (eager launches of the same lists)
    ctx.kernel_profile(1)
    prof_steps = 2
    for _ in range(prof_steps):
        ctx.time_residual(1)
    prof = ctx.kernel_profile(0)
    ctx.close()
    progress("m1: profiled pass done; the momentum-blocked evaluation of the same residual next")
    blocked = blocked_m1(s, opts, t1, t2, float(E), args.steps, args.warmup)
    evals = args.steps * m
    achieved = prof["flops"] / prof["seconds"] if prof["seconds"] > 0 else 0.0
    roofline = {
        "bound": "mfma",
        "achieved": achieved / 1e12,
        "peak": PEAK_FP64_MFMA / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP64_MFMA,
        "traffic": measured_traffic("ueg123"),
        "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "kernel": "gemm_mfma_kernel<128,128,16,*,*> (FP64 MFMA 16x16x4)",
        "launches": prof["launches"],
        "avg_launch_ms": 1e3 * prof["seconds"] / max(prof["launches"], 1),
        "flop_per_launch": prof["flops"] / max(prof["launches"], 1),
        "timing": f"per-launch HIP events on the library stream over {prof_steps} further steps "
                  "(eager launches of the timed graph's lists)",
    } if prof["launches"] > 0 else None
    line = {
        "metric": "tau-point T2 residual evals/s",
        "value": evals / el,
        "unit": "residual evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": dict(cfg, phases="T1/T2 residual (M1)", residual_evals_per_step=m,
                       amplitudes="first-order s(beta/2)", context_setup_s=t_setup,
                       gemm_flop_per_eval=flop_sweep / m,
                       step_gemm_tflops=flop_sweep * args.steps / el / 1e12,
                       step_frac_fp64_mfma=flop_sweep * args.steps / el / PEAK_FP64_MFMA,
                       E_first_order=float(E), momentum_blocked_same_residual=blocked),
        "roofline": roofline,
    }
    return line, s


def blocked_m1(s, opts, t1, t2, e_dense, steps, warmup):
    """The same residual at the same amplitudes through the momentum-blocked path
    (crystal momentum of the plane waves set on the instance; packed blocked
    storage, four node slots): throughput, the energy against the dense path's,
    and the algorithmic bytes against the HBM peak."""
    import torch
    from paper_2004_01729_amd import ftcc as F
    t0 = time.perf_counter()
    ctx = F.Context(1, **opts)
    ctx.set_momentum(0, *s.momentum)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    _, _, e_b = ctx.eval_residual(0, s.mu, s.beta, t1, t2)
    setup = time.perf_counter() - t0
    for _ in range(warmup):
        ctx.time_residual(1)
    torch.cuda.synchronize()
    reps = max(steps, 1) * 20
    sec, fl = ctx.time_residual(reps)
    plan = ctx.plan_info()
    ctx.close()
    m = opts["nodes_per_panel"]
    by = plan["bytes_forward"] / plan["slots"]
    return dict(evals_per_s=reps * m / sec, ms_per_eval=1e3 * sec / (reps * m), reps=reps,
                E_first_order=float(e_b), E_rel_diff_vs_dense=abs(float(e_b) - e_dense) / abs(e_dense),
                blocked_flop_per_eval=fl / m, algorithmic_bytes_per_eval=by,
                achieved_gbps=by * reps * m / sec / 1e9, frac_hbm=by * reps * m / sec / PEAK_HBM,
                dispatches_per_forward_pass=plan["dispatches_forward"], slots=plan["slots"], context_setup_s=setup)


def secondary_57(steps=1, warmup=1):
    """The 57-plane-wave gas through the whole path and the adjoint gradient
    against measured central differences (secondary fields of the default line)."""
    ns = argparse.Namespace(workload="ueg57", momentum=False, steps=steps, warmup=warmup)
    line = step_bench(ns, measure_fd_beta=True)
    keep = ("value", "ms_per_step", "roofline")
    out = {k: line[k] for k in keep}
    out.update(line["config"])
    out["value_unit"] = "residual evals/s of whole-step wall time"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ueg57")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--mode", default="m1",
                    choices=("m1", "step", "residual", "copy", "vendor_gemm", "batch", "numerr", "afm", "exc",
                             "gradient"))
    ap.add_argument("--n-tau", type=int, default=0,
                    help="--mode gradient / residual: tau nodes (0: the workload's)")
    ap.add_argument("--tol", type=float, default=0.0, help="--mode gradient: sweep tolerance (0: the workload's)")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--per-instance", action="store_true")
    ap.add_argument("--group", type=int, default=32, help="--mode batch: instances per context")
    ap.add_argument("--subset", default="all", choices=("all", "rings"))
    ap.add_argument("--momentum", action="store_true")
    ap.add_argument("--dense", action="store_true", help="--mode numerr: dense contractions")
    ap.add_argument("--diis", type=int, default=0, help="--mode batch: DIIS depth of the fixed-point sweeps")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; there is no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2004_01729_amd import ftcc as F

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if args.mode == "copy":
        print(json.dumps(copy_calibration(args.reps)), flush=True)
        return
    if args.mode == "vendor_gemm":
        print(json.dumps(vendor_gemm(args.reps)), flush=True)
        return
    if args.mode == "exc":
        print(json.dumps(exc_bench()), flush=True)
        return
    if args.mode == "afm":
        print(json.dumps(afm_bench()), flush=True)
        return
    if args.mode == "numerr":
        print(json.dumps(numerr_bench(momentum=not args.dense)), flush=True)
        return
    if args.mode == "gradient":
        print(json.dumps(gradient_once(args)), flush=True)
        return
    if args.mode == "batch":
        print(json.dumps(batch_bench(args.per_instance, args.group, args.momentum, args.subset, args.diis)),
              flush=True)
        return
    if args.mode == "residual":
        s, opts, cfg = workload(args.workload)
        if args.n_tau > 0:   # a shorter grid (whole panels): the march of its first panels only
            opts = dict(opts, n_tau=args.n_tau)
            cfg = dict(cfg, n_tau=args.n_tau)
        ctx = F.Context(1, **opts)
        if args.momentum:
            ctx.set_momentum(0, *s.momentum)
        ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
        ctx.solve(s.mu, s.beta)
        progress(f"residual: march of {opts['n_tau']} tau nodes done")
        r = residual_throughput(ctx, args.reps, opts["n_tau"])
        ctx.close()
        print(json.dumps(dict(mode="residual", workload=cfg["workload"], n_tau=opts["n_tau"], reps=args.reps, **r)),
              flush=True)
        return
    if args.mode == "step":
        line = step_bench(args)
        s = workload(args.workload)[0]
    else:
        line, s = m1_bench(args)
        print(f"[bench] m1 done: {line['value']:.3f} residual evals/s", file=sys.stderr, flush=True)
        if not args.no_secondary:
            line["config"]["secondary"] = secondary_57()
            print("[bench] secondary (57 PW whole path) done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(s)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
