"""10-site Hubbard ring, U = 8, mu = U/2, T in {1, 2}: 40 tau nodes (10 panels
x 4), occupation threshold 1e-6, both temperatures in one batched context.

Omega against the oracle values in tests/golden/hubbard10_u8.json (written by
make_hubbard10.py from the oracle alone); dOmega/dmu and dOmega/dU from the
Lambda adjoint against the oracle's discrete adjoint and against central finite
differences of the GPU's own Omega (step 1e-4, Richardson-extrapolated with
step 5e-5) at a frozen reference (orbitals and eps fixed).

At T <= 0.5 the march of the discrete equations has no finite continuation
for this U with a restricted reference: the oracle's own march diverges at
T = 0.5 (plain, damped, four times finer panels, DIIS; pinned in
tests/test_oracle_limits.py), and the GPU must report the instance as failed
(FTCC_EDIVERGE, FTCC_ENONFINITE or, when the sweeps neither settle nor grow
steadily, FTCC_ENOCONV) with a NaN Omega, which the last test checks
at T = 0.5, 0.25 and 0.1."""
import json
import os

import numpy as np
import pytest

import ftcc_inputs as fi

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hubbard10_u8.json")


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_01729_amd import ftcc
    return ftcc


def _ctx(F, g, systems, eri_scale=1.0):
    ctx = F.Context(len(systems), n_tau=g["n_panels"] * g["m"], nodes_per_panel=g["m"], occ_thresh=g["thr"],
                    tol=1e-13)
    for i, s in enumerate(systems):
        ctx.set_hamiltonian(i, s.h, s.eri * eri_scale, s.eps)
    return ctx


def _omega(F, g, systems, dmu=0.0, eri_scale=1.0):
    ctx = _ctx(F, g, systems, eri_scale)
    ctx.solve([s.mu + dmu for s in systems], [s.beta for s in systems])
    om = ctx.grand_potential()[0]
    ctx.close()
    return om


def _richardson(f, h):
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * d2 - d1) / 3


def test_hubbard10_u8_omega_and_gradients(F):
    g = json.load(open(GOLDEN))
    U = g["U"]
    systems = [fi.hubbard_config(L=g["L"], U=U, T=c["T"]) for c in g["cases"]]
    print("[hubbard10] L=10 U=8 T=" + ",".join(str(c["T"]) for c in g["cases"]) + " n_tau=40 thr=1e-6 batched",
          flush=True)
    ctx = _ctx(F, g, systems)
    its, st = ctx.solve([s.mu for s in systems], [s.beta for s in systems])
    om, parts = ctx.grand_potential()
    ctx.lam()
    r = ctx.response(want_mu=True, want_beta=False, want_h=False, deri_dtheta=[s.eri / U for s in systems])
    ctx.close()
    for i, c in enumerate(g["cases"]):
        assert abs(om[i] - c["omega"]) < 1e-10 * abs(c["omega"])
        assert abs(parts[i, 2] - c["omega_cc"]) < 1e-10 * abs(c["omega_cc"])
        assert abs(r["mu"][i] - c["dOmega_dmu"]) < 1e-8 * max(1.0, abs(c["dOmega_dmu"]))
        assert abs(r["theta"][i] - c["dOmega_dU"]) < 1e-8 * max(1.0, abs(c["dOmega_dU"]))
    print("[hubbard10] finite differences", flush=True)
    fd_mu = _richardson(lambda d: _omega(F, g, systems, dmu=d), 1e-4)
    fd_U = _richardson(lambda d: _omega(F, g, systems, eri_scale=(U + d) / U), 1e-4)
    for i in range(len(systems)):
        assert abs(fd_mu[i] - r["mu"][i]) < 1e-7 * max(1.0, abs(r["mu"][i]))
        assert abs(fd_U[i] - r["theta"][i]) < 1e-7 * max(1.0, abs(r["theta"][i]))


def test_hubbard10_u8_low_temperature_reports_failure(F):
    """T = 0.5, 0.25, 0.1 in one batch: every instance fails in its own status
    slot (the oracle's march diverges too) and the call returns promptly (at
    T = 0.5 and 0.1 through the divergence test, at T = 0.25 at max_iter)."""
    import time
    g = json.load(open(GOLDEN))
    systems = [fi.hubbard_config(L=g["L"], U=g["U"], T=T) for T in (0.5, 0.25, 0.1)]
    print("[hubbard10] L=10 U=8 T=0.5,0.25,0.1 n_tau=40 thr=1e-6: expected to fail", flush=True)
    ctx = _ctx(F, g, systems)
    t0 = time.perf_counter()
    _, st = ctx.solve([s.mu for s in systems], [s.beta for s in systems], raise_on_status=False)
    om, _ = ctx.grand_potential()
    ctx.close()
    assert all(int(v) in (F.EDIVERGE, F.ENONFINITE, F.ENOCONV) for v in st), st
    assert np.all(np.isnan(om))
    assert time.perf_counter() - t0 < 60.0
