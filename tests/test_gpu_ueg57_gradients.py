"""Lambda and the gradients of the 57-plane-wave electron gas (the instance of
tests/test_gpu_ueg57_golden.py) against ueg57_gradients.npz, written by
make_ueg57.py from the oracle alone: Lambda of the first and last node, and
dOmega/dmu, dOmega/dbeta, dOmega/dh (1e-8), dense and momentum-blocked."""
import os

import numpy as np
import pytest

from test_gpu_ueg57_golden import F, HERE, _context  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("blocked", [False, True])
def test_ueg57_lambda_and_gradients_against_oracle(F, blocked):
    fw = np.load(os.path.join(HERE, "ueg57_forward.npz"))
    gd = np.load(os.path.join(HERE, "ueg57_gradients.npz"))
    idx = fw["t2_index"]
    print(f"[ueg57 golden] adjoint n=57 n_tau=16 blocked={blocked}", flush=True)
    ctx = _context(F, fw, blocked)
    ctx.lam()
    lams = [ctx.get_lambda(0, int(k), tilde=False)[:2] for k in gd["lam_nodes"]]
    r = ctx.response(want_mu=True, want_beta=True, want_h=True)
    ctx.close()
    for k, (l1, l2) in enumerate(lams):
        sym = 0.5 * (l2 + l2.transpose(1, 0, 3, 2))
        lscale = max(1.0, np.abs(gd["lam2_sym"][k]).max(), np.abs(gd["lam1"][k]).max())
        assert np.abs(l1 - gd["lam1"][k]).max() < 1e-8 * lscale, k
        assert np.abs(sym.ravel()[idx] - gd["lam2_sym"][k]).max() < 1e-8 * lscale, k
    for key, ref in (("mu", float(gd["dOmega_dmu"])), ("beta", float(gd["dOmega_dbeta"]))):
        assert abs(r[key][0] - ref) < 1e-8 * max(1.0, abs(ref)), key
    assert np.abs(r["h"][0] - gd["dOmega_dh"]).max() < 1e-8 * max(1.0, np.abs(gd["dOmega_dh"]).max())
