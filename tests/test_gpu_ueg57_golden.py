"""The 57-plane-wave electron gas at its workload configuration (N = 14,
r_s = 1, Theta = 0.5, thermal HF reference, 16 tau nodes as 4 panels x 4,
exponential collocation) against stored oracle values (tests/golden/
ueg57_forward.npz, written by make_ueg57.py from the oracle alone): Omega and
its parts (1e-10 relative), and the amplitudes of every node of the last panel
(t1 whole, t2 at 20000 sampled momentum-allowed elements; 1e-8 relative to
max(1, max|s|)), for the dense FP64-MFMA path, the momentum-blocked path, and
the blocked path with two rings sharing the instance's context."""
import os

import numpy as np
import pytest

import ftcc_inputs as fi

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_01729_amd import ftcc
    return ftcc


def _context(F, fw, blocked, batch=False):
    """The 57-plane-wave instance first; with batch, two rings (L = 6 and 5) share
    its context and its grouped launches."""
    s = fi.ueg_config(int(fw["n_pw"]), int(fw["n_el"]), float(fw["rs"]), float(fw["theta"]))
    assert abs(s.mu - float(fw["mu"])) < 1e-14 and abs(s.beta - float(fw["beta"])) < 1e-14
    systems = [s] + ([fi.hubbard_config(L=6, U=4.0, T=1.0), fi.hubbard_config(L=5, U=3.0, T=0.8)] if batch else [])
    P, m = int(fw["n_panels"]), int(fw["m"])
    ctx = F.Context(len(systems), n_tau=P * m, nodes_per_panel=m, tol=1e-13)
    for i, x in enumerate(systems):
        if blocked:
            ctx.set_momentum(i, *x.momentum)
        ctx.set_hamiltonian(i, x.h, x.eri, x.eps)
    ctx.solve([x.mu for x in systems], [x.beta for x in systems])
    return ctx


@pytest.mark.parametrize("blocked,batch", [(False, False), (True, False), (True, True)])
def test_ueg57_march_against_oracle(F, blocked, batch):
    fw = np.load(os.path.join(HERE, "ueg57_forward.npz"))
    print(f"[ueg57 golden] forward n=57 n_tau=16 blocked={blocked} batch={batch}", flush=True)
    ctx = _context(F, fw, blocked, batch)
    om, parts = ctx.grand_potential()
    nodes = [ctx.amplitudes(0, int(k)) for k in fw["nodes"]]
    ctx.close()
    assert abs(parts[0, 0] - float(fw["omega0"])) < 1e-12 * abs(float(fw["omega0"]))
    assert abs(parts[0, 1] - float(fw["omega1"])) < 1e-12 * max(1.0, abs(float(fw["omega1"])))
    assert abs(parts[0, 2] - float(fw["omega_cc"])) < 1e-10 * abs(float(fw["omega_cc"]))
    assert abs(om[0] - float(fw["omega"])) < 1e-10 * abs(float(fw["omega"]))
    idx = fw["t2_index"]
    scale = max(1.0, max(np.abs(t[1]).max() for t in nodes))
    for k, (t1, t2) in enumerate(nodes):
        assert np.abs(t1 - fw["t1"][k]).max() < 1e-8 * scale, k
        assert np.abs(t2.ravel()[idx] - fw["t2"][k]).max() < 1e-8 * scale, k
