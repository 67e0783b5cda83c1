"""The largest workload shape, the 123-plane-wave gas (n = 123, N = 14,
r_s = 4, Theta = 1; t2 is 1.83 GB), where no oracle evaluation fits a test:
properties that hold at any size.  One residual evaluation at momentum-
conserving random amplitudes by the dense FP64-MFMA path and by the momentum-
blocked path (two different algorithms for the same equations) agree element
by element; the dense residual has the structure the equations fix (momentum-
forbidden elements zero, S2[ijab] = S2[jiba])."""
import numpy as np
import pytest

import ftcc_inputs as fi

pytestmark = pytest.mark.gpu


def test_residual_n123_dense_equals_blocked():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_01729_amd import ftcc as F
    s = fi.ueg_config(123, 14, 4.0, 1.0)
    n = s.n
    lab = np.asarray(s.momentum[0])
    base = 4 * int(np.abs(lab).max()) + 1
    code = lambda v: (v[..., 0] * base + v[..., 1]) * base + v[..., 2]
    pair = code(lab[:, None, :] + lab[None, :, :])                 # k_i + k_j
    allowed2 = pair[:, :, None, None] == pair[None, None, :, :]
    allowed1 = code(lab)[:, None] == code(lab)[None, :]
    rng = np.random.default_rng(11)
    t1 = rng.standard_normal((n, n)) * 0.02 * allowed1
    t2 = rng.standard_normal((n,) * 4) * 0.02
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    t2 *= allowed2
    out = []
    for blocked in (False, True):
        print(f"[fullsize123] residual n=123 seed=11 blocked={blocked}", flush=True)
        ctx = F.Context(1, n_tau=4, nodes_per_panel=4, occ_thresh=1e-6)
        if blocked:
            ctx.set_momentum(0, *s.momentum)
        ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
        out.append(ctx.eval_residual(0, s.mu, s.beta, t1, t2))
        ctx.close()
    (d1, d2, de), (b1, b2, be) = out
    scale2 = max(1.0, np.abs(d2).max())
    assert np.abs(d1 - b1).max() < 1e-12 * max(1.0, np.abs(d1).max())
    assert np.abs(d2 - b2).max() < 1e-12 * scale2
    assert abs(de - be) < 1e-12 * max(1.0, abs(de))
    assert np.abs(d2[~allowed2]).max() < 1e-14 * scale2 and np.all(b2[~allowed2] == 0.0)
    assert np.abs(d2 - d2.transpose(1, 0, 3, 2)).max() < 1e-13 * scale2


def test_full_configuration_context_fits():
    """The 123-plane-wave context at the workload's full configuration (16 tau
    nodes in 4 panels, checkpointing, occupation threshold 1e-6: about 278 GiB of
    device memory, one executor slot, the permuted-operand caches stopped short
    of a reserve) builds within HBM and evaluates the same residual as a
    4-node context."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_01729_amd import ftcc as F
    s = fi.ueg_config(123, 14, 4.0, 1.0)
    n = s.n
    lab = np.asarray(s.momentum[0])
    base = 4 * int(np.abs(lab).max()) + 1
    code = lambda v: (v[..., 0] * base + v[..., 1]) * base + v[..., 2]
    pair = code(lab[:, None, :] + lab[None, :, :])
    allowed2 = pair[:, :, None, None] == pair[None, None, :, :]
    allowed1 = code(lab)[:, None] == code(lab)[None, :]
    rng = np.random.default_rng(12)
    t1 = rng.standard_normal((n, n)) * 0.02 * allowed1
    t2 = rng.standard_normal((n,) * 4) * 0.02
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    t2 *= allowed2
    out = []
    for n_tau, extra in ((16, dict(checkpoint=1)), (4, {})):
        print(f"[fullsize123] dense context n=123 n_tau={n_tau} {extra}", flush=True)
        ctx = F.Context(1, n_tau=n_tau, nodes_per_panel=4, occ_thresh=1e-6, tol=1e-12, **extra)
        ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
        out.append(ctx.eval_residual(0, s.mu, s.beta, t1, t2))
        ctx.close()
    (a1, a2, ae), (b1, b2, be) = out
    assert np.abs(a1 - b1).max() < 1e-12 * max(1.0, np.abs(b1).max())
    assert np.abs(a2 - b2).max() < 1e-12 * max(1.0, np.abs(b2).max())
    assert abs(ae - be) < 1e-12 * max(1.0, abs(be))


def test_residual_n123_against_oracle_rows():
    """The dense 123-plane-wave residual in the context the benchmark times (16
    tau nodes in 4 panels, checkpointing, occupation threshold 1e-6) against the
    oracle's values at seeded dense random amplitudes (written by
    tests/golden/make_ueg123.py): E, all of S1, and S2 on the rows i in {0, 1, 122},
    j in {4, 5, 122} (136161 elements: both sides of the 128-row tile boundary and
    the last, ragged row)."""
    import os
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_01729_amd import ftcc as F
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "ueg123_residual.npz"))
    s = fi.ueg_config(int(g["n_pw"]), int(g["n_el"]), float(g["rs"]), float(g["theta"]))
    assert abs(s.mu - float(g["mu"])) < 1e-14 and abs(s.beta - float(g["beta"])) < 1e-14
    t1, t2 = fi.random_amplitudes(s.n, seed=int(g["seed"]), scale=float(g["scale"]))
    print("[fullsize123] residual n=123 seed=123 dense against the oracle rows", flush=True)
    ctx = F.Context(1, n_tau=16, nodes_per_panel=4, occ_thresh=float(g["thr"]), tol=1e-12, checkpoint=1)
    ctx.set_hamiltonian(0, s.h, s.eri, s.eps)
    S1, S2, E = ctx.eval_residual(0, s.mu, s.beta, t1, t2)
    ctx.close()
    I, J = g["rows_i"], g["rows_j"]
    rows = S2[np.ix_(I, J)]
    del S2
    assert abs(E - float(g["E"])) < 1e-12 * max(1.0, abs(float(g["E"])))
    assert np.abs(S1 - g["S1"]).max() < 1e-11 * max(1.0, np.abs(g["S1"]).max())
    assert np.abs(rows - g["S2_rows"]).max() < 1e-11 * max(1.0, np.abs(g["S2_rows"]).max())
