"""The seeded input generators that feed both the oracle and the GPU path:
the momentum masks of the electron-gas amplitudes against a brute-force loop
over the plane-wave labels, and the masked random amplitudes' structure."""
import itertools

import numpy as np

import ftcc_inputs as fi


def test_momentum_masks_match_brute_force():
    lab = fi.ueg_shell_basis(19)
    n = len(lab)
    m1, m2 = fi.momentum_masks(lab)
    for i, a in itertools.product(range(n), repeat=2):
        assert m1[i, a] == bool(np.all(lab[i] == lab[a]))
    for i, j, a, b in itertools.product(range(n), repeat=4):
        assert m2[i, j, a, b] == bool(np.all(lab[i] + lab[j] == lab[a] + lab[b]))
    assert m1.sum() == n                      # distinct labels: k_i = k_a only on the diagonal
    assert m2.sum() < n ** 4 // 4


def test_momentum_allowed_amplitudes_structure():
    lab = fi.ueg_shell_basis(19)
    t1, t2 = fi.momentum_allowed_amplitudes(lab, seed=3, scale=0.02)
    m1, m2 = fi.momentum_masks(lab)
    r1, r2 = fi.random_amplitudes(len(lab), seed=3, scale=0.02)
    assert np.array_equal(t1, r1 * m1) and np.array_equal(t2, r2 * m2)
    assert np.all(t2[~m2] == 0.0) and np.count_nonzero(t2[m2]) == m2.sum()
    assert np.array_equal(t2, t2.transpose(1, 0, 3, 2))
