"""The row-restricted residual of the oracle (used where S2 of the 123-plane-wave
gas does not fit in memory) equals the rows of the whole residual, for index
sets that do and do not overlap, in a random real-orbital Hamiltonian and in a
plane-wave gas (integrals without the real-orbital symmetry)."""
import numpy as np
import pytest

import ftcc_inputs as fi
from oracle import restricted as R


@pytest.mark.parametrize("kind", ["random", "ueg"])
def test_residual_rows_equal_whole_residual(kind):
    if kind == "random":
        h, eri, eps = fi.random_hamiltonian(6, seed=3)
        model = R.RestrictedModel(R.RestrictedIntegrals(h, eri, eps, 0.1, 2.0))
    else:
        s = fi.ueg_config(19, 14, 1.0, 0.5)
        model = R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, s.mu, s.beta))
    n = model.n
    t = fi.random_amplitudes(n, seed=4, scale=0.1)
    S1, S2 = model.residual(t)
    for I, J in (([0, 2], [1, 2, n - 1]), ([n - 1], [n - 1]), (list(range(n)), [3])):
        r1, r2 = model.residual_rows(t, I, J)
        assert np.abs(r1 - S1).max() < 1e-13 * max(1.0, np.abs(S1).max())
        assert r2.shape == (len(I), len(J), n, n)
        assert np.abs(r2 - S2[np.ix_(I, J)]).max() < 1e-13 * max(1.0, np.abs(S2).max())
