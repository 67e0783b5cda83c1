"""The spin-orbital oracle with broken-symmetry references (Section IV.A:
Neel state and zero-temperature UHF for the half-filled ring), pinned by
grand-canonical exact diagonalisation (independent of any reference): FT-CCSD
recovers the correlation that the mean-field Omega_0 + Omega_1 misses by
orders of magnitude, with an error that falls like a high power of U; the
amplitudes keep the exact structure (antisymmetry, S_z conservation)."""
import math

import numpy as np
import pytest

import ftcc_inputs as fi
from oracle import ed, grid as G, solver as S, spinorb as so


def _model(s):
    return so.SpinOrbitalModel(so.ThermalIntegrals(s.h, s.eri, s.eps, s.mu, s.beta))


def test_uhf_reference_is_self_consistent():
    """Zero-temperature UHF: the Fock matrix built from the L/2 lowest orbitals of
    each spin is diagonal in those orbitals with the returned energies, and the
    densities alternate (broken spin symmetry)."""
    s = fi.hubbard_unrestricted(L=6, U=4.0, T=1.0, reference="uhf")
    L = 6
    n0 = np.concatenate([np.r_[np.ones(L // 2), np.zeros(L - L // 2)]] * 2)
    vas = s.eri - s.eri.transpose(0, 1, 3, 2)
    f = s.h + np.einsum("prqr,r->pq", vas, n0)
    assert np.abs(f - np.diag(s.eps)).max() < 1e-10
    dens = np.diag(s.meta["C"] @ np.diag(n0) @ s.meta["C"].T)
    m = dens[:L] - dens[L:]
    assert np.all(np.abs(np.abs(m) - abs(m[0])) < 1e-10) and abs(m[0]) > 0.3
    assert np.all(m[::2] * m[1::2] < 0)


@pytest.mark.parametrize("ref", ["neel", "uhf"])
def test_broken_symmetry_reference_against_exact_diagonalisation(ref):
    errs, mfs = [], []
    Us = (0.5, 1.0)
    for U in Us:
        s = fi.hubbard_unrestricted(L=4, U=U, T=1.0, reference=ref)
        hs, es = fi.hubbard_site_basis(4, 1.0, U)
        exact = ed.grand_potential(np.kron(np.eye(2), hs), es, s.mu, s.beta)
        sol = S.solve(_model(s), G.Grid(s.beta, 4, 4), tol=1e-13)
        errs.append(abs(sol.omega - exact))
        mfs.append(abs(sol.omega0 + sol.omega1 - exact))
    assert errs[0] < 2e-5 and errs[0] < 1e-3 * mfs[0]
    assert math.log(errs[1] / errs[0]) / math.log(Us[1] / Us[0]) > 3.5


def test_amplitude_structure():
    s = fi.hubbard_unrestricted(L=4, U=4.0, T=1.0, reference="neel")
    sol = S.solve(_model(s), G.Grid(s.beta, 2, 4), tol=1e-13)
    spin = s.momentum[0][:, 0]
    forbid2 = (spin[:, None, None, None] + spin[None, :, None, None]
               - spin[None, None, :, None] - spin[None, None, None, :]) != 0
    forbid1 = spin[:, None] != spin[None, :]
    for t1, t2 in sol.nodes:
        assert np.abs(t2 + t2.transpose(1, 0, 2, 3)).max() < 1e-13
        assert np.abs(t2 + t2.transpose(0, 1, 3, 2)).max() < 1e-13
        assert np.abs(t2[forbid2]).max() == 0.0 and np.abs(t1[forbid1]).max() == 0.0
