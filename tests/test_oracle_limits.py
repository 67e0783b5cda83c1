"""Limits of the FT-CCSD oracle that textbook results fix.

P7  T -> 0 for a gapped closed-shell reference (slots with occupation below
    1e-10 dropped, which removes only exp(-beta gap) terms): the imaginary-time average
    Omega_CC(beta) = (1/beta) int_0^beta E(tau) dtau approaches the ground-state
    CCSD correlation energy as E_CCSD + C / beta (the transient of s(tau) from
    s(0) = 0 has a finite area C; thermal corrections are exp(-beta gap)), so
    two large beta fix E_CCSD, compared with a textbook zero-temperature
    spin-orbital CCSD written here from the standard Stanton-Gauss equations.
P11 the two propagators (exponential collocation, integrating factor) give the
    same grand potential exactly when every Delta vanishes, and converge to the
    same limit as the tau grid is refined.
"""
import numpy as np
import pytest

import ftcc_inputs as fi
from oracle import grid as G, restricted as R, solver as S


def _gapped_system(seed=11):
    """Four spatial orbitals, two doubly occupied, a gap of about 2.5."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((4, 4)) * 0.05
    h = np.diag([-2.0, -1.6, 1.0, 1.4]) + 0.5 * (a + a.T)
    c = rng.standard_normal((4, 4, 4, 4)) * 0.05
    c = c + c.transpose(1, 0, 2, 3)
    c = c + c.transpose(0, 1, 3, 2)
    c = c + c.transpose(2, 3, 0, 1)
    eri = np.ascontiguousarray(c.transpose(0, 2, 1, 3))      # <pq|rs> = (pr|qs), real orbitals
    nocc = 2
    f = h + 2.0 * np.einsum("prqr->pq", eri[:, :nocc, :, :nocc]) - np.einsum("prrq->pq", eri[:, :nocc, :nocc, :])
    return h, eri, f, nocc


def _ccsd_energy(h, eri, nocc, tol=1e-13, max_iter=500):
    """Zero-temperature closed-shell CCSD correlation energy in spin orbitals
    (orbital 2p + s has spatial part p and spin s), Stanton-Gauss intermediates."""
    n = h.shape[0]
    N = 2 * n
    sp = np.arange(N) // 2
    sg = np.arange(N) % 2
    H = h[np.ix_(sp, sp)] * (sg[:, None] == sg[None, :])
    g = eri[np.ix_(sp, sp, sp, sp)] * ((sg[:, None, None, None] == sg[None, None, :, None])
                                       & (sg[None, :, None, None] == sg[None, None, None, :]))
    A = g - g.transpose(0, 1, 3, 2)                            # <pq||rs>
    o = np.arange(2 * nocc)
    v = np.arange(2 * nocc, N)
    F = H + np.einsum("pmqm->pq", A[:, o][:, :, :, o])
    foo, fov, fvv = F[np.ix_(o, o)], F[np.ix_(o, v)], F[np.ix_(v, v)]
    Aoooo = A[np.ix_(o, o, o, o)]
    Aooov = A[np.ix_(o, o, o, v)]
    Aoovv = A[np.ix_(o, o, v, v)]
    Aovov = A[np.ix_(o, v, o, v)]
    Aovvo = A[np.ix_(o, v, v, o)]
    Aovvv = A[np.ix_(o, v, v, v)]
    Avvvv = A[np.ix_(v, v, v, v)]
    Avvvo = A[np.ix_(v, v, v, o)]
    Aovoo = A[np.ix_(o, v, o, o)]
    Avvoo = A[np.ix_(v, v, o, o)]
    Aoovo = A[np.ix_(o, o, v, o)]
    Dia = np.diag(foo)[:, None] - np.diag(fvv)[None, :]
    Dijab = (np.diag(foo)[:, None, None, None] + np.diag(foo)[None, :, None, None]
             - np.diag(fvv)[None, None, :, None] - np.diag(fvv)[None, None, None, :])
    t1 = fov / Dia
    t2 = Aoovv / Dijab
    fvv_off = fvv - np.diag(np.diag(fvv))
    foo_off = foo - np.diag(np.diag(foo))

    def energy(t1, t2):
        return (np.einsum("ia,ia", fov, t1) + 0.25 * np.einsum("ijab,ijab", Aoovv, t2)
                + 0.5 * np.einsum("ijab,ia,jb", Aoovv, t1, t1))

    e_old = energy(t1, t2)
    for _ in range(max_iter):
        tau_t = t2 + 0.5 * (np.einsum("ia,jb->ijab", t1, t1) - np.einsum("ib,ja->ijab", t1, t1))
        tau = t2 + np.einsum("ia,jb->ijab", t1, t1) - np.einsum("ib,ja->ijab", t1, t1)
        Fae = (fvv_off - 0.5 * np.einsum("me,ma->ae", fov, t1) + np.einsum("mf,mafe->ae", t1, Aovvv)
               - 0.5 * np.einsum("mnaf,mnef->ae", tau_t, Aoovv))
        Fmi = (foo_off + 0.5 * np.einsum("ie,me->mi", t1, fov) + np.einsum("ne,mnie->mi", t1, Aooov)
               + 0.5 * np.einsum("inef,mnef->mi", tau_t, Aoovv))
        Fme = fov + np.einsum("nf,mnef->me", t1, Aoovv)
        Wmnij = (Aoooo + np.einsum("je,mnie->mnij", t1, Aooov) - np.einsum("ie,mnje->mnij", t1, Aooov)
                 + 0.25 * np.einsum("ijef,mnef->mnij", tau, Aoovv))
        Wabef = (Avvvv - np.einsum("mb,amef->abef", t1, -Aovvv.transpose(1, 0, 2, 3))
                 + np.einsum("ma,bmef->abef", t1, -Aovvv.transpose(1, 0, 2, 3))
                 + 0.25 * np.einsum("mnab,mnef->abef", tau, Aoovv))
        Wmbej = (Aovvo + np.einsum("jf,mbef->mbej", t1, Aovvv) - np.einsum("nb,mnej->mbej", t1, Aoovo)
                 - np.einsum("jnfb,mnef->mbej", 0.5 * t2 + np.einsum("jf,nb->jnfb", t1, t1), Aoovv))
        r1 = (fov + np.einsum("ie,ae->ia", t1, Fae) - np.einsum("ma,mi->ia", t1, Fmi)
              + np.einsum("imae,me->ia", t2, Fme) - np.einsum("nf,naif->ia", t1, Aovov)
              - 0.5 * np.einsum("imef,maef->ia", t2, Aovvv) - 0.5 * np.einsum("mnae,nmei->ia", t2, Aoovo))
        Pab = np.einsum("ijae,be->ijab", t2, Fae - 0.5 * np.einsum("mb,me->be", t1, Fme))
        Pij = np.einsum("imab,mj->ijab", t2, Fmi + 0.5 * np.einsum("je,me->mj", t1, Fme))
        ring = np.einsum("imae,mbej->ijab", t2, Wmbej) - np.einsum("ie,ma,mbej->ijab", t1, t1, Aovvo)
        r2 = (Aoovv + Pab - Pab.transpose(0, 1, 3, 2) - Pij + Pij.transpose(1, 0, 2, 3)
              + 0.5 * np.einsum("mnab,mnij->ijab", tau, Wmnij) + 0.5 * np.einsum("ijef,abef->ijab", tau, Wabef)
              + ring - ring.transpose(1, 0, 2, 3) - ring.transpose(0, 1, 3, 2) + ring.transpose(1, 0, 3, 2))
        x = np.einsum("ie,abej->ijab", t1, Avvvo)
        y = np.einsum("ma,mbij->ijab", t1, Aovoo)
        r2 = r2 + x - x.transpose(1, 0, 2, 3) - y + y.transpose(0, 1, 3, 2)
        t1 = r1 / Dia
        t2 = r2 / Dijab
        e = energy(t1, t2)
        if abs(e - e_old) < tol:
            return e
        e_old = e
    raise RuntimeError("CCSD did not converge")


def test_p7_zero_temperature_limit_is_ground_state_ccsd():
    h, eri, f, nocc = _gapped_system()
    e_ccsd = _ccsd_energy(h, eri, nocc)
    eps = np.diag(f).copy()
    mu = 0.5 * (eps[nocc - 1] + eps[nocc])          # inside the gap
    om = {}
    for beta in (30.0, 60.0):
        # slots with occupation below 1e-10 dropped (Section III.A): inverted pairs would
        # otherwise grow like exp(beta |Delta| / 2) while contributing exp(-beta gap)
        model = R.RestrictedModel(R.RestrictedIntegrals(h, eri, eps, mu, beta, 1e-10))
        om[beta] = S.solve(model, G.Grid(beta, int(beta), 4), tol=1e-13).omega_cc
    # Omega_CC(beta) = E + C / beta: eliminate C
    e_limit = (60.0 * om[60.0] - 30.0 * om[30.0]) / 30.0
    assert abs(e_limit - e_ccsd) < 1e-9 * max(1.0, abs(e_ccsd))
    assert abs(om[60.0] - e_ccsd) > 1e-6               # the transient term is really there


def test_p11_propagators_agree_exactly_when_delta_vanishes():
    U, beta = 4.0, 1.0
    h = np.zeros((1, 1))
    eri = np.full((1, 1, 1, 1), U)
    eps = np.array([U / 2])
    model = R.RestrictedModel(R.RestrictedIntegrals(h, eri, eps, U / 2, beta))
    a = S.solve(model, G.Grid(beta, 3, 4, "etd"), tol=1e-14).omega_cc
    b = S.solve(model, G.Grid(beta, 3, 4, "lawson"), tol=1e-14).omega_cc
    assert abs(a - b) < 1e-14 * max(1.0, abs(a))


def test_p11_propagators_converge_to_the_same_limit():
    s = fi.hubbard_config(L=3, U=1.5, T=1.0)
    model = R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, s.mu, s.beta))
    diffs = []
    for P in (1, 2, 4):
        a = S.solve(model, G.Grid(s.beta, P, 4, "etd"), tol=1e-14).omega_cc
        b = S.solve(model, G.Grid(s.beta, P, 4, "lawson"), tol=1e-14).omega_cc
        diffs.append(abs(a - b))
    assert diffs[2] < diffs[1] < diffs[0]
    assert diffs[0] / diffs[2] > 2 ** 8                 # both at least fourth order


def test_ten_site_ring_u8_t05_march_has_no_finite_continuation():
    """The 10-site ring at U = 8, mu = U/2, T = 0.5, 40 tau nodes (10 panels x 4),
    occupation threshold 1e-6: the amplitudes grow to about 25 by the sixth panel
    and the fixed-point sweeps of that panel then blow up (the same happens with
    damping, four times finer panels and DIIS), so the discrete equations have no
    solution reachable by marching from s(0) = 0.  The GPU reports such an
    instance as failed."""
    s = fi.hubbard_config(L=10, U=8.0, T=0.5)
    model = R.RestrictedModel(R.RestrictedIntegrals(s.h, s.eri, s.eps, s.mu, s.beta, 1e-6))
    with pytest.raises((FloatingPointError, RuntimeError)):
        with np.errstate(all="ignore"):
            S.solve(model, G.Grid(s.beta, 10, 4), tol=1e-12, max_iter=200)
