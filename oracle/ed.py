"""Grand-canonical exact diagonalisation (thermal FCI) for small spin-orbital spaces.

TEST INFRASTRUCTURE ONLY (see the package docstring).

H = sum_pq h_pq a_p^+ a_q + 1/2 sum_pqrs <pq|rs> a_p^+ a_q^+ a_s a_r on the
full Fock space of n_so <= 12 spin orbitals;
Omega = -(1/beta) ln Tr exp(-beta (H - mu N)).
"""
from __future__ import annotations

import numpy as np
from scipy.special import logsumexp


def _apply_annihilate(state, p):
    if not (state >> p) & 1:
        return None, 0
    sign = -1 if bin(state & ((1 << p) - 1)).count("1") % 2 else 1
    return state ^ (1 << p), sign


def _apply_create(state, p):
    if (state >> p) & 1:
        return None, 0
    sign = -1 if bin(state & ((1 << p) - 1)).count("1") % 2 else 1
    return state | (1 << p), sign


def hamiltonian(h, eri, tol=0.0):
    n = h.shape[0]
    dim = 1 << n
    H = np.zeros((dim, dim))
    nz1 = [(p, q, h[p, q]) for p in range(n) for q in range(n) if abs(h[p, q]) > tol]
    idx = np.argwhere(np.abs(eri) > tol)
    for st in range(dim):
        for p, q, v in nz1:
            s1, g1 = _apply_annihilate(st, q)
            if s1 is None:
                continue
            s2, g2 = _apply_create(s1, p)
            if s2 is None:
                continue
            H[s2, st] += v * g1 * g2
        for p, q, r, s in idx:
            a1, g1 = _apply_annihilate(st, r)
            if a1 is None:
                continue
            a2, g2 = _apply_annihilate(a1, s)
            if a2 is None:
                continue
            c1, g3 = _apply_create(a2, q)
            if c1 is None:
                continue
            c2, g4 = _apply_create(c1, p)
            if c2 is None:
                continue
            H[c2, st] += 0.5 * eri[p, q, r, s] * g1 * g2 * g3 * g4
    return H


def grand_potential(h, eri, mu, beta):
    """Exact Omega for spin-orbital (h, <pq|rs>)."""
    n = h.shape[0]
    H = hamiltonian(h, eri)
    num = np.array([bin(s).count("1") for s in range(1 << n)], dtype=float)
    H = H - mu * np.diag(num)
    w = np.linalg.eigvalsh(0.5 * (H + H.T))
    return -logsumexp(-beta * w) / beta
