"""Seeded synthetic Hamiltonians and thermal mean-field references.

This module only produces inputs: one-body matrices h, two-electron integrals
<pq|rs> (physicist order, spatial orbitals), reference orbital energies eps,
the chemical potential mu and the inverse temperature beta.  It holds none of
the coupled-cluster arithmetic; both the FP64 oracle and the HIP path take its
output as plain arrays.

Systems (paper, Section IV and Appendix D):
  * the periodic one-dimensional Hubbard ring (Section IV.A), written in the
    Bloch basis where the restricted thermal Hartree-Fock reference is diagonal;
  * the uniform electron gas in a cubic box of plane waves (Section IV.B),
    Coulomb kernel 4 pi / (V q^2) with q = 0 excluded.

The reference orbital energies are the diagonal of the finite-temperature Fock
matrix (Section II.B: the reference energies must be stated).  In both systems
translation symmetry makes the Fock matrix diagonal in the given basis.

Integral convention: eri[p, q, r, s] = <pq|rs> = int phi_p*(1) phi_q*(2)
r12^-1 phi_r(1) phi_s(2).  The arrays are real and satisfy the particle
exchange symmetry <pq|rs> = <qp|sr> and hermiticity <pq|rs> = <rs|pq>; they
do NOT in general satisfy the real-orbital symmetry <pq|rs> = <rq|ps>
(plane waves and Bloch waves are complex).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import expit

__all__ = [
    "System", "hubbard_ring", "ueg_plane_waves", "ueg_shell_basis",
    "restricted_thermal_hf", "hubbard_config", "ueg_config", "batched_configs",
    "random_amplitudes", "random_hamiltonian", "hubbard_site_basis", "hubbard_unrestricted",
    "antisymmetric_amplitudes", "momentum_masks", "momentum_allowed_amplitudes",
]


@dataclasses.dataclass
class System:
    """A restricted (spin-unpolarised) system in a spatial orbital basis."""
    name: str
    h: np.ndarray          # (n, n) one-body matrix
    eri: np.ndarray        # (n, n, n, n) <pq|rs>
    eps: np.ndarray        # (n,) reference orbital energies
    mu: float
    beta: float
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.h.shape[0]

    @property
    def momentum(self):
        """(labels (n, dims) int array, modulus per component, 0 = none) of the
        conserved crystal momentum, or None when the basis carries none."""
        if "momentum_labels" not in self.meta:
            return None
        return self.meta["momentum_labels"], self.meta["momentum_modulus"]


# ---------------------------------------------------------------- Hubbard ring
def hubbard_ring(L: int, t: float, U: float):
    """Periodic 1D Hubbard ring in the Bloch basis k_m = 2 pi m / L.

    Hopping -t sum_i (a_i^+ a_{i+1} + h.c.) with i+1 taken mod L (so for L = 2
    the single bond is counted twice), and on-site U n_up n_dn.  In the Bloch
    basis h_kk = -2 t cos k and <k1 k2|k3 k4> = (U/L) delta(k1+k2 = k3+k4 mod L).
    """
    m = np.arange(L)
    k = 2.0 * np.pi * m / L
    h = np.diag(-2.0 * t * np.cos(k))
    tot12 = (m[:, None] + m[None, :]) % L
    eri = (tot12[:, :, None, None] == tot12[None, None, :, :]).astype(np.float64) * (U / L)
    return h, eri


# ---------------------------------------------------------- electron gas basis
def ueg_shell_basis(n_pw: int) -> np.ndarray:
    """Integer wave vectors of the n_pw lowest plane waves of a cubic box.

    The basis must close a shell of |n|^2 (57 = |n|^2 <= 5, 123 = |n|^2 <= 9).
    Ordered by |n|^2, then lexicographically, so that the ordering is
    reproducible.
    """
    nmax = int(math.isqrt(4 * n_pw)) + 2
    r = np.arange(-nmax, nmax + 1)
    g = np.array(np.meshgrid(r, r, r, indexing="ij")).reshape(3, -1).T
    n2 = (g * g).sum(1)
    order = np.lexsort((g[:, 2], g[:, 1], g[:, 0], n2))
    g, n2 = g[order], n2[order]
    if n_pw > len(g) or (n_pw < len(g) and n2[n_pw - 1] == n2[n_pw]):
        raise ValueError(f"{n_pw} plane waves do not close a |n|^2 shell")
    return g[:n_pw]


def ueg_plane_waves(n_el: int, rs: float, n_pw: int):
    """Uniform electron gas: h = k^2/2, <pq|rs> = 4 pi/(V |k_p-k_r|^2) when
    k_p + k_q = k_r + k_s and k_p != k_r (the q = 0 term is excluded; the
    Madelung constant is a constant shift and is omitted)."""
    g = ueg_shell_basis(n_pw)
    box = (n_el * 4.0 * np.pi * rs ** 3 / 3.0) ** (1.0 / 3.0)
    vol = box ** 3
    kvec = 2.0 * np.pi / box * g.astype(np.float64)
    h = np.diag(0.5 * (kvec * kvec).sum(1))
    # momentum transfer q = k_p - k_r and conservation k_p + k_q = k_r + k_s
    dpr = g[:, None, :] - g[None, :, :]                    # (p, r)
    dsq = g[None, :, :] - g[:, None, :]                    # (q, s) -> k_s - k_q
    q2 = (2.0 * np.pi / box) ** 2 * (dpr * dpr).sum(-1).astype(np.float64)
    with np.errstate(divide="ignore"):
        vq = np.where(q2 > 0, 4.0 * np.pi / (vol * np.where(q2 > 0, q2, 1.0)), 0.0)
    # cons[p, r, q, s] = (k_p - k_r) == (k_s - k_q); vectors encoded as integers
    off, base = 4 * int(np.abs(g).max()) + 1, 8 * int(np.abs(g).max()) + 3
    enc = lambda d: ((d[..., 0] + off) * base + (d[..., 1] + off)) * base + (d[..., 2] + off)
    cons = enc(dpr)[:, :, None, None] == enc(dsq)[None, None, :, :]
    eri_prqs = cons * vq[:, :, None, None]
    eri = np.ascontiguousarray(eri_prqs.transpose(0, 2, 1, 3))   # -> (p, q, r, s)
    return h, eri, dict(box=box, volume=vol, kvec=kvec)


# ----------------------------------------------- restricted thermal mean field
def _fock_diag(h, eri, occ):
    """Diagonal of the restricted Fock matrix f_pp = h_pp + sum_r (2<pr|pr> - <pr|rp>) n_r."""
    idx = np.arange(h.shape[0])
    direct = eri[idx[:, None], idx[None, :], idx[:, None], idx[None, :]]   # <pr|pr>
    exch = eri[idx[:, None], idx[None, :], idx[None, :], idx[:, None]]     # <pr|rp>
    return np.diag(h) + (2.0 * direct - exch) @ occ


def _fermi(eps, mu, beta):
    return expit(-beta * (eps - mu))


def _mu_for_count(eps, beta, n_el):
    lo, hi = eps.min() - 50.0 / beta - 1.0, eps.max() + 50.0 / beta + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if 2.0 * _fermi(eps, mid, beta).sum() < n_el:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def restricted_thermal_hf(h, eri, beta, mu=None, n_el=None, tol=1e-14, max_iter=2000):
    """Self-consistent restricted thermal HF orbital energies in a basis where the
    Fock matrix is diagonal by symmetry.  Either mu is fixed, or it is adjusted
    so that the reference holds n_el electrons (2 sum_p n_p = n_el)."""
    eps = np.diag(h).copy()
    m = mu
    for _ in range(max_iter):
        if n_el is not None:
            m = _mu_for_count(eps, beta, n_el)
        occ = _fermi(eps, m, beta)
        new = _fock_diag(h, eri, occ)
        if np.max(np.abs(new - eps)) < tol:
            eps = new
            break
        eps = 0.5 * eps + 0.5 * new
    if n_el is not None:
        m = _mu_for_count(eps, beta, n_el)
    return eps, m


# ------------------------------------------------------------ named workloads
def hubbard_config(L=6, t=1.0, U=4.0, T=1.0, mu=None):
    """Half-filled Hubbard ring (mu = U/2 unless given) with the restricted thermal
    HF reference at the same temperature."""
    beta = 1.0 / T
    mu = U / 2.0 if mu is None else mu
    h, eri = hubbard_ring(L, t, U)
    eps, _ = restricted_thermal_hf(h, eri, beta, mu=mu)
    return System(f"hubbard_L{L}_U{U:g}_T{T:g}", h, eri, eps, mu, beta,
                  dict(L=L, t=t, U=U, T=T, momentum_labels=np.arange(L).reshape(L, 1),
                       momentum_modulus=[L]))


def ueg_config(n_pw=57, n_el=14, rs=1.0, theta=0.5):
    """Unpolarised UEG: T = theta * T_F with k_F = (9 pi / 4)^(1/3) / r_s and a
    thermal HF reference whose mu gives 2 sum n = n_el."""
    kf = (9.0 * np.pi / 4.0) ** (1.0 / 3.0) / rs
    T = theta * 0.5 * kf * kf
    beta = 1.0 / T
    h, eri, geo = ueg_plane_waves(n_el, rs, n_pw)
    eps, mu = restricted_thermal_hf(h, eri, beta, n_el=n_el)
    return System(f"ueg_{n_pw}pw_rs{rs:g}_theta{theta:g}", h, eri, eps, mu, beta,
                  dict(n_pw=n_pw, n_el=n_el, rs=rs, theta=theta, T=T,
                       momentum_labels=ueg_shell_basis(n_pw).astype(np.int64), momentum_modulus=[0, 0, 0],
                       **{k: v for k, v in geo.items() if k != "kvec"}))


def batched_configs(seed=0, n_pw=57):
    """Mixed batch: 16 UEG points (r_s x theta grid) and 16 Hubbard chains with
    L = 6 + (i mod 9), U ~ U[1, 8], T ~ U[0.1, 2] drawn from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for rs in (0.5, 1.0, 2.0, 4.0):
        for th in (0.25, 0.5, 1.0, 2.0):
            out.append(("ueg", dict(n_pw=n_pw, rs=rs, theta=th)))
    for i in range(16):
        U = float(rng.uniform(1.0, 8.0))
        T = float(rng.uniform(0.1, 2.0))
        out.append(("hubbard", dict(L=6 + (i % 9), U=U, T=T)))
    return out


# ------------------------------------------- unrestricted (spin-orbital) rings
def hubbard_site_basis(L: int, t: float, U: float):
    """Periodic ring in the site basis: hopping matrix h (L x L) and the
    spin-orbital on-site interaction.  Spin orbitals are ordered (alpha sites,
    beta sites); <p q|r s> = U when p, r are one site with one spin and q, s the
    same site with the other spin (U n_up n_dn), zero otherwise."""
    h = np.zeros((L, L))
    for i in range(L):
        h[i, (i + 1) % L] += -t
        h[(i + 1) % L, i] += -t
    N = 2 * L
    eri = np.zeros((N, N, N, N))
    for i in range(L):
        a, b = i, L + i
        eri[a, b, a, b] = U
        eri[b, a, b, a] = U
    return h, eri


def _rotate_spin_orbital(h_site, eri_site, Ca, Cb):
    """Spin-orbital h and <pq|rs> in the orbitals C_alpha, C_beta (columns)."""
    L = h_site.shape[0]
    C = np.zeros((2 * L, 2 * L))
    C[:L, :L] = Ca
    C[L:, L:] = Cb
    hs = np.kron(np.eye(2), h_site)
    h = C.T @ hs @ C
    eri = np.einsum("pqrs,pa,qb,rc,sd->abcd", eri_site, C, C, C, C, optimize=True)
    return h, eri, C


def hubbard_unrestricted(L=4, t=1.0, U=4.0, T=1.0, reference="uhf", mu=None, tol=1e-12, max_iter=5000):
    """Half-filled periodic ring with a broken-spin-symmetry reference (Section IV.A:
    Neel state or zero-temperature UHF; in both the reference energies are the
    diagonal of the zero-temperature Fock matrix).

    reference="neel": site orbitals, alpha electrons on even sites and beta on odd
    ones, eps_{i sigma} = U n_{i, -sigma}.  reference="uhf": the zero-temperature
    unrestricted Hartree-Fock orbitals with L/2 electrons of each spin (iterated
    from the Neel density), eps = their orbital energies.  Returns a spin-orbital
    System (n = 2L) whose meta holds the orbital coefficients `C` (site-spin x
    orbital), spin labels for the conservation of S_z and the sites."""
    beta = 1.0 / T
    mu = U / 2.0 if mu is None else mu
    hsite, esite = hubbard_site_basis(L, t, U)
    na = np.array([1.0 if i % 2 == 0 else 0.0 for i in range(L)])
    nb = 1.0 - na
    if reference == "neel":
        Ca = Cb = np.eye(L)
        eps_a, eps_b = U * nb, U * na
    elif reference == "uhf":
        for _ in range(max_iter):
            ea, Ca = np.linalg.eigh(hsite + np.diag(U * nb))
            eb, Cb = np.linalg.eigh(hsite + np.diag(U * na))
            new_a = (Ca[:, :L // 2] ** 2).sum(1)
            new_b = (Cb[:, :L // 2] ** 2).sum(1)
            if max(np.abs(new_a - na).max(), np.abs(new_b - nb).max()) < tol:
                break
            na, nb = 0.5 * (na + new_a), 0.5 * (nb + new_b)
        eps_a, eps_b = ea, eb
    else:
        raise ValueError(reference)
    h, eri, C = _rotate_spin_orbital(hsite, esite, Ca, Cb)
    eps = np.concatenate([eps_a, eps_b])
    spin = np.concatenate([np.zeros(L, int), np.ones(L, int)]).reshape(-1, 1)
    return System(f"hubbard_L{L}_U{U:g}_T{T:g}_{reference}", h, eri, eps, mu, beta,
                  dict(L=L, t=t, U=U, T=T, reference=reference, C=C,
                       momentum_labels=spin, momentum_modulus=[0]))


def antisymmetric_amplitudes(n, seed=0, scale=0.05):
    """Random spin-orbital amplitudes with t2 antisymmetric in (i, j) and (a, b)."""
    rng = np.random.default_rng(seed)
    t1 = rng.standard_normal((n, n)) * scale
    t2 = rng.standard_normal((n, n, n, n)) * scale
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    return t1, 0.5 * t2


# ------------------------------------------------------------ random tensors
def random_hamiltonian(n, seed=0, scale=0.1):
    """Random real Hamiltonian with the symmetries of real orbitals: h symmetric,
    <pq|rs> symmetric under p<->r, q<->s, (pr)<->(qs).  Orbital energies are the
    diagonal of h plus a random shift, so the reference is not Hartree-Fock."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n)) * scale
    h = 0.5 * (a + a.T) + np.diag(np.sort(rng.uniform(-1.0, 1.0, n)))
    c = rng.standard_normal((n, n, n, n)) * scale          # chemist (pr|qs) raw
    c = c + c.transpose(1, 0, 2, 3)
    c = c + c.transpose(0, 1, 3, 2)
    c = c + c.transpose(2, 3, 0, 1)
    eri = np.ascontiguousarray(c.transpose(0, 2, 1, 3))    # <pq|rs> = (pr|qs)
    eps = np.diag(h) + rng.uniform(-0.05, 0.05, n)
    return h, eri, eps


def random_amplitudes(n, seed=0, scale=0.05):
    """Random restricted amplitudes with T2[i,j,a,b] = T2[j,i,b,a]."""
    rng = np.random.default_rng(seed)
    t1 = rng.standard_normal((n, n)) * scale
    t2 = rng.standard_normal((n, n, n, n)) * scale
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    return t1, t2


def momentum_masks(labels):
    """Boolean masks of the t1 and t2 elements that crystal-momentum labels
    (one integer vector per orbital, no wrap-around) allow: k_i = k_a, and
    k_i + k_j = k_a + k_b."""
    lab = np.asarray(labels, dtype=np.int64)
    base = 4 * int(np.abs(lab).max()) + 1
    code = (lab[:, 0] * base + lab[:, 1]) * base + lab[:, 2]
    pair = code[:, None] + code[None, :]
    return code[:, None] == code[None, :], pair[:, :, None, None] == pair[None, None, :, :]


def momentum_allowed_amplitudes(labels, seed=0, scale=0.05):
    """random_amplitudes(len(labels), seed, scale) with every element that the
    momentum labels forbid set to zero."""
    m1, m2 = momentum_masks(labels)
    t1, t2 = random_amplitudes(len(labels), seed=seed, scale=scale)
    return t1 * m1, t2 * m2
