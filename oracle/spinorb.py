"""Spin-orbital FT-CCSD oracle (plain FP64 NumPy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Appendix A of the paper:
  * occupation numbers n_p = 1 / (1 + exp(beta (eps_p - mu))), the symmetric
    split sqrt(n_p) for hole slots and sqrt(1 - n_p) for particle slots
    (Section II.A, Appendix A);
  * occupation threshold (Section III.A): a hole slot is kept when n_p > thr,
    a particle slot when 1 - n_p > thr; dropped slots get weight zero;
  * thermal one-body integrals f_pq = weights * (<p|f|q> - delta_pq eps_p) with
    the finite-temperature Fock operator <p|f|q> = h_pq + sum_r <pr||qr> n_r.
    The orbital-energy subtraction is applied in all four blocks (oo, ov, vo,
    vv); the paper prints it only for oo and vv (reading documented in the
    design notes);
  * thermal antisymmetrised integrals <pq||rs> = weights * (<pq|rs> - <pq|sr>);
  * the kernels E, S1, S2 of eqn:E, eqn:ccS1, eqn:ccS2 (see terms.py).

Mean-field parts (not written out in the paper; standard definitions):
  Omega_0   = -(1/beta) sum_p ln(1 + exp(-beta (eps_p - mu)))
  Omega_1   = sum_p (h_pp - eps_p) n_p + 1/2 sum_pq <pq||pq> n_p n_q
whose derivative d Omega_1 / d n_q = <q|f|q> - eps_q is the expression of
Appendix B.
"""
from __future__ import annotations

import numpy as np
from scipy.special import expit

from . import terms as T
from .einsum import einsum as _einsum


def spin_orbital_from_spatial(h, eri, eps):
    """Spatial restricted inputs -> spin orbitals ordered (alpha block, beta block)."""
    n = h.shape[0]
    h_so = np.kron(np.eye(2), h)
    eps_so = np.concatenate([eps, eps])
    eri_so = np.zeros((2 * n,) * 4)
    for s1 in range(2):
        for s2 in range(2):
            eri_so[s1 * n:(s1 + 1) * n, s2 * n:(s2 + 1) * n,
                   s1 * n:(s1 + 1) * n, s2 * n:(s2 + 1) * n] = eri
    return h_so, eri_so, eps_so


def occupations(eps, mu, beta):
    """n_p and 1 - n_p, each evaluated directly as a logistic (no cancellation)."""
    x = beta * (np.asarray(eps) - mu)
    return expit(-x), expit(x)


class ThermalIntegrals:
    """Thermal integral blocks for given (h, <pq|rs>, eps, mu, beta, thr)."""

    def __init__(self, h, eri, eps, mu, beta, thr=0.0):
        self.h, self.eri, self.eps = np.asarray(h, float), np.asarray(eri, float), np.asarray(eps, float)
        self.mu, self.beta, self.thr = float(mu), float(beta), float(thr)
        self.n_occ, self.n_vir = occupations(self.eps, self.mu, self.beta)
        self.keep_h = self.n_occ > self.thr
        self.keep_p = self.n_vir > self.thr
        self.wh = np.where(self.keep_h, np.sqrt(self.n_occ), 0.0)
        self.wp = np.where(self.keep_p, np.sqrt(self.n_vir), 0.0)
        self.vas = self.eri - self.eri.transpose(0, 1, 3, 2)            # <pq||rs>
        self.fock = self.h + _einsum("prqr,r->pq", self.vas, self.n_occ)
        self.u = self.fock - np.diag(self.eps)
        self._cache = {}

    def weight(self, kind):
        return self.wh if kind == "o" else self.wp

    def get(self, name, letters):
        pat = T.slot_pattern(letters)
        key = (name, pat)
        if key not in self._cache:
            base = self.u if name == "F" else self.vas
            arr = base
            for axis, kind in enumerate(pat):
                shape = [1] * len(pat)
                shape[axis] = -1
                arr = arr * self.weight(kind).reshape(shape)
            self._cache[key] = arr
        return self._cache[key]

    def derivative(self, dn=None, dh=None, deri=None):
        """Integrals d/d theta of every block, at frozen eps and frozen index sets.

        dn: d n_p / d theta (occupation response); dh, deri: explicit one-body
        and two-electron derivatives.  Returns an object with the same get().
        """
        return _DerivIntegrals(self, dn, dh, deri)


class _DerivIntegrals:
    def __init__(self, base: ThermalIntegrals, dn, dh, deri):
        self.b = base
        n = base.eps.size
        dn = np.zeros(n) if dn is None else np.asarray(dn, float)
        self.dn = dn
        # d sqrt(n) = dn / (2 sqrt n); d sqrt(1-n) = -dn / (2 sqrt(1-n)); zero where dropped
        with np.errstate(divide="ignore", invalid="ignore"):
            self.dwh = np.where(base.keep_h & (base.wh > 0), dn / (2.0 * np.where(base.wh > 0, base.wh, 1.0)), 0.0)
            self.dwp = np.where(base.keep_p & (base.wp > 0), -dn / (2.0 * np.where(base.wp > 0, base.wp, 1.0)), 0.0)
        dvas = np.zeros_like(base.vas) if deri is None else (deri - deri.transpose(0, 1, 3, 2))
        dfock = _einsum("prqr,r->pq", base.vas, dn) + _einsum("prqr,r->pq", dvas, base.n_occ)
        if dh is not None:
            dfock = dfock + dh
        self.du, self.dvas = dfock, dvas
        self._cache = {}

    def get(self, name, letters):
        pat = T.slot_pattern(letters)
        key = (name, pat)
        if key in self._cache:
            return self._cache[key]
        b = self.b
        base, dbase = (b.u, self.du) if name == "F" else (b.vas, self.dvas)
        ws = [b.weight(k) for k in pat]
        dws = [self.dwh if k == "o" else self.dwp for k in pat]

        def scaled(arr, vecs):
            for axis, v in enumerate(vecs):
                shape = [1] * len(pat)
                shape[axis] = -1
                arr = arr * v.reshape(shape)
            return arr

        out = scaled(dbase, ws)
        for k in range(len(pat)):
            vecs = list(ws)
            vecs[k] = dws[k]
            out = out + scaled(base, vecs)
        self._cache[key] = out
        return out


def antisym(x, perm):
    if perm == "":
        return x
    if "ij" in perm:
        x = x - x.transpose(1, 0, 2, 3)
    if "ab" in perm:
        x = x - x.transpose(0, 1, 3, 2)
    return x


class SpinOrbitalModel:
    """E, S and their vector-Jacobian products on spin-orbital amplitudes."""

    def __init__(self, ints: ThermalIntegrals):
        self.ints = ints
        eps = ints.eps
        self.n = eps.size
        self.delta1 = eps[None, :] - eps[:, None]                                   # s1[i, a]
        self.delta2 = (eps[None, None, :, None] + eps[None, None, None, :]
                       - eps[:, None, None, None] - eps[None, :, None, None])    # s2[i, j, a, b]

    # -- amplitudes ---------------------------------------------------------
    def zeros(self):
        n = self.n
        return np.zeros((n, n)), np.zeros((n, n, n, n))

    def _operand(self, name, letters, s, ints):
        if name == "s1":
            return s[0]
        if name == "s2":
            return s[1]
        return ints.get(name, letters)

    def _kernel(self, which, s, ints):
        out = T.OUT[which]
        shape = () if which == "E" else ((self.n,) * len(out))
        acc = np.zeros(shape)
        for coef, perm, factors in T.TERMS[which]:
            specs, ops = [], []
            for f in factors:
                name, letters = T.parse(f)
                specs.append(letters)
                ops.append(self._operand(name, letters, s, ints))
            x = _einsum(",".join(specs) + "->" + out, *ops)
            acc = acc + coef * antisym(x, perm)
        return acc

    def energy(self, s, ints=None):
        return float(self._kernel("E", s, self.ints if ints is None else ints))

    def residual(self, s, ints=None):
        ints = self.ints if ints is None else ints
        return self._kernel("S1", s, ints), self._kernel("S2", s, ints)

    # -- vector-Jacobian products ------------------------------------------
    def _vjp(self, s, ebar, sbar, targets):
        """Transpose every term with respect to the factors named in `targets`.

        d/dX_k of coef * P[einsum(specs -> out)] contracted with cotangent Y is
        coef * einsum(out, other specs -> spec_k)(P Y, others); P is self-adjoint.
        Returns {(name, letters-pattern-or-None): gradient}.
        """
        grads = {}
        cot = {"E": ebar, "S1": sbar[0], "S2": sbar[1]}
        for which in ("E", "S1", "S2"):
            y = cot[which]
            if y is None:
                continue
            out = T.OUT[which]
            for coef, perm, factors in T.TERMS[which]:
                yp = coef * (antisym(y, perm) if which == "S2" else y)
                parsed = [T.parse(f) for f in factors]
                ops = [self._operand(nm, lt, s, self.ints) for nm, lt in parsed]
                for k, (nm, lt) in enumerate(parsed):
                    if nm not in targets:
                        continue
                    specs = [out] + [p[1] for j, p in enumerate(parsed) if j != k]
                    args = [yp] + [o for j, o in enumerate(ops) if j != k]
                    g = _einsum(",".join(specs) + "->" + lt, *args)
                    # integral gradients stay in this term's letter order
                    key = nm if nm in ("s1", "s2") else (nm, T.slot_pattern(lt), lt)
                    grads[key] = grads.get(key, 0.0) + g
        return grads

    def vjp(self, s, ebar, sbar):
        g = self._vjp(s, ebar, sbar, ("s1", "s2"))
        z1, z2 = self.zeros()
        return g.get("s1", z1) + z1, g.get("s2", z2) + z2

    def vjp_fock(self, s, ebar, sbar):
        """Gradient with respect to the unweighted one-body matrix u = f - diag(eps)."""
        g = self._vjp(s, ebar, sbar, ("F",))
        out = np.zeros((self.n, self.n))
        for (nm, pat, lt), gr in g.items():
            w0, w1 = self.ints.weight(pat[0]), self.ints.weight(pat[1])
            out += gr * w0[:, None] * w1[None, :]
        return out

    # -- mean-field parts ----------------------------------------------------
    def omega0(self):
        b = self.ints
        x = b.beta * (b.eps - b.mu)
        return -np.sum(np.logaddexp(0.0, -x)) / b.beta

    def omega1(self):
        b = self.ints
        n = b.n_occ
        d = _einsum("pqpq->pq", b.vas)
        return float(np.dot(np.diag(b.h) - b.eps, n) + 0.5 * n @ d @ n)

    def domega0(self, theta):
        """Explicit d Omega_0 / d mu or d beta at frozen eps."""
        b = self.ints
        if theta == "mu":
            return -float(np.sum(b.n_occ))
        return -self.omega0() / b.beta + float(np.sum((b.eps - b.mu) * b.n_occ)) / b.beta

    def domega0_deps(self):
        """d Omega_0 / d eps_q = n_q (one electron per spin orbital)."""
        return self.ints.n_occ.astype(float)

    def dmf_dh(self):
        """d Omega_1 / d h_pq = n_p delta_pq."""
        return np.diag(self.ints.n_occ).astype(float)

    def domega_mf(self, dn, dh=None, deri=None):
        """d(Omega_0 + Omega_1)/d theta at frozen eps (dn = d n / d theta)."""
        b = self.ints
        n = b.n_occ
        dfq = np.diag(b.fock) - b.eps
        d1 = float(dfq @ dn)
        if dh is not None:
            d1 += float(np.diag(dh) @ n)
        if deri is not None:
            dv = deri - deri.transpose(0, 1, 3, 2)
            d1 += 0.5 * float(n @ _einsum("pqpq->pq", dv) @ n)
        return d1

    def occ_derivs(self):
        """d n / d mu and d n / d beta at frozen eps."""
        b = self.ints
        nn = b.n_occ * b.n_vir
        return b.beta * nn, -(b.eps - b.mu) * nn
