"""Spin-restricted FT-CCSD oracle: the spin-orbital terms summed over spin.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A spin-restricted reference has spin-independent orbitals, energies and
occupations, so the weights sqrt(n) and sqrt(1-n) do not depend on spin and
the closed-shell parametrisation of the amplitudes applies unchanged:

    s_{I}^{A}    = t1[i, a] d(sI, sA)
    s_{IJ}^{AB}  = t2[i, j, a, b] d(sI, sA) d(sJ, sB) - t2[i, j, b, a] d(sI, sB) d(sJ, sA)
    <PQ||RS>     = <pq|rs> d(sP, sR) d(sQ, sS) - <pq|sr> d(sP, sS) d(sQ, sR)
    f_PQ         = u[p, q] d(sP, sQ)

with t2[i, j, a, b] = s_{i alpha, j beta}^{a alpha, b beta}.  Every printed
term of eqn:E, eqn:ccS1 and eqn:ccS2 (terms.py) is evaluated here by explicit
enumeration of the spins of its summed letters, with the output fixed to the
blocks S1[i alpha, a alpha] and S2[i alpha, j beta, a alpha, b beta].  No
algebra is done by hand: each spin assignment and each choice of the direct or
exchange part becomes one spatial einsum.
"""
from __future__ import annotations

import functools
import itertools

import numpy as np
from scipy.special import expit

from . import terms as T
from .einsum import einsum as _einsum

ALPHA, BETA = 0, 1
_OUT_SPINS = {"E": {}, "S1": {"i": ALPHA, "a": ALPHA},
              "S2": {"i": ALPHA, "j": BETA, "a": ALPHA, "b": BETA}}


def _expand_factor(name, letters, spin):
    if name in ("F", "s1"):
        p, q = letters
        return [(1.0, name, letters)] if spin[p] == spin[q] else []
    if name in ("V", "s2"):
        p, q, r, s = letters
        tgt = "G" if name == "V" else "t2"
        out = []
        if spin[p] == spin[r] and spin[q] == spin[s]:
            out.append((1.0, tgt, p + q + r + s))
        if spin[p] == spin[s] and spin[q] == spin[r]:
            out.append((-1.0, tgt, p + q + s + r))
        return out
    raise ValueError(name)


def _antisym_items(which, perm):
    """(sign, output-letter spins, transpose axes) realising P(ij)/P(ab) on a block.

    (P(ij) X)[I, J, A, B] = X[I, J, A, B] - X[J, I, A, B]: the second part is the
    raw term evaluated with the spins of i and j exchanged, transposed on (i, j).
    """
    items = [(1.0, dict(_OUT_SPINS[which]), None)]
    for pair, axes in (("ij", (1, 0, 2, 3)), ("ab", (0, 1, 3, 2))):
        if pair not in perm:
            continue
        p, q = pair
        new = []
        for sgn, spins, ax in items:
            new.append((sgn, spins, ax))
            sw = dict(spins)
            sw[p], sw[q] = spins[q], spins[p]
            new.append((-sgn, sw, _compose(ax, axes)))
        items = new
    return items


def _compose(ax, new):
    if ax is None:
        return new
    return tuple(ax[k] for k in new)


@functools.lru_cache(maxsize=None)
def expanded(which):
    """All spatial einsum items of one kernel: (coef, [(op, subscripts)], axes)."""
    out_letters = T.OUT[which]
    items = []
    for coef, perm, factors in T.TERMS[which]:
        parsed = [T.parse(f) for f in factors]
        letters = sorted({ch for _, lt in parsed for ch in lt})
        for sgn, ospin, axes in _antisym_items(which, perm):
            summed = [ch for ch in letters if ch not in out_letters]
            for combo in itertools.product((ALPHA, BETA), repeat=len(summed)):
                spin = dict(ospin)
                spin.update(zip(summed, combo))
                alts = [_expand_factor(nm, lt, spin) for nm, lt in parsed]
                for choice in itertools.product(*alts):
                    c = coef * sgn
                    ops = []
                    for fs, op, sub in choice:
                        c *= fs
                        ops.append((op, sub))
                    items.append((c, tuple(ops), axes))
    return _merge(items)


def _merge(items):
    acc = {}
    for c, ops, axes in items:
        key = (ops, axes)
        acc[key] = acc.get(key, 0.0) + c
    return [(c, ops, axes) for (ops, axes), c in acc.items() if c != 0.0]


class RestrictedIntegrals:
    """Weighted spatial blocks: F (u = f - diag eps) and G (<pq|rs>, not antisymmetrised)."""

    def __init__(self, h, eri, eps, mu, beta, thr=0.0):
        self.h, self.eri, self.eps = np.asarray(h, float), np.asarray(eri, float), np.asarray(eps, float)
        self.mu, self.beta, self.thr = float(mu), float(beta), float(thr)
        x = self.beta * (self.eps - self.mu)
        self.n_occ, self.n_vir = expit(-x), expit(x)
        self.keep_h = self.n_occ > self.thr
        self.keep_p = self.n_vir > self.thr
        self.wh = np.where(self.keep_h, np.sqrt(self.n_occ), 0.0)
        self.wp = np.where(self.keep_p, np.sqrt(self.n_vir), 0.0)
        self.jk = 2.0 * self.eri - self.eri.transpose(0, 1, 3, 2)       # 2<pq|rs> - <pq|sr>
        self.fock = self.h + _einsum("prqr,r->pq", self.jk, self.n_occ)
        self.u = self.fock - np.diag(self.eps)
        self._cache = {}

    def weight(self, kind):
        return self.wh if kind == "o" else self.wp

    def get(self, name, letters):
        pat = T.slot_pattern(letters)
        key = (name, pat)
        if key not in self._cache:
            arr = self.u if name == "F" else self.eri
            for axis, kind in enumerate(pat):
                shape = [1] * len(pat)
                shape[axis] = -1
                arr = arr * self.weight(kind).reshape(shape)
            self._cache[key] = arr
        return self._cache[key]

    def derivative(self, dn=None, dh=None, deri=None):
        return _RDeriv(self, dn, dh, deri)


class _RDeriv:
    def __init__(self, b, dn, dh, deri):
        n = b.eps.size
        self.b = b
        dn = np.zeros(n) if dn is None else np.asarray(dn, float)
        safe_h = np.where(b.wh > 0, b.wh, 1.0)
        safe_p = np.where(b.wp > 0, b.wp, 1.0)
        self.dwh = np.where(b.keep_h & (b.wh > 0), dn / (2.0 * safe_h), 0.0)
        self.dwp = np.where(b.keep_p & (b.wp > 0), -dn / (2.0 * safe_p), 0.0)
        self.deri = np.zeros_like(b.eri) if deri is None else np.asarray(deri, float)
        djk = 2.0 * self.deri - self.deri.transpose(0, 1, 3, 2)
        du = _einsum("prqr,r->pq", b.jk, dn) + _einsum("prqr,r->pq", djk, b.n_occ)
        if dh is not None:
            du = du + dh
        self.du = du
        self._cache = {}

    def get(self, name, letters):
        pat = T.slot_pattern(letters)
        key = (name, pat)
        if key in self._cache:
            return self._cache[key]
        b = self.b
        base, dbase = (b.u, self.du) if name == "F" else (b.eri, self.deri)
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


def _apply_axes(x, axes):
    return x if axes is None else x.transpose(axes)


class RestrictedModel:
    """Same interface as spinorb.SpinOrbitalModel, on (t1, t2) spatial amplitudes."""

    def __init__(self, ints: RestrictedIntegrals):
        self.ints = ints
        eps = ints.eps
        self.n = eps.size
        self.delta1 = eps[None, :] - eps[:, None]
        self.delta2 = (eps[None, None, :, None] + eps[None, None, None, :]
                       - eps[:, None, None, None] - eps[None, :, None, None])

    def zeros(self):
        n = self.n
        return np.zeros((n, n)), np.zeros((n, n, n, n))

    def _operand(self, op, sub, s, ints):
        if op == "s1":
            return s[0]
        if op == "t2":
            return s[1]
        return ints.get("F" if op == "F" else "V", sub)

    def _kernel(self, which, s, ints):
        out = T.OUT[which]
        acc = np.zeros(() if which == "E" else (self.n,) * len(out))
        for c, ops, axes in expanded(which):
            x = _einsum(",".join(sub for _, sub in ops) + "->" + out,
                          *[self._operand(op, sub, s, ints) for op, sub in ops])
            acc = acc + c * _apply_axes(x, axes)
        return acc

    def residual_rows(self, s, rows_i, rows_j):
        """S1 whole and the rows S2[rows_i][:, rows_j] (shape (|I|, |J|, n, n)),
        for sizes where S2 or the weighted integral blocks do not fit in memory.

        The same items as residual(), each with its output restricted before it
        is evaluated: an item whose result is transposed by `axes` lands its
        axis axes[0] on output axis i and axes[1] on j, so the letters at those
        axes take only the requested indices, in every factor that carries them.
        Weighted integral blocks are formed per item and not kept."""
        out = T.OUT["S2"]
        res = []
        for which, rows in (("S1", None), ("S2", (rows_i, rows_j))):
            shape = (self.n, self.n) if rows is None else (len(rows_i), len(rows_j), self.n, self.n)
            acc = np.zeros(shape)
            for c, ops, axes in expanded(which):
                restrict = {}
                if rows is not None:
                    ax = (0, 1, 2, 3) if axes is None else axes
                    restrict = {out[ax[0]]: np.asarray(rows[0]), out[ax[1]]: np.asarray(rows[1])}
                args = []
                for op, sub in ops:
                    a = self._operand(op, sub, s, self.ints)
                    for k, ch in enumerate(sub):
                        if ch in restrict:
                            a = np.take(a, restrict[ch], axis=k)
                    args.append(a)
                self.ints._cache.clear()
                x = _einsum(",".join(sub for _, sub in ops) + "->" + T.OUT[which], *args)
                acc = acc + c * _apply_axes(x, axes)
            res.append(acc)
        return res[0], res[1]

    def energy(self, s, ints=None):
        return float(self._kernel("E", s, self.ints if ints is None else ints))

    def residual(self, s, ints=None):
        ints = self.ints if ints is None else ints
        return self._kernel("S1", s, ints), self._kernel("S2", s, ints)

    def _vjp(self, s, ebar, sbar, targets):
        grads = {}
        cot = {"E": ebar, "S1": sbar[0], "S2": sbar[1]}
        for which in ("E", "S1", "S2"):
            y = cot[which]
            if y is None:
                continue
            out = T.OUT[which]
            for c, ops, axes in expanded(which):
                yp = c * _apply_axes(y, axes)      # every axes used is an involution
                vals = [self._operand(op, sub, s, self.ints) for op, sub in ops]
                for k, (op, sub) in enumerate(ops):
                    if op not in targets:
                        continue
                    specs = [out] + [o[1] for j, o in enumerate(ops) if j != k]
                    args = [yp] + [v for j, v in enumerate(vals) if j != k]
                    g = _einsum(",".join(specs) + "->" + sub, *args)
                    key = op if op in ("s1", "t2") else (op, T.slot_pattern(sub), sub)
                    grads[key] = grads.get(key, 0.0) + g
        return grads

    def vjp(self, s, ebar, sbar):
        g = self._vjp(s, ebar, sbar, ("s1", "t2"))
        z1, z2 = self.zeros()
        return g.get("s1", z1) + z1, g.get("t2", z2) + z2

    def vjp_fock(self, s, ebar, sbar):
        g = self._vjp(s, ebar, sbar, ("F",))
        out = np.zeros((self.n, self.n))
        for (op, pat, sub), gr in g.items():
            out += gr * self.ints.weight(pat[0])[:, None] * self.ints.weight(pat[1])[None, :]
        return out

    # -- mean-field parts (both spins) ---------------------------------------
    def omega0(self):
        b = self.ints
        x = b.beta * (b.eps - b.mu)
        return -2.0 * np.sum(np.logaddexp(0.0, -x)) / b.beta

    def omega1(self):
        b = self.ints
        n = b.n_occ
        d = 2.0 * _einsum("pqpq->pq", b.eri) - _einsum("pqqp->pq", b.eri)
        return float(2.0 * np.dot(np.diag(b.h) - b.eps, n) + n @ d @ n)

    def domega0(self, theta):
        b = self.ints
        if theta == "mu":
            return -2.0 * float(np.sum(b.n_occ))
        return -self.omega0() / b.beta + 2.0 * float(np.sum((b.eps - b.mu) * b.n_occ)) / b.beta

    def domega0_deps(self):
        """d Omega_0 / d eps_q = 2 n_q (both spins of spatial orbital q)."""
        return 2.0 * self.ints.n_occ

    def dmf_dh(self):
        return 2.0 * np.diag(self.ints.n_occ)

    def domega_mf(self, dn, dh=None, deri=None):
        b = self.ints
        n = b.n_occ
        d1 = 2.0 * float((np.diag(b.fock) - b.eps) @ dn)
        if dh is not None:
            d1 += 2.0 * float(np.diag(dh) @ n)
        if deri is not None:
            dd = 2.0 * _einsum("pqpq->pq", deri) - _einsum("pqqp->pq", deri)
            d1 += float(n @ dd @ n)
        return d1

    def occ_derivs(self):
        b = self.ints
        nn = b.n_occ * b.n_vir
        return b.beta * nn, -(b.eps - b.mu) * nn
