"""Imaginary-time grid and exponential-propagator weights (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper integrates Omega_CC = (1/beta) int_0^beta E[s(tau)] dtau
(eqn:Ecc) with a quadrature g (eqn:g) and obtains the amplitudes from the
integral equation s(tau) = -int_0^tau exp(Delta (tau' - tau)) S[s(tau')] dtau'
(eqn:smu) through a quadrature tensor G (eqn:G).  It does not fix G for
Gauss-Legendre nodes; the reading used here (composite exponential Gauss
collocation) is:

  * [0, beta] is cut into P panels of width h = beta / P; each panel carries
    the m Gauss-Legendre nodes c_1..c_m of [0, 1] with weights b_x, so that
    tau_{p,x} = (p + c_x) h and g_{p,x} = h b_x;
  * inside a panel that starts at state s_b the exact variation-of-constants
    formula s(tau_b + c h) = exp(-Delta c h) s_b
    - h int_0^c exp(Delta h (u - c)) S(tau_b + u h) du is applied with S replaced
    by its Lagrange interpolant through the m nodes, which gives
        s_x   = E_x s_b - sum_x' W_xx' S_x'      (nodes of the panel)
        s_b'  = E_e s_b - sum_x' We_x' S_x'      (state at the panel end)
    with E_x = exp(-Delta h c_x), E_e = exp(-Delta h) and
        W_xx' = h int_0^{c_x} exp(Delta h (u - c_x)) l_x'(u) du,
        We_x' = h int_0^1     exp(Delta h (u - 1))   l_x'(u) du;
  * variant "lawson" interpolates the whole integrand instead (integrating
    factor), which for one panel is the paper's literal
    s(tau_y) = -sum_x G^y_x exp(Delta (tau_x - tau_y)) S(tau_x):
        W_xx' = A_xx' exp(Delta h (c_x' - c_x)),  A_xx' = h int_0^{c_x} l_x'(u) du,
        We_x' = h b_x' exp(Delta h (c_x' - 1)).

The weights are evaluated by plain Gauss-Legendre quadrature with Q = 128
points on each interval, which is exact to rounding for |Delta h| up to ~100.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.legendre import leggauss

Q_SUB = 128


def panel_nodes(m: int):
    """Gauss-Legendre nodes c (ascending) and weights b on [0, 1]."""
    x, w = leggauss(m)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange(c: np.ndarray, u: np.ndarray) -> np.ndarray:
    """l[x', ...] = l_x'(u) for the Lagrange basis on nodes c."""
    u = np.asarray(u, dtype=np.float64)
    out = np.ones((len(c),) + u.shape)
    for k in range(len(c)):
        for j in range(len(c)):
            if j != k:
                out[k] *= (u - c[j]) / (c[k] - c[j])
    return out


class Grid:
    """Composite grid with P panels of m nodes on [0, beta]."""

    def __init__(self, beta: float, n_panels: int, m: int, kind: str = "etd"):
        if kind not in ("etd", "lawson"):
            raise ValueError(kind)
        self.beta, self.P, self.m, self.kind = float(beta), int(n_panels), int(m), kind
        self.c, self.b = panel_nodes(m)
        self.h = self.beta / self.P
        self.n_g = self.P * self.m

    @property
    def tau(self) -> np.ndarray:
        return ((np.arange(self.P)[:, None] + self.c[None, :]) * self.h).ravel()

    @property
    def g(self) -> np.ndarray:
        """Quadrature weights g_x of eqn:g for every node (sum = beta)."""
        return np.tile(self.h * self.b, self.P)

    def weights(self, delta: np.ndarray, h: float | None = None, deriv: bool = False):
        """Exponential weights for an array of Delta values.

        Returns (E, Ee, W, We) with shapes (m,)+d, d, (m, m)+d, (m,)+d; with
        deriv=True also their derivatives with respect to the panel width h.
        """
        h = self.h if h is None else float(h)
        delta = np.asarray(delta, dtype=np.float64)
        uniq, inv = np.unique(delta.ravel(), return_inverse=True)
        res = self._weights_unique(uniq, h, deriv)
        shape = delta.shape
        out = []
        for arr in res:
            lead = arr.shape[:-1]
            out.append(arr[..., inv].reshape(lead + shape))
        return tuple(out)

    def weights_ddelta(self, delta: np.ndarray, h: float | None = None):
        """Derivatives (dE, dEe, dW, dWe) of the exponential weights with respect
        to Delta at fixed h, by the same quadrature of their integral definitions:
        d/dDelta exp(Delta h (u - c)) = h (u - c) exp(Delta h (u - c))."""
        h = self.h if h is None else float(h)
        delta = np.asarray(delta, dtype=np.float64)
        uniq, inv = np.unique(delta.ravel(), return_inverse=True)
        d = uniq
        m, c, b = self.m, self.c, self.b
        dE = -h * c[:, None] * np.exp(-np.outer(c, d) * h)
        dEe = -h * np.exp(-d * h)
        dW = np.zeros((m, m, d.size))
        dWe = np.zeros((m, d.size))
        v, om = panel_nodes(Q_SUB)
        if self.kind == "etd":
            for x in range(m):
                for q in range(Q_SUB):
                    u = c[x] * v[q]
                    ex = np.exp(d * h * (u - c[x]))
                    dW[x] += (h * c[x] * om[q]) * lagrange(c, u)[:, None] * (h * (u - c[x]) * ex)[None, :]
            for q in range(Q_SUB):
                u = v[q]
                ex = np.exp(d * h * (u - 1.0))
                dWe += (h * om[q]) * lagrange(c, u)[:, None] * (h * (u - 1.0) * ex)[None, :]
        else:
            A = np.zeros((m, m))
            for x in range(m):
                for q in range(Q_SUB):
                    A[x] += c[x] * om[q] * lagrange(c, c[x] * v[q])
            for x in range(m):
                for y in range(m):
                    dW[x, y] = h * A[x, y] * h * (c[y] - c[x]) * np.exp(d * h * (c[y] - c[x]))
            for y in range(m):
                dWe[y] = h * b[y] * h * (c[y] - 1.0) * np.exp(d * h * (c[y] - 1.0))
        out = []
        for arr in (dE, dEe, dW, dWe):
            out.append(arr[..., inv].reshape(arr.shape[:-1] + delta.shape))
        return tuple(out)

    def _weights_unique(self, d, h, deriv):
        m, c, b = self.m, self.c, self.b
        E = np.exp(-np.outer(c, d) * h)                        # (m, N)
        Ee = np.exp(-d * h)
        dE = -np.outer(c, d) * E
        dEe = -d * Ee
        W = np.zeros((m, m, d.size))
        We = np.zeros((m, d.size))
        dW = np.zeros((m, m, d.size))
        dWe = np.zeros((m, d.size))
        v, om = panel_nodes(Q_SUB)
        if self.kind == "etd":
            for x in range(m):
                for q in range(Q_SUB):
                    u = c[x] * v[q]
                    arg = d * h * (u - c[x])
                    ex = np.exp(arg)
                    lq = lagrange(c, u)                      # (m,)
                    W[x] += (h * c[x] * om[q]) * lq[:, None] * ex[None, :]
                    dW[x] += (c[x] * om[q]) * lq[:, None] * (ex * (1.0 + arg))[None, :]
            for q in range(Q_SUB):
                u = v[q]
                arg = d * h * (u - 1.0)
                ex = np.exp(arg)
                lq = lagrange(c, u)
                We += (h * om[q]) * lq[:, None] * ex[None, :]
                dWe += om[q] * lq[:, None] * (ex * (1.0 + arg))[None, :]
        else:
            A = np.zeros((m, m))
            for x in range(m):
                for q in range(Q_SUB):
                    A[x] += c[x] * om[q] * lagrange(c, c[x] * v[q])
            for x in range(m):
                for y in range(m):
                    arg = d * h * (c[y] - c[x])
                    ex = np.exp(arg)
                    W[x, y] = h * A[x, y] * ex
                    dW[x, y] = A[x, y] * ex * (1.0 + arg)
            for y in range(m):
                arg = d * h * (c[y] - 1.0)
                ex = np.exp(arg)
                We[y] = h * b[y] * ex
                dWe[y] = b[y] * ex * (1.0 + arg)
        if deriv:
            return E, Ee, W, We, dE, dEe, dW, dWe
        return E, Ee, W, We
