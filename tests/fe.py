"""Independent numpy evaluation of finite-element functions given by coefficient
vectors in the canonical numbering.

Test helper.  It restates the basis of the RT_k x dQ_k spaces (Section 2.3 of the
paper) with numpy's Legendre-series routines, so it shares nothing with either the
oracle or the GPU library:

  L_b(t)   = sqrt(2b+1) P_b(2t-1)                 (orthonormal on [0,1])
  psi_0    = 1-t,  psi_1 = t,  psi_a = int_0^t L_{a-1}   (a >= 2)
  u_x      = psi_a(xi) L_b(eta),   u_y = L_b(xi) psi_a(eta),   p = L_a(xi) L_b(eta)

Global order: x-face dofs, y-face dofs, cell-interior velocity dofs, pressure.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npl


def _e(n):
    c = np.zeros(n + 1)
    c[n] = 1.0
    return c


def L(b, t):
    return np.sqrt(2 * b + 1) * npl.legval(2 * t - 1, _e(b))


def dL(b, t):
    return 2 * np.sqrt(2 * b + 1) * npl.legval(2 * t - 1, npl.legder(_e(b)))


def psi(a, t):
    t = np.asarray(t, dtype=float)
    if a == 0:
        return 1 - t
    if a == 1:
        return t
    m = a - 1
    ic = npl.legint(_e(m), lbnd=-1)      # antiderivative of P_m vanishing at -1
    return np.sqrt(2 * m + 1) * 0.5 * npl.legval(2 * t - 1, ic)


def dpsi(a, t):
    t = np.asarray(t, dtype=float)
    if a == 0:
        return -np.ones_like(t)
    if a == 1:
        return np.ones_like(t)
    return L(a - 1, t)


class Space:
    def __init__(self, n, k):
        self.n, self.k = n, k
        nb = k + 1
        self.nb = nb
        self.n_u = 2 * n * (n + 1) * nb + 2 * k * nb * n * n
        self.n_p = nb * nb * n * n
        self.ndof = self.n_u + self.n_p

    def xface(self, i, cy, b):
        return (cy * (self.n + 1) + i) * self.nb + b

    def yface(self, j, cx, b):
        return self.n * (self.n + 1) * self.nb + (j * self.n + cx) * self.nb + b

    def interior(self, c, comp, a, b):
        return 2 * self.n * (self.n + 1) * self.nb + c * 2 * self.k * self.nb + (comp * self.k + (a - 2)) * self.nb + b

    def pres(self, c, a, b):
        return self.n_u + c * self.nb * self.nb + b * self.nb + a

    def ux_index(self, cx, cy, a, b):
        if a == 0:
            return self.xface(cx, cy, b)
        if a == 1:
            return self.xface(cx + 1, cy, b)
        return self.interior(cy * self.n + cx, 0, a, b)

    def uy_index(self, cx, cy, a, b):
        if a == 0:
            return self.yface(cy, cx, b)
        if a == 1:
            return self.yface(cy + 1, cx, b)
        return self.interior(cy * self.n + cx, 1, a, b)

    def locate(self, x, y):
        n = self.n
        cx = np.minimum((np.asarray(x) * n).astype(int), n - 1)
        cy = np.minimum((np.asarray(y) * n).astype(int), n - 1)
        return cx, cy, x * n - cx, y * n - cy

    def evaluate(self, coef, x, y):
        """u (m,2), grad u (m,2,2) [g[c][d] = du_c/dx_d], div u (m,), p (m,)."""
        x = np.asarray(x, float)
        y = np.asarray(y, float)
        cx, cy, xi, eta = self.locate(x, y)
        n, k, h = self.n, self.k, 1.0 / self.n
        m = x.size
        u = np.zeros((m, 2))
        g = np.zeros((m, 2, 2))
        p = np.zeros(m)
        ux_idx = np.vectorize(self.ux_index)
        uy_idx = np.vectorize(self.uy_index)
        for a in range(k + 2):
            for b in range(k + 1):
                cxa = coef[ux_idx(cx, cy, a, b)]
                u[:, 0] += cxa * psi(a, xi) * L(b, eta)
                g[:, 0, 0] += cxa * dpsi(a, xi) * L(b, eta) / h
                g[:, 0, 1] += cxa * psi(a, xi) * dL(b, eta) / h
                cya = coef[uy_idx(cx, cy, a, b)]
                u[:, 1] += cya * L(b, xi) * psi(a, eta)
                g[:, 1, 0] += cya * dL(b, xi) * psi(a, eta) / h
                g[:, 1, 1] += cya * L(b, xi) * dpsi(a, eta) / h
        c = cy * n + cx
        for b in range(k + 1):
            for a in range(k + 1):
                p += coef[self.n_u + c * (k + 1) ** 2 + b * (k + 1) + a] * L(a, xi) * L(b, eta)
        return u, g, g[:, 0, 0] + g[:, 1, 1], p

    def cell_quadrature(self, q=6):
        """Points and weights of a tensor Gauss rule on every cell (numpy leggauss)."""
        t, w = npl.leggauss(q)
        t, w = 0.5 * (t + 1), 0.5 * w
        n, h = self.n, 1.0 / self.n
        cx, cy, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(q), np.arange(q), indexing="ij")
        X = ((cx + t[ix]) * h).ravel()
        Y = ((cy + t[iy]) * h).ravel()
        W = (w[ix] * w[iy] * h * h).ravel()
        return X, Y, W

    def pressure_mean(self, coef):
        """Mean of p over the unit square (coefficient of L_0 L_0 averaged over cells)."""
        n, k = self.n, self.k
        return coef[self.n_u + np.arange(n * n) * (k + 1) ** 2].mean()

    def remove_pressure_mean(self, coef):
        out = np.array(coef, dtype=float)
        n, k = self.n, self.k
        out[self.n_u + np.arange(n * n) * (k + 1) ** 2] -= self.pressure_mean(coef)
        return out
