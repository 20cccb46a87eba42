"""ctypes wrapper of the plain FP64 CPU oracle (oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU-baseline
leg of bench.py.  The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (OpenMP inside a colour / over rows)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_bp = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        V, I, D, P = None, C.c_int, C.c_double, C.c_void_p
        sig = {
            "orc_create": (P, [I, I, I, D, D, _ip, _dp, I, I, I, I]),
            "orc_destroy": (V, [P]),
            "orc_ndof": (I, [P, I]), "orc_n_u": (I, [P, I]), "orc_N": (I, [P, I]),
            "orc_singular": (I, [P, I]),
            "orc_constrained": (V, [P, I, _bp]),
            "orc_kappa": (V, [P, I, _dp]),
            "orc_nnz": (I, [P, I, I]),
            "orc_csr": (V, [P, I, I, _ip, _ip, _dp]),
            "orc_apply": (V, [P, I, _dp, _dp]),
            "orc_apply_row": (D, [P, I, I, _dp]),
            "orc_npatch": (I, [P, I]),
            "orc_patch_info": (V, [P, I, I, _ip]),
            "orc_patch_dofs": (V, [P, I, I, _ip]),
            "orc_patch_inverse": (V, [P, I, I, _dp]),
            "orc_colour_step": (V, [P, I, I, _dp, _dp]),
            "orc_smooth": (V, [P, I, I, _dp, _dp]),
            "orc_p_nnz": (I, [P, I]),
            "orc_p_csr": (V, [P, I, _ip, _ip, _dp]),
            "orc_prolong_add": (V, [P, I, _dp, _dp]),
            "orc_restrict": (V, [P, I, _dp, _dp]),
            "orc_coarse_solve": (V, [P, _dp, _dp]),
            "orc_vcycle": (V, [P, _dp, _dp]),
            "orc_fgmres": (I, [P, _dp, P, _dp, D, I, I, I, _dp, C.POINTER(D)]),
            "orc_direct_solve": (I, [P, _dp, _dp]),
            "orc_quad_points": (V, [I, I, _dp, _dp]),
            "orc_rhs": (V, [P, _dp, P, P, _dp]),
            "orc_L": (D, [I, D]), "orc_psi": (D, [I, D]),
            "orc_gauss": (V, [I, _dp, _dp]),
            "orc_level_create": (P, [I, I, D, D, _ip, _dp]),
            "orc_level_destroy": (V, [P]),
            "orc_level_ndof": (I, [P]),
            "orc_level_rows": (V, [P, I, _ip, _dp, _dp]),
            "orc_set_smoother": (V, [P, I, D]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def quad_points(n: int, k: int):
    q = k + 2
    cell = np.zeros(n * n * q * q * 2)
    face = np.zeros(4 * n * q * 2)
    lib().orc_quad_points(n, k, cell, face)
    return cell.reshape(n * n * q * q, 2), face.reshape(4 * n * q, 2)


def gauss(q: int):
    x, w = np.zeros(q), np.zeros(q)
    lib().orc_gauss(q, x, w)
    return x, w


class Oracle:
    """One problem: mesh hierarchy, level operators, patches, transfers, coarse solve."""

    def __init__(self, n0, levels, k, mu, sigma, bc, kappa, cycle=1, m_fine=2, colouring=0, smoother=0,
                 omega=0.25, kappa_avg=0):
        """colouring: 0 = S9 ((vx mod 3) + 3 (vy mod 3)), 1 = L8 (cosets of span{(2,2),(2,-2)}).
        smoother: 0 = symmetric multiplicative (Section 3.3), 1 = additive with damping omega.
        kappa_avg: coarse kappa from the four children, 0 arithmetic (Section 4.1), 1 harmonic,
        2 geometric."""
        self.n0, self.J, self.k, self.mu, self.sigma = n0, levels, k, mu, sigma
        self.colouring = colouring
        self.bc = np.ascontiguousarray(bc, dtype=np.int32)
        kap = _f64(kappa)
        n = n0 << levels
        assert kap.size == n * n
        self.h = lib().orc_create(n0, levels, k, mu, sigma, self.bc, kap, cycle, m_fine, colouring, kappa_avg)
        if not self.h:
            raise RuntimeError("oracle setup failed (singular coarse matrix)")
        if smoother:
            lib().orc_set_smoother(self.h, smoother, float(omega))

    @classmethod
    def from_workload(cls, w):
        return cls(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.kappa, w.cycle, w.m_fine)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    # sizes
    def ndof(self, j=None):
        return lib().orc_ndof(self.h, self.J if j is None else j)

    def n_u(self, j=None):
        return lib().orc_n_u(self.h, self.J if j is None else j)

    def N(self, j=None):
        return lib().orc_N(self.h, self.J if j is None else j)

    def singular(self, j=None):
        return bool(lib().orc_singular(self.h, self.J if j is None else j))

    def constrained(self, j=None):
        j = self.J if j is None else j
        out = np.zeros(self.ndof(j), dtype=np.int8)
        lib().orc_constrained(self.h, j, out)
        return out.astype(bool)

    def kappa(self, j):
        out = np.zeros(self.N(j) ** 2)
        lib().orc_kappa(self.h, j, out)
        return out

    def csr(self, j=None, full=False):
        import scipy.sparse as sp
        j = self.J if j is None else j
        n = self.ndof(j)
        nnz = lib().orc_nnz(self.h, j, int(full))
        rp, ci, v = np.zeros(n + 1, np.int32), np.zeros(nnz, np.int32), np.zeros(nnz)
        lib().orc_csr(self.h, j, int(full), rp, ci, v)
        return sp.csr_matrix((v, ci, rp), shape=(n, n))

    def apply(self, x, j=None):
        j = self.J if j is None else j
        y = np.zeros(self.ndof(j))
        lib().orc_apply(self.h, j, _f64(x), y)
        return y

    def apply_row(self, row, x, j=None):
        j = self.J if j is None else j
        return lib().orc_apply_row(self.h, j, int(row), _f64(x))

    # patches
    def npatch(self, j=None):
        return lib().orc_npatch(self.h, self.J if j is None else j)

    def patch(self, p, j=None):
        """(vx, vy, colour, dofs, singular, pseudo-inverse)."""
        j = self.J if j is None else j
        info = np.zeros(5, np.int32)
        lib().orc_patch_info(self.h, j, p, info)
        n = int(info[3])
        dofs = np.zeros(n, np.int32)
        inv = np.zeros(n * n)
        lib().orc_patch_dofs(self.h, j, p, dofs)
        lib().orc_patch_inverse(self.h, j, p, inv)
        return int(info[0]), int(info[1]), int(info[2]), dofs, bool(info[4]), inv.reshape(n, n)

    def colour_step(self, colour, x, b, j=None):
        j = self.J if j is None else j
        x = _f64(x).copy()
        lib().orc_colour_step(self.h, j, colour, x, _f64(b))
        return x

    def smooth(self, steps, x, b, j=None):
        j = self.J if j is None else j
        x = _f64(x).copy()
        lib().orc_smooth(self.h, j, steps, x, _f64(b))
        return x

    def prolongation(self, j):
        import scipy.sparse as sp
        nnz = lib().orc_p_nnz(self.h, j)
        n, m = self.ndof(j), self.ndof(j - 1)
        rp, ci, v = np.zeros(n + 1, np.int32), np.zeros(nnz, np.int32), np.zeros(nnz)
        lib().orc_p_csr(self.h, j, rp, ci, v)
        return sp.csr_matrix((v, ci, rp), shape=(n, m))

    def prolong_add(self, j, xc, xf):
        xf = _f64(xf).copy()
        lib().orc_prolong_add(self.h, j, _f64(xc), xf)
        return xf

    def restrict(self, j, rf):
        out = np.zeros(self.ndof(j - 1))
        lib().orc_restrict(self.h, j, _f64(rf), out)
        return out

    def coarse_solve(self, b):
        x = np.zeros(self.ndof(0))
        lib().orc_coarse_solve(self.h, _f64(b), x)
        return x

    def vcycle(self, r):
        z = np.zeros(self.ndof())
        lib().orc_vcycle(self.h, _f64(r), z)
        return z

    def fgmres(self, b, rtol=1e-10, maxit=200, restart=100, x0=None, precond=True):
        n = self.ndof()
        x = np.zeros(n)
        hist = np.zeros(maxit + 1)
        tr = C.c_double(0.0)
        x0p = None
        if x0 is not None:
            x0a = _f64(x0)
            x0p = x0a.ctypes.data_as(C.c_void_p)
        its = lib().orc_fgmres(self.h, _f64(b), x0p, x, rtol, maxit, restart, int(precond), hist,
                               C.byref(tr))
        return x, its, hist[:abs(its)], tr.value

    def direct_solve(self, b):
        x = np.zeros(self.ndof())
        if lib().orc_direct_solve(self.h, _f64(b), x) != 0:
            raise RuntimeError("direct solve: singular matrix")
        return x

    def rhs(self, f, s=None, g=None):
        """Assemble b from callables f(x, y) -> (..., 2), s(x, y), g(x, y) -> (..., 2)."""
        n = self.N()
        cell, face = quad_points(n, self.k)
        fq = _f64(f(cell[:, 0], cell[:, 1]).reshape(-1))
        keep = []
        sp_ = gp_ = None
        if s is not None:
            sq = _f64(s(cell[:, 0], cell[:, 1]).reshape(-1))
            keep.append(sq)
            sp_ = sq.ctypes.data_as(C.c_void_p)
        if g is not None:
            gq = _f64(g(face[:, 0], face[:, 1]).reshape(-1))
            keep.append(gq)
            gp_ = gq.ctypes.data_as(C.c_void_p)
        b = np.zeros(self.ndof())
        lib().orc_rhs(self.h, fq, sp_, gp_, b)
        return b


class OracleLevel:
    """One level without hierarchy: sampled rows of A x from the integrals."""

    def __init__(self, n, k, mu, sigma, bc, kappa):
        self.bc = np.ascontiguousarray(bc, dtype=np.int32)
        self.h = lib().orc_level_create(n, k, mu, sigma, self.bc, _f64(kappa))

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_level_destroy(self.h)
            self.h = None

    def ndof(self):
        return lib().orc_level_ndof(self.h)

    def rows(self, rows, x):
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        out = np.zeros(rows.size)
        lib().orc_level_rows(self.h, rows.size, rows, _f64(x), out)
        return out
