"""Thin ctypes binding of libbmg.so (include/bmg.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides device memory (tensor data pointers) and the stream.  If the
library is not built, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libbmg.so")

if not os.path.exists(LIBPATH):
    raise ImportError(f"{LIBPATH} is not built; run paper_1602_04858_amd/build.py (hipcc, gfx950)")

# torch first: its HIP runtime (soname libamdhip64.so.7) is then the one libbmg.so
# binds to.  Loading libbmg.so first would bring in a second HIP/HSA runtime from
# the system ROCm, and whichever initialises second finds no device.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIBPATH)

BC_DIRICHLET, BC_OPEN = 0, 1
P_FP64, P_FP32, P_BF16 = 0, 1, 2
CYCLE_STANDARD, CYCLE_VARIABLE = 0, 1
COLOURING_S9, COLOURING_L8 = 0, 1
SMOOTHER_MULTIPLICATIVE, SMOOTHER_ADDITIVE = 0, 1
KAPPA_ARITHMETIC, KAPPA_HARMONIC, KAPPA_GEOMETRIC = 0, 1, 2

STATUS = {0: "BMG_OK", 1: "BMG_E_ARG", 2: "BMG_E_UNSUPPORTED", 3: "BMG_E_NOMEM", 4: "BMG_E_HIP",
          5: "BMG_E_SINGULAR", 6: "BMG_E_NOT_CONVERGED", 7: "BMG_E_NONFINITE", 8: "BMG_E_STATE"}


class Params(C.Structure):
    _fields_ = [("n0", C.c_int32), ("levels", C.c_int32), ("k", C.c_int32), ("mu", C.c_double),
                ("sigma", C.c_double), ("bc", C.c_int32 * 4), ("cycle", C.c_int32), ("m_fine", C.c_int32),
                ("precond_prec", C.c_int32), ("restart", C.c_int32), ("dense_coarse_max", C.c_int32),
                ("n_rhs", C.c_int32), ("colouring", C.c_int32), ("smoother", C.c_int32), ("omega", C.c_double),
                ("coarse_kappa", C.c_int32), ("setup_on_host", C.c_int32), ("rotated_min_n", C.c_int32),
                ("columns_per_block", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32),
                ("rel_residual_estimate", C.c_double), ("rel_residual_true", C.c_double)]


_P, _I32, _I64, _D, _VP = C.POINTER, C.c_int32, C.c_int64, C.c_double, C.c_void_p
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")

_sig = {
    "bmg_plan": [_P(Params), _P(C.c_size_t)],
    "bmg_setup": [_P(Params), _dp, _VP, C.c_size_t, _VP, _P(_VP)],
    "bmg_destroy": [_VP],
    "bmg_sizes": [_VP, _I32, _P(_I32), _P(_I64), _P(_I64)],
    "bmg_apply": [_VP, _I32, _VP, _VP],
    "bmg_vcycle": [_VP, _VP, _VP],
    "bmg_vcycle_noalloc": [_VP, _VP, _VP],
    "bmg_solve": [_VP, _VP, _VP, _D, _I32, _VP, _P(SolveInfo)],
    "bmg_quad_points": [_P(Params), _dp, _dp],
    "bmg_assemble_rhs": [_P(Params), _dp, _VP, _VP, _dp],
    "bmg_colour_step": [_VP, _I32, _I32, _VP, _VP],
    "bmg_smooth": [_VP, _I32, _I32, _VP, _VP],
    "bmg_restrict": [_VP, _I32, _VP, _VP],
    "bmg_prolong_add": [_VP, _I32, _VP, _VP],
    "bmg_coarse_solve": [_VP, _VP, _VP],
    "bmg_export_patch": [_P(Params), _dp, _I32, _I32, _I32, _P(_I32), _ip, _VP, _P(_I32)],
    "bmg_export_level_matrix": [_P(Params), _dp, _I32, _dp],
    "bmg_export_colouring": [_P(Params), _I32, _P(_I32), _VP],
    "bmg_autotune": [_P(Params), _dp, _VP, _I32, _P(Params), _VP],
    "bmg_autotune_tiles": [_P(Params), _dp, _VP, _I32, _P(Params), _VP, _I32, _P(_I32)],
    "bmg_kernel_timing": [_VP, _I32, _I32],
    "bmg_kernel_timing_read": [_VP, _P(_I32), _P(_D), _P(_D)],
    "bmg_batch_setup": [_I32, _P(Params), _P(_P(_D)), _I32, _VP, _P(_VP)],
    "bmg_batch_solve": [_VP, _P(_VP), _P(_VP), _D, _I32, _P(SolveInfo)],
    "bmg_batch_handle_of": [_VP, _I32, _P(_VP)],
    "bmg_batch_destroy": [_VP],
}
EXPORTS = list(_sig) + ["bmg_status_string", "bmg_last_error", "bmg_batch_last_error"]
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.bmg_status_string.argtypes = [C.c_int]
_lib.bmg_status_string.restype = C.c_char_p
_lib.bmg_last_error.argtypes = [_VP]
_lib.bmg_last_error.restype = C.c_char_p
_lib.bmg_batch_last_error.argtypes = [_VP]
_lib.bmg_batch_last_error.restype = C.c_char_p


class BmgError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


def lib():
    return _lib


DENSE_COARSE_DEFAULT = 16384


def make_params(n0, levels, k, mu, sigma, bc, cycle=CYCLE_VARIABLE, m_fine=2, prec=P_FP64, restart=100,
                dense_coarse_max=0, n_rhs=1, colouring=COLOURING_S9, smoother=SMOOTHER_MULTIPLICATIVE, omega=0.25,
                coarse_kappa=KAPPA_ARITHMETIC, setup_on_host=0, rotated_min_n=0, columns_per_block=0):
    p = Params()
    p.n0, p.levels, p.k, p.mu, p.sigma = n0, levels, k, float(mu), float(sigma)
    for i in range(4):
        p.bc[i] = int(bc[i])
    p.cycle, p.m_fine, p.precond_prec, p.restart = cycle, m_fine, prec, restart
    p.dense_coarse_max = dense_coarse_max
    p.n_rhs = n_rhs
    p.colouring = colouring
    p.smoother = smoother
    p.omega = float(omega)
    p.coarse_kappa = coarse_kappa
    p.setup_on_host = setup_on_host
    p.rotated_min_n = rotated_min_n
    p.columns_per_block = columns_per_block
    return p


def plan(params: Params) -> int:
    n = C.c_size_t(0)
    st = _lib.bmg_plan(C.byref(params), C.byref(n))
    if st:
        raise BmgError(st, "plan")
    return n.value


def _ptr(t):
    return C.c_void_p(t.data_ptr())



def _kappa_host(kappa, n_cells):
    """kappa as a contiguous FP64 host array.  The library reads exactly n_cells values
    (the finest mesh's cells) from the pointer it is given, so a shorter array would be
    read past its end: any other size is refused here.  n_cells is None when the
    parameters are out of range; the library then rejects the call itself."""
    kap = np.ascontiguousarray(kappa, dtype=np.float64).reshape(-1)
    if n_cells is not None and kap.size != n_cells:
        raise ValueError(f"kappa has {kap.size} values; the finest mesh has {n_cells} cells")
    return kap


def _cells2(p):
    """Cells of the finest 2-D mesh, (n0 2^levels)^2, or None for out-of-range parameters."""
    return (p.n0 << p.levels) ** 2 if 1 <= p.n0 <= 64 and 0 <= p.levels <= 12 else None


def _cells3(p):
    """Cells of the finest 3-D mesh, (n0 2^(levels-1))^3, or None for out-of-range parameters."""
    return (p.n0 << (p.levels - 1)) ** 3 if 1 <= p.n0 <= 8 and 1 <= p.levels <= 7 else None


class Solver:
    """One problem on the GPU (handle of the C library)."""

    def __init__(self, params: Params, kappa, device="cuda", workspace=None):
        import torch
        self.torch = torch
        self.params = params
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        kap = _kappa_host(kappa, _cells2(params))
        self.stream = torch.cuda.current_stream(self.device)
        ws_ptr, ws_bytes = None, 0
        if workspace == "torch":
            nbytes = plan(params)
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            ws_ptr = C.c_void_p((base + 255) // 256 * 256)
            ws_bytes = nbytes
        h = C.c_void_p()
        st = _lib.bmg_setup(C.byref(params), kap, ws_ptr, ws_bytes, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st:
            raise BmgError(st, f"setup: {_lib.bmg_last_error(None).decode()}")
        self.h = h
        self.J = params.levels
        self.k = params.k
        self.R = max(1, params.n_rhs)

    def close(self):
        if getattr(self, "h", None):
            _lib.bmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st:
            raise BmgError(st, f"{what}: {_lib.bmg_last_error(self.h).decode()}")

    def sizes(self, level=None):
        level = self.J if level is None else level
        N, nu, npr = C.c_int32(), C.c_int64(), C.c_int64()
        self._check(_lib.bmg_sizes(self.h, level, C.byref(N), C.byref(nu), C.byref(npr)), "sizes")
        return N.value, nu.value, npr.value

    def ndof(self, level=None):
        _, a, b = self.sizes(level)
        return a + b

    def zeros(self, level=None):
        """Vector(s) of a level: shape (ndof,) for one right-hand side, (n_rhs, ndof) otherwise."""
        n = self.ndof(level)
        shape = (n,) if self.R == 1 else (self.R, n)
        return self.torch.zeros(shape, dtype=self.torch.float64, device=self.device)

    def _vec(self, t, level=None):
        """Pointer to t after checking that it holds n_rhs FP64 columns of the level on the device."""
        n = self.ndof(level)
        if (t.dtype != self.torch.float64 or t.device != self.device or not t.is_contiguous()
                or t.numel() != self.R * n):
            raise ValueError(f"expected a contiguous float64 tensor of {self.R} x {n} entries on {self.device}, "
                             f"got {tuple(t.shape)} {t.dtype} on {t.device}")
        return _ptr(t)

    def apply(self, x, level=None):
        level = self.J if level is None else level
        y = self.zeros(level)
        self._check(_lib.bmg_apply(self.h, level, self._vec(x, level), _ptr(y)), "apply")
        return y

    def vcycle(self, r):
        z = self.zeros()
        self._check(_lib.bmg_vcycle(self.h, self._vec(r), _ptr(z)), "vcycle")
        return z

    def vcycle_noalloc(self, r, z):
        """z = B_J r into the caller's z, level vectors in the library's static scratch."""
        self._check(_lib.bmg_vcycle_noalloc(self.h, self._vec(r), self._vec(z)), "vcycle_noalloc")
        return z

    def solve(self, b, rtol=1e-10, maxit=500, x0=None, x=None):
        """x, info: one SolveInfo for one right-hand side, a list of n_rhs otherwise."""
        if x is None:
            x = self.zeros()
        infos = (SolveInfo * self.R)()
        st = _lib.bmg_solve(self.h, self._vec(b), self._vec(x), rtol, maxit,
                            self._vec(x0) if x0 is not None else None, infos)
        if st not in (0, 6):
            self._check(st, "solve")
        return x, (infos[0] if self.R == 1 else list(infos))

    def colour_step(self, level, colour, x, b):
        x = x.clone()
        self._check(_lib.bmg_colour_step(self.h, level, colour, self._vec(x, level), self._vec(b, level)),
                    "colour_step")
        return x

    def smooth(self, level, steps, x, b):
        x = x.clone()
        self._check(_lib.bmg_smooth(self.h, level, steps, self._vec(x, level), self._vec(b, level)), "smooth")
        return x

    def restrict(self, level, rf):
        bc = self.zeros(level - 1)
        self._check(_lib.bmg_restrict(self.h, level, self._vec(rf, level), _ptr(bc)), "restrict")
        return bc

    def prolong_add(self, level, xc, xf):
        xf = xf.clone()
        self._check(_lib.bmg_prolong_add(self.h, level, self._vec(xc, level - 1), self._vec(xf, level)),
                    "prolong_add")
        return xf

    def kernel_timing(self, level, max_launches=4096):
        self._check(_lib.bmg_kernel_timing(self.h, level, max_launches), "kernel_timing")

    def kernel_timing_read(self):
        n, ms, by = C.c_int32(), C.c_double(), C.c_double()
        self._check(_lib.bmg_kernel_timing_read(self.h, C.byref(n), C.byref(ms), C.byref(by)), "kernel_timing_read")
        return n.value, ms.value, by.value

    def coarse_solve(self, b):
        x = self.zeros(0)
        self._check(_lib.bmg_coarse_solve(self.h, self._vec(b, 0), _ptr(x)), "coarse_solve")
        return x

class Batch:
    """Independent problems solved together (bmg_batch_*): one handle per problem,
    the solves spread over `nstreams` worker streams."""

    def __init__(self, params_list, kappas, nstreams=4, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        n = len(params_list)
        self.params = list(params_list)
        self._kap = [_kappa_host(kp, _cells2(pp)) for kp, pp in zip(kappas, self.params)]
        if len(kappas) != n:
            raise ValueError("one kappa field per problem")
        arr = (Params * n)(*self.params)
        kptr = (_P(_D) * n)(*[kp.ctypes.data_as(_P(_D)) for kp in self._kap])
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = _lib.bmg_batch_setup(n, arr, kptr, nstreams, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st:
            raise BmgError(st, f"batch_setup: {_lib.bmg_last_error(None).decode()}")
        self.h = h
        self.n = n
        self._del = False

    def close(self):
        if getattr(self, "h", None):
            _lib.bmg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ndof(self, i):
        hi = C.c_void_p()
        st = _lib.bmg_batch_handle_of(self.h, i, C.byref(hi))
        if st:
            raise BmgError(st, "batch_handle_of")
        N, nu, npr = C.c_int32(), C.c_int64(), C.c_int64()
        _lib.bmg_sizes(hi, self.params[i].levels, C.byref(N), C.byref(nu), C.byref(npr))
        return nu.value + npr.value

    def solve(self, bs, rtol=1e-10, maxit=500, xs=None):
        """bs: one device tensor per problem (n_rhs columns as for Solver.solve).
        Returns (xs, infos, status) with one SolveInfo per right-hand side."""
        t = self.torch
        if len(bs) != self.n:
            raise ValueError("one right-hand side per problem")
        if xs is None:
            xs = [t.zeros_like(b) for b in bs]
        nrec = 0
        for i, (b, x) in enumerate(zip(bs, xs)):
            R = max(1, self.params[i].n_rhs)
            n = self.ndof(i) * R
            for v in (b, x):
                if v.dtype != t.float64 or v.device != self.device or not v.is_contiguous() or v.numel() != n:
                    raise ValueError(f"problem {i}: expected a contiguous float64 tensor of {n} entries")
            nrec += R
        bp = (_VP * self.n)(*[b.data_ptr() for b in bs])
        xp = (_VP * self.n)(*[x.data_ptr() for x in xs])
        infos = (SolveInfo * nrec)()
        st = _lib.bmg_batch_solve(self.h, bp, xp, rtol, maxit, infos)
        if st not in (0, 6):
            raise BmgError(st, f"batch_solve: {_lib.bmg_batch_last_error(self.h).decode()}")
        return xs, list(infos), st


def quad_points(params: Params):
    N = params.n0 << params.levels
    q = params.k + 2
    cell = np.zeros(N * N * q * q * 2)
    face = np.zeros(4 * N * q * 2)
    st = _lib.bmg_quad_points(C.byref(params), cell, face)
    if st:
        raise BmgError(st, "quad_points")
    return cell.reshape(-1, 2), face.reshape(-1, 2)


def assemble_rhs(params: Params, f, s=None, g=None):
    """b (numpy, host) from callables f(x, y) -> (..., 2), s(x, y), g(x, y) -> (..., 2)."""
    cell, face = quad_points(params)

    def values(fn, pts, per_point, what):
        # the library reads exactly per_point values per quadrature point
        v = np.ascontiguousarray(fn(pts[:, 0], pts[:, 1]), dtype=np.float64).reshape(-1)
        if v.size != per_point * pts.shape[0]:
            raise ValueError(f"{what} gave {v.size} values for {pts.shape[0]} points ({per_point} per point expected)")
        return v

    fq = values(f, cell, 2, "f")
    keep = []
    sp = gp = None
    if s is not None:
        sq = values(s, cell, 1, "s")
        keep.append(sq)
        sp = sq.ctypes.data_as(C.c_void_p)
    if g is not None:
        gq = values(g, face, 2, "g")
        keep.append(gq)
        gp = gq.ctypes.data_as(C.c_void_p)
    N = params.n0 << params.levels
    k = params.k
    n = 2 * N * (N + 1) * (k + 1) + 2 * k * (k + 1) * N * N + (k + 1) ** 2 * N * N
    b = np.zeros(n)
    st = _lib.bmg_assemble_rhs(C.byref(params), fq, sp, gp, b)
    if st:
        raise BmgError(st, "assemble_rhs")
    return b


def autotune(params: Params, kappa, trials=5, device="cuda"):
    """(parameters with the faster colouring, {"S9": ms, "L8": ms} per V-cycle), by bmg_autotune."""
    import torch
    kap = _kappa_host(kappa, _cells2(params))
    stream = torch.cuda.current_stream(torch.device(device))
    best = Params()
    ms = np.zeros(2)
    st = _lib.bmg_autotune(C.byref(params), kap, C.c_void_p(stream.cuda_stream), trials, C.byref(best),
                           ms.ctypes.data_as(C.c_void_p))
    if st:
        raise BmgError(st, f"autotune: {_lib.bmg_last_error(None).decode()}")
    return best, {"S9": float(ms[0]), "L8": float(ms[1])}


def autotune_tiles(params: Params, kappa, trials=5, device="cuda"):
    """(parameters with the chosen colouring, rotated_min_n and columns_per_block, list of
    (colouring, rotated_min_n, columns_per_block, ms per V-cycle) rows of the timed
    candidates -- empty when the choice came from the per-process cache), by
    bmg_autotune_tiles."""
    import torch
    kap = _kappa_host(kappa, _cells2(params))
    stream = torch.cuda.current_stream(torch.device(device))
    best = Params()
    rep = np.zeros((16, 4))
    nrep = C.c_int32()
    st = _lib.bmg_autotune_tiles(C.byref(params), kap, C.c_void_p(stream.cuda_stream), trials, C.byref(best),
                                 rep.ctypes.data_as(C.c_void_p), 16, C.byref(nrep))
    if st:
        raise BmgError(st, f"autotune_tiles: {_lib.bmg_last_error(None).decode()}")
    return best, [tuple(r) for r in rep[:nrep.value]]


def export_colouring(params: Params, level):
    """(number of colours, colour of every vertex as an (N+1, N+1) array indexed [vy, vx])."""
    N = params.n0 << level
    out = np.zeros((N + 1) * (N + 1), np.int32)
    nc = C.c_int32()
    st = _lib.bmg_export_colouring(C.byref(params), level, C.byref(nc), out.ctypes.data_as(C.c_void_p))
    if st:
        raise BmgError(st, "export_colouring")
    return nc.value, out.reshape(N + 1, N + 1)


def export_patch(params: Params, kappa, level, vx, vy, with_inverse=True):
    """(dofs ascending, pseudo-inverse or None, colour) of vertex patch (vx, vy)."""
    k = params.k
    cap = 12 * (k + 1) + 8 * k * (k + 1) + 4 * (k + 1) ** 2
    dofs = np.zeros(cap, np.int32)
    inv = np.zeros(cap * cap) if with_inverse else None
    n, col = C.c_int32(), C.c_int32()
    kap = _kappa_host(kappa, _cells2(params))
    st = _lib.bmg_export_patch(C.byref(params), kap, level, vx, vy, C.byref(n), dofs,
                               inv.ctypes.data_as(C.c_void_p) if inv is not None else None, C.byref(col))
    if st:
        raise BmgError(st, "export_patch")
    m = n.value
    return dofs[:m].copy(), (inv[:m * m].reshape(m, m).copy() if inv is not None else None), col.value


def export_level_matrix(params: Params, kappa, level):
    N = params.n0 << level
    k = params.k
    n = 2 * N * (N + 1) * (k + 1) + 2 * k * (k + 1) * N * N + (k + 1) ** 2 * N * N
    out = np.zeros(n * n)
    st = _lib.bmg_export_level_matrix(C.byref(params), _kappa_host(kappa, _cells2(params)), level, out)
    if st:
        raise BmgError(st, "export_level_matrix")
    return out.reshape(n, n)


def from_workload(w, prec=P_FP64, restart=100, device="cuda", dense_coarse_max=DENSE_COARSE_DEFAULT, n_rhs=1,
                  colouring=COLOURING_S9, **kw):
    p = make_params(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.cycle, w.m_fine, prec, restart, dense_coarse_max,
                    n_rhs, colouring)
    return Solver(p, w.kappa, device=device, **kw)


# ---------------------------------------------------------------------------------
# 3-D (hexahedral) path: include/bmg3.h
# ---------------------------------------------------------------------------------
class Params3(C.Structure):
    _fields_ = [("n0", C.c_int32), ("levels", C.c_int32), ("k", C.c_int32), ("mu", C.c_double),
                ("sigma", C.c_double), ("cycle", C.c_int32), ("m_fine", C.c_int32), ("restart", C.c_int32),
                ("precond_prec", C.c_int32), ("bc", C.c_int32 * 6)]


_sig3 = {
    "bmg3_setup": [_P(Params3), _dp, _VP, _P(_VP)],
    "bmg3_destroy": [_VP],
    "bmg3_sizes": [_VP, _I32, _P(_I32), _P(_I64), _P(_I64), _P(_I64)],
    "bmg3_assemble_rhs": [_P(Params3), _dp, _dp, _dp, _dp],
    "bmg3_apply": [_VP, _I32, _VP, _VP],
    "bmg3_smooth": [_VP, _I32, _I32, _VP, _VP],
    "bmg3_vcycle": [_VP, _VP, _VP],
    "bmg3_solve": [_VP, _VP, _VP, _D, _I32, _P(SolveInfo)],
    "bmg3_export_patch": [_VP, _I32, _I32, _I32, _I32, _P(_I32), _ip, _VP],
    "bmg3_export_level_csr": [_P(Params3), _dp, _I32, _P(_I64), _VP, _VP, _VP],
    "bmg3_export_patch_host": [_P(Params3), _dp, _I32, _I32, _I32, _I32, _P(_I32), _ip, _VP],
}
EXPORTS += list(_sig3) + ["bmg3_last_error"]
for _name, _args in _sig3.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.bmg3_last_error.argtypes = [_VP]
_lib.bmg3_last_error.restype = C.c_char_p


def make_params3(n0, levels, mu, sigma=6.0, cycle=CYCLE_VARIABLE, m_fine=2, restart=50, k=1, prec=P_FP64,
                 bc=(0, 0, 0, 0, 0, 0)):
    """prec: P_FP64, or P_FP32 for FP32-stored patch pseudo-inverses (FP64 arithmetic);
    bc: BC_DIRICHLET / BC_OPEN per side (x=0, x=1, y=0, y=1, z=0, z=1)."""
    p = Params3()
    p.n0, p.levels, p.k, p.mu, p.sigma = n0, levels, k, float(mu), float(sigma)
    p.cycle, p.m_fine, p.restart, p.precond_prec = cycle, m_fine, restart, prec
    if len(bc) != 6:
        raise ValueError("bc: six sides")
    for i, v in enumerate(bc):
        p.bc[i] = int(v)
    return p


def _ndof3(N, k):
    """Unknowns of the 3-D level with N cells per side (the layout of bmg3.h)."""
    nb = k + 1
    return 3 * (N + 1) * N * N * nb * nb + 3 * k * nb * nb * N ** 3 + nb ** 3 * N ** 3


def assemble_rhs3(params: Params3, kappa, f=(0.0, 0.0, 0.0), g=(1.0, 0.0, 0.0)):
    """Right-hand side for constant body force f and constant boundary data g (host)."""
    N = params.n0 << (params.levels - 1)
    out = np.zeros(_ndof3(N, params.k))
    fv = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    gv = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
    if fv.size != 3 or gv.size != 3:
        raise ValueError("f and g are constant 3-vectors")
    st = _lib.bmg3_assemble_rhs(C.byref(params), _kappa_host(kappa, _cells3(params)), fv, gv, out)
    if st:
        raise BmgError(st, f"assemble_rhs3: {_lib.bmg3_last_error(None).decode()}")
    return out


class Solver3:
    """One 3-D problem on the GPU (handle of the C library; it owns its device memory)."""

    def __init__(self, params: Params3, kappa, device="cuda"):
        import torch
        self.torch = torch
        self.params = params
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = _lib.bmg3_setup(C.byref(params), _kappa_host(kappa, _cells3(params)),
                             C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st:
            raise BmgError(st, f"setup3: {_lib.bmg3_last_error(None).decode()}")
        self.h = h
        self.levels = params.levels

    def close(self):
        if getattr(self, "h", None):
            _lib.bmg3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st:
            raise BmgError(st, f"{what}: {_lib.bmg3_last_error(self.h).decode()}")

    def sizes(self, level=None):
        level = self.levels - 1 if level is None else level
        N, nu, npr, npa = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
        self._check(_lib.bmg3_sizes(self.h, level, C.byref(N), C.byref(nu), C.byref(npr), C.byref(npa)), "sizes")
        return N.value, nu.value, npr.value, npa.value

    def ndof(self, level=None):
        _, a, b, _ = self.sizes(level)
        return a + b

    def _vec(self, t, level=None):
        n = self.ndof(level)
        if t.dtype != self.torch.float64 or t.device != self.device or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"expected a contiguous float64 tensor of {n} entries on {self.device}")
        return _ptr(t)

    def apply(self, x, level=None):
        level = self.levels - 1 if level is None else level
        y = self.torch.empty_like(x)
        self._check(_lib.bmg3_apply(self.h, level, self._vec(x, level), self._vec(y, level)), "apply")
        return y

    def smooth(self, level, steps, x, b):
        self._check(_lib.bmg3_smooth(self.h, level, steps, self._vec(x, level), self._vec(b, level)), "smooth")

    def vcycle(self, r):
        z = self.torch.empty_like(r)
        self._check(_lib.bmg3_vcycle(self.h, self._vec(r), self._vec(z)), "vcycle")
        return z

    def solve(self, b, rtol=1e-10, maxit=200):
        x = self.torch.empty_like(b)
        info = SolveInfo()
        st = _lib.bmg3_solve(self.h, self._vec(b), self._vec(x), float(rtol), int(maxit), C.byref(info))
        if st and st != 6:
            self._check(st, "solve")
        return x, info

    def export_patch(self, level, vx, vy, vz):
        n = C.c_int32()
        dofs = np.zeros(256, dtype=np.int32)
        pinv = np.zeros(256 * 256)
        self._check(_lib.bmg3_export_patch(self.h, level, vx, vy, vz, C.byref(n), dofs,
                                           pinv.ctypes.data_as(C.c_void_p)), "export_patch")
        m = n.value
        return dofs[:m].copy(), pinv[:m * m].reshape(m, m).T.copy()


def export_level_csr3(params: Params3, kappa, level):
    """(rowptr, colidx, values) of the library's level operator (host assembly)."""
    kap = _kappa_host(kappa, _cells3(params))
    nnz = C.c_int64()
    st = _lib.bmg3_export_level_csr(C.byref(params), kap, level, C.byref(nnz), None, None, None)
    if st:
        raise BmgError(st, f"export_level_csr3: {_lib.bmg3_last_error(None).decode()}")
    n = _ndof3(params.n0 << level, params.k)
    rp = np.zeros(n + 1, dtype=np.int32)
    ci = np.zeros(nnz.value, dtype=np.int32)
    v = np.zeros(nnz.value)
    st = _lib.bmg3_export_level_csr(C.byref(params), kap, level, C.byref(nnz), rp.ctypes.data_as(C.c_void_p),
                                    ci.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p))
    if st:
        raise BmgError(st, "export_level_csr3")
    return rp, ci, v


def export_patch_host3(params: Params3, kappa, level, vx, vy, vz):
    """(dofs, pseudo-inverse) of one vertex patch, assembled on the host by the library."""
    n = C.c_int32()
    dofs = np.zeros(256, dtype=np.int32)
    pinv = np.zeros(256 * 256)
    st = _lib.bmg3_export_patch_host(C.byref(params), _kappa_host(kappa, _cells3(params)), level, vx, vy,
                                     vz, C.byref(n), dofs, pinv.ctypes.data_as(C.c_void_p))
    if st:
        raise BmgError(st, f"export_patch_host3: {_lib.bmg3_last_error(None).decode()}")
    m = n.value
    return dofs[:m].copy(), pinv[:m * m].reshape(m, m).T.copy()
