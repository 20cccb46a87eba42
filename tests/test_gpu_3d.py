"""GPU parity of the 3-D path (HIP kernels through the C-ABI) against the 3-D oracle:
RT_1 and RT_0, Brinkman and Darcy, Dirichlet and open sides.  Operator 1e-13, one
smoothing step 1e-11, V-cycle 1e-10 (max norm); FP64 solves: iteration count within
+-1 of the oracle's and the iterate after the same count within 1e-10 (max norm;
zero-mean pressures when every side is Dirichlet)."""
import numpy as np
import pytest

from oracle import oracle3d as o3

torch = pytest.importorskip("torch")
bmg = pytest.importorskip("paper_1602_04858_amd.bmg")

pytestmark = pytest.mark.gpu

MU = 1e-2


def _kappa(n, seed):
    return 10.0 ** np.clip(np.random.default_rng(seed).normal(-3, 1.5, n ** 3), -6, 0)


_cache = {}


def _pair(n0, levels, seed=1, cycle=1, m_fine=2, k=1, mu=MU):
    key = (n0, levels, seed, cycle, m_fine, k, mu)
    if key not in _cache:
        N = n0 << (levels - 1)
        kap = _kappa(N, seed)
        sigma = (k + 1) * (k + 2)  # the penalty of Section 4.1
        print(f"3-D case k={k} mu={mu} n0={n0} levels={levels} N={N} seed={seed}", flush=True)
        s = bmg.Solver3(bmg.make_params3(n0, levels, mu, sigma=sigma, cycle=cycle, m_fine=m_fine, k=k), kap)
        o = o3.Oracle3D(n0, levels, k, mu, sigma, kap, cycle=cycle, m_fine=m_fine)
        _cache[key] = (s, o, kap)
    return _cache[key]


def _oracle_iterate(o, b, its):
    """The oracle's FGMRES iterate after exactly `its` iterations."""
    x, n, _ = o.fgmres(b, rtol=1e-30, maxit=its)
    assert abs(n) == its
    return x


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("level", [0, 1, 2])
def test_apply_3d(level):
    s, o, _ = _pair(1, 3)
    n = o.lev[level].sp.ndof
    x = np.random.default_rng(level).standard_normal(n)
    y = s.apply(_dev(x), level).cpu().numpy()
    yo = o.lev[level].A @ x
    assert np.abs(y - yo).max() <= 1e-13 * np.abs(yo).max()


@pytest.mark.parametrize("level", [1, 2])
def test_smoothing_step_3d(level):
    s, o, _ = _pair(1, 3)
    L = o.lev[level]
    rng = np.random.default_rng(10 + level)
    x = rng.standard_normal(L.sp.ndof)
    x[L.sp.cons] = 0.0
    b = rng.standard_normal(L.sp.ndof)
    xg = _dev(x)
    s.smooth(level, 1, xg, _dev(b))
    xo = x.copy()
    o.sm[level].step(xo, b)
    assert np.abs(xg.cpu().numpy() - xo).max() <= 1e-11 * np.abs(xo).max()


@pytest.mark.parametrize("n0,levels", [(1, 3), (1, 4), (2, 2), (4, 2)])
def test_vcycle_3d(n0, levels):
    s, o, _ = _pair(n0, levels)
    n = o.lev[-1].sp.ndof
    r = np.random.default_rng(5).standard_normal(n)
    z = s.vcycle(_dev(r)).cpu().numpy()
    zo = o.vcycle(r)
    assert np.abs(z - zo).max() <= 1e-10 * np.abs(zo).max()


@pytest.mark.parametrize("n0,levels", [(1, 3), (1, 4), (2, 2), (4, 2)])
def test_solve_3d_matches_oracle(n0, levels):
    s, o, kap = _pair(n0, levels)
    lev = o.lev[-1]
    g = lambda x, y, z: np.array([np.ones_like(x), 0 * x, 0 * x])
    b = lev.rhs(lambda x, y, z: np.zeros((3,) + np.shape(x)), g)
    x, info = s.solve(_dev(b), rtol=1e-10, maxit=100)
    xo, its, tr = o.fgmres(b, rtol=1e-10, maxit=100)
    assert info.converged and info.rel_residual_true <= 1e-10
    assert abs(info.iterations - its) <= 1
    if info.iterations != its:
        xo = _oracle_iterate(o, b, info.iterations)
    xg = x.cpu().numpy()
    d = xg - xo
    d[lev.sp.n_u:] -= o.pressure_mean(xg) - o.pressure_mean(xo)
    # the iterate after the same number of iterations, pressures compared with zero mean
    assert np.abs(d).max() <= 1e-10 * np.abs(xo).max(), np.abs(d).max() / np.abs(xo).max()
    # the library's own right-hand side gives the same solve
    b2 = bmg.assemble_rhs3(s.params, kap, (0.0, 0.0, 0.0), (1.0, 0.0, 0.0))
    assert np.abs(b2 - b).max() <= 1e-13 * np.abs(b).max()


def test_patch_export_matches_host_build_3d():
    s, _, kap = _pair(1, 3)
    for v in [(2, 2, 2), (0, 4, 1), (4, 4, 4)]:
        d1, p1 = s.export_patch(2, *v)
        d2, p2 = bmg.export_patch_host3(s.params, kap, 2, *v)
        assert np.array_equal(d1, d2) and np.array_equal(p1, p2)


def test_zero_rhs_and_coarse_only_3d():
    s, o, _ = _pair(1, 3)
    n = o.lev[-1].sp.ndof
    x, info = s.solve(torch.zeros(n, dtype=torch.float64, device="cuda"))
    assert info.converged and info.iterations == 0 and float(x.abs().max()) == 0.0
    kap = _kappa(2, 4)
    s1 = bmg.Solver3(bmg.make_params3(2, 1, MU), kap)
    o1 = o3.Oracle3D(2, 1, 1, MU, 6.0, kap)
    g = lambda x, y, z: np.array([np.ones_like(x), 0 * x, 0 * x])
    b = o1.lev[0].rhs(lambda x, y, z: np.zeros((3,) + np.shape(x)), g)
    _, info = s1.solve(_dev(b), rtol=1e-10)
    assert info.iterations == 1 and info.rel_residual_true < 1e-12
    s1.close()


def test_solve_3d_at_n16_sampled():
    """N = 16 (5 levels): converged solve; operator checked against the oracle's
    assembly at this size and the true residual recomputed on the host."""
    N = 16
    kap = _kappa(N, 7)
    print("3-D case N=16 levels=5 seed=7", flush=True)
    s = bmg.Solver3(bmg.make_params3(1, 5, MU), kap)
    lev = o3.Level(N, 1, MU, 6.0, kap)
    g = lambda x, y, z: np.array([np.ones_like(x), 0 * x, 0 * x])
    b = bmg.assemble_rhs3(s.params, kap, (0.0, 0.0, 0.0), (1.0, 0.0, 0.0))
    x, info = s.solve(_dev(b), rtol=1e-10, maxit=100)
    xg = x.cpu().numpy()
    assert info.converged and info.iterations <= 20
    assert np.linalg.norm(b - lev.A @ xg) <= 2e-10 * np.linalg.norm(b)
    xr = np.random.default_rng(1).standard_normal(lev.sp.ndof)
    y = s.apply(_dev(xr)).cpu().numpy()
    assert np.abs(y - lev.A @ xr).max() <= 1e-13 * np.abs(y).max()
    s.close()


def test_fp32_stored_inverses_3d():
    """FP32 storage of the patch pseudo-inverses (FP64 arithmetic and vectors): the
    stored entries are the FP64 host ones rounded to nearest, the V-cycle moves by about
    the FP32 rounding of the inverses (each entry relative 2^-24; tolerance 2e-5 allows
    for the sums over the smoothing steps of all levels), and FGMRES still reaches 1e-10
    with at most one more iteration."""
    s, o, kap = _pair(1, 4)
    s32 = bmg.Solver3(bmg.make_params3(1, 4, MU, prec=bmg.P_FP32), kap)
    for v in [(3, 3, 3), (0, 8, 2)]:
        _, p32 = s32.export_patch(3, *v)
        _, p64 = bmg.export_patch_host3(s.params, kap, 3, *v)
        assert np.array_equal(p32, p64.astype(np.float32).astype(np.float64))
    n = o.lev[-1].sp.ndof
    r = np.random.default_rng(21).standard_normal(n)
    z32 = s32.vcycle(_dev(r)).cpu().numpy()
    zo = o.vcycle(r)
    assert np.abs(z32 - zo).max() <= 2e-5 * np.abs(zo).max()
    lev = o.lev[-1]
    g = lambda x, y, z: np.array([np.ones_like(x), 0 * x, 0 * x])
    b = _dev(lev.rhs(lambda x, y, z: np.zeros((3,) + np.shape(x)), g))
    _, i64 = s.solve(b, rtol=1e-10)
    _, i32 = s32.solve(b, rtol=1e-10)
    assert i32.converged and i32.rel_residual_true <= 1e-10 and i32.iterations <= i64.iterations + 1
    s32.close()


def test_not_converged_and_argument_errors_3d():
    import ctypes as C
    s, o, _ = _pair(1, 3)
    lev = o.lev[-1]
    g = lambda x, y, z: np.array([np.ones_like(x), 0 * x, 0 * x])
    b = _dev(lev.rhs(lambda x, y, z: np.zeros((3,) + np.shape(x)), g))
    x, info = s.solve(b, rtol=1e-14, maxit=2)
    assert info.converged == 0 and info.iterations == 2 and info.rel_residual_true > 1e-14
    lib = bmg.lib()
    y = torch.empty_like(b)
    ptr = lambda t: C.c_void_p(t.data_ptr())
    assert lib.bmg3_apply(s.h, 7, ptr(b), ptr(y)) == 1
    assert lib.bmg3_smooth(s.h, 0, 1, ptr(y), ptr(b)) == 1
    assert lib.bmg3_solve(s.h, ptr(b), ptr(y), 0.0, 10, None) == 1
    assert lib.bmg3_solve(s.h, ptr(b), ptr(y), 1e-10, 0, None) == 1
    n = C.c_int32()
    dofs = np.zeros(208, dtype=np.int32)
    assert lib.bmg3_export_patch(s.h, 2, 5, 0, 0, C.byref(n), dofs, None) == 1
    assert lib.bmg3_sizes(s.h, 3, None, None, None, None) == 1


def test_nonfinite_rhs_3d():
    """A NaN or Inf in b is reported as BMG_E_NONFINITE and x is left untouched."""
    import ctypes as C
    s, o, _ = _pair(1, 3)
    n = o.lev[-1].sp.ndof
    lib = bmg.lib()
    ptr = lambda t: C.c_void_p(t.data_ptr())
    for bad in (float("nan"), float("inf")):
        print(f"3-D non-finite right-hand side: {bad}", flush=True)
        b = torch.ones(n, dtype=torch.float64, device="cuda")
        b[n // 2] = bad
        y = torch.full_like(b, 3.0)
        assert lib.bmg3_solve(s.h, ptr(b), ptr(y), 1e-10, 10, None) == 7
        torch.cuda.synchronize()
        assert bool((y == 3.0).all())


# ---------------------------------------------------------------------------------
# RT_0 x dQ_0 (k = 0): Brinkman and the Darcy limit mu = 0
# ---------------------------------------------------------------------------------
KMU0 = [(0, MU), (0, 0.0)]


@pytest.mark.parametrize("k,mu", KMU0)
@pytest.mark.parametrize("level", [0, 1, 2])
def test_apply_rt0_3d(level, k, mu):
    s, o, _ = _pair(1, 3, k=k, mu=mu)
    n = o.lev[level].sp.ndof
    x = np.random.default_rng(level).standard_normal(n)
    y = s.apply(_dev(x), level).cpu().numpy()
    yo = o.lev[level].A @ x
    assert np.abs(y - yo).max() <= 1e-13 * np.abs(yo).max()


@pytest.mark.parametrize("k,mu", KMU0)
@pytest.mark.parametrize("level", [1, 2])
def test_smoothing_step_rt0_3d(level, k, mu):
    s, o, _ = _pair(1, 3, k=k, mu=mu)
    L = o.lev[level]
    rng = np.random.default_rng(10 + level)
    x = rng.standard_normal(L.sp.ndof)
    x[L.sp.cons] = 0.0
    b = rng.standard_normal(L.sp.ndof)
    xg = _dev(x)
    s.smooth(level, 1, xg, _dev(b))
    xo = x.copy()
    o.sm[level].step(xo, b)
    assert np.abs(xg.cpu().numpy() - xo).max() <= 1e-11 * np.abs(xo).max()


@pytest.mark.parametrize("k,mu", KMU0)
@pytest.mark.parametrize("n0,levels", [(1, 3), (1, 4), (2, 3)])
def test_vcycle_rt0_3d(n0, levels, k, mu):
    s, o, _ = _pair(n0, levels, k=k, mu=mu)
    n = o.lev[-1].sp.ndof
    r = np.random.default_rng(5).standard_normal(n)
    r[o.lev[-1].sp.cons] = 0.0
    z = s.vcycle(_dev(r)).cpu().numpy()
    zo = o.vcycle(r)
    assert np.abs(z - zo).max() <= 1e-10 * np.abs(zo).max()


@pytest.mark.parametrize("k,mu", KMU0)
@pytest.mark.parametrize("n0,levels", [(1, 3), (1, 4), (2, 3)])
def test_solve_rt0_3d_matches_oracle(n0, levels, k, mu):
    """FP64 solve: iteration count within +-1 of the oracle's, the iterate after the
    same count within 1e-10 (max norm, zero-mean pressures)."""
    s, o, kap = _pair(n0, levels, k=k, mu=mu)
    lev = o.lev[-1]
    g = lambda x, y, z: np.array([np.ones_like(x), 0 * x, 0 * x])
    f = lambda x, y, z: np.array([0 * x, np.ones_like(x), 0 * x])
    b = lev.rhs(f, g)
    b2 = bmg.assemble_rhs3(s.params, kap, (0.0, 1.0, 0.0), (1.0, 0.0, 0.0))
    assert np.abs(b2 - b).max() <= 1e-13 * np.abs(b).max()
    x, info = s.solve(_dev(b), rtol=1e-10, maxit=200)
    xo, its, tr = o.fgmres(b, rtol=1e-10, maxit=200)
    assert info.converged and info.rel_residual_true <= 1e-10
    assert abs(info.iterations - its) <= 1, (info.iterations, its)
    if info.iterations != its:
        xo = _oracle_iterate(o, b, info.iterations)
    xg = x.cpu().numpy()
    d = xg - xo
    d[lev.sp.n_u:] -= o.pressure_mean(xg) - o.pressure_mean(xo)
    print(f"RT_0 3-D mu={mu} n0={n0} levels={levels}: {info.iterations} iterations (oracle {its}), "
          f"max diff {np.abs(d).max() / np.abs(xo).max():.2e}")
    assert np.abs(d).max() <= 1e-10 * np.abs(xo).max()


def test_rt0_3d_at_n32_sampled():
    """RT_0 Darcy at N = 32 (6 levels), the contrast-1e6 field: converged solve, the
    operator against the oracle's assembly at this size, the true residual recomputed
    on the host."""
    N = 32
    kap = _kappa(N, 8)
    print("3-D case k=0 mu=0 N=32 levels=6 seed=8", flush=True)
    s = bmg.Solver3(bmg.make_params3(1, 6, 0.0, sigma=2.0, k=0), kap)
    lev = o3.Level(N, 0, 0.0, 2.0, kap)
    b = bmg.assemble_rhs3(s.params, kap, (0.0, 0.0, 0.0), (1.0, 0.0, 0.0))
    x, info = s.solve(_dev(b), rtol=1e-10, maxit=200)
    xg = x.cpu().numpy()
    assert info.converged
    assert np.linalg.norm(b - lev.A @ xg) <= 2e-10 * np.linalg.norm(b)
    xr = np.random.default_rng(1).standard_normal(lev.sp.ndof)
    y = s.apply(_dev(xr)).cpu().numpy()
    assert np.abs(y - lev.A @ xr).max() <= 1e-13 * np.abs(y).max()
    print(f"RT_0 3-D Darcy N=32: {info.iterations} iterations", flush=True)
    s.close()


# ---------------------------------------------------------------------------------
# Open sides (natural condition; an open side fixes the pressure level)
# ---------------------------------------------------------------------------------
OPEN_CASES = [(1, MU, (0, 0, 0, 0, 1, 1)), (0, MU, (0, 0, 1, 1, 0, 0)), (0, 0.0, (0, 0, 0, 0, 0, 1)),
              (1, MU, (1, 0, 0, 0, 0, 0))]
_ocache = {}


def _open_pair(k, mu, bc, n0=1, levels=3):
    key = (k, mu, bc, n0, levels)
    if key not in _ocache:
        N = n0 << (levels - 1)
        kap = _kappa(N, 3)
        sigma = (k + 1) * (k + 2)
        print(f"3-D case k={k} mu={mu} bc={bc} n0={n0} levels={levels}", flush=True)
        s = bmg.Solver3(bmg.make_params3(n0, levels, mu, sigma=sigma, k=k, bc=bc), kap)
        o = o3.Oracle3D(n0, levels, k, mu, sigma, kap, bc=bc)
        _ocache[key] = (s, o, kap)
    return _ocache[key]


@pytest.mark.parametrize("k,mu,bc", OPEN_CASES)
def test_open_sides_steps_3d(k, mu, bc):
    """Operator, one smoothing step and the V-cycle against the oracle."""
    s, o, _ = _open_pair(k, mu, bc)
    for level in (0, 1, 2):
        L = o.lev[level]
        x = np.random.default_rng(level).standard_normal(L.sp.ndof)
        y = s.apply(_dev(x), level).cpu().numpy()
        assert np.abs(y - L.A @ x).max() <= 1e-13 * np.abs(L.A @ x).max(), level
    L = o.lev[2]
    rng = np.random.default_rng(12)
    x = rng.standard_normal(L.sp.ndof)
    x[L.sp.cons] = 0.0
    b = rng.standard_normal(L.sp.ndof)
    xg = _dev(x)
    s.smooth(2, 1, xg, _dev(b))
    xo = x.copy()
    o.sm[2].step(xo, b)
    assert np.abs(xg.cpu().numpy() - xo).max() <= 1e-11 * np.abs(xo).max()
    r = rng.standard_normal(L.sp.ndof)
    r[L.sp.cons] = 0.0
    z = s.vcycle(_dev(r)).cpu().numpy()
    zo = o.vcycle(r)
    assert np.abs(z - zo).max() <= 1e-10 * np.abs(zo).max()


@pytest.mark.parametrize("k,mu,bc", OPEN_CASES)
@pytest.mark.parametrize("n0,levels", [(1, 3), (2, 3)])
def test_open_sides_solve_3d(k, mu, bc, n0, levels):
    """FP64 solve with a body force through the open sides: iteration count within +-1
    of the oracle's and the iterate after the same count within 1e-10 (max norm; the
    pressure is determined, nothing removed)."""
    s, o, kap = _open_pair(k, mu, bc, n0, levels)
    lev = o.lev[-1]
    f = lambda x, y, z: np.array([0.3 + 0 * x, -0.2 + 0 * x, np.ones_like(x)])
    g = lambda x, y, z: np.array([np.ones_like(x), 0 * x, 0.5 + 0 * x])
    b = lev.rhs(f, g)
    b2 = bmg.assemble_rhs3(s.params, kap, (0.3, -0.2, 1.0), (1.0, 0.0, 0.5))
    assert np.abs(b2 - b).max() <= 1e-13 * np.abs(b).max()
    x, info = s.solve(_dev(b), rtol=1e-10, maxit=200)
    xo, its, tr = o.fgmres(b, rtol=1e-10, maxit=200)
    assert info.converged and info.rel_residual_true <= 1e-10
    assert abs(info.iterations - its) <= 1, (info.iterations, its)
    if info.iterations != its:
        xo = _oracle_iterate(o, b, info.iterations)
    xg = x.cpu().numpy()
    print(f"open 3-D k={k} mu={mu} bc={bc} n0={n0}: {info.iterations} iterations (oracle {its}), max diff "
          f"{np.abs(xg - xo).max() / np.abs(xo).max():.2e}")
    assert np.abs(xg - xo).max() <= 1e-10 * np.abs(xo).max()


def test_setup_rejects_patches_beyond_the_kernel_limit_3d():
    """RT_1 with every side open on a two-cell level: the centre patch (304 dofs)
    exceeds the colour kernel's 256 rows, and setup says so."""
    with pytest.raises(bmg.BmgError) as e:
        bmg.Solver3(bmg.make_params3(1, 2, MU, bc=(1, 1, 1, 1, 1, 1)), np.ones(8))
    assert e.value.status == 2


@pytest.mark.parametrize("mu", [MU, 0.0])
def test_rt0_coarsest_8_3d(mu):
    """RT_0 with an 8^3 coarsest mesh (2240 unknowns inverted densely, the bench's
    choice for RT_0) and 16^3 on top: V-cycle and solve against the oracle."""
    s, o, kap = _pair(8, 2, k=0, mu=mu)
    lev = o.lev[-1]
    r = np.random.default_rng(6).standard_normal(lev.sp.ndof)
    r[lev.sp.cons] = 0.0
    z = s.vcycle(_dev(r)).cpu().numpy()
    zo = o.vcycle(r)
    assert np.abs(z - zo).max() <= 1e-10 * np.abs(zo).max()
    g = lambda x, y, z_: np.array([np.ones_like(x), 0 * x, 0 * x])
    f = lambda x, y, z_: np.array([0 * x, np.ones_like(x), 0 * x])
    b = lev.rhs(f, g)
    x, info = s.solve(_dev(b), rtol=1e-10, maxit=200)
    xo, its, tr = o.fgmres(b, rtol=1e-10, maxit=200)
    assert info.converged and info.rel_residual_true <= 1e-10
    assert abs(info.iterations - its) <= 1, (info.iterations, its)
    if info.iterations != its:
        xo = _oracle_iterate(o, b, info.iterations)
    xg = x.cpu().numpy()
    d = xg - xo
    d[lev.sp.n_u:] -= o.pressure_mean(xg) - o.pressure_mean(xo)
    print(f"RT_0 3-D coarsest 8^3 mu={mu}: {info.iterations} iterations (oracle {its}), max diff "
          f"{np.abs(d).max() / np.abs(xo).max():.2e}")
    assert np.abs(d).max() <= 1e-10 * np.abs(xo).max()
