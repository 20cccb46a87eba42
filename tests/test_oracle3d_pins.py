"""Pins of the 3-D oracle against what the mathematics fixes (CPU only).

Each test is chosen so that a plausible slip in the 3-D assembly, transfers or smoother
(a dropped face term, a wrong sign of the pressure coupling, a transposed block, a
wrong child offset, a missing Nitsche term) fails at least one of them.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import oracle3d as o3


def _kappa(n, seed, lo=-2.0, hi=0.0):
    return 10.0 ** np.random.default_rng(seed).uniform(lo, hi, n ** 3)


def _cell_kappa(kap, n, x, y, z):
    c = lambda t: np.minimum((np.asarray(t) * n).astype(int), n - 1)
    return kap[(c(z) * n + c(y)) * n + c(x)]


# P1: u = (y, z, x) (divergence free, in RT_1), p = xyz - 1/8 (in dQ_1, mean 0):
# f = -mu lap u + kappa u + grad p; g = u on all sides.  The discrete solution is exact.
@pytest.mark.parametrize("mu", [1.0, 1e-2])
def test_polynomial_solution_is_reproduced_3d(mu):
    n0, levels = 1, 2
    n = n0 << (levels - 1)
    kap = _kappa(n, 5)
    o = o3.Oracle3D(n0, levels, 1, mu, 6.0, kap)
    lev = o.lev[-1]
    k_at = lambda x, y, z: _cell_kappa(kap, n, x, y, z)
    f = lambda x, y, z: np.array([k_at(x, y, z) * y + y * z, k_at(x, y, z) * z + x * z, k_at(x, y, z) * x + x * y])
    g = lambda x, y, z: np.array([y, z, x])
    b = lev.rhs(f, g)
    rng = np.random.default_rng(7)
    P = rng.random((40, 3))
    ue = np.stack([P[:, 1], P[:, 2], P[:, 0]], 1)
    pe = P[:, 0] * P[:, 1] * P[:, 2] - 0.125
    for x in (o.direct_solve(b), o.fgmres(b, rtol=1e-13, maxit=50)[0]):
        U, Pv = o3.evaluate(lev, x, P)
        assert np.abs(U - ue).max() < 1e-11
        assert np.abs(Pv - o.pressure_mean(x) - pe).max() < 1e-10


# P2: f = grad(phi), phi the continuous trilinear hat at an interior vertex, g = 0:
# u_h = 0 and p_h = phi (up to the mean) exactly -- pins the sign and the scaling of
# the pressure coupling against the body force.
def test_hat_gradient_pressure_robustness_3d():
    n0, levels = 2, 2
    n = n0 << (levels - 1)
    h = 1.0 / n
    o = o3.Oracle3D(n0, levels, 1, 1e-2, 6.0, _kappa(n, 9, -6.0, 0.0))
    lev = o.lev[-1]
    v = np.array([2, 1, 3]) * h
    hat1 = lambda t, c: np.maximum(0.0, 1.0 - np.abs(t - c) / h)
    dhat1 = lambda t, c: np.where(np.abs(t - c) < h, -np.sign(t - c) / h, 0.0)
    phi = lambda x, y, z: hat1(x, v[0]) * hat1(y, v[1]) * hat1(z, v[2])
    f = lambda x, y, z: np.array([dhat1(x, v[0]) * hat1(y, v[1]) * hat1(z, v[2]),
                                  hat1(x, v[0]) * dhat1(y, v[1]) * hat1(z, v[2]),
                                  hat1(x, v[0]) * hat1(y, v[1]) * dhat1(z, v[2])])
    zero = lambda x, y, z: np.zeros((3,) + np.shape(x))
    x = o.direct_solve(lev.rhs(f, zero))
    P = np.random.default_rng(3).random((60, 3))
    U, Pv = o3.evaluate(lev, x, P)
    assert np.abs(U).max() < 1e-11
    # the hat integrates to h^3 over the unit cube
    assert np.abs((Pv - o.pressure_mean(x)) - (phi(P[:, 0], P[:, 1], P[:, 2]) - h ** 3)).max() < 1e-10


def test_operator_symmetry_and_essential_rows_3d():
    lev = o3.Level(4, 1, 0.3, 6.0, _kappa(4, 1))
    for A in (lev.A, lev.A_full):
        assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
    cons = np.flatnonzero(lev.sp.cons)
    assert len(cons) == 6 * 16 * 4  # six sides, 16 faces each, (k+1)^2 dofs per face
    Ac = lev.A[cons]
    assert np.array_equal(Ac.indices, cons) and np.all(Ac.data == 1.0)
    # the constant pressure is in the kernel of the operator with essential normals
    assert np.abs(lev.A @ lev.cvec).max() < 1e-13


def test_divergence_free_solution_3d():
    o = o3.Oracle3D(2, 2, 1, 1e-2, 6.0, _kappa(4, 4, -6.0, 0.0))
    lev = o.lev[-1]
    zero = lambda x, y, z: np.zeros((3,) + np.shape(x))
    g = lambda x, y, z: np.array([np.ones_like(x), 0 * x, 0 * x])
    x = o.direct_solve(lev.rhs(zero, g))
    nu = lev.sp.n_u
    div = lev.A_full[nu:, :nu] @ x[:nu]
    assert np.abs(div).max() < 1e-12
    # the essential normal values are those of g: 1 on x-faces at x = 0 and x = 1
    assert np.abs(x[lev.sp.cons] - lev.essential_values(g)[lev.sp.cons]).max() == 0.0


def test_patch_pseudo_inverse_invariants_3d():
    lev = o3.Level(4, 1, 0.5, 6.0, _kappa(4, 2))
    sm = o3.Smoother(lev)
    rng = np.random.default_rng(0)
    sizes = set()
    for pi in rng.choice(len(sm.patches), 12, replace=False).tolist() + [0, len(sm.patches) // 2]:
        (vx, vy, vz), dofs, rows, pinv, singular = sm.patches[pi]
        sizes.add(len(dofs))
        A_S = rows[:, dofs].toarray()
        assert singular
        c = lev.cvec[dofs] / np.linalg.norm(lev.cvec[dofs])
        assert np.abs(A_S @ pinv @ A_S - A_S).max() < 1e-10 * np.abs(A_S).max()
        assert np.abs(pinv @ c).max() < 1e-10 * np.abs(pinv).max()
        assert np.abs(pinv - pinv.T).max() < 1e-10 * np.abs(pinv).max()
        # after one patch correction the local residual lies in the kernel direction
        x = rng.standard_normal(lev.sp.ndof)
        x[lev.sp.cons] = 0.0
        b = rng.standard_normal(lev.sp.ndof)
        r = b[dofs] - rows @ x
        x[dofs] += pinv @ r
        r2 = b[dofs] - rows @ x
        assert np.abs(r2 - c * (c @ r2)).max() < 1e-9 * np.abs(r).max()
    # interior patch: 12 inner faces x 4 + 8 cells x (12 interior + 8 pressure) = 208
    assert 208 in sizes


def test_colour_classes_do_not_interact_3d():
    lev = o3.Level(4, 1, 1.0, 6.0, _kappa(4, 3))
    sm = o3.Smoother(lev)
    A = lev.A.tocsr()
    for col in range(27):
        ps = sm.colours[col]
        for i in range(len(ps)):
            for j in range(i + 1, len(ps)):
                d1, d2 = sm.patches[ps[i]][1], sm.patches[ps[j]][1]
                assert not set(d1.tolist()) & set(d2.tolist())
                assert A[d1][:, d2].nnz == 0


def test_prolongation_is_the_embedding_3d():
    Sc, Sf = o3.Space(2, 1), o3.Space(4, 1)
    P = o3.prolongation(Sc, Sf)
    kap = np.ones(8)
    lc, lf = o3.Level(2, 1, 1.0, 6.0, kap), o3.Level(4, 1, 1.0, 6.0, np.ones(64))
    rng = np.random.default_rng(11)
    xc = rng.standard_normal(Sc.ndof)
    xc[Sc.cons] = 0.0
    xf = P @ xc
    pts = rng.random((50, 3))
    Uc, Pc = o3.evaluate(lc, xc, pts)
    Uf, Pf = o3.evaluate(lf, xf, pts)
    assert np.abs(Uc - Uf).max() < 1e-12
    assert np.abs(Pc - Pf).max() < 1e-12
    assert np.all(np.abs(P[np.flatnonzero(Sf.cons)]).sum(axis=1) == 0)


def test_vcycle_is_symmetric_3d():
    o = o3.Oracle3D(1, 3, 1, 1e-2, 6.0, _kappa(4, 6, -4.0, 0.0))
    n = o.lev[-1].sp.ndof
    free = ~o.lev[-1].sp.cons
    rng = np.random.default_rng(2)
    u, v = rng.standard_normal(n) * free, rng.standard_normal(n) * free
    a, b = u @ o.vcycle(v), v @ o.vcycle(u)
    assert abs(a - b) < 1e-10 * abs(a)


def test_coarse_only_is_exact_3d():
    o = o3.Oracle3D(2, 1, 1, 0.1, 6.0, _kappa(2, 8))
    lev = o.lev[-1]
    g = lambda x, y, z: np.array([np.ones_like(x), 0 * x, 0 * x])
    b = lev.rhs(lambda x, y, z: np.zeros((3,) + np.shape(x)), g)
    _, its, tr = o.fgmres(b, rtol=1e-10, maxit=10)
    assert its == 1 and tr < 1e-12


def test_multigrid_matches_direct_solve_3d():
    o = o3.Oracle3D(2, 3, 1, 1e-2, 6.0, 10.0 ** np.clip(np.random.default_rng(12).normal(-3, 1.5, 512), -6, 0))
    lev = o.lev[-1]
    g = lambda x, y, z: np.array([np.ones_like(x), 0 * x, 0 * x])
    b = lev.rhs(lambda x, y, z: np.zeros((3,) + np.shape(x)), g)
    xm, its, tr = o.fgmres(b, rtol=1e-12, maxit=60)
    xd = o.direct_solve(b)
    d = xm - xd
    d[lev.sp.n_u:] -= o.pressure_mean(xm) - o.pressure_mean(xd)
    assert tr < 1e-11 and its <= 15
    assert np.abs(d).max() < 1e-8 * np.abs(xd).max()


# P3 (3-D): smooth solution u = (sin pi y, sin pi z, sin pi x) (divergence free), p =
# cos pi x cos pi y cos pi z (mean 0), kappa = 1: the L2 velocity error falls as h^2
# and the pressure error at least as h (RT_1 x dQ_1 theory), measured by Gauss
# quadrature over every cell.
def _l2_errors(lev, x, u, p):
    S, rb, N, h = lev.sp, lev.rb, lev.N, lev.h
    X, W = o3.cube_rule(4)
    v, _ = rb.vel(X)
    pv = rb.pres(X)
    nu = len(rb.lu)
    eu = ep = 0.0
    pm = x[S.n_u::S.NB ** 3].mean()
    for t, cc in enumerate(lev.cells):
        d = lev.cell_dof_table[t]
        P = (np.array(cc)[None, :] + X) * h
        uh = np.einsum("i,iqa->qa", x[d[:nu]], v)
        ph = x[d[nu:]] @ pv - pm
        ue = np.stack(u(P[:, 0], P[:, 1], P[:, 2]), -1)
        eu += h ** 3 * np.sum(W[:, None] * (uh - ue) ** 2)
        ep += h ** 3 * np.sum(W * (ph - p(P[:, 0], P[:, 1], P[:, 2])) ** 2)
    return np.sqrt(eu), np.sqrt(ep)


def test_brinkman_convergence_rates_3d():
    mu, pi = 1.0, np.pi
    u = lambda x, y, z: (np.sin(pi * y), np.sin(pi * z), np.sin(pi * x))
    p = lambda x, y, z: np.cos(pi * x) * np.cos(pi * y) * np.cos(pi * z)
    f = lambda x, y, z: np.array([(mu * pi ** 2 + 1.0) * np.sin(pi * y) - pi * np.sin(pi * x) * np.cos(pi * y) * np.cos(pi * z),
                                  (mu * pi ** 2 + 1.0) * np.sin(pi * z) - pi * np.cos(pi * x) * np.sin(pi * y) * np.cos(pi * z),
                                  (mu * pi ** 2 + 1.0) * np.sin(pi * x) - pi * np.cos(pi * x) * np.cos(pi * y) * np.sin(pi * z)])
    g = lambda x, y, z: np.array(u(x, y, z))
    errs = []
    for n in (2, 4, 8):
        lev = o3.Level(n, 1, mu, 6.0, np.ones(n ** 3))
        # sparse direct solve, bordered with the constant pressure (mean zero)
        c = lev.cvec / np.linalg.norm(lev.cvec)
        Bd = sp.bmat([[lev.A, sp.csr_matrix(c[:, None])], [sp.csr_matrix(c[None, :]), None]]).tocsc()
        x = spla.spsolve(Bd, np.concatenate([lev.rhs(f, g), [0.0]]))[:-1]
        errs.append(_l2_errors(lev, x, u, p))
    ru = np.log2(errs[1][0] / errs[2][0])
    rp = np.log2(errs[1][1] / errs[2][1])
    assert ru > 1.8, errs
    assert rp > 0.9, errs


# ---------------------------------------------------------------------------------
# RT_0 x dQ_0 (k = 0, Section 2.3: one normal flux per face, one pressure per cell),
# Brinkman and the Darcy limit mu = 0
# ---------------------------------------------------------------------------------
# P1 (k = 0): constant u = a is in RT_0, divergence free and has no jumps, p = 0:
# f = kappa a, g = a.  The discrete solution is exact for any mu >= 0 and any
# cellwise kappa (a dropped mass term, a wrong lifting or a sign error in the
# pressure coupling leaves an O(1) error).
@pytest.mark.parametrize("mu", [1.0, 1e-2, 0.0])
def test_constant_solution_is_reproduced_rt0_3d(mu):
    n0, levels = 1, 3
    n = n0 << (levels - 1)
    kap = _kappa(n, 5)
    o = o3.Oracle3D(n0, levels, 0, mu, 2.0, kap)
    lev = o.lev[-1]
    a = np.array([0.3, -0.7, 1.1])
    k_at = lambda x, y, z: _cell_kappa(kap, n, x, y, z)
    f = lambda x, y, z: np.array([k_at(x, y, z) * a[0], k_at(x, y, z) * a[1], k_at(x, y, z) * a[2]])
    g = lambda x, y, z: np.array([a[0] + 0 * x, a[1] + 0 * x, a[2] + 0 * x])
    b = lev.rhs(f, g)
    P = np.random.default_rng(7).random((40, 3))
    for x in (o.direct_solve(b), o.fgmres(b, rtol=1e-13, maxit=80)[0]):
        U, Pv = o3.evaluate(lev, x, P)
        assert np.abs(U - a).max() < 1e-10
        assert np.abs(Pv - o.pressure_mean(x)).max() < 1e-10


def test_rt0_sizes_and_patch_3d():
    # N = 4: 3 (N+1) N^2 face fluxes, N^3 pressures; an interior patch holds the 12
    # faces inside its 2 x 2 x 2 block and the 8 cell pressures
    S = o3.Space(4, 0)
    assert S.n_u == 3 * 5 * 16 and S.ndof == S.n_u + 64
    lev = o3.Level(4, 0, 0.5, 2.0, _kappa(4, 2))
    d, cells = o3.patch_dofs(lev.sp, 2, 2, 2)
    assert len(d) == 12 + 8 and len(cells) == 8


@pytest.mark.parametrize("mu", [1e-2, 0.0])
def test_multigrid_matches_direct_solve_rt0_3d(mu):
    # Darcy with contrast 1e2 (at 1e6 the mixed operator's conditioning turns a 1e-12
    # residual into ~1e-7 relative differences between the two solutions)
    kap = 10.0 ** np.clip(np.random.default_rng(12).normal(-3, 1.5, 512), -6, 0) if mu else _kappa(8, 12)
    o = o3.Oracle3D(2, 3, 0, mu, 2.0, kap)
    lev = o.lev[-1]
    g = lambda x, y, z: np.array([np.ones_like(x), 0 * x, 0 * x])
    b = lev.rhs(lambda x, y, z: np.zeros((3,) + np.shape(x)), g)
    xm, its, tr = o.fgmres(b, rtol=1e-12, maxit=100)
    xd = o.direct_solve(b)
    d = xm - xd
    d[lev.sp.n_u:] -= o.pressure_mean(xm) - o.pressure_mean(xd)
    assert tr < 1e-11 and its < 100
    assert np.abs(d).max() < 1e-8 * np.abs(xd).max()


def test_vcycle_is_symmetric_rt0_3d():
    o = o3.Oracle3D(1, 3, 0, 0.0, 2.0, _kappa(4, 6, -4.0, 0.0))
    n = o.lev[-1].sp.ndof
    free = ~o.lev[-1].sp.cons
    rng = np.random.default_rng(2)
    u, v = rng.standard_normal(n) * free, rng.standard_normal(n) * free
    a, b = u @ o.vcycle(v), v @ o.vcycle(u)
    assert abs(a - b) < 1e-10 * abs(a)


# P3 (k = 0, Darcy): u = grad of a smooth p' with kappa = 1 and f = 0 ... written as
# the mixed problem kappa u + grad p = f, div u = 0 with the smooth divergence-free
# u = (sin pi y, sin pi z, sin pi x), p = cos pi x cos pi y cos pi z: f = u + grad p,
# g = u.  RT_0 x dQ_0 converges at first order in L2 for both fields.
def test_darcy_convergence_rates_rt0_3d():
    pi = np.pi
    u = lambda x, y, z: (np.sin(pi * y), np.sin(pi * z), np.sin(pi * x))
    p = lambda x, y, z: np.cos(pi * x) * np.cos(pi * y) * np.cos(pi * z)
    f = lambda x, y, z: np.array([np.sin(pi * y) - pi * np.sin(pi * x) * np.cos(pi * y) * np.cos(pi * z),
                                  np.sin(pi * z) - pi * np.cos(pi * x) * np.sin(pi * y) * np.cos(pi * z),
                                  np.sin(pi * x) - pi * np.cos(pi * x) * np.cos(pi * y) * np.sin(pi * z)])
    g = lambda x, y, z: np.array(u(x, y, z))
    errs = []
    for n in (4, 8, 16):
        lev = o3.Level(n, 0, 0.0, 2.0, np.ones(n ** 3))
        c = lev.cvec / np.linalg.norm(lev.cvec)
        Bd = sp.bmat([[lev.A, sp.csr_matrix(c[:, None])], [sp.csr_matrix(c[None, :]), None]]).tocsc()
        x = spla.spsolve(Bd, np.concatenate([lev.rhs(f, g), [0.0]]))[:-1]
        errs.append(_l2_errors(lev, x, u, p))
    ru = np.log2(errs[1][0] / errs[2][0])
    rp = np.log2(errs[1][1] / errs[2][1])
    assert 0.85 < ru < 1.3, errs
    assert 0.85 < rp < 1.3, errs


# ---------------------------------------------------------------------------------
# Open sides (natural condition mu d_n u - p n = 0, no boundary data)
# ---------------------------------------------------------------------------------
OPEN_Z = (0, 0, 0, 0, 1, 1)  # open at z = 0 and z = 1
OPEN_ONE = (0, 0, 0, 0, 0, 1)


def _junk_on_open(g, bc):
    """g plus a large perturbation on the open sides: the discretisation must not
    evaluate boundary data there."""
    def gj(x, y, z):
        v = np.array(g(x, y, z), dtype=float)
        for d, t in enumerate((x, y, z)):
            for side, val in ((0, 0.0), (1, 1.0)):
                if bc[2 * d + side]:
                    v = v + 7.0 * (np.abs(np.asarray(t) - val) < 1e-14)
        return v
    return gj


# P1 (open sides): u = (0, 0, x) flows through the open z sides (d_z u = 0 there, p =
# 0): f = kappa u, g = u on the Dirichlet sides and junk on the open ones.  RT_1
# holds u, so the discrete solution is exact, pressure included (no constant is free
# with an open side).  Darcy (mu = 0): the same with p = 0 on the open sides.
@pytest.mark.parametrize("mu", [1.0, 1e-2, 0.0])
def test_flow_through_open_sides_is_reproduced_3d(mu):
    n0, levels = 1, 3
    n = n0 << (levels - 1)
    kap = _kappa(n, 5)
    o = o3.Oracle3D(n0, levels, 1, mu, 6.0, kap, bc=OPEN_Z)
    lev = o.lev[-1]
    k_at = lambda x, y, z: _cell_kappa(kap, n, x, y, z)
    f = lambda x, y, z: np.array([0 * x, 0 * x, k_at(x, y, z) * x])
    g = lambda x, y, z: np.array([0 * x, 0 * x, x])
    b = lev.rhs(f, _junk_on_open(g, OPEN_Z))
    P = np.random.default_rng(7).random((40, 3))
    ue = np.stack([0 * P[:, 0], 0 * P[:, 0], P[:, 0]], 1)
    for x in (o.direct_solve(b), o.fgmres(b, rtol=1e-13, maxit=80)[0]):
        U, Pv = o3.evaluate(lev, x, P)
        assert np.abs(U - ue).max() < 1e-10
        assert np.abs(Pv).max() < 1e-10


# P2 (open side): f = grad(phi), phi the trilinear hat at an interior vertex (zero on
# the boundary, so the natural condition holds), g = 0: u_h = 0 and p_h = phi exactly,
# with no constant removed -- an open side fixes the pressure level.
@pytest.mark.parametrize("k", [0, 1])
def test_hat_gradient_fixes_the_pressure_with_an_open_side_3d(k):
    n = 4
    h = 1.0 / n
    lev = o3.Level(n, k, 1e-2, 2.0 if k == 0 else 6.0, _kappa(n, 9, -6.0, 0.0), OPEN_ONE)
    v = np.array([2, 1, 3]) * h
    hat1 = lambda t, c: np.maximum(0.0, 1.0 - np.abs(t - c) / h)
    dhat1 = lambda t, c: np.where(np.abs(t - c) < h, -np.sign(t - c) / h, 0.0)
    f = lambda x, y, z: np.array([dhat1(x, v[0]) * hat1(y, v[1]) * hat1(z, v[2]),
                                  hat1(x, v[0]) * dhat1(y, v[1]) * hat1(z, v[2]),
                                  hat1(x, v[0]) * hat1(y, v[1]) * dhat1(z, v[2])])
    zero = lambda x, y, z: np.zeros((3,) + np.shape(x))
    x = spla.spsolve(lev.A.tocsc(), lev.rhs(f, _junk_on_open(zero, OPEN_ONE)))
    assert np.abs(x[:lev.sp.n_u]).max() < 1e-12
    phi = lambda x_, y_, z_: hat1(x_, v[0]) * hat1(y_, v[1]) * hat1(z_, v[2])
    if k == 1:  # the trilinear hat lies in dQ_1 cellwise
        assert np.abs(x[lev.sp.n_u:] - lev.interpolate_pressure(phi)).max() < 1e-12
    else:       # dQ_0: the cell means of phi
        assert np.abs(x[lev.sp.n_u:] - lev.interpolate_pressure(phi)).max() < 1e-12


def test_open_side_patches_and_operator_3d():
    lev = o3.Level(4, 1, 0.3, 6.0, _kappa(4, 1), OPEN_Z)
    S = lev.sp
    # two open sides: their 2 x 16 faces x (k+1)^2 normal dofs are free
    assert S.cons.sum() == 4 * 16 * 4 and S.open_normal.sum() == 2 * 16 * 4
    assert abs(lev.A - lev.A.T).max() <= 1e-13 * abs(lev.A).max()
    # no pressure constant in the kernel: the operator is nonsingular
    assert np.abs(lev.A @ lev.cvec).max() > 1e-3
    sm = o3.Smoother(lev)
    kinds = {}
    for (vx, vy, vz), dofs, rows, pinv, singular in sm.patches:
        A_S = rows[:, dofs].toarray()
        assert singular == (not S.open_normal[dofs].any())
        kinds[singular] = True
        if not singular:
            assert np.abs(pinv @ A_S - np.eye(len(dofs))).max() < 1e-9
        # only patches with a cell on the first or last layer in z touch an open side
        assert (vz in (0, 1, 3, 4)) or singular
    assert kinds == {True: True, False: True}


@pytest.mark.parametrize("k,mu", [(1, 1e-2), (0, 1e-2), (0, 0.0)])
def test_multigrid_matches_direct_solve_open_3d(k, mu):
    kap = _kappa(8, 12) if mu == 0.0 else 10.0 ** np.clip(np.random.default_rng(12).normal(-3, 1.5, 512), -6, 0)
    o = o3.Oracle3D(2, 3, k, mu, 2.0 if k == 0 else 6.0, kap, bc=OPEN_Z)
    lev = o.lev[-1]
    # a body force along z drives flow through the open sides (for Darcy the only data)
    g = lambda x, y, z: np.array([0 * x, 0 * x, np.ones_like(x)])
    b = lev.rhs(lambda x, y, z: np.array([0 * x, 0 * x, np.ones_like(x)]), g)
    xm, its, tr = o.fgmres(b, rtol=1e-12, maxit=100)
    xd = o.direct_solve(b)
    assert tr < 1e-11 and its < 100
    assert np.abs(xm - xd).max() < 1e-8 * np.abs(xd).max()
    # the V-cycle is a symmetric operator
    n = lev.sp.ndof
    free = ~lev.sp.cons
    rng = np.random.default_rng(2)
    p_, q_ = rng.standard_normal(n) * free, rng.standard_normal(n) * free
    a1, a2 = p_ @ o.vcycle(q_), q_ @ o.vcycle(p_)
    assert abs(a1 - a2) < 1e-10 * abs(a1)


# MAC / cell-centred equivalence of RT_0 (Section 2.3): with the kappa-mass lumped by
# rows (the trapezoidal rule across each face's normal direction, exact for the
# constant transverse factors), the Darcy Schur complement B M_lumped^-1 B^T of the
# oracle's RT_0 blocks is the 7-point cell-centred (two-point flux) operator with face
# transmissibility 2 h / (kappa_K + kappa_L) -- the harmonic mean of the permeabilities
# 1 / kappa -- and no flux through the (essential, zero) boundary faces.  Built here
# independently from kappa alone; a wrong divergence scaling, sign, face numbering or
# boundary treatment in the oracle's RT_0 assembly breaks the equality.
def test_rt0_darcy_lumped_schur_complement_is_the_cell_centred_scheme_3d():
    n = 4
    h = 1.0 / n
    kap = _kappa(n, 21, -3.0, 1.0)
    lev = o3.Level(n, 0, 0.0, 2.0, kap)
    S = lev.sp
    A = lev.A_full.tocsr()
    free_u = np.flatnonzero(~S.cons[:S.n_u])
    # row sums of the whole kappa-mass (the couplings to the essential faces included)
    lumped = np.asarray(A[:S.n_u][:, :S.n_u].sum(axis=1)).ravel()[free_u]
    B = A[S.n_u:][:, :S.n_u].toarray()[:, free_u]
    Schur = B @ np.diag(1.0 / lumped) @ B.T
    T = np.zeros((n ** 3, n ** 3))
    for cz in range(n):
        for cy in range(n):
            for cx in range(n):
                K = S.cell(cx, cy, cz)
                for d in range(3):
                    nb = [cx, cy, cz]
                    nb[d] += 1
                    if nb[d] < n:
                        L = S.cell(*nb)
                        t = 2.0 * h / (kap[K] + kap[L])
                        T[K, L] -= t
                        T[L, K] -= t
                        T[K, K] += t
                        T[L, L] += t
    assert np.abs(Schur - T).max() < 1e-12 * np.abs(T).max()
