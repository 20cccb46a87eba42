"""Host-side checks of the HIP library (no GPU needed).

* the C ABI library loads and exports every function include/bmg.h declares;
* parameter validation and error codes;
* setup products computed on the host -- patch dof maps and colours (bit-exact),
  patch pseudo-inverses, the level matrix from the reference-element blocks the
  kernels use, the right-hand side -- against the CPU oracle.
"""
import math
import os
import re

import numpy as np
import pytest

from oracle import Oracle
from paper_1602_04858_amd import inputs

bmg = pytest.importorskip("paper_1602_04858_amd.bmg")
D, O = inputs.DIRICHLET, inputs.OPEN
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = "".join(open(os.path.join(ROOT, "include", f)).read()
                  for f in sorted(os.listdir(os.path.join(ROOT, "include"))) if f.endswith(".h"))
    declared = set(re.findall(r"^\s*(?:bmg_status|const char\*)\s+(bmg\w*)\s*\(", hdr, re.M))
    assert len(declared) >= 30 and "bmg3_solve" in declared
    lib = bmg.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert declared <= set(bmg.EXPORTS)


def test_status_strings():
    lib = bmg.lib()
    for s in range(9):
        assert lib.bmg_status_string(s)


@pytest.mark.parametrize("change,expect", [
    (dict(k=3), 2), (dict(k=-1), 2), (dict(n0=1), 1), (dict(levels=-1), 1), (dict(mu=-1.0), 1),
    (dict(sigma=0.0), 1), (dict(m_fine=0), 1), (dict(restart=0), 1), (dict(cycle=5), 1),
    (dict(n0=2, levels=12), 1), (dict(prec=7), 1), (dict(dense=-1), 1), (dict(dense=70000), 1),
    (dict(n_rhs=-1), 1), (dict(n_rhs=17), 1), (dict(smoother=2), 1), (dict(smoother=1, omega=0.0), 1),
    (dict(smoother=1, omega=1.5), 1), (dict(colouring=3), 1), (dict(coarse_kappa=3), 1),
    # coarsest level above 4096 unknowns: its dense inverse is not formed (n0 = 64 would need
    # a 98 GB host matrix for RT_2)
    (dict(n0=19, levels=0), 2), (dict(n0=64, levels=0, k=2), 2), (dict(n0=13, levels=1, k=2), 2)])
def test_parameter_validation(change, expect):
    args = dict(n0=2, levels=2, k=1, mu=1.0, sigma=6.0, bc=[D, D, O, O], prec=0)
    args.update(change)
    p = bmg.make_params(args["n0"], args["levels"], args["k"], args["mu"], args["sigma"], args["bc"],
                        prec=args["prec"], m_fine=args.get("m_fine", 2), restart=args.get("restart", 10),
                        cycle=args.get("cycle", 1), dense_coarse_max=args.get("dense", 0),
                        n_rhs=args.get("n_rhs", 1), colouring=args.get("colouring", 0),
                        smoother=args.get("smoother", 0), omega=args.get("omega", 0.25),
                        coarse_kappa=args.get("coarse_kappa", 0))
    with pytest.raises(bmg.BmgError) as e:
        bmg.plan(p)
    assert e.value.status == expect


@pytest.mark.parametrize("n0", [2, 3])
def test_smoother_layout_rule_matches_patch_construction(n0):
    """The colour kernel picks the patch layout from the vertex position alone; setup
    (and plan) refuse with BMG_E_STATE if that rule ever disagrees with the generic
    patch construction.  Every boundary combination, several mesh sizes."""
    for code in range(16):
        bc = [(code >> s) & 1 for s in range(4)]
        for J in (1, 2, 3):
            bmg.plan(bmg.make_params(n0, J, 1, 1e-2, 6.0, bc, restart=4))
            bmg.plan(bmg.make_params(n0, J, 2, 1e-2, 12.0, bc, restart=4))


@pytest.mark.parametrize("n0,k", [(18, 1), (12, 2), (36, 0)])
def test_largest_supported_coarse_mesh(n0, k):
    """The largest coarsest meshes within the 4096-unknown limit are accepted."""
    assert bmg.plan(bmg.make_params(n0, 0, k, 1e-2, (k + 1) * (k + 2), [D, D, O, O], restart=4)) > 0


def test_plan_grows_with_levels():
    sizes = [bmg.plan(bmg.make_params(2, J, 1, 1e-2, 6.0, [D, D, O, O], restart=20)) for J in (2, 3, 4)]
    assert sizes[0] < sizes[1] < sizes[2]


def test_plan_counts_every_right_hand_side():
    """n_rhs columns: Krylov and level vectors grow by n_rhs, the setup products do not;
    n_rhs = 0 is read as 1."""
    def plan(r):
        return bmg.plan(bmg.make_params(2, 4, 1, 1e-2, 6.0, [D, D, O, O], restart=20, n_rhs=r))
    one, zero, four, sixteen = plan(1), plan(0), plan(4), plan(16)
    assert zero == one
    per_rhs = (four - one) / 3
    assert per_rhs > 0 and abs((sixteen - one) - 15 * per_rhs) <= 15 * 4096
    n = 2 * 32 * 33 * 2 + 2 * 2 * 32 * 32 + 4 * 32 * 32  # finest ndof, N = 32, k = 1
    assert per_rhs >= (2 * 20 + 4) * n * 8  # FP64 Krylov vectors of one column


def test_nonfinite_and_negative_kappa_rejected():
    p = bmg.make_params(2, 1, 1, 1.0, 6.0, [D, D, O, O])
    kap = np.ones(16)
    kap[3] = np.nan
    with pytest.raises(bmg.BmgError) as e:
        bmg.export_patch(p, kap, 1, 1, 1)
    assert e.value.status == 7
    kap[3] = -1.0
    with pytest.raises(bmg.BmgError) as e:
        bmg.export_patch(p, kap, 1, 1, 1)
    assert e.value.status == 1
    # zero is the Stokes limit with viscosity, invalid for Darcy
    kap[3] = 0.0
    bmg.export_patch(p, kap, 1, 1, 1)
    with pytest.raises(bmg.BmgError) as e:
        bmg.export_patch(bmg.make_params(2, 1, 1, 0.0, 6.0, [D, D, O, O]), kap, 1, 1, 1)
    assert e.value.status == 1


CASES = [
    (2, 2, 1, 1e-2, 6.0, (D, D, O, O)),
    (2, 2, 1, 1.0, 8.0, (D, D, D, D)),
    (2, 2, 1, 0.0, 6.0, (D, O, D, O)),
    (3, 1, 1, 1e-1, 6.0, (O, O, O, O)),
    (2, 1, 2, 1e-2, 12.0, (D, D, O, O)),
    (2, 1, 2, 0.0, 12.0, (O, D, O, D)),
    (2, 2, 0, 1e-2, 2.0, (D, D, O, O)),
    (3, 1, 0, 0.0, 2.0, (D, D, D, D)),
    (2, 2, 0, 1.0, 2.0, (O, D, O, D)),
]


def _case(case, seed=1):
    n0, J, k, mu, sigma, bc = case
    n = n0 << J
    kap = inputs.kappa_lognormal_channels(n, seed, mean=-2.0, std=1.5, lo=-5.0, hi=0.0, channels=2, width=1)
    return n0, J, k, mu, sigma, bc, kap


@pytest.mark.parametrize("case", CASES)
def test_patch_maps_and_colours_bit_exact(case):
    n0, J, k, mu, sigma, bc, kap = _case(case)
    o = Oracle(n0, J, k, mu, sigma, list(bc), kap, 1, 2)
    p = bmg.make_params(n0, J, k, mu, sigma, bc)
    for j in range(1, J + 1):
        for pi in range(o.npatch(j)):
            vx, vy, col, dofs, sing, _ = o.patch(pi, j)
            d2, _, c2 = bmg.export_patch(p, kap, j, vx, vy, with_inverse=False)
            assert c2 == col
            assert np.array_equal(d2, dofs), (j, vx, vy)


@pytest.mark.parametrize("case", CASES)
def test_patch_pseudo_inverses_match_oracle(case):
    n0, J, k, mu, sigma, bc, kap = _case(case, seed=3)
    o = Oracle(n0, J, k, mu, sigma, list(bc), kap, 1, 2)
    p = bmg.make_params(n0, J, k, mu, sigma, bc)
    j = J
    worst = 0.0
    for pi in range(o.npatch(j)):
        vx, vy, col, dofs, sing, inv = o.patch(pi, j)
        _, inv2, _ = bmg.export_patch(p, kap, j, vx, vy)
        scale = np.abs(inv).max()
        # a patch whose only dof is one pressure has the zero pseudo-inverse (RT_0 corners)
        err = np.abs(inv2 - inv).max() / scale if scale > 0 else np.abs(inv2).max()
        worst = max(worst, err)
    assert worst < 1e-11, worst


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("case", CASES)
def test_level_matrix_matches_oracle(case, mode):
    """Every level's operator (so the coarse kappa of each averaging) against the oracle."""
    n0, J, k, mu, sigma, bc, kap = _case(case, seed=5)
    o = Oracle(n0, J, k, mu, sigma, list(bc), kap, 1, 2, kappa_avg=mode)
    p = bmg.make_params(n0, J, k, mu, sigma, bc, coarse_kappa=mode)
    for j in range(J + 1):
        A = o.csr(j).toarray()
        B = bmg.export_level_matrix(p, kap, j)
        assert np.abs(A - B).max() <= 1e-13 * np.abs(A).max(), j


@pytest.mark.parametrize("case", CASES)
def test_rhs_matches_oracle(case):
    n0, J, k, mu, sigma, bc, kap = _case(case, seed=7)
    o = Oracle(n0, J, k, mu, sigma, list(bc), kap, 1, 2)
    p = bmg.make_params(n0, J, k, mu, sigma, bc)
    f = inputs.smooth_source(17)
    s = lambda x, y: np.sin(3 * x) * np.cos(2 * y)

    def g(x, y):
        # tangential data only (zero normal component on every side)
        out = np.zeros(np.shape(x) + (2,))
        on_x = (x == 0.0) | (x == 1.0)
        out[..., 1] = np.where(on_x, np.sin(math.pi * y) + 0.3, 0.0)
        out[..., 0] = np.where(~on_x, np.cos(2 * x), 0.0)
        return out

    b1 = o.rhs(f, s=s, g=g)
    b2 = bmg.assemble_rhs(p, f, s=s, g=g)
    assert np.abs(b1 - b2).max() <= 1e-13 * np.abs(b1).max()


def test_rhs_rejects_normal_boundary_data():
    p = bmg.make_params(2, 1, 1, 1.0, 6.0, (D, D, O, O))
    g = lambda x, y: np.stack([np.ones_like(x), np.zeros_like(x)], -1)
    with pytest.raises(bmg.BmgError) as e:
        bmg.assemble_rhs(p, inputs.constant_source(1.0, 0.0), g=g)
    assert e.value.status == 2


def test_quadrature_points_match_oracle():
    from oracle import quad_points
    p = bmg.make_params(2, 2, 2, 1.0, 12.0, (D, D, O, O))
    c1, f1 = quad_points(8, 2)
    c2, f2 = bmg.quad_points(p)
    assert np.abs(c1 - c2).max() < 1e-15 and np.abs(f1 - f2).max() < 1e-15


def test_batch_setup_rejects_bad_arguments():
    """Validated before any device work (runs without a GPU)."""
    import ctypes as C
    lib = bmg.lib()
    p = bmg.make_params(2, 1, 1, 1.0, 6.0, [D, D, O, O])
    arr = (bmg.Params * 1)(p)
    kap = np.ones(16)
    kptr = (C.POINTER(C.c_double) * 1)(kap.ctypes.data_as(C.POINTER(C.c_double)))
    h = C.c_void_p()
    assert lib.bmg_batch_setup(0, arr, kptr, 4, None, C.byref(h)) == 1
    assert lib.bmg_batch_setup(1, arr, kptr, 17, None, C.byref(h)) == 1
    assert lib.bmg_batch_setup(1, arr, kptr, -1, None, C.byref(h)) == 1
    bad = (bmg.Params * 1)(bmg.make_params(2, 1, 3, 1.0, 6.0, [D, D, O, O]))
    assert lib.bmg_batch_setup(1, bad, kptr, 4, None, C.byref(h)) == 2
    nullk = (C.POINTER(C.c_double) * 1)()
    assert lib.bmg_batch_setup(1, arr, nullk, 4, None, C.byref(h)) == 1
    assert lib.bmg_batch_solve(None, None, None, 1e-10, 10, None) == 1
    assert lib.bmg_batch_destroy(None) == 1


@pytest.mark.parametrize("colouring", [0, 1])
def test_colouring_export_matches_oracle(colouring):
    """bmg_export_colouring and the colour of bmg_export_patch equal the oracle's
    patch colours, vertex by vertex (S9 and L8)."""
    for n0, J, k in ((2, 2, 1), (3, 2, 1), (2, 2, 2)):
        n = n0 << J
        kap = np.ones(n * n)
        p = bmg.make_params(n0, J, k, 1.0, 6.0, [D, D, O, O], colouring=colouring)
        o = Oracle(n0, J, k, 1.0, 6.0, [D, D, O, O], kap, 1, 2, colouring)
        ncol, col = bmg.export_colouring(p, J)
        assert ncol == (9 if colouring == 0 else 8)
        for pi in range(o.npatch()):
            vx, vy, c, _, _, _ = o.patch(pi)
            assert col[vy, vx] == c
        assert bmg.export_patch(p, kap, J, 1, 2, with_inverse=False)[2] == col[2, 1]


@pytest.mark.parametrize("colouring", [0, 1])
def test_colour_classes_cover_every_vertex(colouring):
    """The kernels enumerate patch p of a colour arithmetically; setup (and plan)
    refuse with BMG_E_STATE unless that enumeration visits every vertex once with its
    own colour.  Many mesh sizes and all boundary combinations."""
    for n0 in (2, 3, 5):
        for J in (1, 2, 3, 4):
            for code in (0, 5, 10, 15):
                bc = [(code >> s) & 1 for s in range(4)]
                bmg.plan(bmg.make_params(n0, J, 1, 1e-2, 6.0, bc, restart=4, colouring=colouring))
    with pytest.raises(bmg.BmgError) as e:
        bmg.plan(bmg.make_params(2, 2, 1, 1e-2, 6.0, [D, D, O, O], colouring=2))
    assert e.value.status == 1


def test_public_headers_compile_as_c_and_cxx():
    import shutil
    import subprocess
    inc = os.path.join(ROOT, "include")
    for name in sorted(os.listdir(inc)):
        if not name.endswith(".h"):
            continue
        for cc, lang in (("gcc", "c"), ("g++", "c++")):
            if shutil.which(cc) is None:
                continue
            r = subprocess.run([cc, "-fsyntax-only", "-Wall", "-x", lang, "-I", inc, os.path.join(inc, name)],
                               capture_output=True, text=True)
            assert r.returncode == 0, (name, lang, r.stderr)


def test_kappa_of_the_wrong_size_is_refused_by_the_binding():
    """The library reads (n0 2^levels)^2 values from kappa; the binding refuses any
    other size before the call (a short array would be read past its end)."""
    p = bmg.make_params(2, 2, 1, 1e-2, 6.0, [D, D, O, O])
    for n in (63, 65, 16):
        with pytest.raises(ValueError):
            bmg.export_patch(p, np.ones(n), 1, 1, 1)
        with pytest.raises(ValueError):
            bmg.export_level_matrix(p, np.ones(n), 1)
    bmg.export_patch(p, np.ones((8, 8)), 1, 1, 1)  # any shape with 64 values


def test_rhs_callables_of_the_wrong_size_are_refused():
    p = bmg.make_params(2, 1, 1, 1e-2, 6.0, [D, D, O, O])
    with pytest.raises(ValueError):
        bmg.assemble_rhs(p, lambda x, y: x)  # one component instead of two
    with pytest.raises(ValueError):
        bmg.assemble_rhs(p, lambda x, y: np.stack([x, y], -1), s=lambda x, y: np.stack([x, y], -1))
    with pytest.raises(ValueError):
        bmg.assemble_rhs(p, lambda x, y: np.stack([x, y], -1), g=lambda x, y: x)
    b = bmg.assemble_rhs(p, lambda x, y: np.stack([x, y], -1), s=lambda x, y: x * y,
                         g=lambda x, y: np.stack([0 * x, 0 * y], -1))
    assert np.isfinite(b).all()


def test_tile_parameters_validated():
    """rotated_min_n in 0..4096 and columns_per_block in 0..16 (0: built-in choice);
    the plan does not depend on them beyond the storage of the inverses."""
    from paper_1602_04858_amd import bmg
    base = dict(n0=2, levels=5, k=1, mu=1e-2, sigma=6.0, bc=(0, 0, 1, 1))
    assert bmg.plan(bmg.make_params(**base)) > 0
    assert bmg.plan(bmg.make_params(**base, rotated_min_n=16, columns_per_block=4)) > 0
    for bad in (dict(rotated_min_n=5000), dict(rotated_min_n=-1), dict(columns_per_block=17),
                dict(columns_per_block=-2)):
        with pytest.raises(bmg.BmgError):
            bmg.plan(bmg.make_params(**base, **bad))
