"""The L8 colouring on the GPU against the oracle run with the same colouring:
single colour steps, V-cycles and solves (the S9 default is covered by the other
parity tests).  Tolerances as there: FP64 steps 1e-12, solves 1e-8 from a tight
oracle solve with the iteration count within +-1."""
import numpy as np
import pytest

from fe import Space
from oracle import Oracle
from paper_1602_04858_amd import inputs

pytestmark = pytest.mark.gpu

D, O = inputs.DIRICHLET, inputs.OPEN
L8 = 1


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def bmg():
    from paper_1602_04858_amd import bmg as b
    return b


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


CASES = [
    (2, 4, 1, 1e-2, 6.0, (D, D, O, O)),
    (3, 3, 1, 1e-3, 6.0, (O, D, O, D)),
    (2, 3, 1, 1.0, 8.0, (D, D, D, D)),
    (3, 2, 2, 1e-2, 12.0, (D, D, O, O)),
]
IDS = ["k1N32", "k1N24", "k1N16dir", "k2N12"]


def _setup(bmg, case, prec=0, dense=0):
    n0, J, k, mu, sigma, bc = case
    n = n0 << J
    kap = inputs.kappa_lognormal_channels(n, 5, channels=3, width=2 if n >= 16 else 1)
    o = Oracle(n0, J, k, mu, sigma, list(bc), kap, 1, 2, L8)
    s = bmg.Solver(bmg.make_params(n0, J, k, mu, sigma, bc, prec=prec, restart=60, dense_coarse_max=dense,
                                   colouring=L8), kap)
    return o, s


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_l8_colour_steps(torch, bmg, case):
    o, s = _setup(bmg, case)
    J = case[1]
    for j in (J, J - 1):
        n = o.ndof(j)
        cons = o.constrained(j)
        x = inputs.random_vector(n, 11)
        b = inputs.random_vector(n, 12)
        x[cons] = 0.0
        b[cons] = 0.0
        xg = torch.as_tensor(x, device="cuda")
        bg = torch.as_tensor(b, device="cuda")
        for colour in range(8):
            xg = s.colour_step(j, colour, xg, bg)
            x = o.colour_step(colour, x, b, j)
            assert _rel(xg.cpu().numpy(), x) < 1e-12, (j, colour)
        xs = s.smooth(j, 2, torch.zeros_like(bg), bg)
        xo = o.smooth(2, np.zeros(n), b, j)
        assert _rel(xs.cpu().numpy(), xo) < 1e-12, j



def _zero_pressure_mean(o, k, v):
    v = np.array(v, dtype=float)
    pidx = o.n_u() + np.arange(o.N() ** 2) * (k + 1) ** 2
    v[pidx] -= v[pidx].mean()
    return v


@pytest.mark.parametrize("case", CASES, ids=IDS)
@pytest.mark.parametrize("dense", [0, 16384])
def test_l8_vcycle_and_solve(torch, bmg, case, dense):
    o, s = _setup(bmg, case, dense=dense)
    n = o.ndof()
    r = inputs.random_vector(n, 21)
    r[o.constrained()] = 0.0
    sp = Space(o.N(), case[2])
    if o.singular():
        # all sides Dirichlet: A has the constant pressure in its kernel, so the
        # right-hand side is made compatible (zero pressure mean) and solutions are
        # compared with their pressure means removed
        r = _zero_pressure_mean(o, case[2], r)
    z = s.vcycle(torch.as_tensor(r, device="cuda")).cpu().numpy()
    zo = o.vcycle(r)
    if o.singular():
        z, zo = sp.remove_pressure_mean(z), sp.remove_pressure_mean(zo)
    assert _rel(z, zo) < 1e-10
    src = inputs.smooth_source(31)
    b_o = o.rhs(src)
    if o.singular():
        b_o = _zero_pressure_mean(o, case[2], b_o)
    x, info = s.solve(torch.as_tensor(b_o, device="cuda"), rtol=1e-10, maxit=300)
    _, its, _, _ = o.fgmres(b_o, rtol=1e-10, maxit=300, restart=60)
    x_tight, _, _, _ = o.fgmres(b_o, rtol=1e-13, maxit=400, restart=60)
    assert info.converged == 1 and abs(info.iterations - abs(its)) <= 1, (info.iterations, its)
    x = x.cpu().numpy()
    if o.singular():
        x, x_tight = sp.remove_pressure_mean(x), sp.remove_pressure_mean(x_tight)
    assert _rel(x, x_tight) < 1e-8


@pytest.mark.parametrize("prec", [1, 2])
def test_l8_mixed_precision_solve(torch, bmg, prec):
    case = CASES[0]
    o, s = _setup(bmg, case, prec=prec, dense=16384)
    src = inputs.smooth_source(41)
    x, info = s.solve(torch.as_tensor(bmg.assemble_rhs(s.params, src), device="cuda"), rtol=1e-10, maxit=300)
    x_tight, its, _, _ = o.fgmres(o.rhs(src), rtol=1e-13, maxit=400, restart=60)
    assert info.converged == 1 and info.rel_residual_true < 2e-10
    assert _rel(x.cpu().numpy(), x_tight) < 1e-8


def test_l8_c2_full_size(torch, bmg):
    """C2 with the L8 colouring: the solve reaches the true residual, within 3
    iterations of the S9 solve, and the solutions agree (both solve A_J x = b)."""
    w = inputs.workload("C2")
    b = torch.as_tensor(bmg.assemble_rhs(bmg.make_params(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc), w.source),
                        device="cuda")
    s8 = bmg.from_workload(w, colouring=L8)
    s9 = bmg.from_workload(w)
    x8, i8 = s8.solve(b, rtol=1e-10, maxit=300)
    x9, i9 = s9.solve(b, rtol=1e-10, maxit=300)
    assert i8.converged == 1 and i8.rel_residual_true < 2e-10
    assert abs(i8.iterations - i9.iterations) <= 3
    assert _rel(x8.cpu().numpy(), x9.cpu().numpy()) < 1e-8


def test_autotune_returns_a_measured_candidate(torch, bmg):
    case = CASES[0]
    n0, J, k, mu, sigma, bc = case
    n = n0 << J
    kap = inputs.kappa_lognormal_channels(n, 5, channels=3, width=2)
    p = bmg.make_params(n0, J, k, mu, sigma, bc, prec=1, restart=20, dense_coarse_max=16384)
    best, ms = bmg.autotune(p, kap, trials=3)
    assert ms["S9"] > 0 and ms["L8"] > 0
    assert best.colouring == (1 if ms["L8"] < ms["S9"] else 0)
    assert (best.n0, best.levels, best.k, best.precond_prec) == (n0, J, k, 1)
