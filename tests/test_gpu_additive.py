"""The additive vertex-patch Schwarz smoother on the GPU against the oracle's
additive smoother (same damping): smoothing steps, V-cycles and solves, both
colourings, one and several right-hand-side columns."""
import numpy as np
import pytest

from fe import Space
from oracle import Oracle
from paper_1602_04858_amd import inputs

pytestmark = pytest.mark.gpu

D, O = inputs.DIRICHLET, inputs.OPEN
OMEGA = 0.25


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
    (2, 4, 1, 1e-2, 6.0, (D, D, O, O), 0),
    (3, 3, 1, 1e-3, 6.0, (O, D, O, D), 1),
    (2, 3, 1, 1.0, 8.0, (D, D, D, D), 0),
    (3, 2, 2, 1e-2, 12.0, (D, D, O, O), 0),
]
IDS = ["k1N32", "k1N24L8", "k1N16dir", "k2N12"]


def _setup(bmg, case, prec=0, dense=0, nrhs=1):
    n0, J, k, mu, sigma, bc, col = case
    n = n0 << J
    kap = inputs.kappa_lognormal_channels(n, 6, channels=3, width=2 if n >= 16 else 1)
    o = Oracle(n0, J, k, mu, sigma, list(bc), kap, 1, 2, col, 1, OMEGA)
    s = bmg.Solver(bmg.make_params(n0, J, k, mu, sigma, bc, prec=prec, restart=100, dense_coarse_max=dense,
                                   colouring=col, smoother=1, omega=OMEGA, n_rhs=nrhs), kap)
    return o, s, kap


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_additive_smoothing_steps(torch, bmg, case):
    o, s, _ = _setup(bmg, case)
    J = case[1]
    for j in (J, J - 1):
        n = o.ndof(j)
        cons = o.constrained(j)
        x = inputs.random_vector(n, 13)
        b = inputs.random_vector(n, 14)
        x[cons] = 0.0
        b[cons] = 0.0
        xs = s.smooth(j, 3, torch.as_tensor(x, device="cuda"), torch.as_tensor(b, device="cuda"))
        xo = o.smooth(3, x, b, j)
        assert _rel(xs.cpu().numpy(), xo) < 1e-12, j


def _zero_pressure_mean(o, k, v):
    v = np.array(v, dtype=float)
    pidx = o.n_u() + np.arange(o.N() ** 2) * (k + 1) ** 2
    v[pidx] -= v[pidx].mean()
    return v


@pytest.mark.parametrize("case", CASES, ids=IDS)
@pytest.mark.parametrize("dense", [0, 16384])
def test_additive_vcycle_and_solve(torch, bmg, case, dense):
    o, s, _ = _setup(bmg, case, dense=dense)
    n = o.ndof()
    sp = Space(o.N(), case[2])
    r = inputs.random_vector(n, 23)
    r[o.constrained()] = 0.0
    if o.singular():
        # all sides Dirichlet: compatible (zero pressure mean) right-hand sides, and
        # solutions compared with their pressure means removed
        r = _zero_pressure_mean(o, case[2], r)
    z = s.vcycle(torch.as_tensor(r, device="cuda")).cpu().numpy()
    zo = o.vcycle(r)
    if o.singular():
        z, zo = sp.remove_pressure_mean(z), sp.remove_pressure_mean(zo)
    assert _rel(z, zo) < 1e-10
    src = inputs.smooth_source(33)
    b_o = o.rhs(src)
    if o.singular():
        b_o = _zero_pressure_mean(o, case[2], b_o)
    x, info = s.solve(torch.as_tensor(b_o, device="cuda"), rtol=1e-10, maxit=400)
    _, its, _, _ = o.fgmres(b_o, rtol=1e-10, maxit=400, restart=100)
    x_tight, _, _, _ = o.fgmres(b_o, rtol=1e-13, maxit=600, restart=100)
    assert info.converged == 1 and abs(info.iterations - abs(its)) <= 1, (info.iterations, its)
    x = x.cpu().numpy()
    if o.singular():
        x, x_tight = sp.remove_pressure_mean(x), sp.remove_pressure_mean(x_tight)
    assert _rel(x, x_tight) < 1e-8


@pytest.mark.parametrize("prec", [1, 2])
def test_additive_mixed_precision(torch, bmg, prec):
    o, s, _ = _setup(bmg, CASES[0], prec=prec, dense=16384)
    src = inputs.smooth_source(43)
    x, info = s.solve(torch.as_tensor(bmg.assemble_rhs(s.params, src), device="cuda"), rtol=1e-10, maxit=400)
    x_tight, _, _, _ = o.fgmres(o.rhs(src), rtol=1e-13, maxit=600, restart=100)
    assert info.converged == 1 and info.rel_residual_true < 2e-10
    assert _rel(x.cpu().numpy(), x_tight) < 1e-8


def test_additive_columns_match_single(torch, bmg):
    _, sm, kap = _setup(bmg, CASES[0], nrhs=3)
    _, s1, _ = _setup(bmg, CASES[0])
    n = s1.ndof()
    r = torch.stack([torch.as_tensor(inputs.random_vector(n, 90 + c), device="cuda") for c in range(3)]).contiguous()
    z = sm.vcycle(r)
    for c in range(3):
        assert _rel(z[c].cpu().numpy(), s1.vcycle(r[c].contiguous()).cpu().numpy()) <= 1e-14, c


def test_additive_c2_full_size(torch, bmg):
    """C2 with the additive smoother (bandwidth-bound levels with rotated inverses):
    converges to the true residual and agrees with the multiplicative solve."""
    w = inputs.workload("C2")
    pa = bmg.make_params(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.cycle, w.m_fine, 0, 100, 16384,
                         smoother=1, omega=OMEGA)
    sa = bmg.Solver(pa, w.kappa)
    b = torch.as_tensor(bmg.assemble_rhs(pa, w.source), device="cuda")
    xa, ia = sa.solve(b, rtol=1e-10, maxit=400)
    sm = bmg.from_workload(w)
    xm, im = sm.solve(b, rtol=1e-10, maxit=400)
    assert ia.converged == 1 and ia.rel_residual_true < 2e-10
    assert _rel(xa.cpu().numpy(), xm.cpu().numpy()) < 1e-8
