"""Coarse-kappa averaging variants (arithmetic, harmonic, geometric) on the GPU
against the oracle with the same averaging: V-cycles and FP64 solves."""
import numpy as np
import pytest

from oracle import Oracle
from paper_1602_04858_amd import inputs

pytestmark = pytest.mark.gpu

D, O = inputs.DIRICHLET, inputs.OPEN


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


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("dense", [0, 16384])
def test_coarse_kappa_variants(torch, bmg, mode, dense):
    w = inputs.scaled_workload("C2", 32)
    o = Oracle(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.kappa, 1, 2, kappa_avg=mode)
    p = bmg.make_params(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.cycle, w.m_fine, 0, 60, dense,
                        coarse_kappa=mode)
    s = bmg.Solver(p, w.kappa)
    n = o.ndof()
    r = inputs.random_vector(n, 51)
    r[o.constrained()] = 0.0
    assert _rel(s.vcycle(torch.as_tensor(r, device="cuda")).cpu().numpy(), o.vcycle(r)) < 1e-10
    x, info = s.solve(torch.as_tensor(bmg.assemble_rhs(p, w.source), device="cuda"), rtol=1e-10, maxit=300)
    b_o = o.rhs(w.source)
    _, its, _, _ = o.fgmres(b_o, rtol=1e-10, maxit=300, restart=60)
    x_tight, _, _, _ = o.fgmres(b_o, rtol=1e-13, maxit=400, restart=60)
    assert info.converged == 1 and abs(info.iterations - abs(its)) <= 1, (info.iterations, its)
    assert _rel(x.cpu().numpy(), x_tight) < 1e-8
