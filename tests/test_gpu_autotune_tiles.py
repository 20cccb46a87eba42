"""Tile parameters and their autotuner: rotated storage below the built-in threshold and
forced columns per block give the V-cycle the oracle gives (the same method, another
storage or launch shape), and bmg_autotune_tiles reports every timed candidate, returns
the fastest, and answers a second call with the same shape from its cache."""
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


CASE = (2, 5, 1, 1e-2, 6.0, (D, D, O, O))  # 64 x 64, RT_1


def _kappa():
    return inputs.kappa_lognormal_channels(64, 9, channels=4, width=2)


@pytest.mark.parametrize("tiles", [dict(rotated_min_n=16), dict(rotated_min_n=4096),
                                   dict(columns_per_block=1), dict(columns_per_block=4)],
                         ids=["rot16", "rot4096", "cpb1", "cpb4"])
def test_tile_parameters_keep_the_vcycle(torch, bmg, tiles):
    n0, J, k, mu, sigma, bc = CASE
    kap = _kappa()
    R = 3
    o = Oracle(n0, J, k, mu, sigma, list(bc), kap, 1, 2)
    s = bmg.Solver(bmg.make_params(n0, J, k, mu, sigma, bc, prec=0, restart=30, n_rhs=R, **tiles), kap)
    n = s.ndof()
    rs = [inputs.random_vector(n, 900 + c) for c in range(R)]
    cons = o.constrained(J)
    for r in rs:
        r[cons] = 0.0
    z = s.vcycle(torch.as_tensor(np.stack(rs), device="cuda")).cpu().numpy()
    for c in range(R):
        assert _rel(z[c], o.vcycle(rs[c])) < 1e-10, c


def test_autotune_tiles_reports_and_caches(torch, bmg):
    n0, J, k, mu, sigma, bc = CASE
    kap = _kappa()
    p = bmg.make_params(n0, J, k, mu, sigma, bc, prec=1, restart=20, dense_coarse_max=0, n_rhs=3)
    best, rows = bmg.autotune_tiles(p, kap, trials=3)
    # 2 colourings, 2 storage thresholds, 3 column counts
    assert len(rows) == 7
    assert all(r[3] > 0 for r in rows)
    fastest = min(rows, key=lambda r: r[3])
    assert (best.colouring, best.rotated_min_n, best.columns_per_block) == tuple(int(v) for v in fastest[:3])
    assert (best.n0, best.levels, best.k, best.precond_prec, best.n_rhs) == (n0, J, k, 1, 3)
    again, rows2 = bmg.autotune_tiles(p, kap, trials=3)
    assert rows2 == []
    assert (again.colouring, again.rotated_min_n, again.columns_per_block) == \
        (best.colouring, best.rotated_min_n, best.columns_per_block)
    # the tuned handle solves like the default one
    src = inputs.smooth_source(3)
    B = np.stack([bmg.assemble_rhs(p, src)] * 3)
    x1, i1 = bmg.Solver(best, kap).solve(torch.as_tensor(B, device="cuda"), rtol=1e-10, maxit=200)
    x0, i0 = bmg.Solver(p, kap).solve(torch.as_tensor(B, device="cuda"), rtol=1e-10, maxit=200)
    assert all(a.converged == 1 for a in i1) and abs(i1[0].iterations - i0[0].iterations) <= 1
    assert _rel(x1[0].cpu().numpy(), x0[0].cpu().numpy()) < 1e-8
