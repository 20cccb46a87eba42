"""Batches of independent problems (bmg_batch_*): every problem of a batch solve
gives what a solve of its own handle gives (same iteration count, same iterates to
rounding), whatever the number of worker streams; two members are also checked
against the oracle."""
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


# (n0, J, k, mu, bc, prec, n_rhs): mixed sizes, degrees, viscosities, precisions
MEMBERS = [
    (2, 4, 1, 1e-2, (D, D, O, O), 1, 1),
    (3, 3, 1, 1e-4, (D, D, O, O), 1, 1),
    (2, 3, 2, 1e-1, (D, D, O, O), 0, 1),
    (2, 5, 1, 3e-3, (D, D, O, O), 2, 2),
    (3, 2, 1, 1.0, (D, D, D, D), 0, 1),
]


def _build(bmg, dense=4000):
    params, kaps, rhs = [], [], []
    for i, (n0, J, k, mu, bc, prec, R) in enumerate(MEMBERS):
        n = n0 << J
        sigma = 6.0 if k == 1 else 12.0
        params.append(bmg.make_params(n0, J, k, mu, sigma, bc, prec=prec, restart=40, dense_coarse_max=dense,
                                      n_rhs=R))
        kaps.append(inputs.kappa_lognormal_channels(n, 4000 + i, channels=3, width=2 if n >= 16 else 1))
        cols = [bmg.assemble_rhs(params[-1], inputs.smooth_source(4100 + 10 * i + c)) for c in range(R)]
        if bc == (D, D, D, D):  # pressure rows of a pure Dirichlet problem: zero mean
            b0 = cols[0]
            nu = b0.size - (k + 1) ** 2 * n * n
            pidx = nu + np.arange(n * n) * (k + 1) ** 2
            for b in cols:
                b[pidx] -= b[pidx].mean()
        rhs.append(np.stack(cols) if R > 1 else cols[0])
    return params, kaps, rhs


@pytest.mark.parametrize("nstreams", [1, 3])
def test_batch_matches_individual_solves(torch, bmg, nstreams):
    params, kaps, rhs = _build(bmg)
    batch = bmg.Batch(params, kaps, nstreams=nstreams)
    bs = [torch.as_tensor(b, device="cuda") for b in rhs]
    xs, infos, st = batch.solve(bs, rtol=1e-10, maxit=300)
    assert st == 0
    torch.cuda.synchronize()
    rec = 0
    for i, p in enumerate(params):
        s = bmg.Solver(p, kaps[i])
        x1, i1 = s.solve(bs[i], rtol=1e-10, maxit=300)
        ii = [i1] if p.n_rhs <= 1 else i1
        for c, one in enumerate(ii):
            assert infos[rec + c].iterations == one.iterations, (i, c)
            assert infos[rec + c].converged == 1 and infos[rec + c].rel_residual_true < 2e-10, (i, c)
        rec += len(ii)
        assert _rel(xs[i].cpu().numpy(), x1.cpu().numpy()) <= 1e-12, i
        s.close()


def test_batch_members_vs_oracle(torch, bmg):
    params, kaps, rhs = _build(bmg)
    batch = bmg.Batch(params, kaps, nstreams=2)
    xs, infos, st = batch.solve([torch.as_tensor(b, device="cuda") for b in rhs], rtol=1e-10, maxit=300)
    assert st == 0
    for i in (0, 2):
        n0, J, k, mu, bc, prec, R = MEMBERS[i]
        o = Oracle(n0, J, k, mu, 6.0 if k == 1 else 12.0, list(bc), kaps[i], 1, 2)
        b_o = o.rhs(inputs.smooth_source(4100 + 10 * i))
        x_tight, _, _, _ = o.fgmres(b_o, rtol=1e-13, maxit=400, restart=60)
        assert _rel(xs[i].cpu().numpy(), x_tight) < 1e-8, i


def test_batch_reports_unconverged_member(torch, bmg):
    params, kaps, rhs = _build(bmg)
    rhs[1] = np.zeros_like(rhs[1])
    batch = bmg.Batch(params, kaps, nstreams=2)
    xs, infos, st = batch.solve([torch.as_tensor(b, device="cuda") for b in rhs], rtol=1e-10, maxit=2)
    assert st == 6
    assert infos[1].converged == 1 and infos[1].iterations == 0
    assert infos[0].converged == 0 and infos[0].iterations == 2
