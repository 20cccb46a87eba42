"""Writes the oracle's attainable-accuracy record of the C3 Darcy generator to tests/golden/.

Runs only the CPU oracle (oracle/) on the seeded C3 Darcy workload scaled to N x N
quads (mu = 0, log-normal kappa with channels, contrast 1e6, f = (1, 0)): FP64
right-preconditioned FGMRES(100) with the variable V-cycle (m_J = 2), as the library
runs it, to the relative tolerance 1e-10 on the Arnoldi estimate, then restarted from
its own iterate (one more cycle at a time) while the true relative residual stays
above 1e-10.  For the first cycle it stores the iteration count, the estimate history,
the true relative residual and the solution at 4000 seeded indices (a GPU solve with
the same number of iterations is compared with these); for every cycle the count and
the true residual.  About 2 minutes at N = 256, 15 at N = 512.

    python tests/golden/make_darcy_floor.py 256 512
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import Oracle  # noqa: E402
from paper_1602_04858_amd import inputs  # noqa: E402

NSAMPLE = 4000
RESTART = 100
CYCLES = 6


def floor_record(n):
    w = inputs.scaled_workload("C3darcy", n)
    t0 = time.time()
    o = Oracle.from_workload(w)
    b = o.rhs(w.source)
    nd = o.ndof()
    print(f"N={n}: ndof {nd}, setup {time.time() - t0:.0f} s", flush=True)
    idx = np.sort(np.random.default_rng(2025).choice(nd, NSAMPLE, replace=False))
    rec = {"workload": w.name, "N": n, "mu": w.mu, "restart": RESTART, "ndof": nd,
           "b_norm": float(np.linalg.norm(b)), "sample_idx": idx.tolist(), "cycles": []}
    x = None
    for cyc in range(CYCLES):
        t1 = time.time()
        x, its, hist, tr = o.fgmres(b, rtol=1e-10, maxit=400, restart=RESTART, x0=x)
        print(f"  cycle {cyc}: its {its}, true residual {tr:.3e}, {time.time() - t1:.0f} s", flush=True)
        c = {"iterations": int(its), "true_rel": tr}
        if cyc == 0:
            c.update({"estimate_history": [float(v) for v in hist], "x_norm": float(np.linalg.norm(x)),
                      "x_max": float(np.abs(x).max()), "x_sample": x[idx].tolist()})
        rec["cycles"].append(c)
        if tr <= 1e-10:
            break
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("sizes", type=int, nargs="+")
    ap.add_argument("--out", default=os.path.join(HERE, "c3darcy_floor_oracle.json"))
    args = ap.parse_args()
    recs = [floor_record(n) for n in args.sizes]
    with open(args.out, "w") as fh:
        json.dump({"records": recs}, fh)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
