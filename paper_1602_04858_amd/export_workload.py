"""Write a workload's permeability field and right-hand-side sources as files for bmg_run.

    python -m paper_1602_04858_amd.export_workload C5 OUTDIR [--n N] [--rhs R]

OUTDIR/kappa.bin: the N*N cellwise kappa values (float64, cell (cx, cy) at cy*N + cx);
OUTDIR/sources.txt: one line per right-hand side, the smooth random source of column r
(the generator's seed 5100 + r for C5) as groups of (amplitude, direction angle, kx, ky,
phase); OUTDIR/args.txt: the bmg_run arguments of the workload (mesh, degree, mu, sigma,
boundary sides, cycle).  Input generation only: nothing here touches the solver.
"""
from __future__ import annotations

import argparse
import os

from paper_1602_04858_amd import inputs


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["C2", "C3", "C3darcy", "C5"])
    ap.add_argument("outdir")
    ap.add_argument("--n", type=int, default=0, help="cells per side (the workload's generator at this size)")
    ap.add_argument("--rhs", type=int, default=16)
    a = ap.parse_args()
    w = inputs.scaled_workload(a.workload, a.n) if a.n else inputs.workload(a.workload)
    os.makedirs(a.outdir, exist_ok=True)
    w.kappa.astype("<f8").tofile(os.path.join(a.outdir, "kappa.bin"))
    with open(os.path.join(a.outdir, "sources.txt"), "w") as f:
        for r in range(a.rhs):
            s = inputs.smooth_source(5100 + r) if a.workload == "C5" else None
            if s is None:
                f.write("1 0 0 0 1.5707963267948966\n")  # f = (1, 0): amplitude 1 along x, sin(pi/2) = 1
                continue
            f.write(" ".join(f"{float(s.amp[i])!r} {float(s.theta[i])!r} {float(s.kx[i])!r} {float(s.ky[i])!r} {float(s.phase[i])!r}"
                             for i in range(len(s.amp))) + "\n")
    with open(os.path.join(a.outdir, "args.txt"), "w") as f:
        f.write(f"--n0 {w.n0} --levels {w.levels} --k {w.k} --mu {w.mu!r} --sigma {w.sigma!r} "
                f"--bc {','.join(str(b) for b in w.bc)} --cycle {w.cycle} --m-fine {w.m_fine}\n")
    print(f"{w.name}: N={w.n}, wrote {a.outdir}/kappa.bin, sources.txt ({a.rhs} lines), args.txt")


if __name__ == "__main__":
    main()
