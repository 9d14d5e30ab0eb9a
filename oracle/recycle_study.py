"""Study (oracle only): Krylov recycling across sources, the paper's proposed improvement.

TEST INFRASTRUCTURE ONLY.  The paper's conclusion proposes GCRO-DR and its block variant to
speed up many right-hand sides.  On the 5 Hz window of oracle/coarse_study.py (573,949 dofs,
64 subdomains, overlap 1, one-level ORAS) with 8 point sources at 0.5 km on a 4 x 2 grid,
tol 1e-6, it prints the preconditioner applications (one per iteration and column) of
  GMRES(40) for each source in turn;
  GCRO-DR(40, k) for each source in turn, the recycle space carried from one to the next;
  block FGMRES(40) over the 8 sources at once (the GPU path's scheme: 8 applications a step).

    python3 -m oracle.recycle_study
"""
from __future__ import annotations

import time

import numpy as np

from . import coarse_study
from . import ddm as odd
from . import fem, krylov, rhs


def run(p, ks=(10, 20), tol=1e-6, m=40, sources=None, label="5 Hz window"):
    """The study on problem p; returns {scheme: (applications, largest residual)}."""
    t0 = time.perf_counter()
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq)
    B = rhs.point_sources(om, p.sources if sources is None else sources).T
    subs, _ = odd.build_subdomains(om, p.velocity, p.freq, None, p.partition, p.n_sub, p.overlap)
    odd.factor_subdomains(subs)
    P = odd.ORAS(A, subs)
    ns = B.shape[1]
    print(f"{label} {p.grid} cubes, n = {om.n}, {p.n_sub} subdomains, {ns} sources, "
          f"set-up {time.perf_counter() - t0:.0f} s", flush=True)
    out = {}
    for label_s, k in [(f"GMRES({m})", 0)] + [(f"GCRO-DR({m}, {k})", k) for k in ks]:
        t = time.perf_counter()
        rec, its, worst = None, [], 0.0
        for c in range(ns):
            x, info, rec = krylov.gcrodr(lambda v: A @ v, B[:, c], P.apply, tol=tol, m=m, k=k, recycle=rec)
            its.append(info["iters"])
            worst = max(worst, info["rel_residual"])
        out[label_s] = (sum(its), worst)
        print(f"{label_s:16s} per source {its}  applications {sum(its):5d}  largest residual {worst:.2e}  "
              f"({time.perf_counter() - t:.0f} s)", flush=True)
    t = time.perf_counter()
    X, info = krylov.block_fgmres(lambda v: A @ v, B, P.apply, tol=tol, m=m, max_iter=400)
    out[f"block FGMRES({m})"] = (info["iters"] * ns, float(info["rel_residual"].max()))
    print(f"{'block FGMRES(%d)' % m:16s} {info['iters']} steps of {ns} columns  applications {info['iters'] * ns:5d}  "
          f"largest residual {info['rel_residual'].max():.2e}  ({time.perf_counter() - t:.0f} s)", flush=True)
    return out


def main():
    return run(coarse_study.problem(n_sources=(4, 2)))


if __name__ == "__main__":
    main()
