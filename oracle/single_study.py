"""Study (oracle only): FGMRES with the whole computation in single precision.

TEST INFRASTRUCTURE ONLY.  The paper runs the whole solve in single precision (section
"Numerical results": the same GMRES iteration count as in double precision at eps = 1e-3,
Table "Cholesky vs ICC").  For one-level ORAS problems and a block of point sources, this
prints the iterations and the final relative residual (recomputed in FP64 with the FP64
operator) of three schemes:
  fp64    local factors, ORAS and FGMRES in complex128;
  mixed   complex64 local factors and ORAS, FGMRES in complex128 (the GPU path's mixed mode);
  single  complex64 local factors and ORAS, and FGMRES (basis, Hessenberg matrix, least
          squares, iterate and residual) in complex64, the operator rounded to complex64;
at the paper's eps = 1e-3 and at 1e-6 (restart 40, at most 400 iterations).

    python3 -m oracle.single_study
"""
from __future__ import annotations

import time

import numpy as np

import workloads as w

from . import ddm as odd
from . import fem, krylov, rhs

PROBLEMS = {
    "unit cube 8^3, k = 8 pi, 8 subdomains": lambda: w.unit_cube_problem(8),
    "layered 16x16x8 cubes, 1 Hz, 32 subdomains": lambda: w.layered_problem(
        freq=1.0, r=1.4, parts=(4, 4, 2), overlap=1, n_sources=(2, 2), max_cubes=(16, 16, 8),
        equal_depth_zcuts=True, coarse_factor=0),
}


def run(name, p, tols=(1e-3, 1e-6)):
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq, p.quality)
    A32 = A.astype(np.complex64)
    if p.sources is not None:
        B = rhs.point_sources(om, p.sources).T
    else:
        B = rhs.point_sources(om, np.array([[0.37, 0.52, 0.61]])).T
    t = time.perf_counter()
    subs, _ = odd.build_subdomains(om, p.velocity, p.freq, p.quality, p.partition, p.n_sub, p.overlap)
    subs32, _ = odd.build_subdomains(om, p.velocity, p.freq, p.quality, p.partition, p.n_sub, p.overlap)
    odd.factor_subdomains(subs)
    odd.factor_subdomains(subs32, np.complex64)
    P64 = odd.ORAS(A, subs)
    P32 = odd.ORAS(A, subs32, dtype=np.complex64)
    print(f"{name}: n = {om.n}, {p.n_sub} subdomains, {B.shape[1]} sources, set-up {time.perf_counter() - t:.1f} s",
          flush=True)
    schemes = {
        "fp64": (lambda x: A @ x, P64.apply, np.complex128),
        "mixed": (lambda x: A @ x, P32.apply, np.complex128),
        "single": (lambda x: A32 @ x, lambda v: P32.apply(v).astype(np.complex64), np.complex64),
    }
    out = {}
    for tol in tols:
        for label, (Af, Pf, dt) in schemes.items():
            X, info = krylov.block_fgmres(Af, B, Pf, tol=tol, m=40, max_iter=400, dtype=dt)
            res = np.linalg.norm(B - A @ X.astype(np.complex128), axis=0) / np.linalg.norm(B, axis=0)
            out[(tol, label)] = (info["iters"], float(res.max()))
            print(f"  tol {tol:.0e}  {label:6s}  iterations {info['iters']:4d}  largest FP64 residual {res.max():.2e}",
                  flush=True)
    return out


def main():
    for name, f in PROBLEMS.items():
        run(name, f())


if __name__ == "__main__":
    main()
