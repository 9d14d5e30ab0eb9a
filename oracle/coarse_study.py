"""Study (oracle only): the coarse space at the 5 Hz resolution, exact and inexact coarse solves.

TEST INFRASTRUCTURE ONLY.  A lateral window of the layered model at 5 Hz with the full depth
and the same cube size as the 5 Hz workload (32 x 32 x 20 cubes, 573,949 dofs), cut into
4 x 4 x 4 boxes at equal depth (64 subdomains), overlap 1, two point sources at 0.5 km,
tol 1e-6, restart 40, at most 300 iterations.  For each preconditioner it prints the
FGMRES iterations and the largest final residual:
  one-level ORAS (eq. oras);
  two-level (eq. 2lvl) with the P1 coarse mesh on every k-th vertex plane of the fine one,
  k = 4, 2 and 1 (about 0.7, 1.4 and 2.8 vertices per minimum wavelength; the paper's coarse
  mesh has 2.5), the coarse problem solved exactly (dense LU) or as the paper does (10 GMRES
  iterations with one-level ORAS on the coarse level, InexactCoarse).

    python3 -m oracle.coarse_study [--parts PX PY PZ] [k ...]      (default: 4 4 4 boxes; k = 4 2 1)
"""
from __future__ import annotations

import sys
import time

import numpy as np

import workloads as w

from . import ddm as odd
from . import fem, krylov, rhs


def problem(n_sources=(2, 1), parts=(4, 4, 4)):
    hxy = 1980.0 / 5.0 / 1000.0 / 2.8  # the family's cube size at 5 Hz (km)
    side = 32 * hxy * 0.999
    return w.layered_problem(freq=5.0, r=1.4, parts=parts, overlap=1, n_sources=n_sources, src_depth=0.5,
                             lateral=(0.0, side, 0.0, side), equal_depth_zcuts=True, coarse_factor=0)


def run(p, factors=(4, 2, 1), tol=1e-6, sources=None, label="5 Hz window"):
    """The study on problem p (its own point sources unless `sources` is given); returns
    {variant name: (iterations, largest residual)}."""
    t0 = time.perf_counter()
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq)
    B = rhs.point_sources(om, p.sources if sources is None else sources).T
    subs, own = odd.build_subdomains(om, p.velocity, p.freq, None, p.partition, p.n_sub, p.overlap)
    odd.factor_subdomains(subs)
    print(f"{label} {p.grid} cubes, n = {om.n}, {p.n_sub} subdomains, set-up {time.perf_counter() - t0:.0f} s",
          flush=True)
    xs = np.unique(p.coords[:, 0])
    ys = np.unique(p.coords[:, 1])
    zs = np.unique(p.coords[:, 2])
    variants = [("one-level", None)]
    for k in factors:
        ct, cc = w.kuhn_mesh(xs[::k], ys[::k], zs[::k])
        Z = odd.coarse_interpolation(om, ct, cc)
        cown = odd.coarse_owners(om, cc, own)
        variants.append((f"two-level {k}x, exact coarse (nc = {cc.shape[0]})", odd.Coarse(Z, A)))
        variants.append((f"two-level {k}x, 10 GMRES + coarse ORAS", odd.InexactCoarse(Z, A, subs, cown)))
        print(f"coarse {k}x: {cc.shape[0]} coarse dofs ({time.perf_counter() - t0:.0f} s)", flush=True)
    out = {}
    for name, coarse in variants:
        t = time.perf_counter()
        P = odd.ORAS(A, subs, coarse)
        X, info = krylov.block_fgmres(lambda x: A @ x, B, P.apply, tol=tol, m=40, max_iter=300)
        res = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
        out[name] = (info["iters"], float(res.max()))
        print(f"{name:44s} iterations {info['iters']:4d}  largest residual {res.max():.2e}  "
              f"({time.perf_counter() - t:.0f} s)", flush=True)
    return out


def main(factors=(4, 2, 1), parts=(4, 4, 4)):
    return run(problem(parts=parts), factors)


if __name__ == "__main__":
    argv = sys.argv[1:]
    parts = (4, 4, 4)
    if argv[:1] == ["--parts"]:
        parts, argv = tuple(int(a) for a in argv[1:4]), argv[4:]
    main(tuple(int(a) for a in argv) or (4, 2, 1), parts)
