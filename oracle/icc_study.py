"""Study (oracle only): ORAS-FGMRES iterations with exact and incomplete local solves.

TEST INFRASTRUCTURE ONLY.  Prints, for the unit cube at k = 8 pi (6 x 6 x 6 cubes, P3, 8
subdomains, overlap 1) and the layered model at 0.4 Hz (8 x 8 x 4 cubes, 4 subdomains,
overlap 1), with one random right-hand side, tol 1e-8, restart 40, at most 200 iterations,
the iteration count and final residual of ORAS-FGMRES with the local operators factored
exactly (SuperLU), by ICC (level 0; natural and, on the cube, reverse Cuthill-McKee order),
and by the same incomplete factorisation on the pattern of A_i^2 (level-one fill and more).

    python3 -m oracle.icc_study
"""
from __future__ import annotations

import time

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

import workloads as w

from . import ddm as odd
from . import fem, icc, krylov


class _Permuted:
    """ICC of P A P^T (P a permutation), optionally on the lower pattern of |A|^2."""

    def __init__(self, A, perm, fill):
        self.p = perm
        self.ip = np.argsort(perm)
        Ap = A[perm][:, perm].tocoo()
        if fill:
            S = abs(Ap.tocsr())
            S2 = (S @ S).tocoo()
            Ap = sp.coo_matrix((np.concatenate([Ap.data, np.zeros(S2.nnz, Ap.dtype)]),
                                (np.concatenate([Ap.row, S2.row]), np.concatenate([Ap.col, S2.col]))), shape=Ap.shape)
        Ap = Ap.tocsr()
        Ap.sum_duplicates()
        self.f = icc.ICC(Ap)

    def solve(self, b):
        b = np.asarray(b)
        return self.f.solve(b[self.p])[self.ip]


def main():
    study(w.unit_cube_problem(6), "unit cube 6^3, k = 8 pi", full=True)
    study(w.layered_problem(freq=0.4, r=1.4, parts=(2, 2, 1), overlap=1, n_sources=(2, 2),
                            max_cubes=(8, 8, 4)), "layered 8x8x4 cubes, 0.4 Hz", full=False)


def study(p, label, full=True):
    """Exact and incomplete local factors on problem p (one random right-hand side, tol 1e-8,
    restart 40, at most 200 iterations); full: also ICC(0) in reverse Cuthill-McKee order."""
    rng = np.random.default_rng(0)
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq, p.quality)
    subs, _ = odd.build_subdomains(om, p.velocity, p.freq, p.quality, p.partition, p.n_sub, p.overlap)
    B = rng.standard_normal((om.n, 1)) + 1j * rng.standard_normal((om.n, 1))
    print(f"{label}, n = {om.n}, subdomains of {min(s.gdofs.size for s in subs)}-{max(s.gdofs.size for s in subs)} dofs")
    variants = [("exact (SuperLU)", None), ("ICC(0), natural order", (False, False))]
    if full:
        variants.append(("ICC(0), reverse Cuthill-McKee", (True, False)))
    variants.append(("incomplete, pattern of A^2", (False, True)))
    for name, v in variants:
        t = time.perf_counter()
        if v is None:
            odd.factor_subdomains(subs)
            entries = sum(s.lu.L.nnz + s.lu.U.nnz for s in subs)
        else:
            rcm, fill = v
            for s in subs:
                A_i = s.A.tocsr()
                perm = reverse_cuthill_mckee(A_i, symmetric_mode=True) if rcm else np.arange(A_i.shape[0])
                s.lu = _Permuted(A_i, perm, fill)
            entries = sum(s.lu.f.L.nnz + s.lu.f.n for s in subs)
        tf = time.perf_counter() - t
        X, info = krylov.block_fgmres(lambda x: A @ x, B, odd.ORAS(A, subs).apply, tol=1e-8, m=40, max_iter=200)
        res = np.linalg.norm(B - A @ X) / np.linalg.norm(B)
        print(f"{name:32s} factor entries {entries:9d}  factor {tf:5.1f} s  iterations {info['iters']:4d}  "
              f"residual {res:.2e}", flush=True)


if __name__ == "__main__":
    main()
