"""Oracle: right-preconditioned block FGMRES(m) with CGS2 Arnoldi, and a dense direct solve.

TEST INFRASTRUCTURE ONLY (tests/, graft smoke check, bench.py CPU baseline).

The paper solves A u = b with GMRES preconditioned by the two-level ORAS operator and
stops on the backward error ||A u - b|| / ||b|| <= eps (sections "Tetrahedral finite
element method" and "Domain decomposition preconditioner").  Readings:
the flexible variant (the preconditioner may run in lower precision), x0 = 0, classical
Gram-Schmidt applied twice, a true block Arnoldi over the source block, QR factors
normalised to a real non-negative diagonal, the least-squares problem solved directly
from the block Hessenberg matrix at every step, and convergence when every column meets
the tolerance on the explicitly recomputed FP64 residual.
"""
from __future__ import annotations

import numpy as np


def qr_pos(W):
    """Thin QR with diag(R) real and >= 0 (Householder via numpy, then signs fixed)."""
    Q, R = np.linalg.qr(W)
    d = np.diag(R).copy()
    ph = np.where(np.abs(d) > 0, d / np.where(np.abs(d) > 0, np.abs(d), 1), 1.0)
    Q = Q * ph[None, :]
    R = np.conj(ph)[:, None] * R
    return Q, R


def block_fgmres(A, B, precond, tol=1e-6, m=40, max_iter=500, fixed_iters=None, x0=None, dtype=np.complex128):
    """Solve A X = B for a block B (n, s).

    A and precond are callables on (n, s) blocks.  Returns X and a dict with the number
    of inner iterations, restarts, per-column true relative residuals and the history of
    least-squares residual estimates.  With fixed_iters=k the first cycle runs exactly k
    steps (tol is ignored) and no restart happens.  dtype=np.complex64 runs every array of
    the method (basis, Hessenberg matrix, least squares, iterate, residual) in single
    precision, the paper's "whole computation in single precision" (section "Numerical
    results"); A and precond must then return complex64 blocks."""
    B = np.asarray(B, dtype)
    if B.ndim == 1:
        B = B[:, None]
    n, s = B.shape
    bnorm = np.linalg.norm(B, axis=0)
    bnorm = np.where(bnorm > 0, bnorm, 1.0)
    X = np.zeros((n, s), dtype) if x0 is None else np.array(x0, dtype).reshape(n, s)
    total = 0
    restarts = 0
    hist = []
    while True:
        R = B - A(X) if (total > 0 or x0 is not None) else B.copy()
        V1, S = qr_pos(R)
        V = [V1]
        Zs = []
        Hbar = np.zeros(((m + 1) * s, m * s), dtype)
        G0 = np.zeros(((m + 1) * s, s), dtype)
        G0[:s] = S
        steps = m if fixed_iters is None else min(m, fixed_iters)
        j_done = 0
        for j in range(steps):
            Zj = precond(V[j])
            W = A(Zj)
            Vb = np.concatenate(V, axis=1)  # (n, (j+1)s)
            Hcol = np.zeros(((j + 1) * s, s), dtype)
            for _ in range(2):  # classical Gram-Schmidt, twice
                Hp = Vb.conj().T @ W
                W = W - Vb @ Hp
                Hcol += Hp
            Vn, Hn = qr_pos(W)
            Hbar[: (j + 1) * s, j * s:(j + 1) * s] = Hcol
            Hbar[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s] = Hn
            V.append(Vn)
            Zs.append(Zj)
            j_done = j + 1
            total += 1
            H = Hbar[: (j + 2) * s, : (j + 1) * s]
            Y, *_ = np.linalg.lstsq(H, G0[: (j + 2) * s], rcond=None)
            est = np.linalg.norm(G0[: (j + 2) * s] - H @ Y, axis=0) / bnorm
            hist.append(est)
            if fixed_iters is None and (np.all(est <= tol) or total >= max_iter):
                break
        H = Hbar[: (j_done + 1) * s, : j_done * s]
        Y, *_ = np.linalg.lstsq(H, G0[: (j_done + 1) * s], rcond=None)
        X = X + np.concatenate(Zs, axis=1) @ Y
        res = np.linalg.norm(B - A(X), axis=0) / bnorm
        if fixed_iters is not None or np.all(res <= tol) or total >= max_iter:
            return X, {"iters": total, "restarts": restarts, "rel_residual": res, "history": hist,
                       "V": np.concatenate(V, axis=1), "Z": np.concatenate(Zs, axis=1),
                       "Hbar": Hbar[: (j_done + 1) * s, : j_done * s]}
        restarts += 1


def dense_solve(A, B):
    """Direct solve with the dense matrix (tiny problems only)."""
    return np.linalg.solve(A.toarray(), np.asarray(B, np.complex128))
