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


def _harmonic_ritz(G, WV, k):
    """k eigenvectors of G^H G p = theta G^H WV p with the smallest |theta| (finite ones)."""
    import scipy.linalg as sla

    th, P = sla.eig(G.conj().T @ G, G.conj().T @ WV)
    th = np.where(np.isfinite(th), th, np.inf)
    return P[:, np.argsort(np.abs(th))[:k]]


def gcrodr(A, b, precond, tol=1e-6, m=40, k=10, max_iter=2000, recycle=None):
    """GCRO-DR(m, k) for one right-hand side (Parks, de Sturler, Mackey, Johnson, Maiti,
    "Recycling Krylov subspaces for sequences of linear systems", 2006), the recycling method
    the paper's conclusion proposes for many sources.  Right-preconditioned with a fixed
    (linear) preconditioner: it solves (A M^{-1}) y = b and returns x = M^{-1} y.

    recycle = (U, C) with (A M^{-1}) U = C and C^H C = I, from an earlier solve with the same
    operator and preconditioner (None: the first cycle is a GMRES(m) cycle).  Each later
    cycle runs m - k Arnoldi steps of (I - C C^H) A M^{-1}, minimises the residual over
    [U, V], and replaces (U, C) by the k harmonic Ritz vectors of the cycle's space.  With
    k = 0 it is restarted GMRES(m).  Returns x, info (iterations = applications of A M^{-1},
    cycles, explicit relative residual) and the recycle pair for the next solve."""
    b = np.asarray(b, np.complex128).ravel()
    Ah = lambda v: np.asarray(A(precond(v[:, None])))[:, 0]
    bn = np.linalg.norm(b)
    y = np.zeros_like(b)
    r = b.copy()
    U, C = (None, None) if recycle is None or k == 0 else recycle
    if U is not None:  # the part of b in range(C) is solved at once
        c = C.conj().T @ r
        y = y + U @ c
        r = r - C @ c
    total = cycles = 0
    while np.linalg.norm(r) > tol * bn and total < max_iter:
        kk = 0 if U is None else k
        p = m - kk
        beta = np.linalg.norm(r)
        V = [r / beta]
        H = np.zeros((p + 1, p), np.complex128)
        Bc = np.zeros((kk, p), np.complex128)
        dn = None if U is None else 1.0 / np.linalg.norm(U, axis=0)

        def small(steps):
            """The cycle's (kk + steps + 1) x (kk + steps) matrix G with A M^{-1} Vhat = What G,
            and What^H r = beta e_{kk+1} (r is orthogonal to C)."""
            G = np.zeros((kk + steps + 1, kk + steps), np.complex128)
            if kk:
                G[:kk, :kk] = np.diag(dn)
                G[:kk, kk:] = Bc[:, :steps]
            G[kk:, kk:] = H[: steps + 1, :steps]
            c = np.zeros(kk + steps + 1, np.complex128)
            c[kk] = beta
            return G, c

        steps = p
        for j in range(p):
            w = Ah(V[j])
            total += 1
            if kk:
                Bc[:, j] = C.conj().T @ w
                w = w - C @ Bc[:, j]
            Vb = np.stack(V, axis=1)
            for _ in range(2):  # classical Gram-Schmidt, twice
                h = Vb.conj().T @ w
                w = w - Vb @ h
                H[: j + 1, j] += h
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j] <= 1e-14 * np.abs(H[: j + 1, j]).max()
            V.append(np.zeros_like(w) if breakdown else w / H[j + 1, j])
            G, c = small(j + 1)
            z, *_ = np.linalg.lstsq(G, c, rcond=None)
            if breakdown or np.linalg.norm(c - G @ z) <= tol * bn or total >= max_iter:
                steps = j + 1
                break
        G, c = small(steps)
        Vm1 = np.stack(V[: steps + 1], axis=1)
        if kk:
            What = np.concatenate([C, Vm1], axis=1)
            Vhat = np.concatenate([U * dn[None, :], Vm1[:, :steps]], axis=1)
            WV = What.conj().T @ Vhat
        else:
            What, Vhat = Vm1, Vm1[:, :steps]
            WV = np.eye(steps + 1, steps)
        z, *_ = np.linalg.lstsq(G, c, rcond=None)
        y = y + Vhat @ z
        r = r - What @ (G @ z)
        cycles += 1
        if k > 0 and G.shape[1] >= k:
            P = _harmonic_ritz(G, WV, k)
            Q, R = np.linalg.qr(G @ P)
            C = What @ Q
            U = Vhat @ P @ np.linalg.inv(R)
    x = np.asarray(precond(y[:, None]))[:, 0]
    res = np.linalg.norm(b - np.asarray(A(x[:, None]))[:, 0]) / bn
    return x, {"iters": total, "cycles": cycles, "rel_residual": res}, (U, C)
