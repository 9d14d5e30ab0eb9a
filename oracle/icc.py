"""Oracle: incomplete Cholesky (ICC) of the local operators, the paper's approximate local solver.

TEST INFRASTRUCTURE ONLY (tests/, graft smoke check, bench.py CPU baseline).

The paper (section "Numerical results", the comparison of Cholesky and ICC for the fine local
matrices) replaces the exact factorisation of A_i in eq. (oras) by an incomplete Cholesky
factorisation.  It names no variant.  Readings:
* level 0, no fill: A_i ~ L D L^T with L unit lower triangular on the lower pattern of A_i;
* the complex symmetric form (transpose, not conjugate transpose), since A_i = A_i^T;
* the local order of A_i (its sorted global dofs), no reordering;
* no shift or pivot modification: a zero pivot is an error.
The factors are the unique ones for which L D L^T equals A_i at every position of the lower
pattern (the defining property, pinned in tests); they are computed row by row in increasing
order, every entry from the entries of earlier rows.  Plain Python loops: small cases only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class ICC:
    """L (unit lower, CSR without the diagonal) and d of A ~ L diag(d) L^T."""

    def __init__(self, A, dtype=np.complex128):
        A = sp.csr_matrix(A)
        n = A.shape[0]
        low = sp.tril(A, format="csr")
        low.sort_indices()
        self.n = n
        self.dtype = dtype
        ptr, col, val = low.indptr, low.indices, low.data.astype(dtype)
        # row i of L: its strictly lower pattern (ascending) and values; d_i
        rows = [dict() for _ in range(n)]
        d = np.zeros(n, dtype)
        for i in range(n):
            Li = rows[i]
            diag = dtype(0)
            for k in range(ptr[i], ptr[i + 1]):
                j = col[k]
                if j == i:
                    diag = val[k]
                    continue
                # l_ij d_j = a_ij - sum over k < j in both patterns of l_ik d_k l_jk
                Lj = rows[j]
                acc = val[k]
                for kk, lik in Li.items():  # entries of row i already computed (columns < j)
                    ljk = Lj.get(kk)
                    if ljk is not None:
                        acc = acc - lik * d[kk] * ljk
                if d[j] == 0:
                    raise ZeroDivisionError(f"ICC: zero pivot {j}")
                Li[j] = dtype(acc / d[j])
            acc = diag
            for kk, lik in Li.items():
                acc = acc - lik * lik * d[kk]
            if acc == 0:
                raise ZeroDivisionError(f"ICC: zero pivot {i}")
            d[i] = acc
        self.d = d
        r, c, v = [], [], []
        for i in range(n):
            for j in sorted(rows[i]):
                r.append(i)
                c.append(j)
                v.append(rows[i][j])
        self.L = sp.csr_matrix((np.array(v, dtype), (np.array(r, np.int64), np.array(c, np.int64))), shape=(n, n))

    def solve(self, b):
        """x = (L D L^T)^{-1} b: forward substitution with unit L (SciPy's sparse triangular
        solve), division by d, backward substitution with L^T."""
        b = np.asarray(b)
        squeeze = b.ndim == 1
        y = np.array(b.reshape(self.n, -1), dtype=self.dtype)
        I = sp.identity(self.n, dtype=self.dtype, format="csr")
        y = spla.spsolve_triangular((I + self.L).tocsr(), y, lower=True, unit_diagonal=True)
        y = y / self.d[:, None]
        y = spla.spsolve_triangular((I + self.L.T).tocsr(), y, lower=False, unit_diagonal=True)
        y = np.asarray(y, self.dtype)
        return y[:, 0] if squeeze else y


def with_square_pattern(A):
    """A with explicit zeros added on the pattern of |A|^2 (every (i, j) joined by a path of
    length two), so that ICC keeps one level of neighbours' fill: the variant the oracle study
    finds convergent."""
    A = sp.csr_matrix(A)
    S = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    P = (S @ S).tocoo()
    Ac = A.tocoo()
    F = sp.coo_matrix((np.concatenate([Ac.data, np.zeros(P.nnz, Ac.data.dtype)]),
                       (np.concatenate([Ac.row, P.row]), np.concatenate([Ac.col, P.col]))), shape=A.shape).tocsr()
    F.sum_duplicates()
    F.sort_indices()
    return F


def factor_subdomains_icc(subs, dtype=np.complex128, square_pattern=False):
    """The ICC factors of every local operator, in place of the exact ones (s.lu gets an
    object with the same solve(b) call); square_pattern: on the pattern of A_i^2."""
    for s in subs:
        s.lu = ICC(with_square_pattern(s.A) if square_pattern else s.A, dtype)
    return subs
