"""Pins of the oracle's incomplete Cholesky (oracle/icc.py), the paper's approximate local solver.

* A matrix whose lower pattern is closed under elimination (tridiagonal) has no fill, so its
  level-0 incomplete factorisation is the exact LDL^T: the ICC solve equals a direct solve.
* The defining property of the level-0 factors: L D L^T equals A at every position of the lower
  pattern of A (checked by an independent sparse product on a P3 local operator with Robin
  faces, whose factorisation does drop fill).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as w
from oracle import ddm as odd
from oracle import fem, icc


def test_icc_is_exact_without_fill():
    rng = np.random.default_rng(3)
    n = 60
    main = rng.standard_normal(n) + 1j * rng.standard_normal(n) + 4.0
    off = rng.standard_normal(n - 1) + 1j * rng.standard_normal(n - 1)
    T = sp.diags([off, main, off], [-1, 0, 1], format="csr")
    b = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    x = icc.ICC(T).solve(b)
    ref = spla.spsolve(T.tocsc(), b)
    assert np.linalg.norm(x - ref) <= 1e-13 * np.linalg.norm(ref)


def test_icc_matches_operator_on_its_pattern():
    p = w.unit_cube_problem(3, freq=2.0, parts=(2, 1, 1), overlap=1)
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    subs, _ = odd.build_subdomains(om, p.velocity, p.freq, None, p.partition, p.n_sub, p.overlap)
    A_i = subs[0].A.tocsr()
    f = icc.ICC(A_i)
    I = sp.identity(f.n, format="csr")
    M = ((I + f.L) @ sp.diags(f.d) @ (I + f.L).T).tocsr()
    low = sp.tril(A_i).tocoo()
    got = np.asarray(M[low.row, low.col]).ravel()
    assert np.max(np.abs(got - low.data)) <= 1e-12 * np.max(np.abs(low.data))
    # and it is incomplete: the product has entries (dropped fill) outside that pattern
    assert sp.tril(M).tocsr().nnz > sp.tril(A_i).nnz


def test_icc_square_pattern_matches_operator_on_its_pattern():
    """ICC on the pattern of A_i^2: L D L^T equals A_i on the lower part of that pattern (zero on
    its fill positions), the pattern contains A_i's, and the filled factors solve closer to the
    exact solution than the level-0 ones."""
    p = w.unit_cube_problem(3, freq=2.0, parts=(2, 1, 1), overlap=1)
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    subs, _ = odd.build_subdomains(om, p.velocity, p.freq, None, p.partition, p.n_sub, p.overlap)
    A_i = subs[0].A.tocsr()
    F2 = icc.with_square_pattern(A_i)
    assert F2.nnz > A_i.nnz
    low = sp.tril(A_i).tocoo()
    low2_all = sp.tril(F2).tocoo()
    pat2 = set(zip(low2_all.row.tolist(), low2_all.col.tolist()))
    assert set(zip(low.row.tolist(), low.col.tolist())) <= pat2
    f = icc.ICC(F2)
    I = sp.identity(f.n, format="csr")
    M = ((I + f.L) @ sp.diags(f.d) @ (I + f.L).T).tocsr()
    low2 = sp.tril(F2).tocoo()
    got = np.asarray(M[low2.row, low2.col]).ravel()
    want = np.asarray(A_i[low2.row, low2.col]).ravel()
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(A_i.data))
    rng = np.random.default_rng(5)
    b = rng.standard_normal(f.n) + 1j * rng.standard_normal(f.n)
    x = spla.spsolve(A_i.tocsc(), b)
    e2 = np.linalg.norm(f.solve(b) - x)
    e0 = np.linalg.norm(icc.ICC(A_i).solve(b) - x)
    assert e2 < e0
