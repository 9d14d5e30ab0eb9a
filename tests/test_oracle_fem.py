"""Pins of the oracle's reference element, dof numbering and assembly.

Each check compares the oracle with something other than itself: exact rationals against
an independent Gauss quadrature, nodal interpolation identities, closed-form counts on the
Kuhn lattice, and invariants of the continuous operators (constants in the kernel of K,
total volume and boundary area, symmetry, sign of the absorbing term)."""
import numpy as np
import pytest
from fractions import Fraction

import workloads as w
from oracle import fem, p3


def _tet_rule(n=8):
    """Collapsed Gauss-Legendre rule on the unit tet (independent of the oracle)."""
    g, wt = np.polynomial.legendre.leggauss(n)
    g, wt = 0.5 * (g + 1), 0.5 * wt
    U, V, W = np.meshgrid(g, g, g, indexing="ij")
    WU, WV, WW = np.meshgrid(wt, wt, wt, indexing="ij")
    x = U
    y = V * (1 - U)
    z = W * (1 - U) * (1 - V)
    jac = (1 - U) ** 2 * (1 - V)
    return np.stack([x.ravel(), y.ravel(), z.ravel()], 1), (WU * WV * WW * jac).ravel()


def _bary(P, X):
    J = np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], axis=1)
    l = np.linalg.solve(J, (X - P[0]).T).T
    return np.concatenate([1 - l.sum(1, keepdims=True), l], axis=1)


def test_basis_is_nodal_and_cubic():
    """phi_i(x_j) = delta_ij on the 20 P3 nodes (unisolvent set), all monomials degree <= 3."""
    nodes = p3.node_barycentrics()
    for i, poly in enumerate(p3.basis()):
        assert all(sum(e) <= 3 for e in poly)
        for j, lam in enumerate(nodes):
            assert p3.evaluate(poly, lam) == (1 if i == j else 0)


def test_reference_sums_exact():
    """sum_ij Mhat = 1 and sum_ij Fhat_f = 1 exactly (the basis sums to one)."""
    assert sum(sum(r) for r in p3.mass_exact()) == Fraction(1)
    for f in range(4):
        assert sum(sum(r) for r in p3.face_mass_exact(f)) == Fraction(1)


@pytest.mark.parametrize("seed", [0, 1])
def test_element_matrices_match_quadrature(seed):
    """K_e, M_e and the face masses on a random tet against Gauss quadrature with
    finite-difference gradients of the nodal basis."""
    rng = np.random.default_rng(seed)
    P = np.array([[0, 0, 0], [1, 0.1, 0], [0.2, 1, 0.1], [0.1, 0.3, 1.2]]) + 0.2 * rng.standard_normal((4, 3))
    tets = np.array([[0, 1, 2, 3]])
    K, M, F = fem.element_parts(tets, P)
    xi, wq = _tet_rule(8)
    J = np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], axis=1)
    X = P[0] + xi @ J.T
    dv = abs(np.linalg.det(J))
    phi = p3.eval_basis_float(_bary(P, X))
    Mq = np.einsum("q,qi,qj->ij", wq * dv, phi, phi)
    h = 1e-5
    grads = np.zeros((X.shape[0], 20, 3))
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        grads[:, :, d] = (p3.eval_basis_float(_bary(P, X + e)) - p3.eval_basis_float(_bary(P, X - e))) / (2 * h)
    Kq = np.einsum("q,qid,qjd->ij", wq * dv, grads, grads)
    np.testing.assert_allclose(M[0], Mq, atol=1e-14 * dv * 100)
    np.testing.assert_allclose(K[0], Kq, atol=1e-6 * abs(Kq).max())
    # face f: triangle rule
    g, wt = np.polynomial.legendre.leggauss(8)
    g, wt = 0.5 * (g + 1), 0.5 * wt
    U, V = np.meshgrid(g, g, indexing="ij")
    WU, WV = np.meshgrid(wt, wt, indexing="ij")
    uu, vv, ww = U.ravel(), (V * (1 - U)).ravel(), (WU * WV * (1 - U)).ravel()
    for f in range(4):
        a, b, c = p3.FACES[f]
        Xf = P[a] + np.outer(uu, P[b] - P[a]) + np.outer(vv, P[c] - P[a])
        area2 = np.linalg.norm(np.cross(P[b] - P[a], P[c] - P[a]))
        ph = p3.eval_basis_float(_bary(P, Xf))
        Fq = np.einsum("q,qi,qj->ij", ww * area2, ph, ph)
        np.testing.assert_allclose(F[0, f], Fq, atol=1e-13 * area2)


def test_dof_counts_kuhn():
    """n = (3nx+1)(3ny+1)(3nz+1), T = 6 nx ny nz; every interior face in exactly 2 tets."""
    for grid in [(1, 1, 1), (2, 3, 1), (3, 2, 2)]:
        xs = [np.linspace(0, 1, g + 1) for g in grid]
        tets, coords = w.kuhn_mesh(*xs)
        td, n = fem.dof_numbering(tets)
        assert n == w.kuhn_ndofs(*grid)
        assert tets.shape[0] == 6 * np.prod(grid)
        nb = fem.face_neighbours(tets)
        nbd = (nb < 0).sum()
        nx, ny, nz = grid
        assert nbd == 4 * (nx * ny + ny * nz + nx * nz)  # 2 triangles per boundary square
        # neighbour relation is symmetric
        for t in range(tets.shape[0]):
            for f in range(4):
                if nb[t, f] >= 0:
                    assert t in nb[nb[t, f]]


def test_dof_numbering_key_order():
    """Dof ids follow the integer key order (vertex < its edges < its faces) and every node
    shared by two tets gets one id."""
    tets, coords = w.kuhn_mesh(*[np.linspace(0, 1, 3)] * 3)
    td, n = fem.dof_numbering(tets)
    keys = fem.dof_keys(tets).reshape(-1, 4)
    ids = td.ravel()
    byid = {}
    for k, i in zip(map(tuple, keys), ids):
        assert byid.setdefault(i, k) == k
    ordered = [byid[i] for i in range(n)]
    assert ordered == sorted(ordered)
    xyz = fem.dof_coordinates(tets, coords, td, n)
    lam = np.array([[float(x) for x in pt] for pt in p3.node_barycentrics()])
    pos = np.einsum("lv,tvd->tld", lam, coords[tets])
    np.testing.assert_allclose(xyz[td], pos, atol=1e-14)


def test_row_counts_kuhn_interior(cube4):
    """Interior rows of the Kuhn P3 lattice: vertex 175, axis/body-diagonal edge 64,
    face-diagonal edge 44, face node 30 (counted from the tets around each node)."""
    p, mesh = cube4
    ip, ix = fem.pattern(mesh.tet_dofs, mesh.n)
    cnt = np.diff(ip)
    xyz = fem.dof_coordinates(mesh.tets, mesh.coords, mesh.tet_dofs, mesh.n)
    interior = np.all((xyz > 0.25 - 1e-12) & (xyz < 0.75 + 1e-12), axis=1)
    keys = fem.dof_keys(mesh.tets).reshape(-1, 4)
    kind = np.empty(mesh.n, object)
    for k, i in zip(keys, mesh.tet_dofs.ravel()):
        if k[1] < 0:
            kind[i] = "v"
        elif k[2] < 0:
            d = np.abs(mesh.coords[k[1]] - mesh.coords[k[0]]) > 1e-12
            kind[i] = {1: "axis", 2: "facediag", 3: "body"}[int(d.sum())]
        else:
            kind[i] = "face"
    expect = {"v": 175, "axis": 64, "body": 64, "facediag": 44, "face": 30}
    for kd, c in expect.items():
        sel = interior & (kind == kd)
        assert sel.any()
        assert np.all(cnt[sel] == c), (kd, np.unique(cnt[sel]))
    # symmetric pattern
    A = fem.assemble_operator(mesh, p.velocity, p.freq)
    S = (A != 0).astype(np.int8)
    assert (S - S.T).nnz == 0


def test_global_invariants(cube4):
    """K 1 = 0; 1^T M 1 = vol; 1^T M_G 1 = boundary area; linear patch test; A = A^T;
    Im(x^H A x) = k x^H M_G x >= 0 for real k."""
    p, mesh = cube4
    K, M, MG = fem.assemble_parts(mesh)
    one = np.ones(mesh.n)
    assert abs(K @ one).max() < 1e-12
    assert abs(one @ (M @ one) - 1.0) < 1e-13
    assert abs(one @ (MG @ one) - 6.0) < 1e-12
    xyz = fem.dof_coordinates(mesh.tets, mesh.coords, mesh.tet_dofs, mesh.n)
    lin = 0.3 * xyz[:, 0] - 1.7 * xyz[:, 1] + 0.9 * xyz[:, 2] + 2.0
    interior = np.all((xyz > 1e-12) & (xyz < 1 - 1e-12), axis=1)
    assert abs((K @ lin)[interior]).max() < 1e-11
    A = fem.assemble_operator(mesh, p.velocity, p.freq)
    assert abs(A - A.T).max() <= 1e-14 * abs(A).max()  # symmetric up to the rounding of K_e
    rng = np.random.default_rng(3)
    x = rng.standard_normal(mesh.n) + 1j * rng.standard_normal(mesh.n)
    k = 2 * np.pi * p.freq
    q = np.vdot(x, A @ x)
    assert abs(q.imag - k * np.vdot(x, MG @ x).real) < 1e-9 * abs(q)
    assert q.imag > 0


def test_dirichlet_rows_identity():
    """Dirichlet dofs: zero row/column except a unit diagonal; the pattern is unchanged."""
    xs = np.linspace(0, 1, 3)
    tets, coords = w.kuhn_mesh(xs, xs, xs)
    bc = w.face_bc_tags(tets, coords, dirichlet_top=True)
    mesh = fem.Mesh(tets, coords, bc)
    assert mesh.dirichlet.sum() == 7 * 7  # nodes of the top plane
    vel = np.ones(tets.shape[0])
    A = fem.assemble_operator(mesh, vel, 1.0)
    ip, ix = fem.pattern(mesh.tet_dofs, mesh.n)
    np.testing.assert_array_equal(A.indptr, ip)
    np.testing.assert_array_equal(A.indices, ix)
    D = np.nonzero(mesh.dirichlet)[0]
    Ad = A[D].toarray()
    assert np.all(Ad[np.arange(D.size), D] == 1)
    Ad[np.arange(D.size), D] = 0
    assert np.all(Ad == 0)
    assert np.all(A[:, D].toarray()[~mesh.dirichlet] == 0)


def test_assemble_rows_matches_full(cube4):
    p, mesh = cube4
    A = fem.assemble_operator(mesh, p.velocity, p.freq)
    rows = [0, 17, mesh.n // 2, mesh.n - 1]
    out = fem.assemble_rows(mesh, p.velocity, p.freq, None, rows)
    for r in rows:
        cols, vals = out[r]
        np.testing.assert_array_equal(cols, A.indices[A.indptr[r]:A.indptr[r + 1]])
        np.testing.assert_allclose(vals, A.data[A.indptr[r]:A.indptr[r + 1]], rtol=0, atol=1e-13 * abs(vals).max())


def test_paper_dof_to_element_ratio():
    """The paper's mesh table lists ~4.5 dofs per element (16M elts / 74M dofs, 131M / 575M,
    63M / 286M, 506M / 2285M); the P3 count on Kuhn meshes tends to 27/6 = 4.5, and the
    5-ppwl regular Overthrust mesh (h = 88 m, 227 x 227 x 53 cubes) gives 16.4M / 74.4M."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_mesh_table.json")))
    for row in g["rows"]:
        assert 4.3 < row["dofs_M"] / row["elts_M"] < 4.7
    nx, ny, nz = 227, 227, 53
    assert abs(6 * nx * ny * nz / 1e6 - 16.4) < 0.05
    assert abs(w.kuhn_ndofs(nx, ny, nz) / 1e6 - 74.4) < 0.1
    # and on small meshes the oracle's own count equals the closed form
    tets, _ = w.kuhn_mesh(*[np.linspace(0, 1, 4)] * 3)
    assert fem.dof_numbering(tets)[1] == w.kuhn_ndofs(3, 3, 3)
