"""Pins of the oracle's loads, decomposition, coarse space and block FGMRES.

Pins: fourth-order convergence of P3 to a plane-wave manufactured solution (textbook
O(h^{p+1}) in L2), agreement with a dense direct solve on tiny meshes, reciprocity of the
Green's function (A^T = A), the exact partition-of-unity identity, the one-subdomain
special case (ORAS = exact inverse), constants reproduced by the P1 coarse space, and the
Arnoldi identities of FGMRES."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as w
from oracle import ddm, fem, krylov, p3, rhs


def _cube(n, freq=1.0, parts=(2, 2, 2), overlap=1):
    p = w.unit_cube_problem(n, freq=freq, parts=parts, overlap=overlap)
    return p, fem.Mesh(p.tets, p.coords, p.face_bc)


def test_plane_wave_fourth_order():
    """||u_h - I_h u||_M / ||I_h u||_M drops ~16x per halving of h (P3: O(h^4))."""
    errs = []
    for n in (2, 4, 8):
        p, mesh = _cube(n, freq=1.0)
        A = fem.assemble_operator(mesh, p.velocity, p.freq)
        f = rhs.plane_wave_load(mesh, p.velocity, p.freq, p.extra["direction"])
        u = spla.spsolve(A.tocsc(), f)
        xyz = fem.dof_coordinates(mesh.tets, mesh.coords, mesh.tet_dofs, mesh.n)
        ui = rhs.plane_wave_nodal(mesh, p.velocity, p.freq, p.extra["direction"], xyz)
        _, M, _ = fem.assemble_parts(mesh)
        e = u - ui
        errs.append(np.sqrt(abs(np.vdot(e, M @ e)) / abs(np.vdot(ui, M @ ui))))
    order = np.log2(errs[1] / errs[2])
    assert order >= 3.5, errs
    assert errs[2] < 5e-4


def test_point_source_partition_of_unity():
    """sum_j phi_j(x) = 1 inside the mesh and the source at a node is a unit vector."""
    p, mesh = _cube(3)
    rng = np.random.default_rng(5)
    xs = rng.uniform(0.05, 0.95, (6, 3))
    f = rhs.point_sources(mesh, xs)
    np.testing.assert_allclose(f.sum(axis=1), 1.0, atol=1e-12)
    xyz = fem.dof_coordinates(mesh.tets, mesh.coords, mesh.tet_dofs, mesh.n)
    j = 123
    g = rhs.point_sources(mesh, xyz[j][None])
    assert abs(g[0, j] - 1) < 1e-12 and abs(g[0]).sum() - 1 < 1e-10


def test_partition_of_unity_identity():
    """sum_i R_i^T D_i R_i = I exactly (each dof owned by one subdomain)."""
    p, mesh = _cube(4, parts=(2, 2, 2), overlap=1)
    subs, own = ddm.build_subdomains(mesh, p.velocity, p.freq, None, p.partition, p.n_sub, p.overlap)
    acc = np.zeros(mesh.n, np.int64)
    for s in subs:
        acc[s.gdofs[s.owned]] += 1
        assert np.all(np.diff(s.gdofs) > 0)
        assert abs(s.A - s.A.T).max() <= 1e-14 * abs(s.A).max()
    assert np.all(acc == 1)
    # overlap grows the subdomain strictly beyond its owned dofs
    assert all(s.gdofs.size > s.owned.sum() for s in subs)


def test_local_operator_without_cuts_is_global():
    """One subdomain with no overlap: A_1 = A and ORAS = A^{-1}, FGMRES converges in 1 step."""
    p, mesh = _cube(3, parts=(1, 1, 1), overlap=0)
    A = fem.assemble_operator(mesh, p.velocity, p.freq)
    P = ddm.build_preconditioner(mesh, A, p.velocity, p.freq, None, p.partition, 1, 0)
    assert abs(P.subs[0].A - A).max() == 0
    b = rhs.plane_wave_load(mesh, p.velocity, p.freq, p.extra["direction"])
    X, info = krylov.block_fgmres(lambda x: A @ x, b, P.apply, tol=1e-12, m=10)
    assert info["iters"] == 1 and info["rel_residual"][0] < 1e-12


def test_robin_on_cut_faces():
    """A 2-subdomain split: the local operator differs from the restricted global operator
    exactly by i k |f| Fhat on the cut faces (checked through its imaginary part)."""
    p, mesh = _cube(2, parts=(2, 1, 1), overlap=0)
    subs, _ = ddm.build_subdomains(mesh, p.velocity, p.freq, None, p.partition, 2, 0)
    s = subs[0]
    k = 2 * np.pi * p.freq
    cut = s.robin_faces & ~mesh.impedance[s.tets]
    assert cut.sum() == 2 * 2 * 2  # 2x2 cube faces, 2 triangles each
    _, _, F = fem.element_parts(mesh.tets, mesh.coords, sel=s.tets)
    # total imaginary mass of the local operator = k * (physical impedance area + cut area)
    one = np.ones(s.gdofs.size)
    area_phys = (mesh.impedance[s.tets][:, :, None, None] * F).sum()
    area_cut = (cut[:, :, None, None] * F).sum()
    assert abs(area_cut - 1.0) < 1e-13  # the cut is the plane x = 1/2 of the unit cube
    assert abs((one @ (s.A.imag @ one)) - k * (area_phys + area_cut)) < 1e-10


@pytest.mark.parametrize("n,parts,overlap", [(2, (2, 1, 1), 1), (3, (2, 2, 1), 1), (4, (2, 2, 2), 1)])
def test_oras_fgmres_matches_dense(n, parts, overlap):
    """ORAS-FGMRES at tol 1e-12 agrees with numpy.linalg.solve to 1e-9 (multi-RHS block)."""
    p, mesh = _cube(n, freq=1.0, parts=parts, overlap=overlap)
    A = fem.assemble_operator(mesh, p.velocity, p.freq)
    P = ddm.build_preconditioner(mesh, A, p.velocity, p.freq, None, p.partition, p.n_sub, overlap)
    rng = np.random.default_rng(n)
    B = rng.standard_normal((mesh.n, 3)) + 1j * rng.standard_normal((mesh.n, 3))
    X, info = krylov.block_fgmres(lambda x: A @ x, B, P.apply, tol=1e-12, m=60, max_iter=200)
    Xd = krylov.dense_solve(A, B)
    assert np.all(info["rel_residual"] <= 1e-12)
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) < 1e-9


def test_reciprocity():
    """G(s,r) = phi(r)^T A^{-1} phi(s) = G(r,s), since A is complex symmetric."""
    p, mesh = _cube(3, freq=1.5)
    A = fem.assemble_operator(mesh, p.velocity, p.freq)
    srcs = np.array([[0.2, 0.3, 0.4], [0.7, 0.55, 0.15], [0.45, 0.8, 0.9]])
    F = rhs.point_sources(mesh, srcs).T
    U = krylov.dense_solve(A, F)
    G = F.T @ U
    assert abs(G - G.T).max() <= 1e-12 * abs(G).max()
    P = ddm.build_preconditioner(mesh, A, p.velocity, p.freq, None, p.partition, p.n_sub, 1)
    X, info = krylov.block_fgmres(lambda x: A @ x, F, P.apply, tol=1e-10, m=60)
    Gi = F.T @ X
    assert abs(Gi - Gi.T).max() <= 1e-8 * abs(Gi).max()


def test_fgmres_arnoldi_identities():
    """V orthonormal to 1e-13, A Z_j = V_{j+1} Hbar_j to 1e-13, and the least-squares
    residual estimate equals the explicit residual."""
    p, mesh = _cube(3, freq=1.0)
    A = fem.assemble_operator(mesh, p.velocity, p.freq)
    P = ddm.build_preconditioner(mesh, A, p.velocity, p.freq, None, p.partition, p.n_sub, 1)
    rng = np.random.default_rng(1)
    B = rng.standard_normal((mesh.n, 2)) + 1j * rng.standard_normal((mesh.n, 2))
    X, info = krylov.block_fgmres(lambda x: A @ x, B, P.apply, fixed_iters=4, m=10)
    V, Z, H = info["V"], info["Z"], info["Hbar"]
    assert abs(V.conj().T @ V - np.eye(V.shape[1])).max() < 1e-13
    assert abs(A @ Z - V @ H).max() < 1e-13 * abs(A @ Z).max()
    est = info["history"][-1]
    np.testing.assert_allclose(est, info["rel_residual"], rtol=1e-8)


def test_coarse_space_invariants():
    """Z 1 = 1 on non-Dirichlet rows (P1 reproduces constants), E = E^T, and the two-level
    preconditioner needs no more iterations than the one-level one."""
    p, mesh = _cube(8, freq=2.0, parts=(2, 2, 2), overlap=1)
    xs = np.linspace(0, 1, 9)
    ct, cc = w.kuhn_mesh(xs[::4], xs[::4], xs[::4])
    Z = ddm.coarse_interpolation(mesh, ct, cc)
    np.testing.assert_allclose(Z @ np.ones(Z.shape[1]), 1.0, atol=1e-12)
    assert Z.shape == (mesh.n, 27) and Z.nnz <= 4 * mesh.n
    A = fem.assemble_operator(mesh, p.velocity, p.freq)
    C = ddm.Coarse(Z, A)
    assert abs(C.E - C.E.T).max() <= 1e-12 * abs(C.E).max()
    f = rhs.plane_wave_load(mesh, p.velocity, p.freq, p.extra["direction"])
    P1 = ddm.build_preconditioner(mesh, A, p.velocity, p.freq, None, p.partition, p.n_sub, 1)
    P2 = ddm.ORAS(A, P1.subs, C)
    _, i1 = krylov.block_fgmres(lambda x: A @ x, f, P1.apply, tol=1e-8, m=80)
    _, i2 = krylov.block_fgmres(lambda x: A @ x, f, P2.apply, tol=1e-8, m=80)
    assert i2["iters"] <= i1["iters"]


def test_dirichlet_coarse_rows_zero():
    xs = np.linspace(0, 1, 5)
    tets, coords = w.kuhn_mesh(xs, xs, xs)
    mesh = fem.Mesh(tets, coords, w.face_bc_tags(tets, coords, dirichlet_top=True))
    ct, cc = w.kuhn_mesh(xs[::2], xs[::2], xs[::2])
    Z = ddm.coarse_interpolation(mesh, ct, cc)
    rs = np.asarray(abs(Z).sum(axis=1)).ravel()
    assert np.all(rs[mesh.dirichlet] == 0)
    np.testing.assert_allclose((Z @ np.ones(Z.shape[1]))[~mesh.dirichlet], 1.0, atol=1e-12)


def test_fgmres_single_precision_option():
    """The whole computation in complex64 (the paper's single-precision runs): every array is
    complex64, the Arnoldi relation holds to single-precision rounding, the fixed-iteration
    iterate is the FP64 one to single-precision accuracy, and a solve to the paper's 1e-3
    takes the FP64 iteration count."""
    p, mesh = _cube(3, freq=1.0)
    A = fem.assemble_operator(mesh, p.velocity, p.freq)
    A32 = A.astype(np.complex64)
    subs, _ = ddm.build_subdomains(mesh, p.velocity, p.freq, None, p.partition, p.n_sub, 1)
    ddm.factor_subdomains(subs, np.complex64)
    P32 = ddm.ORAS(A, subs, dtype=np.complex64)
    P64 = ddm.build_preconditioner(mesh, A, p.velocity, p.freq, None, p.partition, p.n_sub, 1)
    rng = np.random.default_rng(2)
    B = rng.standard_normal((mesh.n, 2)) + 1j * rng.standard_normal((mesh.n, 2))
    X32, i32 = krylov.block_fgmres(lambda x: A32 @ x, B, lambda v: P32.apply(v).astype(np.complex64),
                                   fixed_iters=4, m=10, dtype=np.complex64)
    X64, _ = krylov.block_fgmres(lambda x: A @ x, B, P64.apply, fixed_iters=4, m=10)
    assert X32.dtype == np.complex64 and i32["V"].dtype == np.complex64 and i32["Hbar"].dtype == np.complex64
    V, Z, H = (i32[k].astype(np.complex128) for k in ("V", "Z", "Hbar"))
    assert abs(A32 @ i32["Z"] - i32["V"] @ i32["Hbar"]).max() < 1e-5 * abs(A @ Z).max()
    assert abs(V.conj().T @ V - np.eye(V.shape[1])).max() < 1e-5
    assert np.linalg.norm(X32 - X64) / np.linalg.norm(X64) < 1e-4
    _, a = krylov.block_fgmres(lambda x: A32 @ x, B, lambda v: P32.apply(v).astype(np.complex64), tol=1e-3,
                               dtype=np.complex64)
    _, b = krylov.block_fgmres(lambda x: A @ x, B, P64.apply, tol=1e-3)
    assert a["iters"] == b["iters"]


def _cube_with_coarse(n, parts, overlap=1, freq=1.0, k=2):
    p, mesh = _cube(n, freq=freq, parts=parts, overlap=overlap)
    xs = np.linspace(0.0, 1.0, n + 1)[::k]
    ct, cc = w.kuhn_mesh(xs, xs, xs)
    A = fem.assemble_operator(mesh, p.velocity, p.freq)
    subs, own = ddm.build_subdomains(mesh, p.velocity, p.freq, None, p.partition, p.n_sub, overlap)
    Z = ddm.coarse_interpolation(mesh, ct, cc)
    cown = ddm.coarse_owners(mesh, cc, own)
    return p, mesh, A, subs, Z, cown


def test_inexact_coarse_one_subdomain_is_exact():
    """With one subdomain and no overlap the local operator is the global one, so the coarse
    ORAS is E^{-1} itself and one GMRES step gives the exact coarse solve."""
    p, mesh, A, subs, Z, cown = _cube_with_coarse(4, (1, 1, 1), overlap=0)
    rng = np.random.default_rng(4)
    V = rng.standard_normal((mesh.n, 3)) + 1j * rng.standard_normal((mesh.n, 3))
    exact = ddm.Coarse(Z, A).solve(V)
    for iters in (1, 10):
        q = ddm.InexactCoarse(Z, A, subs, cown, iters=iters).solve(V)
        assert np.linalg.norm(q - exact) <= 1e-10 * np.linalg.norm(exact), iters


def test_inexact_coarse_full_krylov_space_is_exact():
    """As many GMRES iterations as coarse dofs span the whole coarse space: the result is the
    exact coarse solve whatever the coarse preconditioner (four subdomains, overlap 1)."""
    p, mesh, A, subs, Z, cown = _cube_with_coarse(4, (2, 2, 1))
    nc = Z.shape[1]
    rng = np.random.default_rng(5)
    v = rng.standard_normal((mesh.n, 1)) + 1j * rng.standard_normal((mesh.n, 1))
    exact = ddm.Coarse(Z, A).solve(v)
    q = ddm.InexactCoarse(Z, A, subs, cown, iters=nc).solve(v)
    assert np.linalg.norm(q - exact) <= 1e-8 * np.linalg.norm(exact)
    # ten iterations do not reach it, but reduce the coarse residual
    ic = ddm.InexactCoarse(Z, A, subs, cown, iters=10)
    r = Z.T @ v
    y, _ = krylov.block_fgmres(lambda x: ic.E @ x, r, ic.precond, fixed_iters=10, m=10)
    assert np.linalg.norm(ic.E @ y - r) < 0.5 * np.linalg.norm(r)


def test_coarse_partition_of_unity_owns_each_coarse_dof_once():
    """Every coarse dof is in some coarse subdomain and owned by exactly one of them, the one
    owning the fine dof at its vertex (the lowest subdomain id whose own tets hold it)."""
    p, mesh, A, subs, Z, cown = _cube_with_coarse(4, (2, 2, 2))
    ic = ddm.InexactCoarse(Z, A, subs, cown)
    owned = np.concatenate([J[o] for J, _, o in ic.loc])
    assert np.array_equal(np.sort(owned), np.arange(Z.shape[1]))
    # the vertex at the origin lies in subdomain 0 only; the centre vertex (2,2,2) of the 4^3
    # cube touches all eight boxes, so it belongs to the lowest id, 0; the far corner to box 7
    cc = w.kuhn_mesh(*(np.linspace(0.0, 1.0, 5)[::2],) * 3)[1]
    at = {tuple(np.round(c * 2).astype(int)): j for j, c in enumerate(cc)}
    assert cown[at[(0, 0, 0)]] == 0 and cown[at[(1, 1, 1)]] == 0 and cown[at[(2, 2, 2)]] == 7


def test_gcrodr_without_recycling_is_restarted_gmres():
    """GCRO-DR with k = 0 is GMRES(m): with a fixed preconditioner the flexible oracle runs the
    same iteration, so iterations and iterate agree (restarts forced by m = 8)."""
    p, mesh = _cube(3, freq=1.0)
    A = fem.assemble_operator(mesh, p.velocity, p.freq)
    P = ddm.build_preconditioner(mesh, A, p.velocity, p.freq, None, p.partition, p.n_sub, 1)
    rng = np.random.default_rng(6)
    b = rng.standard_normal(mesh.n) + 1j * rng.standard_normal(mesh.n)
    x, info, _ = krylov.gcrodr(lambda v: A @ v, b, P.apply, tol=1e-10, m=8, k=0)
    xo, io = krylov.block_fgmres(lambda v: A @ v, b[:, None], P.apply, tol=1e-10, m=8)
    assert info["iters"] == io["iters"] and info["iters"] > 8
    assert np.linalg.norm(x - xo[:, 0]) <= 1e-8 * np.linalg.norm(xo)


def test_gcrodr_recycle_space_and_recycled_solves():
    """After a solve, the recycle pair satisfies A M^{-1} U = C with C^H C = I; solves of new
    right-hand sides that start from it reach the direct solution."""
    p, mesh = _cube(3, freq=1.5)
    A = fem.assemble_operator(mesh, p.velocity, p.freq)
    P = ddm.build_preconditioner(mesh, A, p.velocity, p.freq, None, p.partition, p.n_sub, 1)
    rng = np.random.default_rng(7)
    Bs = rng.standard_normal((mesh.n, 3)) + 1j * rng.standard_normal((mesh.n, 3))
    Xd = krylov.dense_solve(A, Bs)
    rec = None
    for c in range(3):
        x, info, rec = krylov.gcrodr(lambda v: A @ v, Bs[:, c], P.apply, tol=1e-10, m=10, k=4, recycle=rec)
        assert info["rel_residual"] <= 1e-9
        assert np.linalg.norm(x - Xd[:, c]) <= 1e-7 * np.linalg.norm(Xd[:, c])
        U, C = rec
        assert U.shape[1] == 4
        assert abs(C.conj().T @ C - np.eye(4)).max() <= 1e-10
        AU = A @ P.apply(U)
        assert np.linalg.norm(AU - C) <= 1e-8 * np.linalg.norm(C)


def test_gcrodr_recycling_deflates_a_positive_definite_operator():
    """The case the method is built for: restarted GMRES(20) stalls on a stiffness-dominated
    (symmetric positive definite) operator, GCRO-DR(20, 8) converges, and each later right-hand
    side that starts from the recycled space takes fewer iterations than the first."""
    p, mesh = _cube(3, freq=1.0)
    K, M, _ = fem.assemble_parts(mesh)
    A = (K + 0.01 * M).astype(np.complex128)
    rng = np.random.default_rng(1)
    Bs = rng.standard_normal((mesh.n, 3)) + 1j * rng.standard_normal((mesh.n, 3))
    _, g, _ = krylov.gcrodr(lambda v: A @ v, Bs[:, 0], lambda v: v, tol=1e-8, m=20, k=0, max_iter=250)
    assert g["rel_residual"] > 1e-6
    rec, its = None, []
    for c in range(3):
        x, info, rec = krylov.gcrodr(lambda v: A @ v, Bs[:, c], lambda v: v, tol=1e-8, m=20, k=8, recycle=rec,
                                     max_iter=1500)
        assert info["rel_residual"] <= 1e-8
        its.append(info["iters"])
    assert its[0] < 250 and its[1] < 0.8 * its[0] and its[2] < 0.8 * its[0], its


def test_inexact_coarse_full_overlap_is_exact():
    """Two subdomains that each grow over the whole cube: every local coarse operator is E,
    so the coarse ORAS (each coarse dof taken from its owner only) is E^{-1} itself (summing the
    two subdomains' results instead would give 2 E^{-1}), and one GMRES step is exact."""
    p, mesh, A, subs, Z, cown = _cube_with_coarse(4, (2, 1, 1), overlap=4)
    assert all(s.gdofs.size == mesh.n for s in subs)
    ic = ddm.InexactCoarse(Z, A, subs, cown, iters=1)
    rng = np.random.default_rng(8)
    r = rng.standard_normal((Z.shape[1], 2)) + 1j * rng.standard_normal((Z.shape[1], 2))
    Ed = ic.E.toarray()
    assert np.linalg.norm(ic.precond(r) - np.linalg.solve(Ed, r)) <= 1e-10 * np.linalg.norm(np.linalg.solve(Ed, r))
    V = rng.standard_normal((mesh.n, 2)) + 1j * rng.standard_normal((mesh.n, 2))
    exact = ddm.Coarse(Z, A).solve(V)
    assert np.linalg.norm(ic.solve(V) - exact) <= 1e-10 * np.linalg.norm(exact)
