"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Indices (dof map, CSR pattern, R_i, D_i, Z pattern) must match bit for bit.  Floating
point: assembled values within 1e-13 relative (summation order differs), FP64
preconditioner and fixed-iteration FGMRES iterates within 1e-10 relative, mixed precision
at the stated residual with its error against the FP64 oracle reported."""
import numpy as np
import pytest

import workloads as w
from oracle import ddm as odd
from oracle import fem, krylov, rhs

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2004_07930_amd import hz

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    c = hz.Context(0, stream=torch.cuda.current_stream())
    yield c
    c.close()


def _small_layered(freq=0.4, grid=(8, 8, 4), parts=(2, 2, 1), overlap=1, with_q=False):
    return w.layered_problem(freq=freq, r=1.4, parts=parts, overlap=overlap, n_sources=(2, 2),
                             max_cubes=grid, with_q=with_q)


CASES = {
    "cube3": lambda: w.unit_cube_problem(3, freq=1.5, parts=(2, 2, 1), overlap=1),
    "cube6": lambda: w.unit_cube_problem(6, freq=2.0, parts=(2, 2, 2), overlap=1),
    "layered": lambda: _small_layered(),
    "layered_q": lambda: _small_layered(with_q=True, overlap=2),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, ctx):
    p = CASES[request.param]()
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    gm = ctx.mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq, p.quality)
    gop = ctx.assemble(gm, p.velocity, p.freq, p.quality)
    return request.param, p, om, gm, A, gop


def test_dofmap_bit_exact(case, ctx):
    name, p, om, gm, A, gop = case
    assert gm.n == om.n
    np.testing.assert_array_equal(ctx.dofmap(gm), om.tet_dofs)


def test_csr_pattern_bit_exact_values_close(case, ctx):
    name, p, om, gm, A, gop = case
    rp, ci, va = ctx.csr(gop)
    np.testing.assert_array_equal(rp, A.indptr)
    np.testing.assert_array_equal(ci, A.indices)
    err = np.abs(va - A.data).max() / np.abs(A.data).max()
    assert err <= 1e-13, err
    # the GPU operator is exactly symmetric (mirrored packed element entries)
    import scipy.sparse as sp

    G = sp.csr_matrix((va, ci, rp), shape=A.shape)
    assert abs(G - G.T).max() == 0


# both kernels, partial column groups, odd and even widths, blocks split into 32-column chunks
SPMM_WIDTHS = (1, 3, 8, 12, 16, 17, 31, 32, 40, 57, 64, 70)


def test_spmm_matches(case, ctx):
    name, p, om, gm, A, gop = case
    rng = np.random.default_rng(7)
    for s in SPMM_WIDTHS:
        X = rng.standard_normal((s, om.n)) + 1j * rng.standard_normal((s, om.n))
        Y = ctx.spmm(gop, X)
        assert _rel(Y, (A @ X.T).T) <= 1e-13, s


def test_spmm_complex64_input(case, ctx):
    """The product the mixed-precision solve applies to its complex64 vectors: the exact
    widening of x times the FP64 operator, to FP64 rounding (the oracle multiplies the same
    widened values), from host and from device blocks."""
    import torch

    name, p, om, gm, A, gop = case
    rng = np.random.default_rng(17)
    for s in SPMM_WIDTHS:
        X = (rng.standard_normal((s, om.n)) + 1j * rng.standard_normal((s, om.n))).astype(np.complex64)
        ref = (A @ X.astype(np.complex128).T).T
        assert _rel(ctx.spmm_c64x(gop, X), ref) <= 1e-13, s
        Yd = ctx.spmm_c64x(gop, torch.from_numpy(X).cuda())
        assert _rel(Yd.cpu().numpy(), ref) <= 1e-13, s


def test_spmm_device_tensors_and_repeatable(case, ctx):
    import torch

    name, p, om, gm, A, gop = case
    rng = np.random.default_rng(8)
    X = rng.standard_normal((5, om.n)) + 1j * rng.standard_normal((5, om.n))
    Xd = torch.from_numpy(X).cuda()
    Y1 = ctx.spmm(gop, Xd)
    Y2 = ctx.spmm(gop, Xd)
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)
    assert _rel(Y1.cpu().numpy(), (A @ X.T).T) <= 1e-13


def test_point_sources(case, ctx):
    name, p, om, gm, A, gop = case
    lo, hi = p.coords.min(0), p.coords.max(0)
    rng = np.random.default_rng(3)
    xyz = lo + (hi - lo) * rng.uniform(0.05, 0.95, (4, 3))
    if p.sources is not None:
        xyz = np.concatenate([xyz, p.sources])
    F = ctx.point_sources(gm, xyz)
    Fo = rhs.point_sources(om, xyz)
    assert np.abs(F - Fo).max() <= 1e-12


@pytest.fixture(scope="module")
def ddm_case(case, ctx):
    name, p, om, gm, A, gop = case
    d = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap)
    subs, own = odd.build_subdomains(om, p.velocity, p.freq, p.quality, p.partition, p.n_sub, p.overlap)
    return d, subs


def test_subdomains_bit_exact(case, ddm_case, ctx):
    name, p, om, gm, A, gop = case
    d, subs = ddm_case
    for i, s in enumerate(subs):
        g, own, rp, ci, va = ctx.subdomain(d, i)
        np.testing.assert_array_equal(g, s.gdofs)
        np.testing.assert_array_equal(own, s.owned)
        np.testing.assert_array_equal(rp, s.A.indptr)
        np.testing.assert_array_equal(ci, s.A.indices)
        assert np.abs(va - s.A.data).max() <= 1e-13 * np.abs(s.A.data).max()


def test_precond_one_level_c128(case, ddm_case, ctx):
    name, p, om, gm, A, gop = case
    d, subs = ddm_case
    odd.factor_subdomains(subs)
    P = odd.ORAS(A, subs)
    rng = np.random.default_rng(11)
    # 1 and 4 columns: vector-unit sweeps; 8..32: FP64 matrix-core sweeps (partial column
    # groups at 8, 21; the first apply of each group width also times both tile sizes)
    for s in (1, 4, 8, 16, 21, 32):
        V = rng.standard_normal((s, om.n)) + 1j * rng.standard_normal((s, om.n))
        Z = ctx.precond(d, V)
        Zo = P.apply(V.T).T
        assert _rel(Z, Zo) <= 1e-10, (s, _rel(Z, Zo))
    st = ctx.ddm_stats(d)
    assert st["static_pivots"] == 0


def test_ddm_levels_consistent(case, ddm_case, ctx):
    """Per-level elimination statistics add up to the whole-ddm ones, and every local dof of
    the oracle's subdomains is a pivot exactly once."""
    name, p, om, gm, A, gop = case
    d, subs = ddm_case
    st = ctx.ddm_stats(d)
    lv = ctx.ddm_levels(d)
    assert len(lv) == st["n_levels"]
    assert sum(x["n_fronts"] for x in lv) == st["n_fronts"]
    assert sum(x["sum_pivots"] for x in lv) == st["local_dofs_total"] == sum(len(s.gdofs) for s in subs)
    assert sum(x["factor_useful"] for x in lv) == st["factor_useful"]
    assert max(x["max_front"] for x in lv) == st["max_front"]
    assert all(x["max_pivots"] <= x["max_front"] and x["sum_pivots"] <= x["sum_front"] for x in lv)


def test_precond_one_level_mixed(case, ddm_case, ctx):
    """complex64 factors and sweeps (vector kernels below 8 columns, matrix-core kernels from
    8 on, 16-column groups with a ragged last group, wider blocks in 32-column chunks): each
    column within 1e-4 of the FP64 oracle's ORAS application, and a column's result
    independent of the block it sits in (to single-precision rounding)."""
    from paper_2004_07930_amd import hz

    name, p, om, gm, A, gop = case
    d, subs = ddm_case
    if subs[0].lu is None:
        odd.factor_subdomains(subs)
    P = odd.ORAS(A, subs)
    d32 = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap, precision=hz.HZ_PREC_MIXED)
    rng = np.random.default_rng(13)
    V = rng.standard_normal((64, om.n)) + 1j * rng.standard_normal((64, om.n))
    Zo = P.apply(V.T).T
    Z1 = ctx.precond(d32, V[:1])
    for s in (1, 3, 8, 16, 21, 32, 45, 64):
        Z = ctx.precond(d32, V[:s])
        errs = [_rel(Z[c], Zo[c]) for c in range(s)]
        print(f"{name} s={s}: max column error vs FP64 oracle {max(errs):.2e}")
        assert max(errs) <= 1e-4, (s, max(errs))
        assert _rel(Z[0], Z1[0]) <= 1e-5, (s, _rel(Z[0], Z1[0]))
    # the second chunk of a 64-column block against the same columns applied alone
    Zh = ctx.precond(d32, V[32:])
    assert max(_rel(Z[32 + c], Zh[c]) for c in range(32)) <= 1e-5
    ctx.release(d32)


def test_fgmres_fixed_iterations_c128(case, ddm_case, ctx):
    """Same algorithm, same iteration count: the iterate is unique, FP64 parity 1e-10."""
    name, p, om, gm, A, gop = case
    d, subs = ddm_case
    if subs[0].lu is None:
        odd.factor_subdomains(subs)
    P = odd.ORAS(A, subs)
    rng = np.random.default_rng(12)
    # 3 columns: vector-unit Gram-Schmidt kernels; 16 and 32: FP64 matrix-core kernels
    for s, ks in ((3, (1, 4)), (16, (3,)), (32, (2,))):
        B = rng.standard_normal((s, om.n)) + 1j * rng.standard_normal((s, om.n))
        for k in ks:
            X, info = ctx.solve(d, B, fixed_iters=k, restart=k)
            Xo, io = krylov.block_fgmres(lambda x: A @ x, B.T, P.apply, fixed_iters=k, m=k)
            assert info[0]["iters"] == k
            assert _rel(X, Xo.T) <= 1e-10, (s, k, _rel(X, Xo.T))
            np.testing.assert_allclose([i["rel_residual"] for i in info], io["rel_residual"], rtol=1e-8)


def test_fgmres_fixed_iterations_wide_block(ctx):
    """12 steps of a 32-column block (a least-squares problem of 384 x 384 blocks of 32, over
    the 10240 entries of the small register layout of the back substitution) on a problem that
    is still far from converged after them (cube 6 at 8 Hz, no overlap, so no column becomes
    dependent): FP64 parity 1e-10 and equal residual estimates."""
    p = w.unit_cube_problem(6, freq=8.0, parts=(2, 2, 2), overlap=0)
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq, p.quality)
    gm = ctx.mesh(p.tets, p.coords, p.face_bc)
    gop = ctx.assemble(gm, p.velocity, p.freq, p.quality)
    d = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap)
    subs, own = odd.build_subdomains(om, p.velocity, p.freq, p.quality, p.partition, p.n_sub, p.overlap)
    odd.factor_subdomains(subs)
    P = odd.ORAS(A, subs)
    rng = np.random.default_rng(21)
    B = rng.standard_normal((32, om.n)) + 1j * rng.standard_normal((32, om.n))
    X, info = ctx.solve(d, B, fixed_iters=12, restart=12)
    Xo, io = krylov.block_fgmres(lambda x: A @ x, B.T, P.apply, fixed_iters=12, m=12)
    assert min(io["rel_residual"]) > 1e-3  # not converged: every Arnoldi block has full rank
    assert _rel(X, Xo.T) <= 1e-10, _rel(X, Xo.T)
    np.testing.assert_allclose([i["rel_residual"] for i in info], io["rel_residual"], rtol=1e-8)
    ctx.release(d)


def test_fgmres_long_restart_wide_block(ctx):
    """A 32-column block at restart 48, run for 42 steps: the least-squares problem (43 x 42
    blocks of 32, 43,008 entries of Y) is past the 40,960 entries a register-resident back
    substitution could hold, and the restart length is used as asked (no shortening): FP64
    parity 1e-10 with the oracle at the same step count, reported m and block width (the block
    reaches residuals near 1e-10 by then)."""
    p = w.unit_cube_problem(6, freq=8.0, parts=(2, 2, 2), overlap=0)
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq, p.quality)
    gm = ctx.mesh(p.tets, p.coords, p.face_bc)
    gop = ctx.assemble(gm, p.velocity, p.freq, p.quality)
    d = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap)
    subs, own = odd.build_subdomains(om, p.velocity, p.freq, p.quality, p.partition, p.n_sub, p.overlap)
    odd.factor_subdomains(subs)
    P = odd.ORAS(A, subs)
    B = w.seeded_rhs_block(om.n, 32, 22)
    X, info = ctx.solve(d, B, fixed_iters=42, restart=48, block=32)
    assert all(i["restart_len"] == 48 and i["block"] == 32 and i["iters"] == 42 for i in info)
    Xo, io = krylov.block_fgmres(lambda x: A @ x, B.T, P.apply, fixed_iters=42, m=48)
    assert _rel(X, Xo.T) <= 1e-10, _rel(X, Xo.T)
    # residuals near 1e-10 after 42 steps: equal to rounding (absolute floor 1e-14)
    np.testing.assert_allclose([i["rel_residual"] for i in info], io["rel_residual"], rtol=1e-3, atol=1e-14)
    ctx.release(d)


def test_solve_to_tolerance_matches_direct(ctx):
    """cube 4, 8 subdomains: ORAS-FGMRES to 1e-12 equals the dense direct solve to 1e-9."""
    p = w.unit_cube_problem(4, freq=1.0, parts=(2, 2, 2), overlap=1)
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq)
    gm = ctx.mesh(p.tets, p.coords, p.face_bc)
    gop = ctx.assemble(gm, p.velocity, p.freq)
    d = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap)
    rng = np.random.default_rng(2)
    B = rng.standard_normal((5, om.n)) + 1j * rng.standard_normal((5, om.n))
    X, info = ctx.solve(d, B, tol=1e-12, max_iter=300)
    Xd = krylov.dense_solve(A, B.T).T
    assert all(i["rel_residual"] <= 1e-12 for i in info)
    assert _rel(X, Xd) <= 1e-9


def test_delayed_reorthogonalisation_restarts_and_convergence(ctx):
    """16- and 32-column blocks take the delayed-reorthogonalisation path, whose Hessenberg
    columns complete one step late: restarted cycles (restart 3) that end on the tolerance must
    stop after the same number of steps as the CGS2 oracle, with the same restarts and the same
    iterate; and a block iterated on past convergence (its Krylov blocks become dependent)
    must end its cycle with a finite, converged result (32 columns: test_solve_failure_paths)."""
    p = w.unit_cube_problem(4, freq=1.0, parts=(2, 2, 2), overlap=1)
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq)
    gm = ctx.mesh(p.tets, p.coords, p.face_bc)
    gop = ctx.assemble(gm, p.velocity, p.freq)
    d = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap)
    subs, own = odd.build_subdomains(om, p.velocity, p.freq, None, p.partition, p.n_sub, p.overlap)
    odd.factor_subdomains(subs)
    P = odd.ORAS(A, subs)
    rng = np.random.default_rng(33)
    for s, m, tol in ((16, 3, 1e-9), (16, 40, 1e-10), (32, 3, 1e-9)):
        B = rng.standard_normal((s, om.n)) + 1j * rng.standard_normal((s, om.n))
        X, info = ctx.solve(d, B, tol=tol, max_iter=200, restart=m)
        Xo, io = krylov.block_fgmres(lambda x: A @ x, B.T, P.apply, tol=tol, m=m, max_iter=200)
        print(f"{s} columns, restart {m}: GPU {info[0]['iters']} steps, {info[0]['restarts']} restarts; "
              f"oracle {io['iters']}, {io['restarts']}; iterate difference {_rel(X, Xo.T):.2e}")
        assert info[0]["iters"] == io["iters"] and info[0]["restarts"] == io["restarts"]
        assert all(i["rel_residual"] <= tol for i in info)
        assert _rel(X, Xo.T) <= 1e-8, _rel(X, Xo.T)
    # past convergence: cube 3 at 1.5 Hz converges to rounding in a few steps of 16 columns
    p = w.unit_cube_problem(3, freq=1.5, parts=(2, 2, 1), overlap=1)
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq)
    gm = ctx.mesh(p.tets, p.coords, p.face_bc)
    gop = ctx.assemble(gm, p.velocity, p.freq)
    d2 = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap)
    B16 = rng.standard_normal((16, om.n)) + 1j * rng.standard_normal((16, om.n))
    X, info = ctx.solve(d2, B16, fixed_iters=12, restart=12)
    assert np.isfinite(X).all()
    res = np.linalg.norm(B16.T - A @ X.T, axis=0) / np.linalg.norm(B16, axis=1)
    assert res.max() <= 1e-8 and info[0]["iters"] <= 12, (res.max(), info[0]["iters"])
    np.testing.assert_allclose(res, [i["rel_residual"] for i in info], rtol=1e-3, atol=1e-13)
    ctx.release(d)
    ctx.release(d2)


def test_delayed_reorthogonalisation_past_convergence_seeds(ctx):
    """Blocks iterated far past convergence make the once-projected block rounding noise,
    whose Gram matrix has many dependent directions: over several right-hand sides, 16 and
    32 columns and both precisions, every solve ends finite, converged, and with the reported
    residual equal to the true one."""
    from paper_2004_07930_amd import hz

    p = w.unit_cube_problem(3, freq=1.5, parts=(2, 2, 1), overlap=1)
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq)
    gm = ctx.mesh(p.tets, p.coords, p.face_bc)
    gop = ctx.assemble(gm, p.velocity, p.freq)
    for prec, tol in ((hz.HZ_PREC_C128, 1e-8), (hz.HZ_PREC_MIXED, 1e-5)):
        d = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap, precision=prec)
        for seed in (1, 2, 3, 4):
            rng = np.random.default_rng(seed)
            for s in (16, 32):
                B = rng.standard_normal((s, om.n)) + 1j * rng.standard_normal((s, om.n))
                X, info = ctx.solve(d, B, fixed_iters=12, restart=12)
                assert np.isfinite(X).all(), (prec, seed, s)
                res = np.linalg.norm(B.T - A @ X.T, axis=0) / np.linalg.norm(B, axis=1)
                assert res.max() <= tol, (prec, seed, s, res.max())
                np.testing.assert_allclose(res, [i["rel_residual"] for i in info], rtol=1e-3, atol=1e-13)
        ctx.release(d)


def test_config1_plane_wave(ctx):
    """Unit cube 8^3 (15,625 dofs), k = 8 pi, impedance everywhere, 8 subdomains, overlap 1,
    one-level ORAS, c128, tol 1e-8: same iteration count as the oracle and the iterate at
    that count within 1e-10 of the oracle's."""
    p = w.unit_cube_problem(8)
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq)
    b = rhs.plane_wave_load(om, p.velocity, p.freq, p.extra["direction"])
    P = odd.build_preconditioner(om, A, p.velocity, p.freq, None, p.partition, p.n_sub, p.overlap)
    Xo, io = krylov.block_fgmres(lambda x: A @ x, b, P.apply, tol=p.tol, m=40)
    gm = ctx.mesh(p.tets, p.coords, p.face_bc)
    gop = ctx.assemble(gm, p.velocity, p.freq)
    d = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap)
    X, info = ctx.solve(d, b[None], tol=p.tol, max_iter=200)
    assert info[0]["rel_residual"] <= p.tol
    assert abs(info[0]["iters"] - io["iters"]) <= 1
    Xk, _ = ctx.solve(d, b[None], fixed_iters=io["iters"], restart=io["iters"])
    assert _rel(Xk[0], Xo[:, 0]) <= 1e-10
    # discretisation error against the exact plane wave stays that of the oracle's solution
    xyz = fem.dof_coordinates(om.tets, om.coords, om.tet_dofs, om.n)
    ui = rhs.plane_wave_nodal(om, p.velocity, p.freq, p.extra["direction"], xyz)
    assert abs(_rel(X[0], ui) - _rel(Xo[:, 0], ui)) <= 1e-6


def test_coarse_space_and_two_level(ctx):
    p = _small_layered(freq=0.4, grid=(8, 8, 4), parts=(2, 2, 1), overlap=1)
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq)
    gm = ctx.mesh(p.tets, p.coords, p.face_bc)
    gop = ctx.assemble(gm, p.velocity, p.freq)
    d = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap, coarse=(p.coarse_tets, p.coarse_coords))
    Z = odd.coarse_interpolation(om, p.coarse_tets, p.coarse_coords)
    nc, rp, ci, va = ctx.coarse(d)
    assert nc == Z.shape[1]
    np.testing.assert_array_equal(rp, Z.indptr)
    np.testing.assert_array_equal(ci, Z.indices)
    assert np.abs(va - Z.data).max() <= 1e-14
    P = odd.build_preconditioner(om, A, p.velocity, p.freq, None, p.partition, p.n_sub, p.overlap,
                                 p.coarse_tets, p.coarse_coords)
    rng = np.random.default_rng(5)
    V = rng.standard_normal((32, om.n)) + 1j * rng.standard_normal((32, om.n))
    Zo = P.apply(V.T).T
    # blocks of 1..32 columns: the prolongation takes a fine row's columns 16 at a time (one
    # ragged chunk, one full chunk, two chunks)
    for s in (1, 3, 16, 17, 32):
        assert _rel(ctx.precond(d, V[:s]), Zo[:s]) <= 1e-10, s
    from paper_2004_07930_amd import hz

    d32 = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap, coarse=(p.coarse_tets, p.coarse_coords),
                        precision=hz.HZ_PREC_MIXED)
    for s in (1, 3, 16, 17, 32):
        Z = ctx.precond(d32, V[:s])
        assert max(_rel(Z[c], Zo[c]) for c in range(s)) <= 1e-4, s
    ctx.release(d32)
    F = ctx.point_sources(gm, p.sources)
    X, info = ctx.solve(d, F, fixed_iters=5, restart=5)
    Xo, io = krylov.block_fgmres(lambda x: A @ x, F.T, P.apply, fixed_iters=5, m=5)
    assert _rel(X, Xo.T) <= 1e-10


def test_mixed_precision_reaches_tolerance(ctx):
    """complex64 factors / ORAS / coarse inside FP64 FGMRES reach the 1e-6 residual; the
    iteration count is within one of the FP64 solve's and the solution error against the
    FP64 oracle is reported (and bounded by the conditioning estimate)."""
    p = _small_layered(freq=0.4, grid=(8, 8, 4), parts=(2, 2, 1), overlap=1)
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq)
    gm = ctx.mesh(p.tets, p.coords, p.face_bc)
    gop = ctx.assemble(gm, p.velocity, p.freq)
    co = (p.coarse_tets, p.coarse_coords)
    from paper_2004_07930_amd import hz

    d64 = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap, coarse=co, precision=hz.HZ_PREC_C128)
    d32 = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap, coarse=co, precision=hz.HZ_PREC_MIXED)
    F = ctx.point_sources(gm, p.sources)
    X64, i64 = ctx.solve(d64, F, tol=1e-6)
    X32, i32 = ctx.solve(d32, F, tol=1e-6)
    assert all(i["rel_residual"] <= 1e-6 for i in i32)
    assert abs(i32[0]["iters"] - i64[0]["iters"]) <= 1
    Xo = krylov.dense_solve(A, F.T).T
    err = _rel(X32, Xo)
    # the FP64 oracle's own FGMRES at the same 1e-6 residual
    P = odd.build_preconditioner(om, A, p.velocity, p.freq, None, p.partition, p.n_sub, p.overlap,
                                 p.coarse_tets, p.coarse_coords)
    Xf, io = krylov.block_fgmres(lambda x: A @ x, F.T, P.apply, tol=1e-6, m=40)
    err_f = _rel(X32, Xf.T)
    print(f"mixed vs exact: {err:.3e}; fp64 vs exact: {_rel(X64, Xo):.3e}; mixed vs FP64 oracle FGMRES "
          f"at 1e-6: {err_f:.3e}; FP64 GPU vs FP64 oracle FGMRES: {_rel(X64, Xf.T):.3e}")
    assert err <= 1e-4
    assert err_f <= 1e-5  # mixed vs FP64 at the same 1e-6 residual


def test_solve_failure_paths(ctx):
    """Non-finite right-hand side -> HZ_ERR_ARG; max_iter reached -> HZ_ERR_NOT_CONVERGED with
    the best iterate and its residual returned (the residual is that of the returned x); a
    block with dependent columns -> HZ_ERR_ARG; a block that becomes dependent while iterating
    (every column converged to rounding) ends its cycle instead of breaking down."""
    from paper_2004_07930_amd import hz

    p = w.unit_cube_problem(3, freq=1.5, parts=(2, 2, 1), overlap=1)
    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    A = fem.assemble_operator(om, p.velocity, p.freq)
    gm = ctx.mesh(p.tets, p.coords, p.face_bc)
    gop = ctx.assemble(gm, p.velocity, p.freq)
    d = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap)
    rng = np.random.default_rng(21)
    B = rng.standard_normal((2, om.n)) + 1j * rng.standard_normal((2, om.n))  # full column rank
    keep = B[1, 5]
    B[1, 5] = np.nan
    with pytest.raises(hz.HzError) as e:
        ctx.solve(d, B)
    assert e.value.code == hz.HZ_ERR_ARG
    B[1, 5] = keep
    with pytest.raises(hz.HzError) as e:
        ctx.solve(d, B, tol=1e-14, max_iter=1)
    assert e.value.code == hz.HZ_ERR_NOT_CONVERGED
    X, info = ctx.solve(d, B, tol=1e-14, max_iter=1, raise_on_not_converged=False)
    assert all(i["status"] == hz.HZ_ERR_NOT_CONVERGED and i["iters"] == 1 for i in info)
    res = np.linalg.norm(B.T - A @ X.T, axis=0) / np.linalg.norm(B, axis=1)
    np.testing.assert_allclose(res, [i["rel_residual"] for i in info], rtol=1e-8)
    assert res.max() < 1.0  # one preconditioned step already reduces the residual
    # dependent columns (block CholQR breakdown at the start) -> HZ_ERR_ARG, nothing solved
    with pytest.raises(hz.HzError) as e:
        ctx.solve(d, np.stack([B[0], B[1], 2j * B[0]]))
    assert e.value.code == hz.HZ_ERR_ARG and "rank deficient" in str(e.value)
    # iterating on past convergence: the Krylov block becomes dependent, the cycle ends at
    # that step and the solution is returned converged and finite (no breakdown NaN)
    B32 = rng.standard_normal((32, om.n)) + 1j * rng.standard_normal((32, om.n))
    X, info = ctx.solve(d, B32, fixed_iters=12, restart=12)
    assert np.isfinite(X).all()
    res = np.linalg.norm(B32.T - A @ X.T, axis=0) / np.linalg.norm(B32, axis=1)
    assert res.max() <= 1e-8 and info[0]["iters"] <= 12, (res.max(), info[0]["iters"])
    np.testing.assert_allclose(res, [i["rel_residual"] for i in info], rtol=1e-3, atol=1e-13)
    ctx.release(d)


@pytest.mark.parametrize("prec", ["mixed", "c128"])
def test_sweep_tile_tuning(case, ctx, prec):
    """The first matrix-core apply times both tile sizes on every level and keeps the faster;
    tile sizes do not change results, so the tuning apply (which ends on the larger tiles) and
    the tuned apply agree bit for bit (complex64 and complex128 sweeps)."""
    from paper_2004_07930_amd import hz

    name, p, om, gm, A, gop = case
    pr = hz.HZ_PREC_MIXED if prec == "mixed" else hz.HZ_PREC_C128
    dd = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap, precision=pr)
    assert all(l["fwd_tile_rows"] == 0 and l["bwd_tile_cols"] == 0 for l in ctx.ddm_levels(dd))
    rng = np.random.default_rng(17)
    V = rng.standard_normal((16, om.n)) + 1j * rng.standard_normal((16, om.n))
    Z1 = ctx.precond(dd, V)
    lv = ctx.ddm_levels(dd)
    print(name, prec, "tiles", [(l["fwd_tile_rows"], l["bwd_tile_cols"]) for l in lv])
    assert all(l["fwd_tile_rows"] in (64, 128) and l["bwd_tile_cols"] in (64, 128) for l in lv)
    Z2 = ctx.precond(dd, V)
    assert np.array_equal(Z1, Z2)
    ctx.release(dd)
