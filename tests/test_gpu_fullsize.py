"""Parity at the full size of the benchmark workload (layered 2.5 Hz: 1,742,293 dofs, 82.6M
nonzeros, 64 subdomains, overlap 2, P1 coarse space, 16 point sources), in the configuration
bench.py times (mixed precision, tol 1e-6).

The oracle handles this size for everything but the preconditioner: the dof map and the CSR
pattern must match bit for bit, the values and the point sources to 1e-13 / 1e-12, and the
explicit residual of every column of the GPU solution, recomputed with the oracle's operator,
must meet the tolerance and agree with the residual the library reports; the mixed-precision
solution is within 1e-5 of the FP64 solve at the same residual."""
import time

import numpy as np
import pytest

import workloads as w
from oracle import fem, rhs

pytestmark = pytest.mark.gpu


def _log(msg, t0):
    print(f"[fullsize] {msg} ({time.perf_counter() - t0:.1f} s)", flush=True)


def test_benchmark_workload_full_size():
    import torch
    from paper_2004_07930_amd import hz

    t0 = time.perf_counter()
    p = w.layered_problem(freq=2.5, r=1.4, parts=(8, 8, 1), overlap=2, n_sources=(4, 4), src_depth=0.5)
    ctx = hz.Context(0, stream=torch.cuda.current_stream())
    try:
        gm = ctx.mesh(p.tets, p.coords, p.face_bc)
        gop = ctx.assemble(gm, p.velocity, p.freq, p.quality)
        d = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap, coarse=(p.coarse_tets, p.coarse_coords),
                          precision=hz.HZ_PREC_MIXED)
        F = ctx.point_sources(gm, p.sources)
        X, info = ctx.solve(d, F, tol=1e-6, max_iter=500)
        ctx.release(d)
        d64 = ctx.setup_ddm(gop, p.partition, p.n_sub, p.overlap, coarse=(p.coarse_tets, p.coarse_coords),
                            precision=hz.HZ_PREC_C128)
        X64, info64 = ctx.solve(d64, F, tol=1e-6, max_iter=500)
        ctx.release(d64)
        rp, ci, va = ctx.csr(gop)
        tet_dofs = ctx.dofmap(gm)
        _log(f"GPU side done: n={gm.n}, {info[0]['iters']} iterations", t0)
    finally:
        ctx.close()

    om = fem.Mesh(p.tets, p.coords, p.face_bc)
    assert om.n == gm.n == 1742293
    np.testing.assert_array_equal(tet_dofs, om.tet_dofs)
    _log("dof map bit-exact", t0)
    Fo = rhs.point_sources(om, p.sources)
    assert np.abs(F - Fo).max() <= 1e-12
    _log("point sources match", t0)
    A = fem.assemble_operator(om, p.velocity, p.freq, p.quality)
    np.testing.assert_array_equal(rp, A.indptr)
    np.testing.assert_array_equal(ci, A.indices)
    assert np.abs(va - A.data).max() <= 1e-13 * np.abs(A.data).max()
    _log(f"CSR pattern bit-exact, values close ({A.nnz} nonzeros)", t0)
    R = Fo.T - A @ X.T
    res = np.linalg.norm(R, axis=0) / np.linalg.norm(Fo, axis=1)
    rep = np.array([i["rel_residual"] for i in info])
    _log(f"explicit residuals {res.min():.3e}..{res.max():.3e}; reported {rep.min():.3e}..{rep.max():.3e}", t0)
    assert res.max() <= 1e-6 * (1 + 1e-6)
    np.testing.assert_allclose(res, rep, rtol=1e-6, atol=1e-12)
    # the mixed-precision solution against the FP64 solve at the same 1e-6 residual
    err = np.linalg.norm(X - X64) / np.linalg.norm(X64)
    _log(f"mixed vs FP64 solution: {err:.3e} ({info[0]['iters']} vs {info64[0]['iters']} iterations)", t0)
    assert err <= 1e-5
