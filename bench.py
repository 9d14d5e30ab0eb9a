"""Benchmark: sources solved per second at a 1e-6 relative residual, mixed vs FP64.

Workload (default): the layered synthetic stand-in for the Overthrust box of the paper --
20 x 20 x 4.65 km, v(z) = 2200 + 3800 z / 4.65 m/s with 12 seeded Gaussian anomalies and
3 dipping step layers, 2.5 Hz, graded Kuhn tets (72 x 72 x 12 cubes, 1,742,293 P3 dofs),
free surface on top and absorbing elsewhere, 64 subdomains (8 x 8 columns) with overlap 2,
P1 coarse space on a 4x coarser grid, 16 point sources on a 4 x 4 grid at 500 m depth.

A step is one hz_solve of the 16-source block to 1e-6 with the operator and factors
resident in HBM (set-up is timed separately).  The headline value uses the mixed
precision preconditioner (complex64 factors, ORAS and coarse solve inside FP64 FGMRES);
the FP64 solve is timed the same way and reported beside it.

The roofline object is computed live: the library brackets every launch of its main
kernel classes with HIP events on the solve stream during the timed steps and sums each
launch's algorithmic bytes (hz_profile_*); the class with the largest time is reported.

The CPU baseline times the oracle (NumPy / SciPy, one thread) on a bounded sample of the
same workload -- one overlapped subdomain -- and scales it to sources per second.

Prints ONE JSON line.  More than one GPU is not supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sources solved/s at 1e-6 rel. residual, mixed vs FP64; p50/p99 solve latency"
HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s


def build_workload(name):
    import workloads as w

    if name == "layered-2.5hz":
        p = w.layered_problem(freq=2.5, r=1.4, parts=(8, 8, 1), overlap=2, n_sources=(4, 4), src_depth=0.5)
        desc = ("layered 20x20x4.65 km, 2.5 Hz, Kuhn P3 %dx%dx%d cubes, 64 subdomains, overlap 2, "
                "P1 coarse (4x coarser), 16 point sources at 0.5 km, tol 1e-6" % p.grid)
        return p, desc
    if name == "cube8":
        p = w.unit_cube_problem(8)
        return p, "unit cube 8^3 x 6 tets, k = 8 pi, impedance, 8 subdomains, overlap 1, tol 1e-8"
    if name == "layered-1hz":
        p = w.layered_problem(freq=1.0, r=1.4, parts=(4, 4, 1), overlap=2, n_sources=(4, 4), src_depth=0.5)
        return p, "layered 20x20x4.65 km, 1 Hz, %dx%dx%d cubes, 16 subdomains, overlap 2, P1 coarse" % p.grid
    raise SystemExit(f"unknown workload {name}")


def counter_traffic(kernel_class, workload):
    """HBM bytes per launch of a kernel class from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (profiles/traffic_<workload>.json), or None when there is no record or
    the kernel's source file has changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel_class)
    if rec is None:
        return None
    src = os.path.join(ROOT, rec["source"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"] / 1e9  # GB per launch, same unit basis as "achieved"


def cpu_baseline(p, n_global, iters, s):
    """Oracle on one overlapped subdomain of the workload, scaled to sources/s.

    The sample is the corner column of the partition with its overlap (the tets of
    11 x 11 cubes over the full depth) as a standalone mesh: assembly, SuperLU factor,
    one s-RHS local solve, one local SpMM and one CGS pass against 20 s-blocks.  A full
    oracle iteration is then n_sub local solves plus (n / n_i) times the local SpMM and
    four CGS passes; a source block needs `iters` iterations (the GPU's count for the
    same algorithm)."""
    import scipy.sparse.linalg as spla
    from threadpoolctl import threadpool_limits

    import workloads as w
    from oracle import fem

    nx, ny, nz = p.grid
    ex = p.overlap + (nx // int(round(np.sqrt(p.n_sub))))
    cubes = np.arange(p.tets.shape[0]) // 6
    ci, cj = cubes % nx, (cubes // nx) % ny
    sel = np.nonzero((ci < ex) & (cj < ex))[0]
    used, inv = np.unique(p.tets[sel].ravel(), return_inverse=True)
    lt = inv.reshape(-1, 4).astype(np.int32)
    lc = p.coords[used]
    t0 = time.perf_counter()
    with threadpool_limits(1):
        m = fem.Mesh(lt, lc, w.face_bc_tags(lt, lc, dirichlet_top=True))
        A = fem.assemble_operator(m, p.velocity[sel], p.freq, None if p.quality is None else p.quality[sel])
        t1 = time.perf_counter()
        lu = spla.splu(A.tocsc(), permc_spec="MMD_AT_PLUS_A")
        t2 = time.perf_counter()
        rng = np.random.default_rng(0)
        B = rng.standard_normal((m.n, s)) + 1j * rng.standard_normal((m.n, s))
        lu.solve(B)
        t3 = time.perf_counter()
        A @ B
        t4 = time.perf_counter()
        V = rng.standard_normal((m.n, 20 * s)) + 0j
        H = V.conj().T @ B
        B - V @ H
        t5 = time.perf_counter()
    scale = n_global / m.n
    t_iter = p.n_sub * (t3 - t2) + scale * ((t4 - t3) + 4 * (t5 - t4))
    return {
        "value": s / (iters * t_iter),
        "unit": "sources/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"one overlapped subdomain ({m.n} dofs, {len(sel)} tets) of the same workload: SuperLU factor "
                   f"{t2 - t1:.1f} s, {s}-RHS local solve {t3 - t2:.2f} s, SpMM {t4 - t3:.3f} s, CGS pass "
                   f"{t5 - t4:.2f} s; extrapolated to {p.n_sub} subdomains x {iters} iterations "
                   f"({t_iter:.1f} s per iteration); sample wall {time.perf_counter() - t0:.1f} s"),
        "extrapolated": True,
        "setup_s_extrapolated": p.n_sub * (t2 - t1),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="layered-2.5hz",
                    choices=["layered-2.5hz", "cube8", "layered-1hz"])
    ap.add_argument("--restart", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device copy (reference for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no collectives); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2004_07930_amd import hz

    def log(*a):
        if args.verbose:
            print(*a, file=sys.stderr, flush=True)

    if args.copy_calibration:  # 1 GiB read + 1 GiB written by one copy kernel
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    p, desc = build_workload(args.workload)
    stream = torch.cuda.current_stream()
    ctx = hz.Context(0, stream=stream)
    t0 = time.perf_counter()
    mesh = ctx.mesh(p.tets, p.coords, p.face_bc)
    op = ctx.assemble(mesh, p.velocity, p.freq, p.quality)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    log(f"mesh+assembly {t_asm:.2f}s n={mesh.n}")
    coarse = (p.coarse_tets, p.coarse_coords) if p.coarse_tets is not None else None
    if p.sources is not None:
        B = ctx.point_sources(mesh, p.sources,
                              out=torch.empty((len(p.sources), mesh.n), dtype=torch.complex128, device="cuda"))
    else:
        from oracle import fem, rhs  # manufactured load of the unit-cube case (test input only)

        om = fem.Mesh(p.tets, p.coords, p.face_bc)
        B = torch.from_numpy(rhs.plane_wave_load(om, p.velocity, p.freq, p.extra["direction"])[None]).cuda()
    s = B.shape[0]
    X = torch.empty_like(B)
    results = {}
    precisions = [("mixed", hz.HZ_PREC_MIXED)] + ([] if args.no_fp64 else [("fp64", hz.HZ_PREC_C128)])
    for label, prec in precisions:
        t0 = time.perf_counter()
        d = ctx.setup_ddm(op, p.partition, p.n_sub, p.overlap, coarse=coarse, precision=prec)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        st = ctx.ddm_stats(d)
        log(f"{label}: setup {t_setup:.2f}s {st}")
        kw = dict(tol=p.tol, max_iter=500, restart=args.restart, block=args.block, out=X)
        for _ in range(args.warmup):
            ctx.solve(d, B, **kw)
        torch.cuda.synchronize()
        ctx.profile(True)
        lat = []
        infos = None
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            a = time.perf_counter()
            _, infos = ctx.solve(d, B, **kw)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - a)
        torch.cuda.synchronize()
        el = time.perf_counter() - t_start
        kstats = ctx.profile_stats()
        ctx.profile(False)
        results[label] = dict(
            sources_per_s=s * args.steps / el, ms_per_step=1e3 * el / args.steps,
            p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
            iters=infos[0]["iters"], max_rel_residual=max(i["rel_residual"] for i in infos),
            setup_s=t_setup, static_pivots=st["static_pivots"], factor_entries=st["factor_entries"],
            device_gb=st["device_bytes"] / 1e9, n_fronts=st["n_fronts"], levels=st["n_levels"],
            max_front=st["max_front"], local_dofs=st["local_dofs_total"],
            kernels={k: dict(launches=v["launches"], seconds=v["seconds"],
                             gbps=(v["bytes"] / v["seconds"] / 1e9) if v["seconds"] > 0 else None,
                             tflops=(v["flops"] / v["seconds"] / 1e12) if v["seconds"] > 0 else None)
                     for k, v in kstats.items()},
            _kraw=kstats)
        log(label, {k: v for k, v in results[label].items() if k != "_kraw"})
        ctx.release(d)
    head = results["mixed"]
    kraw = head.pop("_kraw")
    if "fp64" in results:
        results["fp64"].pop("_kraw")
    dom = max(kraw, key=lambda k: kraw[k]["seconds"])
    kd = kraw[dom]
    achieved = kd["bytes"] / kd["seconds"] if kd["seconds"] > 0 else 0.0
    roofline = {"kernel": dom, "bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK, "traffic": counter_traffic(dom, args.workload),
                "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE x fetch scale + WRITE_SIZE x write scale)",
                "launches": kd["launches"], "avg_launch_ms": 1e3 * kd["seconds"] / max(1, kd["launches"]),
                "algorithmic_bytes_per_launch": kd["bytes"] / max(1, kd["launches"])}
    cpu = None
    if not args.no_cpu_baseline and p.sources is not None:
        cpu = cpu_baseline(p, mesh.n, head["iters"], s)
    out = {
        "metric": METRIC,
        "value": head["sources_per_s"],
        "unit": "sources/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 preconditioner, f64 Krylov",
        "data": "synthetic",
        "config": {"workload": desc, "n_dofs": mesh.n, "nnz": int(ctx.csr(op, values=False)[1].size),
                   "n_sources": s, "n_sub": p.n_sub, "overlap": p.overlap, "tol": p.tol,
                   "assembly_s": t_asm},
        "latency": {"p50_s": head["p50_s"], "p99_s": head["p99_s"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "mixed": head,
        "fp64": results.get("fp64"),
        "mixed_over_fp64": (head["sources_per_s"] / results["fp64"]["sources_per_s"]) if "fp64" in results else None,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
