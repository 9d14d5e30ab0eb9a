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


SERVE_FREQS = (2.5, 3.5)


def serve_workloads():
    """Operators of the serving run: the layered model at 2.5 Hz (8 x 8 columns) and 3.5 Hz
    (8 x 8 x 2 boxes cut at equal depth), overlap 2, P1 coarse space, mixed precision."""
    import workloads as w

    out = []
    for f in SERVE_FREQS:
        parts = (8, 8, 1) if f <= 2.5 else (8, 8, 2)
        out.append(w.layered_problem(freq=f, r=1.4, parts=parts, overlap=2, n_sources=(4, 4), src_depth=0.5,
                                     equal_depth_zcuts=parts[2] > 1))
    return out


def serve_requests(n_req, seed=4):
    """Poisson arrivals (mean gap 0.25 s); operator uniform; n_src = round(exp(U[0, ln 128]));
    the sources are the first n_src of a seeded permutation of a 16 x 8 grid at 0.5 km depth
    (x = 0.625 + 1.25 i km, y = 1.25 + 2.5 j km)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grid = np.array([[0.625 + 1.25 * i, 1.25 + 2.5 * j, 0.5] for j in range(8) for i in range(16)])
    t, reqs = 0.0, []
    for _ in range(n_req):
        t += rng.exponential(0.25)
        op = int(rng.integers(0, len(SERVE_FREQS)))
        ns = int(round(np.exp(rng.uniform(0.0, np.log(128.0)))))
        perm = rng.permutation(len(grid))
        reqs.append((t, op, grid[perm[:ns]]))
    return reqs


def run_serve(args):
    """Continuous-batching run: every request is submitted at its arrival time to one serving
    context holding both operators; prints one JSON line with p50 / p99 latency (submission to
    completion) and sources per second."""
    import torch

    from paper_2004_07930_amd import hz

    reqs = serve_requests(args.serve)
    probs = serve_workloads()
    free0, _ = torch.cuda.mem_get_info()
    # caller-side tensors (right-hand sides and solutions of every request) are torch's,
    # outside the library's accounting: keep them out of the serving budget
    import workloads as w

    n = [w.kuhn_ndofs(*q.grid) for q in probs]
    caller = sum(2 * len(src) * n[op] * 16 for _, op, src in reqs)
    ctx = hz.Context(0, stream=torch.cuda.current_stream(), hbm_budget=int(0.8 * free0) - caller)
    ops, setup = [], {}
    for k, q in enumerate(probs):
        t0 = time.perf_counter()
        mesh = ctx.mesh(q.tets, q.coords, q.face_bc)
        op = ctx.assemble(mesh, q.velocity, q.freq, q.quality)
        d = ctx.setup_ddm(op, q.partition, q.n_sub, q.overlap, coarse=(q.coarse_tets, q.coarse_coords),
                          precision=hz.HZ_PREC_MIXED)
        torch.cuda.synchronize()
        setup[SERVE_FREQS[k]] = dict(n_dofs=mesh.n, n_sub=q.n_sub, seconds=time.perf_counter() - t0,
                                    ddm_gb=ctx.ddm_stats(d)["device_bytes"] / 1e9)
        ops.append((mesh, d))
        print(f"serve: {SERVE_FREQS[k]} Hz ready {setup[SERVE_FREQS[k]]}", file=sys.stderr, flush=True)
    rhs = [ctx.point_sources(ops[op][0], src, out=torch.empty((len(src), ops[op][0].n), dtype=torch.complex128,
                                                                device="cuda")) for _, op, src in reqs]
    torch.cuda.synchronize()
    ctx.serve_start(max_slots=8)
    tickets = []
    t_start = time.perf_counter()
    try:
        for (t_arr, op, src), b in zip(reqs, rhs):
            delay = t_start + t_arr - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets.append(ctx.submit(ops[op][1], b, tol=1e-6))
        done = []
        for k, tk in enumerate(tickets):
            done.append(ctx.wait(tk))
            print(f"serve: request {k} done ({len(reqs[k][2])} sources at {SERVE_FREQS[reqs[k][1]]} Hz)",
                  file=sys.stderr, flush=True)
        st = ctx.serve_stats()
    finally:
        ctx.serve_stop()
    wall = time.perf_counter() - t_start
    ok = all(status == 0 and all(i["rel_residual"] <= 1e-6 for i in info) for _, info, status in done)
    n_src = sum(len(r[2]) for r in reqs)
    print(json.dumps({
        "metric": "served sources/s at 1e-6 rel. residual with p50/p99 request latency", "value": st["sources_per_s"],
        "unit": "sources/s", "n_gpus": 1, "higher_is_better": True, "dtype": "c64 preconditioner, f64 Krylov",
        "data": "synthetic",
        "config": {"workload": "serving: layered model at 2.5 and 3.5 Hz resident, Poisson arrivals (mean gap "
                               "0.25 s, seed 4), n_src log-uniform in [1, 128], tol 1e-6, 8 slots",
                   "requests": len(reqs), "sources": n_src, "operators": setup},
        "latency": {"p50_s": st["p50_s"], "p99_s": st["p99_s"]}, "wall_s": wall,
        "completed": st["completed"], "rejected": st["rejected"], "all_converged": ok,
        "iters": [max(i["iters"] for i in info) for _, info, _ in done]}))


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
    ap.add_argument("--serve", type=int, default=0, metavar="N",
                    help="instead: serve N requests on the 2.5 and 3.5 Hz operators (continuous batching)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no collectives); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        run_serve(args)
        return

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
    src = p.sources if p.sources is not None else np.array([[0.37, 0.52, 0.61]])  # unit cube: one interior source
    B = ctx.point_sources(mesh, src, out=torch.empty((len(src), mesh.n), dtype=torch.complex128, device="cuda"))
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
