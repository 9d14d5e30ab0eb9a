"""ctypes binding of libhz (include/hz.h).

Argument marshalling only: every step of the solver runs in the library's HIP kernels.
Device buffers are torch tensors on the context's GPU (torch is used for memory and the
stream); host buffers are numpy arrays.  The binding raises if libhz.so is missing: there
is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhz.so")

HZ_OK, HZ_ERR_ARG, HZ_ERR_OOM, HZ_ERR_HIP, HZ_ERR_NOT_CONVERGED = 0, -1, -2, -3, -4
HZ_ERR_SINGULAR, HZ_ERR_BUSY, HZ_ERR_STATE, HZ_ERR_ABI = -5, -6, -7, -8
HZ_BC_NONE, HZ_BC_IMPEDANCE, HZ_BC_DIRICHLET = 0, 1, 2
HZ_PREC_C128, HZ_PREC_MIXED = 0, 1
HZ_MEM_HOST, HZ_MEM_DEVICE = 0, 1
HZ_POU_BOOLEAN, HZ_POU_SMOOTH = 0, 1
HZ_LOCAL_EXACT, HZ_LOCAL_ICC, HZ_LOCAL_ICC_A2 = 0, 1, 2

_STATUS = {0: "HZ_OK", -1: "HZ_ERR_ARG", -2: "HZ_ERR_OOM", -3: "HZ_ERR_HIP", -4: "HZ_ERR_NOT_CONVERGED",
           -5: "HZ_ERR_SINGULAR", -6: "HZ_ERR_BUSY", -7: "HZ_ERR_STATE", -8: "HZ_ERR_ABI"}

EXPORTS = [
    "hz_init", "hz_finalize", "hz_last_error", "hz_release", "hz_mesh", "hz_assemble", "hz_setup_ddm",
    "hz_setup_ddm_ex", "hz_get_pou",
    "hz_solve", "hz_solve_ex", "hz_point_sources", "hz_spmm", "hz_spmm_c64x", "hz_spmm_noalloc", "hz_precond", "hz_ddm_stats_get", "hz_ddm_levels",
    "hz_serve_start", "hz_serve_submit", "hz_serve_poll", "hz_serve_wait", "hz_serve_stats_get",
    "hz_serve_stop", "hz_get_dofmap", "hz_get_csr_size", "hz_get_csr", "hz_get_subdomain_size",
    "hz_get_subdomain", "hz_get_coarse_size", "hz_get_coarse", "hz_profile_enable", "hz_profile_get",
]

HZ_K_SPMM, HZ_K_ORAS_FWD, HZ_K_ORAS_BWD, HZ_K_CGS_GRAM, HZ_K_CGS_UPDATE = range(5)
KERNEL_CLASSES = {"spmm": 0, "oras_fwd": 1, "oras_bwd": 2, "cgs_gram": 3, "cgs_update": 4}


class HzError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class InitOpts(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("device", C.c_int), ("hbm_budget", C.c_size_t), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("alloc_user", C.c_void_p), ("stream", C.c_void_p)]


class CoarseMesh(C.Structure):
    _fields_ = [("n_tets", C.c_int64), ("tets", C.c_void_p), ("n_verts", C.c_int64), ("coords", C.c_void_p)]


class ColInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("rel_residual", C.c_double), ("status", C.c_int32),
                ("restart_len", C.c_int32), ("block", C.c_int32)]


def _info_dicts(arr):
    return [dict(iters=i.iters, restarts=i.restarts, rel_residual=i.rel_residual, status=i.status,
                 restart_len=i.restart_len, block=i.block) for i in arr]


class DdmOpts(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("precision", C.c_int), ("pou", C.c_int), ("local_solver", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("tol", C.c_double), ("max_iter", C.c_int32), ("restart", C.c_int32),
                ("fixed_iters", C.c_int32), ("block", C.c_int32)]


class DdmStats(C.Structure):
    _fields_ = [("n_dofs", C.c_int64), ("nnz", C.c_int64), ("n_sub", C.c_int64), ("local_dofs_total", C.c_int64),
                ("factor_entries", C.c_int64), ("n_fronts", C.c_int64), ("n_levels", C.c_int64),
                ("max_front", C.c_int64), ("n_coarse", C.c_int64), ("static_pivots", C.c_int64),
                ("update_entries", C.c_int64), ("factor_useful", C.c_int64),
                ("device_bytes", C.c_int64), ("setup_seconds", C.c_double), ("factor_seconds", C.c_double),
                ("factor_flops", C.c_double), ("local_solver", C.c_int64), ("icc_entries", C.c_int64),
                ("icc_levels", C.c_int64)]


class DdmLevel(C.Structure):
    _fields_ = [("n_fronts", C.c_int64), ("max_pivots", C.c_int64), ("max_front", C.c_int64),
                ("sum_pivots", C.c_int64), ("sum_front", C.c_int64), ("factor_useful", C.c_int64),
                ("fwd_tile_rows", C.c_int32), ("bwd_tile_cols", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("ddm", C.c_uint64), ("n_rhs", C.c_int64), ("rhs", C.c_void_p),
                ("x", C.c_void_p), ("mem", C.c_int), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("info", C.c_void_p)]


class KernelStat(C.Structure):
    _fields_ = [("launches", C.c_int64), ("seconds", C.c_double), ("bytes", C.c_double), ("flops", C.c_double)]


class ServeStats(C.Structure):
    _fields_ = [("p50_s", C.c_double), ("p99_s", C.c_double), ("sources_per_s", C.c_double),
                ("completed", C.c_int64), ("rejected", C.c_int64), ("parts_done", C.c_int64),
                ("steps", C.c_int64), ("active_parts", C.c_int64)]


_lib = None


def load(path: str | None = None):
    """Load libhz.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"libhz.so not found at {p}: build it with `python -m paper_2004_07930_amd.build`")
    # torch (ROCm) ships its own libamdhip64.so.7; load it first so that libhz binds to the
    # same HIP runtime that owns torch's streams and allocations
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(p)
    vp, i64, i32, u64 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64
    sig = {
        "hz_init": [C.POINTER(vp), C.POINTER(InitOpts)],
        "hz_finalize": [vp],
        "hz_last_error": [vp],
        "hz_release": [vp, u64],
        "hz_mesh": [vp, i64, vp, i64, vp, vp, C.POINTER(u64), C.POINTER(i64)],
        "hz_assemble": [vp, u64, vp, vp, C.c_double, C.POINTER(u64)],
        "hz_setup_ddm": [vp, u64, vp, i32, i32, C.POINTER(CoarseMesh), C.c_int, C.POINTER(u64)],
        "hz_setup_ddm_ex": [vp, u64, vp, i32, i32, C.POINTER(CoarseMesh), C.POINTER(DdmOpts), C.POINTER(u64)],
        "hz_get_pou": [vp, u64, i32, vp],
        "hz_solve": [vp, u64, i64, vp, C.c_int, C.c_double, i32, vp, C.c_int, vp],
        "hz_solve_ex": [vp, u64, i64, vp, C.c_int, C.POINTER(SolveOpts), vp, C.c_int, vp],
        "hz_point_sources": [vp, u64, i64, vp, vp, vp, C.c_int],
        "hz_spmm": [vp, u64, i64, vp, C.c_int, vp, C.c_int],
        "hz_spmm_c64x": [vp, u64, i64, vp, C.c_int, vp, C.c_int],
        "hz_spmm_noalloc": [vp, u64, i64, vp, vp],
        "hz_precond": [vp, u64, i64, vp, C.c_int, vp, C.c_int],
        "hz_ddm_stats_get": [vp, u64, C.POINTER(DdmStats)],
        "hz_ddm_levels": [vp, u64, C.POINTER(DdmLevel), C.c_int32, C.POINTER(C.c_int32)],
        "hz_serve_start": [vp, i32],
        "hz_serve_submit": [vp, C.POINTER(Request), C.POINTER(u64)],
        "hz_serve_poll": [vp, u64, C.POINTER(C.c_int)],
        "hz_serve_wait": [vp, u64, C.POINTER(i32)],
        "hz_serve_stats_get": [vp, C.POINTER(ServeStats)],
        "hz_serve_stop": [vp],
        "hz_get_dofmap": [vp, u64, vp],
        "hz_get_csr_size": [vp, u64, C.POINTER(i64), C.POINTER(i64)],
        "hz_get_csr": [vp, u64, vp, vp, vp],
        "hz_get_subdomain_size": [vp, u64, i32, C.POINTER(i64), C.POINTER(i64)],
        "hz_get_subdomain": [vp, u64, i32, vp, vp, vp, vp, vp],
        "hz_get_coarse_size": [vp, u64, C.POINTER(i64), C.POINTER(i64)],
        "hz_get_coarse": [vp, u64, vp, vp, vp],
        "hz_profile_enable": [vp, C.c_int],
        "hz_profile_get": [vp, C.c_int, C.POINTER(KernelStat)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = None if name == "hz_finalize" else (C.c_char_p if name == "hz_last_error" else C.c_int)
    _lib = lib
    return lib


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _block_arg(x, n):
    """(pointer, mem kind, keepalive) for a complex128 block of shape (s, n)."""
    if _is_torch(x):
        import torch

        if x.dtype != torch.complex128 or not x.is_contiguous():
            raise TypeError("device blocks must be contiguous torch.complex128 tensors")
        if x.shape[-1] != n:
            raise ValueError(f"block has {x.shape[-1]} dofs, expected {n}")
        return C.c_void_p(x.data_ptr()), (HZ_MEM_DEVICE if x.is_cuda else HZ_MEM_HOST), x
    a = np.ascontiguousarray(x, dtype=np.complex128)
    if a.shape[-1] != n:
        raise ValueError(f"block has {a.shape[-1]} dofs, expected {n}")
    return _np_ptr(a), HZ_MEM_HOST, a


class Mesh:
    def __init__(self, ctx, handle, n_dofs, n_tets):
        self.ctx, self.handle, self.n, self.n_tets = ctx, handle, n_dofs, n_tets


class Operator:
    def __init__(self, ctx, handle, mesh):
        self.ctx, self.handle, self.mesh, self.n = ctx, handle, mesh, mesh.n


class Ddm:
    def __init__(self, ctx, handle, op, precision):
        self.ctx, self.handle, self.op, self.n, self.precision = ctx, handle, op, op.n, precision


_live_contexts = weakref.WeakSet()


@atexit.register
def _close_live_contexts():
    # release library memory while torch's allocator is still alive
    for c in list(_live_contexts):
        try:
            c.close()
        except Exception:
            pass


def _torch_allocator(device):
    """(alloc, free) callbacks over torch's stream-ordered caching allocator."""
    import torch

    def _alloc(nbytes, stream, user):
        for attempt in range(2):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device, int(stream or 0))
            except Exception:  # out of memory or a bad request: the library reports HZ_ERR_OOM
                if attempt:
                    return None
                # blocks torch keeps cached (of other sizes) go back to the device, then retry once
                torch.cuda.empty_cache()
        return None

    def _free(ptr, stream, user):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    return ALLOC_FN(_alloc), FREE_FN(_free)


class Context:
    """One GPU; all work on `stream` (a torch.cuda.Stream, a raw hipStream_t int, or None).
    allocator="torch" routes the library's device memory through torch's caching allocator
    on that stream; "hip" uses hipMalloc / hipFree."""

    def __init__(self, device=0, stream=None, hbm_budget=0, allocator="torch"):
        self.lib = load()
        self.h = None
        self._alloc_cbs = None
        o = InitOpts()
        o.struct_size, o.device, o.hbm_budget = C.sizeof(InitOpts), device, hbm_budget
        if stream is not None:
            o.stream = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        if allocator == "torch":
            self._alloc_cbs = _torch_allocator(device)  # kept alive as long as the context
            o.alloc, o.free = self._alloc_cbs
        elif allocator != "hip":
            raise ValueError("allocator must be 'torch' or 'hip'")
        h = C.c_void_p()
        st = self.lib.hz_init(C.byref(h), C.byref(o))
        if st != HZ_OK:
            raise HzError(st, "hz_init failed")
        self.h = h
        _live_contexts.add(self)

    def close(self):
        if self.h:
            self.lib.hz_finalize(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow=()):
        if st != HZ_OK and st not in allow:
            raise HzError(st, self.lib.hz_last_error(self.h).decode())
        return st

    def release(self, obj):
        self._check(self.lib.hz_release(self.h, obj.handle))

    # ---------------------------------------------------------------- setup
    def mesh(self, tets, coords, face_bc=None):
        t = np.ascontiguousarray(tets, np.int32)
        x = np.ascontiguousarray(coords, np.float64)
        fb = None if face_bc is None else np.ascontiguousarray(face_bc, np.int8)
        h, n = C.c_uint64(), C.c_int64()
        self._check(self.lib.hz_mesh(self.h, t.shape[0], _np_ptr(t), x.shape[0], _np_ptr(x),
                                     None if fb is None else _np_ptr(fb), C.byref(h), C.byref(n)))
        return Mesh(self, h.value, n.value, t.shape[0])

    def assemble(self, mesh, velocity, freq, Q=None):
        v = np.ascontiguousarray(velocity, np.float64)
        q = None if Q is None else np.ascontiguousarray(Q, np.float64)
        h = C.c_uint64()
        self._check(self.lib.hz_assemble(self.h, mesh.handle, _np_ptr(v), None if q is None else _np_ptr(q),
                                         float(freq), C.byref(h)))
        return Operator(self, h.value, mesh)

    def setup_ddm(self, op, partition, n_sub, overlap, coarse=None, precision=HZ_PREC_C128, pou=HZ_POU_BOOLEAN,
                  local_solver=HZ_LOCAL_EXACT):
        p = np.ascontiguousarray(partition, np.int32)
        cm = None
        keep = []
        if coarse is not None:
            ct = np.ascontiguousarray(coarse[0], np.int32)
            cc = np.ascontiguousarray(coarse[1], np.float64)
            keep += [ct, cc]
            cm = CoarseMesh(ct.shape[0], ct.ctypes.data, cc.shape[0], cc.ctypes.data)
        h = C.c_uint64()
        if self._alloc_cbs is not None:
            # memory that earlier calls returned to torch's cache goes back to the device: the
            # set-up sizes its factorisation groups by the device's free memory
            import torch

            torch.cuda.empty_cache()
        o = DdmOpts(C.sizeof(DdmOpts), int(precision), int(pou), int(local_solver))
        st = self.lib.hz_setup_ddm_ex(self.h, op.handle, _np_ptr(p), int(n_sub), int(overlap),
                                      None if cm is None else C.byref(cm), C.byref(o), C.byref(h))
        if self._alloc_cbs is not None:
            # the factorisation's transient buffers went back to torch's cache: hand them back to
            # the device, where the library's free-memory queries (Krylov sizing) see them
            import torch

            torch.cuda.empty_cache()
        self._check(st)
        return Ddm(self, h.value, op, precision)

    # ---------------------------------------------------------------- compute
    def solve(self, ddm, rhs, tol=1e-6, max_iter=500, restart=0, fixed_iters=0, block=0, out=None,
              raise_on_not_converged=True):
        """Solve A X = B for B of shape (s, n); returns (X, list of per-column info dicts)."""
        rp, rm, keep = _block_arg(rhs, ddm.n)
        s = int(np.prod(rhs.shape[:-1])) if len(rhs.shape) > 1 else 1
        if out is None:
            if _is_torch(rhs):
                import torch

                out = torch.empty_like(rhs)
            else:
                out = np.empty((s, ddm.n), np.complex128)
        xp, xm, keep2 = _block_arg(out, ddm.n)
        info = (ColInfo * s)()
        o = SolveOpts(C.sizeof(SolveOpts), float(tol), int(max_iter), int(restart), int(fixed_iters), int(block))
        st = self.lib.hz_solve_ex(self.h, ddm.handle, s, rp, rm, C.byref(o), xp, xm, info)
        self._check(st, allow=() if raise_on_not_converged else (HZ_ERR_NOT_CONVERGED,))
        return out, _info_dicts(info)

    def point_sources(self, mesh, xyz, amp=None, out=None):
        x = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
        a = None if amp is None else np.ascontiguousarray(np.asarray(amp, np.complex128))
        if out is None:
            out = np.empty((x.shape[0], mesh.n), np.complex128)
        op_, om, keep = _block_arg(out, mesh.n)
        self._check(self.lib.hz_point_sources(self.h, mesh.handle, x.shape[0], _np_ptr(x),
                                              None if a is None else _np_ptr(a), op_, om))
        return out

    def spmm(self, op, x, out=None):
        xp, xm, keep = _block_arg(x, op.n)
        s = int(np.prod(x.shape[:-1])) if len(x.shape) > 1 else 1
        if out is None:
            out = np.empty((s, op.n), np.complex128) if not _is_torch(x) else x.new_empty(x.shape)
        yp, ym, keep2 = _block_arg(out, op.n)
        self._check(self.lib.hz_spmm(self.h, op.handle, s, xp, xm, yp, ym))
        return out

    def spmm_noalloc(self, op, x, out):
        """y = A x through the library's static scratch memory (no device allocation); x and out
        are contiguous complex128 device tensors of shape (s, n)."""
        for t in (x, out):
            if not (_is_torch(t) and t.is_cuda and t.is_contiguous()) or str(t.dtype) != "torch.complex128":
                raise TypeError("x and out must be contiguous complex128 device tensors")
            if t.shape[-1] != op.n:
                raise ValueError(f"block has {t.shape[-1]} dofs, expected {op.n}")
        s = int(np.prod(x.shape[:-1])) if len(x.shape) > 1 else 1
        if tuple(out.shape) != tuple(x.shape):
            raise ValueError("out must have the shape of x")
        self._check(self.lib.hz_spmm_noalloc(self.h, op.handle, s, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr())))
        return out

    def spmm_c64x(self, op, x):
        """y = A x for a complex64 block x (widened exactly, FP64 products); y complex128."""
        if _is_torch(x):
            import torch

            if x.dtype != torch.complex64 or not x.is_contiguous():
                raise TypeError("device blocks must be contiguous torch.complex64 tensors")
            xp, xm, keep = C.c_void_p(x.data_ptr()), (HZ_MEM_DEVICE if x.is_cuda else HZ_MEM_HOST), x
            out = torch.empty(x.shape, dtype=torch.complex128, device=x.device)
        else:
            keep = np.ascontiguousarray(x, dtype=np.complex64)
            xp, xm = _np_ptr(keep), HZ_MEM_HOST
            out = np.empty(keep.shape, np.complex128)
        if x.shape[-1] != op.n:
            raise ValueError(f"block has {x.shape[-1]} dofs, expected {op.n}")
        s = int(np.prod(x.shape[:-1])) if len(x.shape) > 1 else 1
        yp, ym, keep2 = _block_arg(out, op.n)
        self._check(self.lib.hz_spmm_c64x(self.h, op.handle, s, xp, xm, yp, ym))
        return out

    def precond(self, ddm, v, out=None):
        vp, vm, keep = _block_arg(v, ddm.n)
        s = int(np.prod(v.shape[:-1])) if len(v.shape) > 1 else 1
        if out is None:
            out = np.empty((s, ddm.n), np.complex128) if not _is_torch(v) else v.new_empty(v.shape)
        zp, zm, keep2 = _block_arg(out, ddm.n)
        self._check(self.lib.hz_precond(self.h, ddm.handle, s, vp, vm, zp, zm))
        return out

    # ---------------------------------------------------------------- serving
    def serve_start(self, max_slots=8):
        """Start the scheduler thread; until serve_stop only the serving calls are valid."""
        self._check(self.lib.hz_serve_start(self.h, int(max_slots)))

    def submit(self, ddm, rhs, tol=1e-6, max_iter=500, out=None):
        """Queue a solve request; returns a ticket (rhs / out must stay alive until wait)."""
        rp, rm, keep = _block_arg(rhs, ddm.n)
        s = int(np.prod(rhs.shape[:-1])) if len(rhs.shape) > 1 else 1
        if out is None:
            if _is_torch(rhs):
                import torch

                out = torch.empty_like(rhs)
            else:
                out = np.empty((s, ddm.n), np.complex128)
        xp, xm, keep2 = _block_arg(out, ddm.n)
        if xm != rm:
            raise ValueError("rhs and out must both be host or both be device blocks")
        info = (ColInfo * s)()
        req = Request(C.sizeof(Request), ddm.handle, s, rp.value, xp.value, rm, float(tol), int(max_iter),
                      C.cast(info, C.c_void_p).value)
        t = C.c_uint64()
        self._check(self.lib.hz_serve_submit(self.h, C.byref(req), C.byref(t)))
        return {"id": t.value, "out": out, "info": info, "keep": (keep, keep2, rhs)}

    def poll(self, ticket):
        done = C.c_int()
        self._check(self.lib.hz_serve_poll(self.h, ticket["id"], C.byref(done)))
        return bool(done.value)

    def wait(self, ticket):
        st = C.c_int32()
        self._check(self.lib.hz_serve_wait(self.h, ticket["id"], C.byref(st)))
        return ticket["out"], _info_dicts(ticket["info"]), st.value

    def serve_stats(self):
        s = ServeStats()
        self._check(self.lib.hz_serve_stats_get(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ServeStats._fields_}

    def serve_stop(self):
        self._check(self.lib.hz_serve_stop(self.h))

    # ---------------------------------------------------------------- measurement
    def profile(self, on=True):
        """Start (clear) or stop live event timing of the kernel classes in KERNEL_CLASSES."""
        self._check(self.lib.hz_profile_enable(self.h, 1 if on else 0))

    def profile_stats(self):
        out = {}
        for name, k in KERNEL_CLASSES.items():
            st = KernelStat()
            self._check(self.lib.hz_profile_get(self.h, k, C.byref(st)))
            out[name] = dict(launches=st.launches, seconds=st.seconds, bytes=st.bytes, flops=st.flops)
        return out

    # ---------------------------------------------------------------- introspection
    def ddm_stats(self, ddm):
        s = DdmStats()
        self._check(self.lib.hz_ddm_stats_get(self.h, ddm.handle, C.byref(s)))
        return {k: getattr(s, k) for k, _ in DdmStats._fields_}

    def ddm_levels(self, ddm):
        """Per elimination level (leaves first): fronts, largest p and f, sums of p and f, and
        stored factor nonzeros."""
        n = C.c_int32()
        self._check(self.lib.hz_ddm_levels(self.h, ddm.handle, None, 0, C.byref(n)))
        arr = (DdmLevel * max(1, n.value))()
        self._check(self.lib.hz_ddm_levels(self.h, ddm.handle, arr, n.value, C.byref(n)))
        return [{k: getattr(arr[i], k) for k, _ in DdmLevel._fields_} for i in range(n.value)]

    def dofmap(self, mesh):
        out = np.empty((mesh.n_tets, 20), np.int32)
        self._check(self.lib.hz_get_dofmap(self.h, mesh.handle, _np_ptr(out)))
        return out

    def csr(self, op, values=True):
        n, nnz = C.c_int64(), C.c_int64()
        self._check(self.lib.hz_get_csr_size(self.h, op.handle, C.byref(n), C.byref(nnz)))
        rp = np.empty(n.value + 1, np.int64)
        ci = np.empty(nnz.value, np.int32)
        va = np.empty(nnz.value, np.complex128) if values else None
        self._check(self.lib.hz_get_csr(self.h, op.handle, _np_ptr(rp), _np_ptr(ci), None if va is None else _np_ptr(va)))
        return rp, ci, va

    def subdomain(self, ddm, i, values=True):
        n, nnz = C.c_int64(), C.c_int64()
        self._check(self.lib.hz_get_subdomain_size(self.h, ddm.handle, int(i), C.byref(n), C.byref(nnz)))
        g = np.empty(n.value, np.int32)
        own = np.empty(n.value, np.uint8)
        rp = np.empty(n.value + 1, np.int64)
        ci = np.empty(nnz.value, np.int32)
        va = np.empty(nnz.value, np.complex128) if values else None
        self._check(self.lib.hz_get_subdomain(self.h, ddm.handle, int(i), _np_ptr(g), _np_ptr(own), _np_ptr(rp),
                                              _np_ptr(ci), None if va is None else _np_ptr(va)))
        return g, own.astype(bool), rp, ci, va

    def pou_weights(self, ddm, i):
        """Partition-of-unity weights of subdomain i, aligned with its sorted dofs."""
        n, nnz = C.c_int64(), C.c_int64()
        self._check(self.lib.hz_get_subdomain_size(self.h, ddm.handle, int(i), C.byref(n), C.byref(nnz)))
        out = np.empty(n.value, np.float64)
        self._check(self.lib.hz_get_pou(self.h, ddm.handle, int(i), _np_ptr(out)))
        return out

    def coarse(self, ddm):
        nc, nnz = C.c_int64(), C.c_int64()
        self._check(self.lib.hz_get_coarse_size(self.h, ddm.handle, C.byref(nc), C.byref(nnz)))
        rp = np.empty(ddm.n + 1, np.int64)
        ci = np.empty(nnz.value, np.int32)
        va = np.empty(nnz.value, np.float64)
        self._check(self.lib.hz_get_coarse(self.h, ddm.handle, _np_ptr(rp), _np_ptr(ci), _np_ptr(va)))
        return nc.value, rp, ci, va
