"""Thin ctypes binding of libhdg.so (include/hdg.h).

Argument marshalling only: torch supplies device memory (``tensor.data_ptr()``) and the
stream (``torch.cuda.current_stream().cuda_stream``); every step of the condensation path runs
in the library's HIP kernels.  Importing this module never falls back to anything else: if
the shared library is missing, loading fails with an error that says how to build it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhdg.so")

ACOUSTIC, ELASTIC, MAXWELL, MAXWELL_GLM = 0, 1, 2, 3
FP64, MIXED_FP32, MIXED_BF16 = 0, 1, 2
BACKWARD_EULER, DIRK33 = 0, 1
PHYSICS = {"acoustic": ACOUSTIC, "elastic": ELASTIC, "maxwell": MAXWELL, "maxwell_glm": MAXWELL_GLM}
PRECISION = {"fp64": FP64, "mixed_fp32": MIXED_FP32, "mixed_bf16": MIXED_BF16}
STATUS = {0: "HDG_OK", 1: "HDG_E_ARG", 2: "HDG_E_MESH", 3: "HDG_E_ALLOC", 4: "HDG_E_HIP",
          5: "HDG_E_SINGULAR", 6: "HDG_E_NOCONV", 7: "HDG_E_STATE", 8: "HDG_E_UNSUPPORTED"}
Q = dict(n_elem=0, n_faces=1, n_bfaces=2, n_local_dofs=3, n_trace_dofs=4, n_vol_points=5,
         n_bnd_points=6, last_iters=7, last_refine=8, m_local=9, m_trace=10, schedule=11,
         step_graph=12, step_graph_iters=13, n_colors=14)
PRECOND = {"jacobi": 0, "ssor": 1}

# every function declared in include/hdg.h
EXPORTS = ["hdg_init_mesh", "hdg_query", "hdg_condense", "hdg_condense_rhs", "hdg_trace_solve", "hdg_recover",
           "hdg_step", "hdg_apply_mass", "hdg_volume_points", "hdg_project_volume",
           "hdg_boundary_points", "hdg_project_boundary", "hdg_point_sources",
           "hdg_element_data", "hdg_last_timing", "hdg_reference_table", "hdg_destroy",
           "hdg_last_error", "hdg_last_residual", "hdg_trace_solve_static",
           "hdg_hbm_probe"]


class HDGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_vert", C.c_int64), ("xyz", C.c_void_p),
                ("n_elem", C.c_int64), ("elem_vert", C.c_void_p), ("degree", C.c_void_p),
                ("bface_tag", C.c_void_p)]


class PhysDesc(C.Structure):
    _fields_ = [("physics", C.c_int), ("elem_par", C.c_void_p), ("stab_scale", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("k", C.c_int), ("nrhs", C.c_int),
                ("krylov_tol", C.c_double), ("krylov_maxit", C.c_int),
                ("refine_tol", C.c_double), ("refine_maxit", C.c_int),
                ("refine_inner_tol", C.c_double), ("cache_factors", C.c_int),
                ("autotune", C.c_int), ("autotune_table", C.c_char_p), ("use_graph", C.c_int),
                ("graph_step", C.c_int), ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN),
                ("alloc_user", C.c_void_p), ("precond", C.c_int)]


class TorchAllocator:
    """Device workspaces of a context from torch's caching allocator (options.dev_alloc /
    dev_free): each block is a uint8 tensor kept alive until the library returns it."""

    def __init__(self, device=None):
        import torch
        self._torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        self.blocks = {}
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    def _alloc(self, user, nbytes):
        try:
            t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=self.device)
        except RuntimeError:
            return None
        p = t.data_ptr()
        self.blocks[p] = t
        return p

    def _free(self, user, ptr):
        self.blocks.pop(ptr, None)

    @property
    def nbytes(self):
        return sum(t.numel() for t in self.blocks.values())


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhdg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_1807_00086_amd.build` "
                          "(or __graft_entry__.build()); there is no fallback implementation")
    lib = C.CDLL(path)
    vp, i64, dbl, cint = C.c_void_p, C.c_int64, C.c_double, C.c_int
    sig = {
        "hdg_init_mesh": (cint, [C.POINTER(vp), C.POINTER(MeshDesc), C.POINTER(PhysDesc),
                                 C.POINTER(Options), vp]),
        "hdg_query": (cint, [vp, cint, C.POINTER(i64)]),
        "hdg_condense": (cint, [vp, dbl, vp, vp]),
        "hdg_condense_rhs": (cint, [vp, dbl, vp, vp]),
        "hdg_trace_solve": (cint, [vp, vp, C.POINTER(cint), C.POINTER(dbl)]),
        "hdg_recover": (cint, [vp, vp, vp]),
        "hdg_step": (cint, [vp, dbl, dbl, cint, vp, vp, vp, vp]),
        "hdg_apply_mass": (cint, [vp, dbl, vp, vp]),
        "hdg_volume_points": (cint, [vp, vp]),
        "hdg_project_volume": (cint, [vp, vp, vp]),
        "hdg_boundary_points": (cint, [vp, vp]),
        "hdg_project_boundary": (cint, [vp, vp, vp]),
        "hdg_point_sources": (cint, [vp, cint, vp, vp]),
        "hdg_element_data": (cint, [vp, cint, i64, i64, vp]),
        "hdg_last_timing": (cint, [vp, cint, C.POINTER(dbl)]),
        "hdg_reference_table": (i64, [cint, cint, cint, cint, vp, i64]),
        "hdg_destroy": (None, [vp]),
        "hdg_last_error": (C.c_char_p, [vp]),
        "hdg_last_residual": (cint, [vp, vp]),
        "hdg_trace_solve_static": (cint, [vp, vp, C.POINTER(cint), C.POINTER(dbl)]),
        "hdg_hbm_probe": (cint, [vp, vp, i64, cint, cint, vp, C.POINTER(dbl)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    """Host pointer of a contiguous numpy array (host-side helpers only)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def check_device_vector(t, n, name):
    """Device pointer of `t` after checking that it is a contiguous FP64 torch tensor on the GPU
    with at least `n` elements: the library's kernels read and write exactly that many, so a
    host array, another dtype, a strided view or a short buffer is rejected here (HDG_E_ARG)
    instead of being handed to them."""
    if not (hasattr(t, "data_ptr") and hasattr(t, "is_cuda")):
        raise HDGError(1, f"{name}: expected a torch tensor on the GPU, got {type(t).__name__}")
    if not t.is_cuda:
        raise HDGError(1, f"{name}: tensor is on {t.device}, the library needs device memory")
    if str(t.dtype) != "torch.float64":
        raise HDGError(1, f"{name}: dtype {t.dtype}, the library reads and writes float64")
    if not t.is_contiguous():
        raise HDGError(1, f"{name}: tensor is not contiguous")
    if t.numel() < n:
        raise HDGError(1, f"{name}: {t.numel()} elements, {n} needed")
    return C.c_void_p(t.data_ptr())


def hbm_probe(src, dst=None, reps=10, blocks_per_cu=8, stream=None):
    """Milliseconds per launch of the library's streaming read (dst None) or copy pass over the
    FP64 device tensor src (diagnostic)."""
    lib = load_library()
    n = src.numel()
    check_device_vector(src, n, "src")
    if dst is not None:
        check_device_vector(dst, n, "dst")
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    ms = C.c_double()
    st = lib.hdg_hbm_probe(C.c_void_p(src.data_ptr()), None if dst is None else C.c_void_p(dst.data_ptr()),
                           n, int(reps), int(blocks_per_cu), C.c_void_p(stream), C.byref(ms))
    if st != 0:
        raise HDGError(st, "hdg_hbm_probe failed")
    return ms.value


def reference_table(dim, k, kF, which):
    lib = load_library()
    cap = 8 * 6 * 200000
    out = np.zeros(cap)
    n = lib.hdg_reference_table(dim, k, kF, which, _ptr(out), cap)
    if n < 0:
        raise HDGError(-n, "hdg_reference_table failed")
    return out[:n].copy()


class Solver:
    """One HDG context (mesh + physics + options) bound to a HIP stream."""

    def __init__(self, xyz, elem_vert, physics, elem_par, k=None, degree=None, precision="fp64",
                 nrhs=1, stab_scale=1.0, krylov_tol=1e-13, krylov_maxit=5000, refine_tol=1e-13,
                 refine_maxit=10, refine_inner_tol=1e-6, cache_factors=False, autotune=False,
                 autotune_table=None, use_graph=False, graph_step=False, bface_tag=None, allocator=None,
                 precond="jacobi", stream=None):
        self.lib = load_library()
        self._xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self._ev = np.ascontiguousarray(elem_vert, dtype=np.int64)
        par = np.zeros((self._ev.shape[0], 3))
        ep = np.asarray(elem_par, dtype=np.float64)
        par[:, :ep.shape[1]] = ep
        self._par = np.ascontiguousarray(par)
        self._deg = None if degree is None else np.ascontiguousarray(degree, dtype=np.int8)
        self._tag = None
        if bface_tag is not None:
            self._tag = np.ascontiguousarray(bface_tag, dtype=np.int8)
            if self._tag.shape != self._ev.shape:
                raise ValueError(f"bface_tag: shape {self._tag.shape}, expected {self._ev.shape}")
        self.dim = self._xyz.shape[1]
        self.physics = PHYSICS[physics] if isinstance(physics, str) else int(physics)
        self.nrhs = int(nrhs)
        md = MeshDesc(self.dim, self._xyz.shape[0], _ptr(self._xyz).value, self._ev.shape[0],
                      _ptr(self._ev).value, None if self._deg is None else _ptr(self._deg).value,
                      None if self._tag is None else _ptr(self._tag).value)
        pd = PhysDesc(self.physics, _ptr(self._par).value, float(stab_scale))
        prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
        od = Options(prec, int(k if k is not None else (int(degree[0]) if degree is not None else 1)),
                     self.nrhs, float(krylov_tol), int(krylov_maxit), float(refine_tol),
                     int(refine_maxit), float(refine_inner_tol), int(bool(cache_factors)),
                     int(bool(autotune)), None if autotune_table is None else os.fsencode(autotune_table),
                     int(bool(use_graph)), int(bool(graph_step)))
        # allocator: None (hipMalloc) or "torch" / a TorchAllocator (torch's caching allocator)
        self.allocator = TorchAllocator() if allocator == "torch" else allocator
        if self.allocator is not None:
            od.dev_alloc = self.allocator.alloc_fn
            od.dev_free = self.allocator.free_fn
        od.precond = PRECOND[precond] if isinstance(precond, str) else int(precond)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        self.ctx = C.c_void_p()
        st = self.lib.hdg_init_mesh(C.byref(self.ctx), C.byref(md), C.byref(pd), C.byref(od),
                                    C.c_void_p(stream))
        if st != 0:
            raise HDGError(st, self.lib.hdg_last_error(None).decode())

    # ------------------------------------------------------------------ helpers
    def _check(self, st):
        if st != 0:
            raise HDGError(st, self.lib.hdg_last_error(self.ctx).decode())

    def schedules(self):
        """{degree: schedule} of the block-structured condensation's classes chosen so far."""
        v = self.query("schedule")
        return {k: ((v >> (4 * (k - 1))) & 15) - 1 for k in range(1, 6) if (v >> (4 * (k - 1))) & 15}

    def query(self, key):
        v = C.c_int64()
        self._check(self.lib.hdg_query(self.ctx, Q[key] if isinstance(key, str) else key, C.byref(v)))
        return v.value

    def close(self):
        if self.ctx:
            self.lib.hdg_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ path
    def _nl(self):
        return self.query("n_local_dofs") * self.nrhs

    def _nt(self):
        return self.query("n_trace_dofs") * self.nrhs

    def condense(self, a, f_loc, lam_bnd):
        self._check(self.lib.hdg_condense(self.ctx, float(a), check_device_vector(f_loc, self._nl(), "f_loc"),
                                          check_device_vector(lam_bnd, self._nt(), "lam_bnd")))

    def condense_rhs(self, a, f_loc, lam_bnd):
        """Condense a new right-hand side with the factors of the last condense (same a)."""
        self._check(self.lib.hdg_condense_rhs(self.ctx, float(a), check_device_vector(f_loc, self._nl(), "f_loc"),
                                              check_device_vector(lam_bnd, self._nt(), "lam_bnd")))

    def trace_solve(self, lam):
        it = C.c_int()
        rr = C.c_double()
        self._check(self.lib.hdg_trace_solve(self.ctx, check_device_vector(lam, self._nt(), "lambda"),
                                             C.byref(it), C.byref(rr)))
        return it.value, rr.value

    def trace_solve_static(self, lam):
        """hdg_trace_solve without any allocation (library-owned static scratch)."""
        it = C.c_int()
        rr = C.c_double()
        self._check(self.lib.hdg_trace_solve_static(self.ctx, check_device_vector(lam, self._nt(), "lambda"),
                                                    C.byref(it), C.byref(rr)))
        return it.value, rr.value

    def recover(self, lam, u):
        self._check(self.lib.hdg_recover(self.ctx, check_device_vector(lam, self._nt(), "lambda"),
                                         check_device_vector(u, self._nl(), "u_loc")))

    def last_residual(self):
        """Relative FP64 residual per column of the last mixed-precision recover."""
        out = np.zeros(self.nrhs)
        self._check(self.lib.hdg_last_residual(self.ctx, _ptr(out)))
        return out

    def step(self, t, dt, scheme, u, lam, lam_bnd_stages, src=None):
        sc = {"be": BACKWARD_EULER, "dirk33": DIRK33}.get(scheme, scheme)
        ns = 3 if sc == DIRK33 else 1
        self._check(self.lib.hdg_step(self.ctx, float(t), float(dt), int(sc), check_device_vector(u, self._nl(), "u"),
                                      check_device_vector(lam, self._nt(), "lambda"),
                                      check_device_vector(lam_bnd_stages, ns * self._nt(), "lam_bnd"),
                                      None if src is None else check_device_vector(src, self._nl(), "src")))

    def apply_mass(self, a, u, f):
        self._check(self.lib.hdg_apply_mass(self.ctx, float(a), check_device_vector(u, self._nl(), "u"),
                                            check_device_vector(f, self._nl(), "f")))

    # ------------------------------------------------------------------ host helpers
    def volume_points(self):
        n = self.query("n_vol_points")
        out = np.zeros((n, self.dim))
        self._check(self.lib.hdg_volume_points(self.ctx, _ptr(out)))
        return out

    def project_volume(self, vals):
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        u = np.zeros(self.query("n_local_dofs"))
        self._check(self.lib.hdg_project_volume(self.ctx, _ptr(vals), _ptr(u)))
        return u

    def boundary_points(self):
        n = self.query("n_bnd_points")
        out = np.zeros((n, self.dim))
        self._check(self.lib.hdg_boundary_points(self.ctx, _ptr(out)))
        return out

    def project_boundary(self, vals):
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        lam = np.zeros(self.query("n_trace_dofs"))
        self._check(self.lib.hdg_project_boundary(self.ctx, _ptr(vals), _ptr(lam)))
        return lam

    def point_sources(self, pts):
        pts = np.ascontiguousarray(pts, dtype=np.float64)
        f = np.zeros((self.query("n_local_dofs"), pts.shape[0]))
        self._check(self.lib.hdg_point_sources(self.ctx, pts.shape[0], _ptr(pts), _ptr(f)))
        return f

    def element_data(self, which, e0, count, block):
        out = np.zeros(count * block)
        w = {"K": 0, "r": 1, "Z": 2, "z": 3}.get(which, which)
        self._check(self.lib.hdg_element_data(self.ctx, w, int(e0), int(count), _ptr(out)))
        return out

    def timing(self, which):
        ms = C.c_double()
        w = {"condense": 0, "assemble": 1, "solve": 2, "recover": 3, "refine_elem": 4,
             "refine_solve": 5}.get(which, which)
        self._check(self.lib.hdg_last_timing(self.ctx, w, C.byref(ms)))
        return ms.value
