"""Thin ctypes binding of libnlq (include/nlq.h): argument marshalling only.

Every step of the assembly and solve runs in the library's HIP kernels; this
module converts numpy arrays to pointers and status codes to exceptions.  It
raises ImportError-like errors loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnlq.so")

NLQ_OK, NLQ_EINVAL, NLQ_ENOMEM, NLQ_EDEVICE, NLQ_ENOTREADY, NLQ_ECANCELLED, NLQ_EBUSY, \
    NLQ_ENOCONV = 0, -1, -2, -3, -4, -5, -6, -7
NLQ_ETA_CONST, NLQ_ETA_GAUSS = 0, 1
NLQ_FORM_SYM4, NLQ_FORM_PAPER2, NLQ_FORM_PAPER2_INNER = 0, 1, 2
NLQ_FP64_PLAIN, NLQ_FP32_MIXED = 0, 1
NLQ_SHAPE_SIMPLEX, NLQ_SHAPE_BOX = 0, 1

STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOTREADY",
                -5: "ECANCELLED", -6: "EBUSY", -7: "ENOCONV"}

# every extern "C" symbol declared in include/nlq.h
EXPORTS = [
    "nlq_ctx_create", "nlq_ctx_set_stream", "nlq_ctx_memory", "nlq_ctx_destroy",
    "nlq_mesh_create", "nlq_mesh_create_order", "nlq_mesh_create_shape", "nlq_mesh_box", "nlq_mesh_info", "nlq_mesh_copy", "nlq_mesh_destroy",
    "nlq_assemble", "nlq_prepare", "nlq_integrate_range", "nlq_integrate_ranges", "nlq_assemble_batch", "nlq_assemble_info_get",
    "nlq_autotune", "nlq_tune_save", "nlq_tune_load", "nlq_reassemble", "nlq_set_data",
    "nlq_set_data_device", "nlq_solve", "nlq_solve_noalloc", "nlq_solution_device",
    "nlq_info", "nlq_csr_copy", "nlq_csr_device", "nlq_pairs_copy", "nlq_rhs_copy",
    "nlq_pair_blocks", "nlq_system_destroy", "nlq_serve_start", "nlq_submit", "nlq_wait",
    "nlq_cancel", "nlq_result_release", "nlq_serve_stats_get", "nlq_serve_stop", "nlq_last_error",
]


class NlqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class nlq_params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("kernel", C.c_int32), ("delta", C.c_double),
                ("eps", C.c_double), ("scale", C.c_double), ("lmin", C.c_int32),
                ("lmax", C.c_int32), ("form", C.c_int32), ("precision", C.c_int32),
                ("deterministic", C.c_int32), ("min_dist_l2", C.c_int32)]


class nlq_assemble_info(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("n_leaf", C.c_int64 * 9), ("n_evals", C.c_int64),
                ("nnz", C.c_int64), ("t_tables", C.c_double), ("t_pairs", C.c_double),
                ("t_pattern", C.c_double), ("t_integrate", C.c_double), ("t_total", C.c_double),
                ("t_kernel", C.c_double), ("n_leaf_zero", C.c_int64)]


class nlq_tune_info(C.Structure):
    _fields_ = [("occupancy_variant", C.c_int32), ("workgroups_per_cu", C.c_int32),
                ("pairs_per_item", C.c_int32), ("work_items_per_element", C.c_int32),
                ("candidates", C.c_int32), ("best_ms", C.c_double), ("default_ms", C.c_double),
                ("stack_capacity", C.c_int32), ("leaf_capacity", C.c_int32)]


class nlq_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32),
                ("rel_residual", C.c_double), ("seconds", C.c_double)]


class nlq_request(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32), ("k_gamma", C.c_int32),
                ("params", nlq_params), ("f_nodal", C.c_void_p), ("g_nodal", C.c_void_p),
                ("rtol", C.c_double), ("maxit", C.c_int32)]


class nlq_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_nodes", C.c_int64), ("n_pairs", C.c_int64),
                ("n_free", C.c_int64), ("u", C.POINTER(C.c_double)), ("cg_iterations", C.c_int32),
                ("rel_residual", C.c_double), ("latency_s", C.c_double), ("queue_s", C.c_double),
                ("assemble_s", C.c_double), ("solve_s", C.c_double), ("launches", C.c_int32),
                ("cache_hit", C.c_int32), ("setup_s", C.c_double)]


class nlq_serve_config(C.Structure):
    _fields_ = [("max_active", C.c_int32), ("target_launch_ms", C.c_double), ("cache_systems", C.c_int32)]


class nlq_serve_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("cancelled", C.c_int64), ("launches", C.c_int64), ("launch_segments", C.c_int64),
                ("max_per_launch", C.c_int32), ("max_admitted", C.c_int32), ("cache_hits", C.c_int64),
                ("peak_bytes", C.c_uint64), ("launch_s", C.c_double)]


_lib = None


def lib():
    """Load libnlq.so; fail loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2101_08825_amd/build.py "
                               "(there is no fallback implementation)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        P = C.POINTER
        sig = {
            "nlq_ctx_create": [i32, u64, P(vp)],
            "nlq_ctx_set_stream": [vp, vp],
            "nlq_ctx_memory": [vp, P(u64), P(u64)],
            "nlq_ctx_destroy": [vp],
            "nlq_mesh_create": [vp, i32, i64, vp, i64, vp, vp, P(vp)],
            "nlq_mesh_create_order": [vp, i32, i32, i64, vp, i64, vp, vp, P(vp)],
            "nlq_mesh_create_shape": [vp, i32, i32, i32, i64, vp, i64, vp, vp, P(vp)],
            "nlq_mesh_box": [vp, i32, i32, i32, P(vp)],
            "nlq_mesh_info": [vp, P(i32), P(i64), P(i64), P(i64)],
            "nlq_mesh_copy": [vp, vp, vp, vp],
            "nlq_mesh_destroy": [vp],
            "nlq_assemble": [vp, vp, P(nlq_params), P(vp)],
            "nlq_assemble_batch": [vp, i32, vp, vp, vp],
            "nlq_prepare": [vp, vp, P(nlq_params), P(vp)],
            "nlq_integrate_range": [vp, i64, i64, P(d), vp],
            "nlq_integrate_ranges": [vp, i32, vp, vp, P(d), vp, vp],
            "nlq_autotune": [vp, d, P(nlq_tune_info)],
            "nlq_tune_save": [vp, C.c_char_p],
            "nlq_tune_load": [vp, C.c_char_p, P(i32)],
            "nlq_assemble_info_get": [vp, P(nlq_assemble_info)],
            "nlq_reassemble": [vp],
            "nlq_set_data": [vp, vp, vp],
            "nlq_set_data_device": [vp, vp, vp],
            "nlq_solve": [vp, d, i32, vp, P(nlq_solve_info)],
            "nlq_solve_noalloc": [vp, d, i32, vp, P(nlq_solve_info)],
            "nlq_solution_device": [vp, P(vp)],
            "nlq_info": [vp, P(i64), P(i64), P(i64), P(i64)],
            "nlq_csr_copy": [vp, vp, vp, vp],
            "nlq_csr_device": [vp, P(vp), P(vp), P(vp)],
            "nlq_pairs_copy": [vp, vp, vp],
            "nlq_rhs_copy": [vp, vp],
            "nlq_pair_blocks": [vp, i64, vp, vp, vp],
            "nlq_system_destroy": [vp],
            "nlq_serve_start": [vp, P(nlq_serve_config)],
            "nlq_serve_stats_get": [vp, P(nlq_serve_stats)],
            "nlq_submit": [vp, P(nlq_request), P(u64)],
            "nlq_wait": [vp, u64, i32, P(nlq_result)],
            "nlq_cancel": [vp, u64],
            "nlq_result_release": [vp, u64],
            "nlq_serve_stop": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int32
        L.nlq_last_error.argtypes = []
        L.nlq_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(st):
    if st != NLQ_OK:
        raise NlqError(st, lib().nlq_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data


def params(dim, delta, eps, lmax, lmin=1, kernel=NLQ_ETA_CONST, form=NLQ_FORM_SYM4,
           precision=NLQ_FP64_PLAIN, scale=0.0, deterministic=False, min_dist_l2=0):
    return nlq_params(int(dim), int(kernel), float(delta), float(eps), float(scale), int(lmin),
                      int(lmax), int(form), int(precision), int(bool(deterministic)),
                      int(min_dist_l2))


class Context:
    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = C.c_void_p()
        _check(lib().nlq_ctx_create(device, hbm_budget_bytes, C.byref(h)))
        self.h = h
        self._meshes = weakref.WeakSet()

    def set_stream(self, hip_stream: int | None):
        _check(lib().nlq_ctx_set_stream(self.h, C.c_void_p(hip_stream or 0)))

    def memory(self):
        u, b = C.c_uint64(), C.c_uint64()
        _check(lib().nlq_ctx_memory(self.h, C.byref(u), C.byref(b)))
        return u.value, b.value

    def tune_save(self, path):
        """nlq_tune_save: write the context's tuned launch configurations."""
        _check(lib().nlq_tune_save(self.h, os.fsencode(path)))

    def tune_load(self, path):
        """nlq_tune_load: read tuned configurations of this device's architecture; returns their number."""
        n = C.c_int32()
        _check(lib().nlq_tune_load(self.h, os.fsencode(path), C.byref(n)))
        return n.value

    def close(self):
        """Destroy the context after every mesh (and system) made from it."""
        if self.h:
            for m in list(self._meshes):
                m.close()
            _check(lib().nlq_ctx_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Mesh:
    def __init__(self, ctx: Context, h, order: int = 1, shape: int = 0):
        self.ctx = ctx
        self.h = h
        self.order = order
        self.shape = shape
        self._systems = weakref.WeakSet()
        ctx._meshes.add(self)
        d, nn, ne, nf = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().nlq_mesh_info(h, C.byref(d), C.byref(nn), C.byref(ne), C.byref(nf)))
        self.dim, self.n_nodes, self.n_elems, self.n_free = d.value, nn.value, ne.value, nf.value
        # nodes per element: the vertices (corners), then (order 2) the edge midpoints
        if shape == NLQ_SHAPE_BOX:
            self.nb = (1 << self.dim) if order == 1 else (8 if self.dim == 2 else 20)
        else:
            self.nb = (self.dim + 1) if order == 1 else (self.dim + 1) * (self.dim + 2) // 2

    @classmethod
    def create(cls, ctx, coords, conn, constrained, order: int = 1, shape: int = 0):
        """Simplices (shape 0): P1 (order 1, conn [e][dim+1]) or P2 (order 2,
        conn [e][(dim+1)(dim+2)/2]: vertices, then the edge midpoints of edges
        (0,1),(0,2),... in lexicographic order).  Quadrilaterals / hexahedra
        (shape 1): Q1 (corners in tensor order) or serendipity (then the edge
        midpoints), see nlq_mesh_create_shape."""
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        cst = np.ascontiguousarray(constrained, dtype=np.uint8)
        h = C.c_void_p()
        _check(lib().nlq_mesh_create_shape(ctx.h, coords.shape[1], shape, order, coords.shape[0], _ptr(coords),
                                           conn.shape[0], _ptr(conn), _ptr(cst), C.byref(h)))
        return cls(ctx, h, order, shape)

    @classmethod
    def box(cls, ctx, dim, n, k_gamma):
        h = C.c_void_p()
        _check(lib().nlq_mesh_box(ctx.h, dim, n, k_gamma, C.byref(h)))
        return cls(ctx, h)

    def copy(self):
        coords = np.zeros((self.n_nodes, self.dim))
        conn = np.zeros((self.n_elems, self.nb), dtype=np.int32)
        cst = np.zeros(self.n_nodes, dtype=np.uint8)
        _check(lib().nlq_mesh_copy(self.h, _ptr(coords), _ptr(conn), _ptr(cst)))
        return coords, conn, cst

    def close(self):
        """Destroy the mesh after every system assembled on it."""
        if self.h:
            for s in list(self._systems):
                s.close()
            _check(lib().nlq_mesh_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            if self.ctx.h:
                self.close()
        except Exception:
            pass


class System:
    def __init__(self, ctx: Context, mesh: Mesh, prm: nlq_params, handle=None):
        h = handle
        if h is None:
            h = C.c_void_p()
            _check(lib().nlq_assemble(ctx.h, mesh.h, C.byref(prm), C.byref(h)))
        self.h = h
        self.ctx, self.mesh, self.prm = ctx, mesh, prm
        mesh._systems.add(self)

    @staticmethod
    def prepare(ctx: Context, mesh: Mesh, prm: nlq_params):
        """nlq_prepare: pair list and pattern only (values zero)."""
        h = C.c_void_p()
        _check(lib().nlq_prepare(ctx.h, mesh.h, C.byref(prm), C.byref(h)))
        return System(ctx, mesh, prm, handle=h)

    def integrate_range(self, lo, hi):
        """nlq_integrate_range: kernel seconds and leaf counts of outer elements [lo, hi)."""
        t = C.c_double()
        leaves = np.zeros(9, dtype=np.int64)
        _check(lib().nlq_integrate_range(self.h, int(lo), int(hi), C.byref(t), _ptr(leaves)))
        return t.value, leaves

    def integrate_ranges(self, lo, hi):
        """nlq_integrate_ranges: one launch over the disjoint outer-element ranges
        [lo[k], hi[k]); kernel seconds, leaf counts per level and the leaves not
        evaluated (all-zero integrals), summed over them."""
        lo_a = np.ascontiguousarray(lo, dtype=np.int64)
        hi_a = np.ascontiguousarray(hi, dtype=np.int64)
        if lo_a.shape != hi_a.shape or lo_a.ndim != 1:
            raise ValueError("lo and hi must be 1-D of one length")
        t = C.c_double()
        leaves = np.zeros(9, dtype=np.int64)
        zero = np.zeros(1, dtype=np.int64)
        _check(lib().nlq_integrate_ranges(self.h, int(lo_a.shape[0]), _ptr(lo_a), _ptr(hi_a), C.byref(t),
                                          _ptr(leaves), _ptr(zero)))
        return t.value, leaves, int(zero[0])

    @staticmethod
    def batch(ctx: Context, meshes, prms):
        """nlq_assemble_batch: systems whose integrations share launches."""
        n = len(meshes)
        mh = (C.c_void_p * n)(*[m.h.value for m in meshes])
        pa = (nlq_params * n)(*prms)
        out = (C.c_void_p * n)()
        _check(lib().nlq_assemble_batch(ctx.h, n, mh, pa, out))
        return [System(ctx, meshes[i], prms[i], handle=C.c_void_p(out[i])) for i in range(n)]

    def info(self):
        i = nlq_assemble_info()
        _check(lib().nlq_assemble_info_get(self.h, C.byref(i)))
        return i

    def sizes(self):
        a, b, c, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().nlq_info(self.h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return dict(n_rows=a.value, nnz=b.value, n_pairs=c.value, n_free=d.value)

    def reassemble(self):
        _check(lib().nlq_reassemble(self.h))

    def autotune(self, budget_s=2.0):
        """nlq_autotune: choose the integration launch configuration (values are recomputed)."""
        t = nlq_tune_info()
        _check(lib().nlq_autotune(self.h, float(budget_s), C.byref(t)))
        return {k: getattr(t, k) for k, _ in nlq_tune_info._fields_}

    def set_data(self, f_nodal, g_nodal):
        f = np.ascontiguousarray(f_nodal, dtype=np.float64)
        g = np.ascontiguousarray(g_nodal, dtype=np.float64)
        _check(lib().nlq_set_data(self.h, _ptr(f), _ptr(g)))

    def set_data_device(self, f_ptr: int, g_ptr: int):
        """f, g as device pointers (e.g. torch.Tensor.data_ptr() of float64 tensors)."""
        _check(lib().nlq_set_data_device(self.h, C.c_void_p(f_ptr), C.c_void_p(g_ptr)))

    def solve(self, rtol=1e-12, maxit=20000, copy=True):
        u = np.zeros(self.mesh.n_nodes) if copy else None
        inf = nlq_solve_info()
        st = lib().nlq_solve(self.h, float(rtol), int(maxit), _ptr(u), C.byref(inf))
        if st not in (NLQ_OK, NLQ_ENOCONV):
            _check(st)
        return u, inf

    def solve_noalloc(self, u_dev_ptr: int, rtol=1e-12, maxit=20000):
        """nlq_solve_noalloc: the solve without any device allocation; u is
        written to the caller's device buffer u_dev_ptr [n_nodes] (e.g. the
        data_ptr() of a float64 torch tensor)."""
        inf = nlq_solve_info()
        st = lib().nlq_solve_noalloc(self.h, float(rtol), int(maxit), C.c_void_p(u_dev_ptr), C.byref(inf))
        if st not in (NLQ_OK, NLQ_ENOCONV):
            _check(st)
        return inf

    def solution_device(self) -> int:
        p = C.c_void_p()
        _check(lib().nlq_solution_device(self.h, C.byref(p)))
        return p.value or 0

    def csr(self):
        s = self.sizes()
        rp = np.zeros(s["n_rows"] + 1, dtype=np.int64)
        col = np.zeros(s["nnz"], dtype=np.int32)
        val = np.zeros(s["nnz"])
        _check(lib().nlq_csr_copy(self.h, _ptr(rp), _ptr(col), _ptr(val)))
        return rp, col, val

    def csr_device(self):
        rp, col, val = C.c_void_p(), C.c_void_p(), C.c_void_p()
        _check(lib().nlq_csr_device(self.h, C.byref(rp), C.byref(col), C.byref(val)))
        return rp.value, col.value, val.value

    def pairs(self):
        s = self.sizes()
        off = np.zeros(self.mesh.n_elems + 1, dtype=np.int64)
        pm = np.zeros(max(s["n_pairs"], 1), dtype=np.int32)
        _check(lib().nlq_pairs_copy(self.h, _ptr(off), _ptr(pm)))
        return off, pm[:s["n_pairs"]]

    def rhs(self):
        out = np.zeros(self.mesh.n_nodes)
        _check(lib().nlq_rhs_copy(self.h, _ptr(out)))
        return out

    def pair_blocks(self, l, m):
        l = np.ascontiguousarray(l, dtype=np.int32)
        m = np.ascontiguousarray(m, dtype=np.int32)
        n2 = 2 * self.mesh.nb
        out = np.zeros((l.shape[0], n2, n2))
        _check(lib().nlq_pair_blocks(self.h, l.shape[0], _ptr(l), _ptr(m), _ptr(out)))
        return out

    def close(self):
        if self.h:
            _check(lib().nlq_system_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            if self.mesh.h and self.ctx.h:
                self.close()
        except Exception:
            pass


class Server:
    """Serving loop of a context (nlq_serve_*): requests on Kuhn box meshes."""

    def __init__(self, ctx: Context, max_active=0, target_launch_ms=0.0, cache_systems=False):
        cfg = nlq_serve_config(int(max_active), float(target_launch_ms), int(bool(cache_systems)))
        _check(lib().nlq_serve_start(ctx.h, C.byref(cfg)))
        self.ctx = ctx
        self.running = True

    def submit(self, dim, n, k_gamma, prm: nlq_params, f_nodal, g_nodal, rtol=1e-10, maxit=10000) -> int:
        f = np.ascontiguousarray(f_nodal, dtype=np.float64)
        g = np.ascontiguousarray(g_nodal, dtype=np.float64)
        if f.shape[0] != (n + 1) ** dim or g.shape[0] != (n + 1) ** dim:
            raise ValueError("f and g need (n+1)^dim nodal values")
        req = nlq_request(int(dim), int(n), int(k_gamma), prm, f.ctypes.data, g.ctypes.data,
                          float(rtol), int(maxit))
        t = C.c_uint64()
        _check(lib().nlq_submit(self.ctx.h, C.byref(req), C.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1, release: bool = True):
        """Result dict (u copied) or None on timeout."""
        r = nlq_result()
        st = lib().nlq_wait(self.ctx.h, C.c_uint64(ticket), int(timeout_ms), C.byref(r))
        if st == NLQ_ENOTREADY:
            return None
        _check(st)
        u = None
        if r.u:
            u = np.ctypeslib.as_array(r.u, shape=(r.n_nodes,)).copy()
        out = dict(status=r.status, error=(lib().nlq_last_error().decode() if r.status else ""),
                   n_nodes=r.n_nodes, n_pairs=r.n_pairs, n_free=r.n_free, u=u,
                   cg_iterations=r.cg_iterations, rel_residual=r.rel_residual,
                   latency_s=r.latency_s, queue_s=r.queue_s, assemble_s=r.assemble_s,
                   solve_s=r.solve_s, launches=r.launches, cache_hit=bool(r.cache_hit), setup_s=r.setup_s)
        if release:
            _check(lib().nlq_result_release(self.ctx.h, C.c_uint64(ticket)))
        return out

    def cancel(self, ticket: int):
        _check(lib().nlq_cancel(self.ctx.h, C.c_uint64(ticket)))

    def stats(self):
        s = nlq_serve_stats()
        _check(lib().nlq_serve_stats_get(self.ctx.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in nlq_serve_stats._fields_}

    def stop(self):
        if self.running:
            _check(lib().nlq_serve_stop(self.ctx.h))
            self.running = False
