"""ctypes wrapper of the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py.  The library under test never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no FMA contraction)."""
    stale = (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class _Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_nodes", C.c_int64), ("n_elems", C.c_int64),
                ("coords", C.c_void_p), ("conn", C.c_void_p), ("order", C.c_int32),
                ("shape", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("delta", C.c_double), ("eps", C.c_double), ("scale", C.c_double),
                ("kernel", C.c_int32), ("lmin", C.c_int32), ("lmax", C.c_int32),
                ("form", C.c_int32), ("min_l2", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        d, i32, i64, vp = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        L.or_xi.restype = d
        L.or_xi.argtypes = [d]
        L.or_mu.restype = d
        L.or_mu.argtypes = [d, d, d]
        L.or_kernel_constant.restype = d
        L.or_kernel_constant.argtypes = [i32, i32, d, d]
        L.or_rule.restype = i32
        L.or_rule.argtypes = [i32, vp, vp]
        L.or_children.restype = None
        L.or_children.argtypes = [i32, vp, vp]
        L.or_box_rule.restype = i32
        L.or_box_rule.argtypes = [i32, vp, vp]
        L.or_box_basis.restype = None
        L.or_box_basis.argtypes = [i32, i32, vp, vp]
        L.or_box_children.restype = None
        L.or_box_children.argtypes = [i32, vp, vp]
        L.or_aprxmax.restype = d
        L.or_aprxmax.argtypes = [i32, vp, vp, vp, vp]
        L.or_aprxmin.restype = d
        L.or_aprxmin.argtypes = [i32, vp, vp, vp, vp]
        L.or_elem_measure.restype = d
        L.or_elem_measure.argtypes = [vp, i64]
        L.or_pairs.restype = i64
        L.or_pairs.argtypes = [vp, d, i32, vp, vp]
        L.or_pairs_of.restype = i64
        L.or_pairs_of.argtypes = [vp, d, i64, vp]
        L.or_pattern.restype = i64
        L.or_pattern.argtypes = [vp, vp, vp, vp, vp]
        L.or_pair_block.restype = i32
        L.or_pair_block.argtypes = [vp, vp, i64, i64, vp, vp, vp]
        L.or_assemble.restype = i32
        L.or_assemble.argtypes = [vp, vp, i32, vp, vp, i64, vp, vp, vp, vp, vp, vp]
        L.or_leaf_counts.restype = None
        L.or_leaf_counts.argtypes = [vp, vp, i32, i64, vp, vp]
        L.or_outer_blocks.restype = d
        L.or_outer_blocks.argtypes = [vp, vp, i32, i64, vp, vp, vp]
        L.or_rows.restype = i64
        L.or_rows.argtypes = [vp, vp, d, i32, i64, vp, vp, vp, vp]
        L.or_load.restype = None
        L.or_load.argtypes = [vp, vp, vp, vp]
        L.or_lift.restype = None
        L.or_lift.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp]
        L.or_cg.restype = i32
        L.or_cg.argtypes = [i64, vp, vp, vp, vp, vp, d, i32, vp, vp]
        L.or_lu_solve.restype = i32
        L.or_lu_solve.argtypes = [i64, vp, vp, vp, vp, vp, vp]
        L.or_cholesky_solve.restype = i32
        L.or_cholesky_solve.argtypes = [i64, vp, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data if a is not None else None


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


class OracleMesh:
    """Holds the arrays alive for the C struct."""

    def __init__(self, coords, conn, order=1, shape=0):
        """shape 0: simplices (P1 / P2); shape 1: quadrilaterals / hexahedra
        (Q1 / serendipity), corners in tensor order, then the edge midpoints."""
        self.coords = np.ascontiguousarray(coords, dtype=np.float64)
        self.conn = np.ascontiguousarray(conn, dtype=np.int32)
        self.dim = int(self.coords.shape[1])
        self.order = int(order)
        self.shape = int(shape)
        if self.shape:
            nb = (8 if self.dim == 2 else 20) if self.order == 2 else 1 << self.dim
        else:
            nb = (self.dim + 1) * (self.dim + 2) // 2 if self.order == 2 else self.dim + 1
        if self.conn.shape[1] != nb:
            raise ValueError(f"order {order} elements need {nb} nodes, conn has {self.conn.shape[1]}")
        self.nb = nb
        self.s = _Mesh(self.dim, self.coords.shape[0], self.conn.shape[0],
                       self.coords.ctypes.data, self.conn.ctypes.data, self.order, self.shape)

    @property
    def ref(self):
        return C.byref(self.s)


def params(delta, eps, lmax, lmin=1, kernel=0, form=0, scale=0.0, min_l2=0):
    return _Params(float(delta), float(eps), float(scale), int(kernel), int(lmin),
                   int(lmax), int(form), int(min_l2))


# ------------------------------------------------------------------ scalars

def xi(r: float) -> float:
    return lib().or_xi(float(r))


def mu(d: float, delta: float, eps: float) -> float:
    return lib().or_mu(float(d), float(delta), float(eps))


def kernel_constant(dim, kernel, delta, eps) -> float:
    return lib().or_kernel_constant(int(dim), int(kernel), float(delta), float(eps))


def rule(dim):
    bary = np.zeros((15, 4))
    w = np.zeros(15)
    n = lib().or_rule(int(dim), _p(bary), _p(w))
    return bary.reshape(-1)[: n * (dim + 1)].reshape(n, dim + 1).copy(), w[:n].copy()


def box_rule(dim):
    xi = np.zeros((27, 3))
    w = np.zeros(27)
    n = lib().or_box_rule(int(dim), _p(xi), _p(w))
    return xi.reshape(-1)[: n * dim].reshape(n, dim).copy(), w[:n].copy()


def box_basis(dim, order, xi):
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    nb = (8 if dim == 2 else 20) if order == 2 else 1 << dim
    phi = np.zeros(nb)
    lib().or_box_basis(int(dim), int(order), _p(xi), _p(phi))
    return phi


def box_children(P: np.ndarray) -> np.ndarray:
    P = np.ascontiguousarray(P, dtype=np.float64)
    dim = P.shape[1]
    out = np.zeros((1 << dim, 1 << dim, dim))
    lib().or_box_children(dim, _p(P), _p(out))
    return out


def children(v: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64)
    dim = v.shape[1]
    out = np.zeros((1 << dim, dim + 1, dim))
    lib().or_children(dim, _p(v), _p(out))
    return out


def aprxmax(lo1, hi1, lo2, hi2) -> float:
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (lo1, hi1, lo2, hi2)]
    return lib().or_aprxmax(len(a[0]), *[_p(x) for x in a])


def aprxmin(lo1, hi1, lo2, hi2) -> float:
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (lo1, hi1, lo2, hi2)]
    return lib().or_aprxmin(len(a[0]), *[_p(x) for x in a])


# ------------------------------------------------------------------ mesh level

def pairs(mesh: OracleMesh, thr: float, nthreads: int | None = None):
    nt = nthreads or default_threads()
    ne = mesh.conn.shape[0]
    off = np.zeros(ne + 1, dtype=np.int64)
    total = lib().or_pairs(mesh.ref, float(thr), nt, _p(off), None)
    pm = np.zeros(max(total, 1), dtype=np.int32)
    lib().or_pairs(mesh.ref, float(thr), nt, _p(off), _p(pm))
    return off, pm[:total]


def pairs_of(mesh: OracleMesh, thr: float, l: int):
    out = np.zeros(mesh.conn.shape[0], dtype=np.int32)
    n = lib().or_pairs_of(mesh.ref, float(thr), int(l), _p(out))
    return out[:n].copy()


def pattern(mesh: OracleMesh, off, pm):
    nn = mesh.coords.shape[0]
    row_ptr = np.zeros(nn + 1, dtype=np.int64)
    nnz = lib().or_pattern(mesh.ref, _p(off), _p(pm), _p(row_ptr), None)
    col = np.zeros(max(nnz, 1), dtype=np.int32)
    lib().or_pattern(mesh.ref, _p(off), _p(pm), _p(row_ptr), _p(col))
    return row_ptr, col[:nnz]


def pair_block(mesh: OracleMesh, prm, l: int, m: int, lmax: int | None = None):
    ne2 = 2 * mesh.nb
    E = np.zeros((ne2, ne2))
    leaves = np.zeros(16, dtype=np.int64)
    evals = np.zeros(2, dtype=np.int64)
    lib().or_pair_block(mesh.ref, C.byref(prm), int(l), int(m), _p(E), _p(leaves), _p(evals))
    return E, leaves, evals


def assemble(mesh: OracleMesh, prm, off, pm, row_ptr, col, sel=None, nthreads=None):
    nt = nthreads or default_threads()
    val = np.zeros(col.shape[0])
    leaves = np.zeros(16, dtype=np.int64)
    evals = np.zeros(2, dtype=np.int64)
    sel_a = None if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    st = lib().or_assemble(mesh.ref, C.byref(prm), nt, _p(off), _p(pm),
                           0 if sel_a is None else sel_a.shape[0], _p(sel_a),
                           _p(row_ptr), _p(col), _p(val), _p(leaves), _p(evals))
    if st != 0:
        raise RuntimeError("oracle assembly: entry outside the pattern")
    return val, leaves, evals


def leaf_counts(mesh: OracleMesh, prm, outer, nthreads=None):
    """Leaf integrations per level (index = level) of Algorithm 1 for the outer
    elements `outer`, counted without evaluating them."""
    nt = nthreads or default_threads()
    sel = np.ascontiguousarray(outer, dtype=np.int64)
    leaves = np.zeros(16, dtype=np.int64)
    lib().or_leaf_counts(mesh.ref, C.byref(prm), nt, sel.shape[0], _p(sel), _p(leaves))
    return leaves


def outer_blocks(mesh: OracleMesh, prm, outer, nthreads=None):
    """Algorithm 1 with evaluation for the outer elements `outer` (each with its
    brute-force J_l), blocks discarded; returns (leaves, evals, checksum)."""
    nt = nthreads or default_threads()
    sel = np.ascontiguousarray(outer, dtype=np.int64)
    leaves = np.zeros(16, dtype=np.int64)
    evals = np.zeros(2, dtype=np.int64)
    cs = lib().or_outer_blocks(mesh.ref, C.byref(prm), nt, sel.shape[0], _p(sel), _p(leaves), _p(evals))
    return leaves, evals, cs


def rows(mesh: OracleMesh, prm, thr, row_ids, values=True, nthreads=None):
    """Pattern (and values) of selected rows; returns list of (cols, vals)."""
    nt = nthreads or default_threads()
    r = np.ascontiguousarray(row_ids, dtype=np.int64)
    rl = np.zeros(r.shape[0], dtype=np.int64)
    total = lib().or_rows(mesh.ref, C.byref(prm), float(thr), nt, r.shape[0], _p(r), _p(rl),
                          None, None)
    cols = np.zeros(max(total, 1), dtype=np.int32)
    vals = np.zeros(max(total, 1)) if values else None
    lib().or_rows(mesh.ref, C.byref(prm), float(thr), nt, r.shape[0], _p(r), _p(rl),
                  _p(cols), _p(vals))
    out = []
    o = 0
    for k in range(r.shape[0]):
        n = int(rl[k])
        out.append((cols[o:o + n].copy(), None if vals is None else vals[o:o + n].copy()))
        o += n
    return out


def load(mesh: OracleMesh, f_nodal, constrained):
    F = np.zeros(mesh.coords.shape[0])
    f = np.ascontiguousarray(f_nodal, dtype=np.float64)
    cst = np.ascontiguousarray(constrained, dtype=np.uint8)
    lib().or_load(mesh.ref, _p(f), _p(cst), _p(F))
    return F


def lift(row_ptr, col, val, constrained, g, F):
    n = row_ptr.shape[0] - 1
    Ft = np.zeros(n)
    cst = np.ascontiguousarray(constrained, dtype=np.uint8)
    gg = np.ascontiguousarray(g, dtype=np.float64)
    FF = np.ascontiguousarray(F, dtype=np.float64)
    lib().or_lift(n, _p(row_ptr), _p(col), _p(val), _p(cst), _p(gg), _p(FF), _p(Ft))
    return Ft


def cg(row_ptr, col, val, constrained, rhs, rtol=1e-14, maxit=20000):
    n = row_ptr.shape[0] - 1
    w = np.zeros(n)
    rel = np.zeros(1)
    cst = np.ascontiguousarray(constrained, dtype=np.uint8)
    b = np.ascontiguousarray(rhs, dtype=np.float64)
    it = lib().or_cg(n, _p(row_ptr), _p(col), _p(val), _p(cst), _p(b), float(rtol), int(maxit),
                     _p(w), _p(rel))
    return w, int(it), float(rel[0])


def cholesky_solve(row_ptr, col, val, constrained, rhs):
    n = row_ptr.shape[0] - 1
    w = np.zeros(n)
    cst = np.ascontiguousarray(constrained, dtype=np.uint8)
    b = np.ascontiguousarray(rhs, dtype=np.float64)
    st = lib().or_cholesky_solve(n, _p(row_ptr), _p(col), _p(val), _p(cst), _p(b), _p(w))
    if st != 0:
        raise RuntimeError(f"cholesky failed ({st})")
    return w


def lu_solve(row_ptr, col, val, constrained, rhs):
    """Dense LU with partial pivoting on the free block (non-symmetric matrices)."""
    n = row_ptr.shape[0] - 1
    w = np.zeros(n)
    cst = np.ascontiguousarray(constrained, dtype=np.uint8)
    b = np.ascontiguousarray(rhs, dtype=np.float64)
    st = lib().or_lu_solve(n, _p(row_ptr), _p(col), _p(val), _p(cst), _p(b), _p(w))
    if st != 0:
        raise RuntimeError(f"lu failed ({st})")
    return w


class Solution:
    pass


def solve_problem(mesh_arrays, prm, f_nodal, g_nodal, rtol=1e-14, nthreads=None,
                  direct=False, order=1, shape=0):
    """Full oracle pipeline: pairs, pattern, assembly, load, lifting, solve."""
    coords, conn, constrained = mesh_arrays
    m = OracleMesh(coords, conn, order, shape)
    thr = prm.delta + prm.eps
    s = Solution()
    s.off, s.pm = pairs(m, thr, nthreads)
    s.row_ptr, s.col = pattern(m, s.off, s.pm)
    s.val, s.leaves, s.evals = assemble(m, prm, s.off, s.pm, s.row_ptr, s.col,
                                        nthreads=nthreads)
    s.F = load(m, f_nodal, constrained)
    s.Ft = lift(s.row_ptr, s.col, s.val, constrained, g_nodal, s.F)
    if prm.form != 0:
        # the two-term forms are not symmetric: Gaussian elimination (CG does not apply)
        w = lu_solve(s.row_ptr, s.col, s.val, constrained, s.Ft)
        s.iters, s.relres = 0, 0.0
    elif direct:
        w = cholesky_solve(s.row_ptr, s.col, s.val, constrained, s.Ft)
        s.iters, s.relres = 0, 0.0
    else:
        w, s.iters, s.relres = cg(s.row_ptr, s.col, s.val, constrained, s.Ft, rtol)
    cst = np.asarray(constrained, dtype=bool)
    s.u = np.where(cst, g_nodal, w)
    s.mesh = m
    return s
