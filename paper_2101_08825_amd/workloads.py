"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

This module generates problem *inputs* only: meshes, constrained-node flags,
manufactured solutions sampled at the nodes, and the serving request stream.
It holds none of the method's arithmetic (no kernel, quadrature, pair test,
refinement or assembly), so both the library under test and the oracle can
consume the same arrays without sharing any computation.

Mesh layout (Kuhn / Freudenthal split of the unit cube into simplices):
  * nodes x = (i0/n, i1/n[, i2/n]) with one correctly rounded FP64 division;
    node id = i0 + (n+1)*(i1 + (n+1)*i2);
  * cell id = c0 + n*(c1 + n*c2);
  * element id = (#permutations)*cell + p, where p enumerates the
    permutations pi of {0..N-1} in lexicographic order and the vertices follow
    the Kuhn path v0 = cell origin, v_{k+1} = v_k + e_{pi(k)}.
Every simplex contains the cell diagonal, so its bounding box is its cell.

The interaction layer Gamma (Section 2, eq. interaction-domain) of a box mesh is
the closed layer of width K cells at the boundary of [0,1]^N: a node is
constrained when some index i_k <= K or i_k >= n - K.  The mesh covers
Omega u Gamma; Omega is the open interior.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    dim: int
    n: int                      # cells per direction
    coords: np.ndarray          # [n_nodes, dim] float64
    conn: np.ndarray            # [n_elems, dim+1] int32
    constrained: np.ndarray     # [n_nodes] uint8, 1 = node in Gamma
    k_gamma: int                # width of Gamma in cells

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[0])

    @property
    def h(self) -> float:
        return 1.0 / self.n


def kuhn_mesh(dim: int, n: int, k_gamma: int) -> Mesh:
    """Kuhn simplicial mesh of [0,1]^dim with n cells per direction."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    if n < 1 or k_gamma < 0:
        raise ValueError("bad mesh size")
    nn = n + 1
    idx = np.arange(nn, dtype=np.int64)
    if dim == 2:
        i1, i0 = np.meshgrid(idx, idx, indexing="ij")
        ii = [i0.ravel(), i1.ravel()]
    else:
        i2, i1, i0 = np.meshgrid(idx, idx, idx, indexing="ij")
        ii = [i0.ravel(), i1.ravel(), i2.ravel()]
    coords = np.stack([k.astype(np.float64) / float(n) for k in ii], axis=1)
    constrained = np.zeros(coords.shape[0], dtype=np.uint8)
    for k in ii:
        constrained |= ((k <= k_gamma) | (k >= n - k_gamma)).astype(np.uint8)

    perms = list(itertools.permutations(range(dim)))
    cidx = np.arange(n, dtype=np.int64)
    if dim == 2:
        c1, c0 = np.meshgrid(cidx, cidx, indexing="ij")
        cc = [c0.ravel(), c1.ravel()]
    else:
        c2, c1, c0 = np.meshgrid(cidx, cidx, cidx, indexing="ij")
        cc = [c0.ravel(), c1.ravel(), c2.ravel()]
    n_cells = cc[0].shape[0]
    conn = np.zeros((n_cells, len(perms), dim + 1), dtype=np.int64)

    def node_id(v):
        out = v[0].copy()
        mul = nn
        for k in range(1, dim):
            out += mul * v[k]
            mul *= nn
        return out

    for p, pi in enumerate(perms):
        v = [c.copy() for c in cc]
        conn[:, p, 0] = node_id(v)
        for k in range(dim):
            v[pi[k]] = v[pi[k]] + 1
            conn[:, p, k + 1] = node_id(v)
    conn = conn.reshape(n_cells * len(perms), dim + 1).astype(np.int32)
    return Mesh(dim=dim, n=n, coords=coords, conn=conn,
                constrained=constrained, k_gamma=k_gamma)


def kuhn_mesh_p2(dim: int, n: int, k_gamma: int) -> Mesh:
    """The Kuhn mesh of `kuhn_mesh` with P2 Lagrange elements: nodes on the grid of
    spacing h/2, x = i/(2n) (one correctly rounded FP64 division), node id =
    i0 + (2n+1)(i1 + (2n+1) i2); element e has the vertices of the P1 element e
    (at even grid indices) followed by its edge midpoints in the order (0,1),
    (0,2), (1,2) [2D] or (0,1), (0,2), (0,3), (1,2), (1,3), (2,3) [3D].  A node
    is constrained when some index i_k <= 2K or i_k >= 2n - 2K (the same layer of
    K cells)."""
    p1 = kuhn_mesh(dim, n, k_gamma)
    nn = 2 * n + 1
    idx = np.arange(nn, dtype=np.int64)
    if dim == 2:
        i1, i0 = np.meshgrid(idx, idx, indexing="ij")
        ii = [i0.ravel(), i1.ravel()]
    else:
        i2, i1, i0 = np.meshgrid(idx, idx, idx, indexing="ij")
        ii = [i0.ravel(), i1.ravel(), i2.ravel()]
    coords = np.stack([k.astype(np.float64) / float(2 * n) for k in ii], axis=1)
    constrained = np.zeros(coords.shape[0], dtype=np.uint8)
    for k in ii:
        constrained |= ((k <= 2 * k_gamma) | (k >= 2 * n - 2 * k_gamma)).astype(np.uint8)
    # P1 node id -> fine grid index vector (even entries)
    p1_idx = np.stack(np.unravel_index(np.arange(p1.n_nodes), [n + 1] * dim, order="F"), axis=1) * 2
    fine = lambda v: sum(v[..., k] * nn ** k for k in range(dim))
    V = p1_idx[p1.conn]                       # [e, nv, dim] fine indices of the vertices
    nv = dim + 1
    cols = [fine(V[:, i, :]) for i in range(nv)]
    for i in range(nv):
        for j in range(i + 1, nv):
            cols.append(fine((V[:, i, :] + V[:, j, :]) // 2))
    conn = np.stack(cols, axis=1).astype(np.int32)
    return Mesh(dim=dim, n=n, coords=coords, conn=conn, constrained=constrained, k_gamma=k_gamma)


def jittered_mesh(dim: int, n: int, k_gamma: int, frac: float = 0.2, seed: int = 0) -> Mesh:
    """The Kuhn mesh of `kuhn_mesh` with every node that is not on the boundary of
    [0,1]^dim moved by independent U(-frac h, frac h) offsets per coordinate
    (seeded PCG64): a general simplicial mesh whose element boxes are no longer
    its cells.  Connectivity and constrained flags are those of the Kuhn mesh.
    frac <= 0.2 keeps every simplex positively oriented: the smallest height of a
    Kuhn simplex is h / sqrt(2), and each of its vertices moves by at most
    frac h sqrt(dim)."""
    m = kuhn_mesh(dim, n, k_gamma)
    rng = np.random.default_rng(seed)
    off = rng.uniform(-frac, frac, size=m.coords.shape) / float(n)
    inner = np.all((m.coords > 0.0) & (m.coords < 1.0), axis=1)
    coords = m.coords.copy()
    coords[inner] += off[inner]
    return Mesh(dim=dim, n=n, coords=coords, conn=m.conn, constrained=m.constrained,
                k_gamma=k_gamma)


def box_mesh(dim: int, n: int, k_gamma: int, order: int = 1, frac: float = 0.0, seed: int = 0,
             cells=None) -> Mesh:
    """Structured mesh of squares / cubes of side h = 1/n, n cells per axis
    ([0,1]^dim) or cells[k] along axis k ([0, cells[k]/n] per axis), cell id
    c0 + n0*(c1 + n1*c2), quadrilateral or hexahedral elements.
      * order 1 (Q1): nodes x = i/n (one correctly rounded FP64 division), node id
        i0 + (n+1)*(i1 + (n+1)*i2); element nodes = the cell's corners in tensor
        order (corner c = c0 + 2 c1 + 4 c2 at offset (c0, c1, c2));
      * order 2 (serendipity, 8 / 20 nodes): nodes on the half grid x = j/(2n),
        j_k in 0..2n, with at most one odd j_k (no face or cell centres), ids in
        increasing j0 + (2n+1)*(j1 + (2n+1)*j2); element nodes = the corners in
        tensor order, then the edge midpoints in increasing t0 + 3 t1 + 9 t2 of
        their offset t in half cells (exactly one t_k = 1).
    (With cells given, the strides n+1 / 2n+1 above are cells[k]+1 / 2 cells[k]+1
    per axis and the coordinates i/n, j/(2n) run to cells[k]/n.)
    A node is constrained when some coordinate index lies in the layer of K =
    k_gamma cells (i_k <= K or >= n_k - K; half-grid j_k <= 2K or >= 2n_k - 2K).
    frac > 0 moves every corner node not on the boundary of [0,1]^dim by
    independent U(-frac h, frac h) offsets per coordinate (seeded PCG64), giving
    non-affine (bilinear / trilinear) elements; edge midpoints are then placed
    at the midpoints of their moved corners (straight edges)."""
    if dim not in (2, 3) or order not in (1, 2):
        raise ValueError("dim must be 2 or 3, order 1 or 2")
    if n < 1 or k_gamma < 0:
        raise ValueError("bad mesh size")
    rng = np.random.default_rng(seed)
    nc = [int(c) for c in cells] if cells is not None else [n] * dim
    s = 2 if order == 2 else 1          # grid steps per cell
    ngk = [s * c + 1 for c in nc]
    grid = np.array(list(itertools.product(*[range(g) for g in ngk[::-1]])))[:, ::-1]   # j0 fastest
    if order == 2:
        keep = (grid % 2 == 1).sum(axis=1) <= 1
        grid = grid[keep]
    stride = [int(np.prod(ngk[:k])) for k in range(dim)]
    key = sum(grid[:, k].astype(np.int64) * stride[k] for k in range(dim))
    ident = -np.ones(int(np.prod(ngk)), dtype=np.int64)
    ident[key] = np.arange(grid.shape[0])
    coords = grid.astype(np.float64) / float(s * n)
    constrained = np.zeros(grid.shape[0], dtype=np.uint8)
    for k in range(dim):
        constrained |= ((grid[:, k] <= s * k_gamma) | (grid[:, k] >= s * (nc[k] - k_gamma))).astype(np.uint8)
    cells_ = np.array(list(itertools.product(*[range(c) for c in nc[::-1]])))[:, ::-1]     # c0 fastest
    offsets = [tuple(2 * ((c >> k) & 1) for k in range(dim)) for c in range(1 << dim)]
    if order == 2:
        offsets += [t for t in (tuple((q // 3 ** k) % 3 for k in range(dim)) for q in range(3 ** dim))
                    if sum(x == 1 for x in t) == 1]
    cols = []
    for t in offsets:
        j = cells_ * s + np.array(t) * s // 2
        cols.append(ident[sum(j[:, k].astype(np.int64) * stride[k] for k in range(dim))])
    conn = np.stack(cols, axis=1).astype(np.int32)
    if frac > 0.0:
        off = rng.uniform(-frac, frac, size=coords.shape) / float(n)
        even = np.all(grid % s == 0, axis=1)
        inner = np.all((grid > 0) & (grid < np.array(ngk) - 1), axis=1) & even
        coords[inner] += off[inner]
        if order == 2:
            for e_col in range(1 << dim, conn.shape[1]):
                t = np.array(offsets[e_col])
                ax = int(np.argmax(t == 1))
                a = t.copy()
                b = t.copy()
                a[ax], b[ax] = 0, 2
                ca = conn[:, offsets.index(tuple(int(x) for x in a))]
                cb = conn[:, offsets.index(tuple(int(x) for x in b))]
                coords[conn[:, e_col]] = (coords[ca] + coords[cb]) * 0.5
    return Mesh(dim=dim, n=n, coords=coords, conn=conn, constrained=constrained, k_gamma=k_gamma)


def stratified_ranges(n_elems: int, fraction: float, n_strata: int = 32, seed: int = 0):
    """A seeded sample of about `fraction` of the outer elements spread over the
    whole mesh: the ids 1..n_elems-2 cut into n_strata equal strata, one run of
    round(fraction * stratum) consecutive ids at a seeded position in each.
    Returns (lo, hi) arrays of the runs [lo_k, hi_k) (0 < lo_k < hi_k < n_elems)."""
    rng = np.random.default_rng(seed)
    first, last = 1, n_elems - 1          # usable ids [first, last)
    edges = np.linspace(first, last, n_strata + 1).astype(np.int64)
    lo, hi = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        run = max(1, int(round(fraction * (b - a))))
        run = min(run, int(b - a))
        start = int(a + rng.integers(0, b - a - run + 1))
        lo.append(start)
        hi.append(start + run)
    return np.array(lo, dtype=np.int64), np.array(hi, dtype=np.int64)


# ---------------------------------------------------------------------------
# Manufactured data.  A quadratic u = sum a_k x_k^2 + sum_{k<l} b_kl x_k x_l
# + c.x + d has Laplacian 2*sum a_k; f = -Laplacian(u) is then constant.
# ---------------------------------------------------------------------------
@dataclass
class Quadratic:
    a: np.ndarray                       # [dim]
    b: np.ndarray = field(default=None)  # [dim, dim] strictly upper part used
    c: np.ndarray = field(default=None)  # [dim]
    d: float = 0.0

    def __post_init__(self):
        dim = len(self.a)
        if self.b is None:
            self.b = np.zeros((dim, dim))
        if self.c is None:
            self.c = np.zeros(dim)

    def __call__(self, x: np.ndarray) -> np.ndarray:
        dim = x.shape[1]
        out = np.full(x.shape[0], float(self.d))
        for k in range(dim):
            out += self.a[k] * x[:, k] * x[:, k] + self.c[k] * x[:, k]
            for l in range(k + 1, dim):
                out += self.b[k, l] * x[:, k] * x[:, l]
        return out

    def laplacian(self) -> float:
        return float(2.0 * np.sum(self.a))


def nodal_data(mesh: Mesh, u: Quadratic):
    """Nodal u (exact solution), f = -Laplacian(u) and g = u (read on Gamma)."""
    uu = u(mesh.coords)
    f = np.full(mesh.n_nodes, -u.laplacian())
    return uu, f, uu.copy()


# ---------------------------------------------------------------------------
# Workload configurations (sizes of the paper-shaped problems).
# ---------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    dim: int
    n: int
    k_delta: int            # delta = k_delta * h
    eps_div: int            # eps = delta / eps_div
    lmax: int
    kernel: int             # 0 = constant eta, 1 = truncated Gaussian eta
    u: Quadratic
    shape: int = 0          # 0: Kuhn simplices; 1: squares / cubes (box_mesh)
    order: int = 1          # 1: P1 / Q1; 2: P2 / serendipity

    @property
    def h(self) -> float:
        return 1.0 / self.n

    @property
    def delta(self) -> float:
        return self.k_delta / self.n

    @property
    def eps(self) -> float:
        return self.delta / self.eps_div

    def mesh(self) -> Mesh:
        if self.shape == 1:
            return box_mesh(self.dim, self.n, self.k_delta, self.order)
        if self.order == 2:
            return kuhn_mesh_p2(self.dim, self.n, self.k_delta)
        return kuhn_mesh(self.dim, self.n, self.k_delta)


def _ux1sq(dim):
    a = np.zeros(dim)
    a[0] = 1.0
    return Quadratic(a)


WORKLOADS = {
    # 2D 16x16, delta = 2h, eps = delta/16, depth 3, u = x1^2
    "c1_2d16": Workload("c1_2d16", 2, 16, 2, 16, 3, 0, _ux1sq(2)),
    # 2D 128x128, delta in {2h, 4h}, eps = delta/32, depth 5, u = x1^2 + x2^2
    "c2a_2d128_d2h": Workload("c2a_2d128_d2h", 2, 128, 2, 32, 5, 0, Quadratic(np.ones(2))),
    "c2b_2d128_d4h": Workload("c2b_2d128_d4h", 2, 128, 4, 32, 5, 0, Quadratic(np.ones(2))),
    # 3D 24^3 x 6 tets, delta = 3h (= 0.125), eps = delta/16, depth 4, u = x1^2
    "c3_3d24": Workload("c3_3d24", 3, 24, 3, 16, 4, 0, _ux1sq(3)),
    # 3D 48^3 x 6 tets, truncated Gaussian, delta = 3h, eps = delta/32, depth 6
    "c5_3d48_gauss": Workload("c5_3d48_gauss", 3, 48, 3, 32, 6, 1, _ux1sq(3)),
    # other element types (FP64), with the ratios of the paper's runs:
    # 20-node serendipity hexahedra, the 3D scaling run's delta = 4h, eps = h/2,
    # depth 2, on a 24^3 cube (13,824 hexes, 60,625 nodes)
    "hex20_3d24": Workload("hex20_3d24", 3, 24, 4, 8, 2, 0, _ux1sq(3), shape=1, order=2),
    # 8-node serendipity quadrilaterals, delta = 4h, eps = h/2, depth 3, 128^2
    "quad8_2d128": Workload("quad8_2d128", 2, 128, 4, 8, 3, 0, Quadratic(np.ones(2)), shape=1, order=2),
    # 10-node P2 tetrahedra, delta = 3h, eps = delta/16, depth 3, 16^3 x 6
    "p2tet_3d16": Workload("p2tet_3d16", 3, 16, 3, 16, 3, 0, _ux1sq(3), order=2),
}


def random_quadratic(rng: np.random.Generator, dim: int) -> Quadratic:
    """u = sum a_k x_k^2 + sum_{k<l} b_kl x_k x_l + c.x + d, all U(-1,1)."""
    a = rng.uniform(-1, 1, dim)
    b = np.triu(rng.uniform(-1, 1, (dim, dim)), 1)
    c = rng.uniform(-1, 1, dim)
    d = float(rng.uniform(-1, 1))
    return Quadratic(a, b, c, d)


@dataclass
class Request:
    rid: int
    arrival_s: float
    dim: int
    n: int
    k_delta: int
    eps_div: int
    lmax: int
    u: Quadratic


def serving_stream(n_requests: int = 256, rate_per_s: float = 20.0, seed: int = 0,
                   lmax: int = 3, eps_div: int = 16) -> list[Request]:
    """Poisson arrivals; 2D meshes 8^2..96^2 and 3D 6^3..20^3 with sizes
    uniform in log; delta in {2h, 3h, 4h}; random quadratic u."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        dim = 2 if rng.uniform() < 0.5 else 3
        lo, hi = (8, 96) if dim == 2 else (6, 20)
        n = int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))
        k_delta = int(rng.integers(2, 5))
        out.append(Request(rid, t, dim, n, k_delta, eps_div, lmax,
                           random_quadratic(rng, dim)))
    return out
