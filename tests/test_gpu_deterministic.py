"""Deterministic (fixed-order) accumulation on the GPU.

* The same system assembled twice gives bit-identical values, and so does the
  assembly cut into many slabs (the sums do not depend on the slab size).
* The values equal the atomic path's to the FP64 reordering of additions
  (relative Frobenius 1e-13), with identical pair lists, patterns and leaf
  counts; the four-term matrix is exactly symmetric.
* A deterministic system in a batch equals its single assembly bit for bit.
* Served requests give bit-identical solutions alone and in a mix (the CG's
  reductions have a fixed order too).
"""
import os

import numpy as np
import pytest

from paper_2101_08825_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = [
    # dim, n, k_delta, eps_div, lmax, form
    (2, 16, 2, 16, 4, 0),
    (2, 12, 3, 8, 3, 1),
    (3, 5, 2, 16, 3, 0),
    (3, 4, 2, 4, 2, 1),
]


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


@pytest.fixture(scope="module")
def nlq_mod():
    import torch
    from paper_2101_08825_amd import nlq
    assert torch.cuda.is_available()
    return nlq


def _mesh(nlq, ctx, case):
    dim, n, kd, ed, lmax, form = case
    wl = W.Workload(f"d{dim}_{n}", dim, n, kd, ed, lmax, 0, W._ux1sq(dim))
    m = wl.mesh()
    return wl, m, nlq.Mesh.create(ctx, m.coords, m.conn, m.constrained)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("case", CASES)
def test_repeatable_and_equal_to_atomic(nlq_mod, case, precision):
    nlq = nlq_mod
    dim, n, kd, ed, lmax, form = case
    print(f"[case] deterministic {case} precision={precision}", flush=True)
    ctx = nlq.Context(0)
    wl, m, mh = _mesh(nlq, ctx, case)
    prm_d = nlq.params(dim, wl.delta, wl.eps, lmax, form=form, precision=precision, deterministic=True)
    prm_a = nlq.params(dim, wl.delta, wl.eps, lmax, form=form, precision=precision)
    a = nlq.System(ctx, mh, prm_d)
    ra, ca, va = a.csr()
    a.reassemble()
    _, _, va2 = a.csr()
    assert np.array_equal(va, va2), "two deterministic assemblies differ"
    # many slabs: a slab of about one element's pairs
    os.environ["NLQ_DET_SLAB_PAIRS"] = "1"
    try:
        a.reassemble()
        _, _, va3 = a.csr()
    finally:
        del os.environ["NLQ_DET_SLAB_PAIRS"]
    assert np.array_equal(va, va3), "slab size changed the values"
    b = nlq.System(ctx, mh, prm_a)
    rb, cb, vb = b.csr()
    assert np.array_equal(ra, rb) and np.array_equal(ca, cb)
    assert list(a.info().n_leaf) == list(b.info().n_leaf)
    err = _rel(va, vb)
    print(f"  deterministic vs atomic: {err:.2e}", flush=True)
    assert err <= 1e-13
    if form == 0:
        import scipy.sparse as sp
        A = sp.csr_matrix((va, ca, ra), shape=(m.n_nodes, m.n_nodes))
        assert (A - A.T).count_nonzero() == 0 or sp.linalg.norm(A - A.T) == 0.0
    a.close()
    b.close()
    mh.close()
    ctx.close()


def test_batch_member_equals_single(nlq_mod):
    nlq = nlq_mod
    print("[case] deterministic in a batch", flush=True)
    ctx = nlq.Context(0)
    meshes, prms = [], []
    for k, case in enumerate(CASES[:3]):
        dim, n, kd, ed, lmax, form = case
        wl, m, mh = _mesh(nlq, ctx, case)
        meshes.append(mh)
        prms.append(nlq.params(dim, wl.delta, wl.eps, lmax, form=form, precision=1, deterministic=(k != 1)))
    batch = nlq.System.batch(ctx, meshes, prms)
    for k in (0, 2):
        single = nlq.System(ctx, meshes[k], prms[k])
        assert np.array_equal(batch[k].csr()[2], single.csr()[2]), k
        single.close()
    for s in batch:
        s.close()
    for mh in meshes:
        mh.close()
    ctx.close()


def test_served_alone_equals_mix(nlq_mod):
    nlq = nlq_mod
    rng = np.random.default_rng(11)
    spec = [(2, 12, 2, 3), (2, 16, 3, 3), (3, 5, 2, 2), (2, 20, 2, 3), (3, 4, 2, 3)]
    reqs = [W.Request(i, 0.0, d, n, kd, 16, lm, W.random_quadratic(rng, d)) for i, (d, n, kd, lm) in enumerate(spec)]
    ctx = nlq.Context(0)
    srv = nlq.Server(ctx, cache_systems=False, target_launch_ms=5.0)

    def submit(r):
        mesh = W.kuhn_mesh(r.dim, r.n, r.k_delta)
        _, f, g = W.nodal_data(mesh, r.u)
        delta = r.k_delta / r.n
        prm = nlq.params(r.dim, delta, delta / r.eps_div, r.lmax, precision=1, deterministic=True)
        return srv.submit(r.dim, r.n, r.k_delta, prm, f, g, rtol=1e-12, maxit=20000)

    print("[case] deterministic serving", flush=True)
    alone = []
    for r in reqs:
        x = srv.wait(submit(r))
        assert x["status"] == 0, x["error"]
        alone.append(x["u"])
    mix = [srv.wait(t) for t in [submit(r) for r in reqs]]
    srv.stop()
    ctx.close()
    for r, a, x in zip(reqs, alone, mix):
        assert x["status"] == 0, x["error"]
        assert np.array_equal(a, x["u"]), (r.dim, r.n)
