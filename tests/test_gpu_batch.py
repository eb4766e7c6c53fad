"""Shared integration launches (nlq_assemble_batch) against one launch per system.

Several systems of different meshes, horizons, depths and forms are assembled
in one batch; each must equal its own nlq_assemble result: pair list, pattern
and leaf counts bit-exact, values within the FP64 reordering of atomics
(relative Frobenius 1e-13), and the mixed path within its own tolerance of the
oracle-checked FP64 values.
"""
import numpy as np
import pytest

from paper_2101_08825_amd import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


CASES = [
    # dim, n, k_delta, eps_div, lmax, form
    (2, 16, 2, 16, 3, 0),
    (2, 12, 3, 8, 4, 0),
    (2, 16, 2, 16, 3, 1),
    (2, 20, 4, 32, 3, 0),
    (3, 5, 2, 16, 3, 0),
    (3, 4, 2, 4, 2, 1),
]


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single(precision):
    import torch
    from paper_2101_08825_amd import nlq
    assert torch.cuda.is_available()
    ctx = nlq.Context(0)
    meshes, prms = [], []
    for (dim, n, kd, ed, lmax, form) in CASES:
        wl = W.Workload(f"b{dim}_{n}", dim, n, kd, ed, lmax, 0, W._ux1sq(dim))
        m = wl.mesh()
        meshes.append(nlq.Mesh.create(ctx, m.coords, m.conn, m.constrained))
        prms.append(nlq.params(dim, wl.delta, wl.eps, lmax, form=form, precision=precision))
    print(f"[case] batch precision={precision} systems={len(CASES)}", flush=True)
    batch = nlq.System.batch(ctx, meshes, prms)
    for k, (mh, prm) in enumerate(zip(meshes, prms)):
        single = nlq.System(ctx, mh, prm)
        a, b = batch[k], single
        ia, ib = a.info(), b.info()
        assert list(ia.n_leaf) == list(ib.n_leaf), CASES[k]
        assert ia.n_pairs == ib.n_pairs
        oa, pa = a.pairs()
        ob, pb = b.pairs()
        assert np.array_equal(oa, ob) and np.array_equal(pa, pb)
        ra, ca, va = a.csr()
        rb, cb, vb = b.csr()
        assert np.array_equal(ra, rb) and np.array_equal(ca, cb)
        err = _rel(va, vb)
        print(f"  system {k} {CASES[k]}: rel diff {err:.2e}", flush=True)
        assert err <= (1e-13 if precision == 0 else 1e-6), (CASES[k], err)
        single.close()
    for s in batch:
        s.close()
    for m in meshes:
        m.close()
    ctx.close()
