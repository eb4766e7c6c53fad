"""CG with the 8-iteration check blocks replayed as a HIP graph vs plain launches.

The graph holds the same kernels in the same order, so every iterate must be
identical bit for bit.  Each maxit below stops CG after a different number of
replays (2 .. 5, with the host's copy + synchronisation between replays), and
the iterate left there is compared with the plain-launch run.
"""
import os

import numpy as np
import pytest

from paper_2101_08825_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
def test_cg_graph_equals_plain(precision):
    import torch
    from paper_2101_08825_amd import nlq
    assert torch.cuda.is_available()
    wl = W.Workload("cg", 2, 32, 3, 16, 3, 0, W.Quadratic(np.array([1.0, 0.5])))
    mesh = wl.mesh()
    _, f, g = W.nodal_data(mesh, wl.u)
    ctx = nlq.Context(0)
    m = nlq.Mesh.create(ctx, mesh.coords, mesh.conn, mesh.constrained)
    s = nlq.System(ctx, m, nlq.params(2, wl.delta, wl.eps, wl.lmax, precision=precision))
    s.set_data(f, g)
    old = os.environ.get("NLQ_CG_GRAPH")
    try:
        for maxit in (16, 24, 32, 40):
            print(f"[case] cg graph precision={precision} maxit={maxit}", flush=True)
            os.environ["NLQ_CG_GRAPH"] = "0"
            u0, i0 = s.solve(rtol=1e-30, maxit=maxit)
            os.environ["NLQ_CG_GRAPH"] = "1"
            u1, i1 = s.solve(rtol=1e-30, maxit=maxit)
            assert i0.iterations == i1.iterations == maxit
            assert np.array_equal(u0, u1), float(np.max(np.abs(u0 - u1)))
            assert i0.rel_residual == i1.rel_residual
        # and a converged solve
        os.environ["NLQ_CG_GRAPH"] = "0"
        u0, i0 = s.solve(rtol=1e-12)
        os.environ["NLQ_CG_GRAPH"] = "1"
        u1, i1 = s.solve(rtol=1e-12)
        assert i0.converged and i1.converged and i0.iterations == i1.iterations
        assert np.array_equal(u0, u1)
    finally:
        if old is None:
            os.environ.pop("NLQ_CG_GRAPH", None)
        else:
            os.environ["NLQ_CG_GRAPH"] = old
    s.close()
    m.close()
    ctx.close()
