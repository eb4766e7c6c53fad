"""Failure paths on the GPU, forced from the host: malformed input gives C-ABI
status codes, an injected device-allocation failure at any point of the
mesh / assemble / load / solve sequence gives NLQ_ENOMEM and leaves the context
usable (a retry gives the clean result and nothing leaks), and the serving loop
returns u = g for a request without free nodes and keeps serving after a
request fails."""
import os

import numpy as np
import pytest

from paper_2101_08825_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nlq_mod():
    import torch
    from paper_2101_08825_amd import nlq
    assert torch.cuda.is_available()
    return nlq


def _status(nlq, fn):
    try:
        fn()
    except nlq.NlqError as e:
        return e.status
    return nlq.NLQ_OK


def test_malformed_input(nlq_mod):
    nlq = nlq_mod
    print("[case] malformed input", flush=True)
    ctx = nlq.Context(0)
    mesh = W.kuhn_mesh(2, 4, 1)
    bad = mesh.conn.copy()
    bad[3, 1] = mesh.n_nodes
    assert _status(nlq, lambda: nlq.Mesh.create(ctx, mesh.coords, bad, mesh.constrained)) == nlq.NLQ_EINVAL
    flat = mesh.conn.copy()
    flat[0, 2] = flat[0, 1]
    assert _status(nlq, lambda: nlq.Mesh.create(ctx, mesh.coords, flat, mesh.constrained)) == nlq.NLQ_EINVAL
    nan = mesh.coords.copy()
    nan[5, 0] = np.nan
    assert _status(nlq, lambda: nlq.Mesh.create(ctx, nan, mesh.conn, mesh.constrained)) == nlq.NLQ_EINVAL
    m = nlq.Mesh.create(ctx, mesh.coords, mesh.conn, mesh.constrained)
    for prm in (nlq.params(2, 0.25, 0.25, 3),              # eps = delta
                nlq.params(2, 0.25, 0.01, 9),              # lmax too large
                nlq.params(3, 0.25, 0.01, 3),              # dim of another mesh
                nlq.params(2, 0.25, 0.01, 3, lmin=4)):     # lmin > lmax
        assert _status(nlq, lambda: nlq.System(ctx, m, prm)) == nlq.NLQ_EINVAL
    p = nlq.params(2, 0.25, 0.01, 3)
    p.deterministic = 2
    assert _status(nlq, lambda: nlq.System(ctx, m, p)) == nlq.NLQ_EINVAL
    # still usable
    s = nlq.System(ctx, m, nlq.params(2, 0.25, 0.01, 3))
    assert s.info().n_pairs > 0
    s.close()
    m.close()
    ctx.close()


def _run(nlq, ctx, mesh, f, g, wl, det):
    m = nlq.Mesh.create(ctx, mesh.coords, mesh.conn, mesh.constrained)
    try:
        s = nlq.System(ctx, m, nlq.params(2, wl.delta, wl.eps, wl.lmax, deterministic=det))
        try:
            s.set_data(f, g)
            u, _ = s.solve(rtol=1e-12)
            return s.csr()[2], u
        finally:
            s.close()
    finally:
        m.close()


@pytest.mark.parametrize("det", [False, True])
def test_injected_allocation_failure(nlq_mod, det):
    nlq = nlq_mod
    wl = W.WORKLOADS["c1_2d16"]
    mesh = wl.mesh()
    _, f, g = W.nodal_data(mesh, wl.u)
    ctx = nlq.Context(0)
    ref_val, ref_u = _run(nlq, ctx, mesh, f, g, wl, det)
    base_used = ctx.memory()[0]
    ctx.close()
    failures = 0
    for k in range(200):
        os.environ["NLQ_FAIL_ALLOC_AT"] = str(k)
        try:
            ctx = nlq.Context(0)
        finally:
            del os.environ["NLQ_FAIL_ALLOC_AT"]
        try:
            st = nlq.NLQ_OK
            try:
                _run(nlq, ctx, mesh, f, g, wl, det)
            except nlq.NlqError as e:
                st = e.status
            if st == nlq.NLQ_OK:
                print(f"  allocation {k}: past the last allocation; {failures} injected failures", flush=True)
                break
            assert st == nlq.NLQ_ENOMEM, (k, st)
            failures += 1
            # the injection fired once: the same sequence now succeeds, equal to the clean run
            val, u = _run(nlq, ctx, mesh, f, g, wl, det)
            tol = 0.0 if det else 1e-13
            assert np.linalg.norm(val - ref_val) <= tol * np.linalg.norm(ref_val), k
            assert np.linalg.norm(u - ref_u) <= max(tol, 1e-12) * np.linalg.norm(ref_u), k
            assert ctx.memory()[0] <= base_used, (k, ctx.memory()[0], base_used)
        finally:
            ctx.close()
    assert failures > 10


def test_serving_zero_free_nodes_and_failed_request(nlq_mod):
    nlq = nlq_mod
    print("[case] serving: no free nodes; a failing request", flush=True)
    ctx = nlq.Context(0)
    srv = nlq.Server(ctx, cache_systems=False)
    rng = np.random.default_rng(3)
    u0 = W.random_quadratic(rng, 3)
    mesh = W.kuhn_mesh(3, 6, 4)
    assert not np.any(mesh.constrained == 0)
    _, f, g = W.nodal_data(mesh, u0)
    prm = nlq.params(3, 4 / 6, 4 / 6 / 16, 2)
    x = srv.wait(srv.submit(3, 6, 4, prm, f, g))
    assert x["status"] == 0, x["error"]
    assert np.array_equal(x["u"], g)
    # a request whose parameters fail at setup (lmax too large) ends with its
    # status; the next one is served
    mesh2 = W.kuhn_mesh(2, 8, 2)
    _, f2, g2 = W.nodal_data(mesh2, W.random_quadratic(rng, 2))
    bad = srv.wait(srv.submit(2, 8, 2, nlq.params(2, 0.25, 0.01, 9), f2, g2))
    assert bad["status"] == nlq.NLQ_EINVAL
    ok = srv.wait(srv.submit(2, 8, 2, nlq.params(2, 0.25, 0.25 / 16, 3), f2, g2))
    assert ok["status"] == 0, ok["error"]
    st = srv.stats()
    srv.stop()
    ctx.close()
    assert st["failed"] == 1 and st["completed"] == 2
