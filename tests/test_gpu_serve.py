"""Serving loop on the GPU: continuous batching, residency, admission, cancel.

* Each request's solution is the same alone and in a mix whose integrations
  share launches (relative 2-norm 1e-9 in FP64, 1e-6 in the mixed path: the
  matrices differ only by the order of FP64 atomics, CG stops at rtol 1e-12).
* The small requests are also checked against the FP64 oracle's assemble +
  Cholesky solve on the same mesh and data.
* A resident matrix is reused for an equal request (cache hit, same answer).
* A small HBM budget limits how many requests are admitted at once.
"""
import numpy as np
import pytest

from paper_2101_08825_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _requests(seed=3):
    """A mix of 2D / 3D meshes, horizons 2h..4h, depths 2..3, random quadratics."""
    rng = np.random.default_rng(seed)
    spec = [(2, 8, 2, 3), (2, 12, 3, 3), (2, 16, 4, 2), (2, 24, 2, 3), (2, 10, 4, 3),
            (3, 4, 2, 2), (3, 5, 2, 3), (3, 6, 3, 2), (2, 20, 3, 3), (2, 32, 2, 2)]
    out = []
    for dim, n, kd, lmax in spec:
        out.append(W.Request(len(out), 0.0, dim, n, kd, 16, lmax, W.random_quadratic(rng, dim)))
    return out


def _submit(nlq, srv, r, precision):
    mesh = W.kuhn_mesh(r.dim, r.n, r.k_delta)
    _, f, g = W.nodal_data(mesh, r.u)
    h = 1.0 / r.n
    delta = r.k_delta * h
    prm = nlq.params(r.dim, delta, delta / r.eps_div, r.lmax, precision=precision)
    return srv.submit(r.dim, r.n, r.k_delta, prm, f, g, rtol=RTOL, maxit=20000)


@pytest.fixture(scope="module")
def nlq_mod():
    import torch
    from paper_2101_08825_amd import nlq
    assert torch.cuda.is_available()
    return nlq


@pytest.mark.parametrize("precision", [0, 1])
def test_alone_equals_mix(nlq_mod, oracle_lib, precision):
    nlq = nlq_mod
    reqs = _requests()
    ctx = nlq.Context(0)
    srv = nlq.Server(ctx, cache_systems=False, target_launch_ms=5.0)
    alone = []
    for r in reqs:
        print(f"[case] alone precision={precision} dim={r.dim} n={r.n} kd={r.k_delta} lmax={r.lmax}", flush=True)
        res = srv.wait(_submit(nlq, srv, r, precision))
        assert res["status"] == 0, res["error"]
        alone.append(res["u"])
    print(f"[case] mix precision={precision} requests={len(reqs)}", flush=True)
    tickets = [_submit(nlq, srv, r, precision) for r in reqs]
    mix = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.stop()
    tol = 1e-9 if precision == 0 else 1e-6
    for r, a, m in zip(reqs, alone, mix):
        assert m["status"] == 0, m["error"]
        err = _rel(m["u"], a)
        print(f"  dim={r.dim} n={r.n} kd={r.k_delta}: alone vs mix {err:.2e}, launches {m['launches']}",
              flush=True)
        assert err <= tol, (r, err)
    # the mix shared integration launches
    assert st["max_per_launch"] >= 2, st
    assert st["completed"] == 2 * len(reqs) and st["failed"] == 0
    # the small 2D requests against the oracle (FP64 assembly + Cholesky)
    O = oracle_lib
    for r, m in zip(reqs[:3], mix[:3]):
        mesh = W.kuhn_mesh(r.dim, r.n, r.k_delta)
        _, f, g = W.nodal_data(mesh, r.u)
        h = 1.0 / r.n
        prm = O.params(r.k_delta * h, r.k_delta * h / r.eps_div, r.lmax)
        ref = O.solve_problem((mesh.coords, mesh.conn, mesh.constrained), prm, f, g, direct=True)
        err = _rel(m["u"], ref.u)
        print(f"  oracle dim={r.dim} n={r.n}: {err:.2e}", flush=True)
        assert err <= (1e-9 if precision == 0 else 1e-5), err
    ctx.close()


def test_resident_matrix_reused(nlq_mod):
    nlq = nlq_mod
    ctx = nlq.Context(0)
    srv = nlq.Server(ctx, cache_systems=True)
    r = _requests()[1]
    print("[case] cache", flush=True)
    a = srv.wait(_submit(nlq, srv, r, 0))
    b = srv.wait(_submit(nlq, srv, r, 0))
    st = srv.stats()
    srv.stop()
    ctx.close()
    assert a["status"] == 0 and b["status"] == 0
    assert not a["cache_hit"] and b["cache_hit"] and st["cache_hits"] == 1
    assert b["assemble_s"] == 0.0 and b["launches"] == 0
    assert _rel(b["u"], a["u"]) <= 1e-12


def test_admission_by_memory(nlq_mod):
    nlq = nlq_mod
    # budget for roughly two of these requests at a time
    ctx = nlq.Context(0, hbm_budget_bytes=96 << 20)
    srv = nlq.Server(ctx, cache_systems=False)
    rng = np.random.default_rng(5)
    reqs = [W.Request(i, 0.0, 2, 48, 4, 16, 2, W.random_quadratic(rng, 2)) for i in range(6)]
    print("[case] admission", flush=True)
    tickets = [_submit(nlq, srv, r, 1) for r in reqs]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.stop()
    used, budget = ctx.memory()
    ctx.close()
    assert all(x["status"] == 0 for x in res), [x["error"] for x in res]
    assert st["max_admitted"] < len(reqs), st
    assert st["peak_bytes"] <= budget


def test_cancel_pending(nlq_mod):
    nlq = nlq_mod
    ctx = nlq.Context(0)
    srv = nlq.Server(ctx, max_active=1)
    rng = np.random.default_rng(7)
    reqs = [W.Request(i, 0.0, 2, 16, 2, 16, 3, W.random_quadratic(rng, 2)) for i in range(4)]
    print("[case] cancel", flush=True)
    tickets = [_submit(nlq, srv, r, 0) for r in reqs]
    srv.cancel(tickets[-1])
    res = [srv.wait(t) for t in tickets]
    srv.stop()
    ctx.close()
    assert res[-1]["status"] == nlq.NLQ_ECANCELLED
    assert all(x["status"] == 0 for x in res[:-1])
