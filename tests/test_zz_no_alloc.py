"""nlq_solve_noalloc (the solve for callers that cannot allocate device memory)
against nlq_solve on the same systems, through the C-ABI: two calls in a row,
the second on a smaller system, each equal to nlq_solve's solution; a system
beyond the scratch limit is refused with a status."""
import numpy as np
import pytest

from paper_2101_08825_amd import workloads as W

pytestmark = pytest.mark.gpu


def _system(nlq, ctx, dim, n, kd, ed, lmax, precision):
    mesh = W.kuhn_mesh(dim, n, kd)
    u = W.Quadratic(np.linspace(0.5, 1.0, dim))
    _, f, g = W.nodal_data(mesh, u)
    m = nlq.Mesh.create(ctx, mesh.coords, mesh.conn, mesh.constrained)
    delta = kd / n
    s = nlq.System(ctx, m, nlq.params(dim, delta, delta / ed, lmax, precision=precision))
    s.set_data(f, g)
    return m, s


def test_noalloc_solve_equals_solve():
    import torch
    from paper_2101_08825_amd import nlq
    assert torch.cuda.is_available()
    ctx = nlq.Context(0)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    # the larger system first, then a smaller one: the second call reuses the
    # scratch the first one left behind
    cases = [(2, 40, 3, 16, 3, nlq.NLQ_FP32_MIXED), (3, 6, 2, 16, 2, nlq.NLQ_FP64_PLAIN),
             (2, 12, 2, 16, 3, nlq.NLQ_FP64_PLAIN)]
    for dim, n, kd, ed, lmax, prec in cases:
        print(f"[case] noalloc dim={dim} n={n} kd={kd} precision={prec}", flush=True)
        m, s = _system(nlq, ctx, dim, n, kd, ed, lmax, prec)
        u_ref, info_ref = s.solve(rtol=1e-12)
        u_dev = torch.full((m.n_nodes,), float("nan"), dtype=torch.float64, device="cuda")
        info = s.solve_noalloc(u_dev.data_ptr(), rtol=1e-12)
        torch.cuda.synchronize()
        u = u_dev.cpu().numpy()
        err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
        print(f"  nodes {m.n_nodes}: iterations {info.iterations} vs {info_ref.iterations}, "
              f"|u - u_solve| / |u_solve| = {err:.3e}", flush=True)
        assert info.converged == 1 and info.iterations == info_ref.iterations
        assert np.all(np.isfinite(u)) and err <= 1e-12
        s.close()
        m.close()
    ctx.close()


def test_noalloc_refuses_beyond_scratch():
    import torch
    from paper_2101_08825_amd import nlq
    ctx = nlq.Context(0)
    # 2D 560^2 cells: 314,721 nodes, beyond the 16 MiB scratch (about 290,000)
    mesh = W.kuhn_mesh(2, 560, 2)
    m = nlq.Mesh.create(ctx, mesh.coords, mesh.conn, mesh.constrained)
    s = nlq.System.prepare(ctx, m, nlq.params(2, 2 / 560, 2 / 560 / 16, 1, precision=nlq.NLQ_FP64_PLAIN))
    s.set_data(np.zeros(m.n_nodes), np.zeros(m.n_nodes))
    u_dev = torch.zeros(m.n_nodes, dtype=torch.float64, device="cuda")
    with pytest.raises(nlq.NlqError) as e:
        s.solve_noalloc(u_dev.data_ptr())
    print(f"  refused: {e.value}", flush=True)
    assert "scratch" in str(e.value)
    s.close()
    m.close()
    ctx.close()
