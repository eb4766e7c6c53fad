"""Autotuner of the integration launch (nlq_autotune).

The tuned configuration must not change what is computed: after tuning, the
system's values equal an untuned assembly (FP64 atomics reordering only), the
pair list and leaf counts are unchanged, and a later assembly with the same key
(which picks the tuned configuration up from the context) gives the same matrix.
"""
import numpy as np
import pytest

from paper_2101_08825_amd import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dim,n,kd,ed,lmax,precision", [
    (2, 48, 4, 32, 4, 1), (2, 48, 4, 32, 4, 0), (3, 8, 3, 16, 2, 1)])
def test_autotune_keeps_values(dim, n, kd, ed, lmax, precision):
    import torch
    from paper_2101_08825_amd import nlq
    assert torch.cuda.is_available()
    print(f"[case] autotune dim={dim} n={n} kd={kd} lmax={lmax} precision={precision}", flush=True)
    wl = W.Workload("tune", dim, n, kd, ed, lmax, 0, W._ux1sq(dim))
    mesh = wl.mesh()
    ref_ctx = nlq.Context(0)
    ref_m = nlq.Mesh.create(ref_ctx, mesh.coords, mesh.conn, mesh.constrained)
    prm = nlq.params(dim, wl.delta, wl.eps, lmax, precision=precision)
    ref = nlq.System(ref_ctx, ref_m, prm)
    _, _, v_ref = ref.csr()
    leaves_ref = list(ref.info().n_leaf)

    ctx = nlq.Context(0)
    m = nlq.Mesh.create(ctx, mesh.coords, mesh.conn, mesh.constrained)
    s = nlq.System(ctx, m, prm)
    t = s.autotune(budget_s=3.0)
    print(f"  tuned: {t}", flush=True)
    assert t["candidates"] >= 1 and t["best_ms"] > 0 and t["best_ms"] <= t["default_ms"] * 1.0001
    assert t["work_items_per_element"] >= 1 and t["workgroups_per_cu"] >= 1
    _, _, v = s.csr()
    assert list(s.info().n_leaf) == leaves_ref
    assert _rel(v, v_ref) <= 1e-13
    # a new system with the same key uses the tuned configuration
    s2 = nlq.System(ctx, m, prm)
    _, _, v2 = s2.csr()
    assert list(s2.info().n_leaf) == leaves_ref
    assert _rel(v2, v_ref) <= 1e-13
    for x in (s, s2):
        x.close()
    m.close()
    ctx.close()
    ref.close()
    ref_m.close()
    ref_ctx.close()
