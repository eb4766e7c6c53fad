"""Autotuner of the integration launch (nlq_autotune).

The tuned configuration must not change what is computed: after tuning, the
system's values equal an untuned assembly, the pair list and leaf counts are
unchanged, and a later assembly with the same key (which picks the tuned
configuration up from the context) gives the same matrix.  The launch shape
reorders only the FP64 atomics (1e-13); the stack and leaf-buffer capacities
also regroup each pair's partial sums (the order in which leaves are popped and
flushed), which moves FP32-mixed values by FP32 rounding (2e-6 relative) and
FP64 values by FP64 rounding.
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
    assert 64 <= t["stack_capacity"] <= 512 and 64 <= t["leaf_capacity"] <= 256
    regrouped = precision == 1 and (t["stack_capacity"], t["leaf_capacity"]) != (128, 128)
    bar = 2e-6 if regrouped else 1e-13
    _, _, v = s.csr()
    assert list(s.info().n_leaf) == leaves_ref
    assert _rel(v, v_ref) <= bar
    # a new system with the same key uses the tuned configuration
    s2 = nlq.System(ctx, m, prm)
    _, _, v2 = s2.csr()
    assert list(s2.info().n_leaf) == leaves_ref
    assert _rel(v2, v_ref) <= bar
    for x in (s, s2):
        x.close()
    m.close()
    ctx.close()
    ref.close()
    ref_m.close()
    ref_ctx.close()


def test_tuning_cache_file(tmp_path):
    """nlq_tune_save / nlq_tune_load: a new context loads what an earlier one
    tuned (lines of another architecture are skipped, a malformed line is an
    error), and saving it again writes the same file."""
    import torch
    from paper_2101_08825_amd import nlq
    assert torch.cuda.is_available()
    print("[case] tuning cache file", flush=True)
    wl = W.Workload("tune", 2, 48, 4, 32, 4, 0, W._ux1sq(2))
    mesh = wl.mesh()
    ctx = nlq.Context(0)
    m = nlq.Mesh.create(ctx, mesh.coords, mesh.conn, mesh.constrained)
    s = nlq.System(ctx, m, nlq.params(2, wl.delta, wl.eps, 4, precision=1))
    s.autotune(budget_s=1.0)
    s.close()
    m.close()
    a = tmp_path / "a.txt"
    ctx.tune_save(a)
    ctx.close()
    lines = a.read_text().splitlines()
    assert lines[0].startswith("#") and len(lines) == 2
    arch = lines[1].split()[0]
    assert arch.startswith("gfx")
    other = tmp_path / "other.txt"
    assert len(lines[1].split()) == 12            # arch + 11 fields (format v2)
    # a line of another architecture is skipped; a line of the first format
    # (no order, no capacities) still parses
    other.write_text(a.read_text() + "gfx000 2 1 1 0 4 9 1 3 256 128 128\n" + "gfx000 2 1 0 4 9 1 3 256\n")
    ctx2 = nlq.Context(0)
    assert ctx2.tune_load(other) == 1
    b = tmp_path / "b.txt"
    ctx2.tune_save(b)
    assert b.read_text() == a.read_text()
    bad = tmp_path / "bad.txt"
    bad.write_text(a.read_text() + f"{arch} 2 1 0\n")
    with pytest.raises(nlq.NlqError) as e:
        ctx2.tune_load(bad)
    assert e.value.status == nlq.NLQ_EINVAL
    with pytest.raises(nlq.NlqError):
        ctx2.tune_load(tmp_path / "missing.txt")
    ctx2.close()


@pytest.mark.parametrize("dim,n,kd,ed,lmax,precision", [(3, 8, 3, 16, 3, 1), (2, 32, 4, 32, 4, 0)])
def test_capacities_keep_values(tmp_path, dim, n, kd, ed, lmax, precision):
    """Traversal stack and leaf buffer capacities at the ends of the tuner's
    range (loaded from a cache file for the system's key): leaf counts equal,
    values equal to FP32 (2e-6) / FP64 (1e-13) rounding."""
    import torch
    from paper_2101_08825_amd import nlq
    assert torch.cuda.is_available()
    print(f"[case] capacities dim={dim} n={n} lmax={lmax} precision={precision}", flush=True)
    wl = W.Workload("cap", dim, n, kd, ed, lmax, 0, W._ux1sq(dim))
    mesh = wl.mesh()
    prm = nlq.params(dim, wl.delta, wl.eps, lmax, precision=precision)
    ctx = nlq.Context(0)
    m = nlq.Mesh.create(ctx, mesh.coords, mesh.conn, mesh.constrained)
    ref = nlq.System(ctx, m, prm)
    _, _, v_ref = ref.csr()
    leaves_ref = list(ref.info().n_leaf)
    ref.autotune(budget_s=0.5)        # puts the system's key into the cache file
    path = tmp_path / "t.txt"
    ctx.tune_save(path)
    ref.close()
    m.close()
    ctx.close()
    head, line = path.read_text().splitlines()[:2]
    f = line.split()
    bar = 2e-6 if precision == 1 else 1e-13
    for stack_cap, leaf_cap in ((64, 64), (512, 256), (1024, 512)):
        # arch dim order precision kernel lmax size_class | occ wg ppi stack leaf
        f[7], f[8], f[9], f[10], f[11] = "0", "0", "256" if dim == 3 else "512", str(stack_cap), str(leaf_cap)
        path.write_text(head + "\n" + " ".join(f) + "\n")
        c2 = nlq.Context(0)
        assert c2.tune_load(path) == 1
        m2 = nlq.Mesh.create(c2, mesh.coords, mesh.conn, mesh.constrained)
        s2 = nlq.System(c2, m2, prm)
        _, _, v = s2.csr()
        err = _rel(v, v_ref)
        print(f"  stack {stack_cap} leaf {leaf_cap}: rel {err:.3e}", flush=True)
        assert list(s2.info().n_leaf) == leaves_ref
        assert err <= bar
        s2.close()
        m2.close()
        c2.close()
