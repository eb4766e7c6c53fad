"""3D configurations at full size on the GPU, checked on sampled outputs.

* 24^3 x 6 tets, delta = 3h, eps = delta/16, depth 4 (constant kernel): the whole
  matrix is assembled in the FP32-mixed path; the pair count equals the closed
  Kuhn form, sampled J_l equal the oracle's brute force, the leaf integrations
  per level over the whole mesh equal the oracle's (tests/golden/c3_oracle.json,
  written by the committed oracle script beside it) and their total the
  independent count, four whole rows of the assembled matrix equal the oracle's
  rows, sampled per-pair blocks equal the oracle's (both precisions), and the
  matrix is symmetric with zero row sums.
* 48^3 x 6 tets, truncated Gaussian kernel, delta = 3h, eps = delta/32, depth 6:
  too large to integrate whole in a test (about 9e15 kernel evaluations); the
  system is prepared (pair list, pattern), the pair count is checked against the
  closed form, sampled J_l and per-pair blocks against the oracle, and a seeded
  sample of outer elements spread over the whole mesh (32 strata) is integrated
  in one launch and timed; its leaf integrations per level equal the oracle's.
"""
import json
import os

import numpy as np
import pytest

from paper_2101_08825_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _kuhn_pairs(dim, n, delta, eps):
    """Ordered pairs of a Kuhn mesh: (dim!)^2 prod_k [n(2K+1) - K(K+1)], with K the
    largest cell offset whose bbox gap max(K-1, 0) h is below delta + eps."""
    h = 1.0 / n
    K = 0
    while max(K, 0) * h < delta + eps:
        K += 1
    types = 2 if dim == 2 else 6
    return types ** 2 * (n * (2 * K + 1) - K * (K + 1)) ** dim


def _blocks_rel(got, exp):
    return float(np.linalg.norm((got - exp).ravel()) / np.linalg.norm(exp.ravel()))


def _check_vals(got, exp, tol):
    err = float(np.linalg.norm(got - exp) / np.linalg.norm(exp))
    emax = float(np.max(np.abs(got - exp)) / np.max(np.abs(exp)))
    print(f"  rel Frobenius {err:.3e}, max entry error / max entry {emax:.3e}", flush=True)
    assert err <= tol and emax <= tol, (err, emax)


# leaf integrations of the 24^3 problem from a count independent of both
# implementations
C3_LEAVES = 78429899232
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_oracle.json")


@pytest.fixture(scope="module")
def nlq_mod():
    import torch
    from paper_2101_08825_amd import nlq
    assert torch.cuda.is_available()
    return nlq


def _sampled_checks(nlq, O, s, mesh, wl, prm_o, precision, n_elems_sample, n_pairs_sample, seed):
    om = O.OracleMesh(mesh.coords, mesh.conn)
    thr = wl.delta + wl.eps
    off, pm = s.pairs()
    rng = np.random.default_rng(seed)
    for l in rng.choice(mesh.n_elems, n_elems_sample, replace=False):
        ref = O.pairs_of(om, thr, int(l))
        assert np.array_equal(pm[off[l]:off[l + 1]], ref), l
    pick = rng.choice(len(pm), n_pairs_sample, replace=False)
    ls = (np.searchsorted(off, pick, side="right") - 1).astype(np.int32)
    ms = pm[pick]
    got = s.pair_blocks(ls, ms)
    exp = np.stack([O.pair_block(om, prm_o, int(a), int(b))[0] for a, b in zip(ls, ms)])
    err = _blocks_rel(got, exp)
    print(f"  sampled pair blocks ({n_pairs_sample}): stacked rel Frobenius {err:.3e}", flush=True)
    assert err <= (TOL64 if precision == 0 else TOL32)
    return off


def test_c3_full_size(nlq_mod, oracle_lib):
    nlq, O = nlq_mod, oracle_lib
    wl = W.WORKLOADS["c3_3d24"]
    print("[case] c3 full size, FP32-mixed", flush=True)
    mesh = wl.mesh()
    ctx = nlq.Context(0)
    m = nlq.Mesh.create(ctx, mesh.coords, mesh.conn, mesh.constrained)
    s = nlq.System(ctx, m, nlq.params(3, wl.delta, wl.eps, wl.lmax, precision=nlq.NLQ_FP32_MIXED))
    info = s.info()
    print(f"  pairs {info.n_pairs} leaves {list(info.n_leaf)[1:5]} evals {info.n_evals:.3e} "
          f"t_kernel {info.t_kernel:.2f}s t_total {info.t_total:.2f}s", flush=True)
    assert info.n_pairs == _kuhn_pairs(3, 24, wl.delta, wl.eps) == 271063296
    gold = json.load(open(GOLDEN))
    assert list(info.n_leaf)[1:5] == gold["leaves_per_level"][1:5]
    assert sum(gold["leaves_per_level"]) == C3_LEAVES
    prm_o = O.params(wl.delta, wl.eps, wl.lmax)
    _sampled_checks(nlq, O, s, mesh, wl, prm_o, 1, 6, 24, seed=3)
    rp, col, val = s.csr()
    for name, row in gold["rows"].items():
        r = row["node"]
        assert np.array_equal(col[rp[r]:rp[r + 1]], np.array(row["cols"], dtype=np.int32)), name
        exp = np.array([float.fromhex(v) for v in row["vals"]])
        print(f"  row {name} ({r}, {len(exp)} entries):", flush=True)
        _check_vals(val[rp[r]:rp[r + 1]], exp, TOL32)
    n = mesh.n_nodes
    rows_of = np.repeat(np.arange(n), np.diff(rp))
    rowsum = np.bincount(rows_of, weights=val, minlength=n)
    rowabs = np.bincount(rows_of, weights=np.abs(val), minlength=n)
    rs = float(np.max(np.abs(rowsum) / rowabs))
    import scipy.sparse as sp
    A = sp.csr_matrix((val, col, rp), shape=(n, n))
    asym = sp.linalg.norm(A - A.T) / sp.linalg.norm(A)
    print(f"  nnz {len(val)}; max |row sum| / row abs sum {rs:.3e}; |A - A^T|/|A| {asym:.3e}", flush=True)
    assert len(val) == 14706125
    assert rs <= 1e-13 and asym == 0.0
    s.close()
    # the FP64 plain path on sampled blocks of a prepared system
    p64 = nlq.System.prepare(ctx, m, nlq.params(3, wl.delta, wl.eps, wl.lmax, precision=nlq.NLQ_FP64_PLAIN))
    _sampled_checks(nlq, O, p64, mesh, wl, prm_o, 0, 2, 24, seed=4)
    p64.close()
    m.close()
    ctx.close()


def test_c5_sampled(nlq_mod, oracle_lib):
    nlq, O = nlq_mod, oracle_lib
    wl = W.WORKLOADS["c5_3d48_gauss"]
    print("[case] c5 prepared, sampled, slab timing", flush=True)
    mesh = wl.mesh()
    ctx = nlq.Context(0)
    m = nlq.Mesh.create(ctx, mesh.coords, mesh.conn, mesh.constrained)
    prm = nlq.params(3, wl.delta, wl.eps, wl.lmax, kernel=nlq.NLQ_ETA_GAUSS, precision=nlq.NLQ_FP32_MIXED)
    s = nlq.System.prepare(ctx, m, prm)
    info = s.info()
    sz = s.sizes()
    print(f"  pairs {sz['n_pairs']} nnz {sz['nnz']} t_pairs {info.t_pairs:.2f}s t_pattern {info.t_pattern:.2f}s",
          flush=True)
    assert sz["n_pairs"] == _kuhn_pairs(3, 48, wl.delta, wl.eps) == 2517643008
    assert sz["nnz"] == 131872229
    prm_o = O.params(wl.delta, wl.eps, wl.lmax, kernel=1)
    _sampled_checks(nlq, O, s, mesh, wl, prm_o, 1, 4, 8, seed=5)
    # a seeded 1/1024 of the outer elements, spread over the mesh in 32 strata,
    # integrated in one launch and timed; leaf counts per level against the oracle
    ne = mesh.n_elems
    lo, hi = W.stratified_ranges(ne, 1.0 / 1024, 32, seed=5)
    t, leaves, nzero = s.integrate_ranges(lo, hi)
    sel = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)])
    lv_o = O.leaf_counts(O.OracleMesh(mesh.coords, mesh.conn), prm_o, sel)
    evals = int(np.sum(leaves)) * 15 * 15
    print(f"  sample {len(sel)} elements: {t:.3f} s, leaves {list(leaves[1:7])}, {evals / t / 1e9:.1f} Gevals/s, "
          f"whole mesh extrapolated {t * ne / len(sel) / 60:.1f} min", flush=True)
    assert list(leaves[1:7]) == list(lv_o[1:7])
    assert evals > 0
    s.close()
    m.close()
    ctx.close()
