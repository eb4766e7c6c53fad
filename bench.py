"""Benchmark of the hot path on one MI355X.

Headline (`value`): the 3D problem of 24^3 cubes x 6 Kuhn tetrahedra (82,944 P1
tets, 15,625 nodes), delta = 3h = 0.125, eps = delta/16, depth <= 4, 15-point
rule, constant kernel, u = x1^2, f = -2.  A step is one pass of the whole path
(element tables, pair list, CSR pattern, Algorithm 1 + leaf integration, FP64
CSR accumulation, load vector + lifting, CG solve) with mesh and data resident
in HBM; `value` = element-pair integrals per second of the FP32-mixed path over
exactly the K timed steps.  The FP64 plain path runs the same step.

Beside it, each section skipped (and said so) when the run's time budget would
not hold it:
 * errors: four whole rows of the oracle's matrix of the headline problem
   (tests/golden/c3_oracle.json, written by the CPU oracle) against both paths;
   the FP32 matrix and solution against the FP64 path's, itself pinned to the
   oracle at 1e-12;
 * the 48^3 x 6 problem with the truncated Gaussian kernel (663,552 tets,
   delta = 3h, eps = delta/32, depth 6, about 9e15 kernel evaluations):
   prepared whole, integrated on a seeded 1/1024 sample of outer elements
   spread over the mesh (32 strata, one launch), whole-mesh time extrapolated by
   the sample's share of the pairs;
 * the 2D 128^2 problems (delta = 2h and 4h, eps = delta/32, depth 5);
 * other element types in FP64, whole assembly + solve: 20-node serendipity
   hexahedra (24^3, the paper's 3D scaling ratios delta = 4h, eps = h/2, depth
   2), 10-node P2 tetrahedra (16^3 x 6, delta = 3h, eps = delta/16, depth 3),
   8-node serendipity quadrilaterals (128^2, delta = 4h, eps = h/2, depth 3),
   each with the oracle on one seeded outer element on one core;
 * serving: the seeded 256-request stream (2D 8^2..96^2 / 3D 6^3..20^3, delta
   2h..4h, eps = delta/16, depth 3) replayed open loop, first at 20 requests/s
   (beyond capacity: its wall time gives the capacity), then at 0.8 of that
   capacity for both precisions: p50 / p99 of submit -> solution;
 * the CPU oracle on a bounded seeded sample of the headline problem's outer
   elements, on all host threads (up to 16) and on one.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2101_08825_amd import workloads as W  # noqa: E402

METRIC = "element-pair integrals/s + p50/p99 assemble+solve latency vs FP64 plain"
HEADLINE = "c3_3d24"
LARGE = "c5_3d48_gauss"
WORKLOADS_2D = ("c2a_2d128_d2h", "c2b_2d128_d4h")
# other element types, FP64: (workload, contraction rows per evaluation)
ELEMENT_WORKLOADS = (("hex20_3d24", 90), ("p2tet_3d16", 35), ("quad8_2d128", 22))
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
GOLDEN = os.path.join(ROOT, "tests", "golden", "c3_oracle.json")


def flops_per_eval(dim: int) -> int:
    """Algorithmic flops of one kernel evaluation: distance (dim subtractions,
    dim multiply-adds) plus the contraction into the N+1 + N(N+1)/2 rows of
    the per-pair accumulators (one multiply-add each)."""
    nv = dim + 1
    rows = nv + nv * (nv - 1) // 2
    return dim + 2 * dim + 2 * rows - 1


T0 = time.perf_counter()


def elapsed():
    return time.perf_counter() - T0


def progress(msg):
    print(f"[bench {elapsed():7.1f}s] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("nlq_integrate.hip", "nlq_device.hpp", "nlq_refine.hpp"):
        with open(os.path.join(ROOT, "paper_2101_08825_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(profile):
    """HBM bytes per integration launch from a committed counter profile
    (FETCH_SIZE, WRITE_SIZE scaled by a plain copy), or None when the kernel
    sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_source_sha256_16"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    if fields.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return float(fields["traffic_bytes_per_launch"])


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else float("nan")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def maxrel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


class Problem:
    """A mesh and its data resident on the device."""

    def __init__(self, nlq, ctx, torch, name):
        self.wl = W.WORKLOADS[name]
        self.host = self.wl.mesh()
        _, f, g = W.nodal_data(self.host, self.wl.u)
        self.mesh = nlq.Mesh.create(ctx, self.host.coords, self.host.conn, self.host.constrained)
        self.f = torch.as_tensor(f, dtype=torch.float64, device="cuda")
        self.g = torch.as_tensor(g, dtype=torch.float64, device="cuda")

    def params(self, nlq, precision, **kw):
        wl = self.wl
        return nlq.params(self.host.dim, wl.delta, wl.eps, wl.lmax, precision=precision, kernel=wl.kernel, **kw)


def run_steps(nlq, ctx, torch, problems, precision, steps, warmup, label, keep_last=False):
    """Warm-up steps, then exactly `steps` timed steps; a step assembles, loads,
    lifts and solves every problem of `problems`."""
    step_times, kernel, lat = [], [], []
    pairs = evals = zero_evals = 0
    kept = []
    for it in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pairs = evals = zero_evals = 0
        kt = []
        systems = []
        for p in problems:
            r0 = time.perf_counter()
            s = nlq.System(ctx, p.mesh, p.params(nlq, precision))
            s.set_data_device(p.f.data_ptr(), p.g.data_ptr())
            s.solve(rtol=1e-10, copy=False)
            info = s.info()
            lat.append(time.perf_counter() - r0)
            nq2 = (7 if p.host.dim == 2 else 15) ** 2
            pairs += info.n_pairs
            evals += info.n_evals
            zero_evals += info.n_leaf_zero * nq2
            kt.append((info.t_kernel, info.n_evals - info.n_leaf_zero * nq2))
            systems.append(s)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        last = it == warmup + steps - 1
        for s in systems:
            if keep_last and last:
                kept.append(s)
            else:
                s.close()
        if it >= warmup:
            step_times.append(dt)
            kernel.extend(kt)
        else:
            lat.clear()
        progress(f"{label} step {it + 1}/{warmup + steps} {1e3 * dt:.1f} ms")
    ms = 1e3 * float(np.mean(step_times)) if step_times else float("nan")
    return dict(step_times=step_times, ms=ms, lat=lat, kernel=kernel, pairs=pairs, evals=evals,
                zero_evals=zero_evals, value=pairs / (ms * 1e-3) if step_times else None, kept=kept)


def element_case(nlq, ctx, torch, name, rows):
    """One warm and one timed FP64 assembly + load + solve of an element workload."""
    wl = W.WORKLOADS[name]
    host = wl.mesh()
    mesh = nlq.Mesh.create(ctx, host.coords, host.conn, host.constrained, order=wl.order, shape=wl.shape)
    _, f, g = W.nodal_data(host, wl.u)
    fd = torch.as_tensor(f, dtype=torch.float64, device="cuda")
    gd = torch.as_tensor(g, dtype=torch.float64, device="cuda")
    prm = nlq.params(host.dim, wl.delta, wl.eps, wl.lmax, kernel=wl.kernel, precision=nlq.NLQ_FP64_PLAIN)
    res = None
    for it in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = nlq.System(ctx, mesh, prm)
        s.set_data_device(fd.data_ptr(), gd.data_ptr())
        s.solve(rtol=1e-10, copy=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        info = s.info()
        s.close()
        nq = (9 if host.dim == 2 else 27) if wl.shape == 1 else (7 if host.dim == 2 else 15)
        evaluated = info.n_evals - info.n_leaf_zero * nq * nq
        fpe = 3 * host.dim - 1 + 2 * rows
        res = {"pairs": int(info.n_pairs), "ms_per_step": 1e3 * dt, "pairs_per_s": info.n_pairs / dt,
               "kernel_ms": 1e3 * info.t_kernel, "nnz": int(info.nnz),
               "evaluated_kernel_evals": int(evaluated), "flops_per_eval": fpe,
               "kernel_tflops": evaluated * fpe / info.t_kernel / 1e12,
               "frac_of_fp64_peak": evaluated * fpe / info.t_kernel / 1e12 / FP64_PEAK_TFLOPS}
        progress(f"{name} step {it + 1}/2 {1e3 * dt:.1f} ms")
    mesh.close()
    # the oracle on one seeded outer element away from the boundary, one core
    import oracle
    om = oracle.OracleMesh(host.coords, host.conn, order=wl.order, shape=wl.shape)
    opr = oracle.params(wl.delta, wl.eps, wl.lmax, kernel=wl.kernel)
    c = host.n // 2
    if wl.shape == 1:
        sel = [c + host.n * (c + (host.n * c if host.dim == 3 else 0))]
    else:
        per = 2 if host.dim == 2 else 6
        sel = [per * (c + host.n * (c + (host.n * c if host.dim == 3 else 0)))]
    k = 8 if host.dim == 2 else 1
    sel = np.arange(sel[0], sel[0] + k, dtype=np.int64)
    pairs = int(sum(len(oracle.pairs_of(om, wl.delta + wl.eps, int(l))) for l in sel))
    t0 = time.perf_counter()
    oracle.outer_blocks(om, opr, sel, nthreads=1)
    secs = time.perf_counter() - t0
    res["cpu_oracle_one_core"] = {"pairs_per_s": pairs / secs, "sample": f"{k} outer element(s), {pairs} pairs, "
                                                                        f"{secs:.2f} s"}
    return res


def stream(rate):
    return W.serving_stream(rate_per_s=rate)


def serve_replay(nlq, ctx, precision, reqs, label, deadline_s):
    """Open-loop replay of a request stream through the serving loop."""
    srv = nlq.Server(ctx)
    data = []
    for r in reqs:
        mesh = W.kuhn_mesh(r.dim, r.n, r.k_delta)
        _, f, g = W.nodal_data(mesh, r.u)
        delta = r.k_delta / r.n
        prm = nlq.params(r.dim, delta, delta / r.eps_div, r.lmax, precision=precision)
        data.append((r, prm, f, g))
    t0 = time.perf_counter()
    tickets = []
    for (r, prm, f, g) in data:
        wait = r.arrival_s - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        tickets.append(srv.submit(r.dim, r.n, r.k_delta, prm, f, g, rtol=1e-10))
    progress(f"serving {label}: {len(tickets)} requests submitted")
    res = []
    for k, t in enumerate(tickets):
        while True:
            x = srv.wait(t, timeout_ms=5000)
            if x is not None:
                break
            progress(f"serving {label}: waiting for request {k}: {srv.stats()}")
            if time.perf_counter() - t0 > deadline_s:
                progress(f"serving {label} did not finish within {deadline_s:.0f} s; exiting")
                os._exit(3)
        res.append(x)
        if k % 32 == 31 or k == len(tickets) - 1:
            progress(f"serving {label}: {k + 1} done, last {1e3 * x['latency_s']:.1f} ms")
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.stop()
    bad = [x for x in res if x["status"] != 0]
    if bad:
        raise RuntimeError(f"serving: {len(bad)} requests failed: {bad[0]['error']}")
    lat = [x["latency_s"] for x in res]
    phases = {"queue": [x["queue_s"] for x in res], "setup": [x["setup_s"] for x in res],
              "integrate": [x["assemble_s"] - x["setup_s"] for x in res], "solve": [x["solve_s"] for x in res]}
    return {"requests": len(res), "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
            "mean_ms": 1e3 * float(np.mean(lat)), "wall_s": wall, "requests_per_s": len(res) / wall,
            "arrival_rate_per_s": len(reqs) / reqs[-1].arrival_s if reqs else None,
            "phase_p50_ms": {k: 1e3 * percentile(v, 50) for k, v in phases.items()},
            "pairs": int(sum(x["n_pairs"] for x in res)), "launches": st["launches"],
            "mean_requests_per_launch": st["launch_segments"] / max(st["launches"], 1),
            "max_requests_per_launch": st["max_per_launch"], "max_admitted": st["max_admitted"],
            "peak_hbm_gib": st["peak_bytes"] / 2**30}


def cpu_baseline(n_all=16, n_one=1, seed=0):
    """The oracle on seeded samples of the headline problem's outer elements:
    Algorithm 1 with every leaf integrated, over all pairs of each (the blocks
    are formed, not scattered into a matrix)."""
    import oracle
    wl = W.WORKLOADS[HEADLINE]
    mesh = wl.mesh()
    m = oracle.OracleMesh(mesh.coords, mesh.conn)
    prm = oracle.params(wl.delta, wl.eps, wl.lmax)
    nt = max(1, min(16, os.cpu_count() or 1))
    rng = np.random.default_rng(seed)
    out = {}
    for key, k, threads in (("all", max(n_all, nt), nt), ("one", n_one, 1)):
        sel = np.sort(rng.choice(mesh.n_elems, k, replace=False))
        pairs = int(sum(len(oracle.pairs_of(m, wl.delta + wl.eps, int(l))) for l in sel))
        t0 = time.perf_counter()
        oracle.outer_blocks(m, prm, sel, nthreads=threads)
        secs = time.perf_counter() - t0
        out[key] = (pairs / secs, pairs, k, secs, threads)
        progress(f"cpu baseline ({threads} threads): {k} outer elements, {pairs} pairs, {secs:.1f} s")
    v, pairs, k, secs, nt = out["all"]
    v1, pairs1, k1, secs1, _ = out["one"]
    return {"value": v, "unit": "pairs/s", "cores": nt, "kind": "oracle",
            "sample": f"{k} seeded outer elements of the 24^3 x 6 tets problem ({pairs} pairs, "
                      f"Algorithm 1 + integration of every pair's block), {secs:.1f} s on {nt} threads",
            "single_core": {"value": v1, "unit": "pairs/s", "cores": 1,
                            "sample": f"{k1} seeded outer elements ({pairs1} pairs), {secs1:.1f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--budget-s", type=float, default=540.0,
                    help="wall-clock budget: optional sections that would pass it are skipped")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--large-fraction", type=float, default=1.0 / 1024)
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-2d", action="store_true")
    ap.add_argument("--no-elements", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU only (the path has no cross-GPU sharding); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    progress("importing torch")
    import torch
    from paper_2101_08825_amd import nlq
    assert torch.cuda.is_available(), "bench needs the GPU"
    torch.cuda.init()
    ctx = nlq.Context(0)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    head = Problem(nlq, ctx, torch, HEADLINE)
    torch.cuda.synchronize()
    progress("headline problem resident")
    skipped = {}

    def fits(section, estimate_s):
        if elapsed() + estimate_s <= args.budget_s:
            return True
        skipped[section] = f"estimated {estimate_s:.0f} s beyond the {args.budget_s:.0f} s budget " \
                           f"at {elapsed():.0f} s"
        progress(f"skipping {section}: {skipped[section]}")
        return False

    tuned = {}
    if not args.no_autotune:
        for precision in (nlq.NLQ_FP32_MIXED,) + (() if args.skip_fp64 else (nlq.NLQ_FP64_PLAIN,)):
            s = nlq.System.prepare(ctx, head.mesh, head.params(nlq, precision))
            tuned[f"{HEADLINE}/{'fp32' if precision else 'fp64'}"] = s.autotune(budget_s=4.0)
            s.close()
        progress(f"autotuned: {tuned}")

    # ---- headline: K timed steps, FP32-mixed
    mixed = run_steps(nlq, ctx, torch, [head], nlq.NLQ_FP32_MIXED, args.steps, args.warmup, "c3 fp32",
                      keep_last=True)
    plain = None
    if not args.skip_fp64 and fits("fp64_plain", 2.6 * mixed["ms"] * 1e-3 * args.fp64_steps):
        plain = run_steps(nlq, ctx, torch, [head], nlq.NLQ_FP64_PLAIN, args.fp64_steps, 0, "c3 fp64",
                          keep_last=True)

    # ---- errors against the oracle's rows and the FP64 path
    errors = {}
    gold = json.load(open(GOLDEN))
    s32 = mixed["kept"][0]
    rp, col, v32 = s32.csr()
    u32, _ = s32.solve(rtol=1e-10)
    for key, s_ in (("fp32_mixed", s32),) + ((("fp64_plain", plain["kept"][0]),) if plain else ()):
        _, _, v = (rp, col, v32) if s_ is s32 else s_.csr()
        got = np.concatenate([v[rp[r["node"]]:rp[r["node"] + 1]] for r in gold["rows"].values()])
        exp = np.concatenate([[float.fromhex(x) for x in r["vals"]] for r in gold["rows"].values()])
        errors[f"{key}_vs_oracle_rows"] = {"rel_frobenius": rel(got, exp), "max_entry_rel": maxrel(got, exp),
                                           "entries": int(exp.size)}
    if plain:
        _, _, v64 = plain["kept"][0].csr()
        u64, _ = plain["kept"][0].solve(rtol=1e-12)
        errors["fp32_vs_fp64_matrix"] = {"rel_frobenius": rel(v32, v64), "max_entry_rel": maxrel(v32, v64)}
        errors["fp32_vs_fp64_solution_rel_l2"] = rel(u32, u64)
        ux = head.wl.u(head.host.coords)
        errors["solution_vs_exact_u_rel_l2"] = {"fp32_mixed": rel(u32, ux), "fp64_plain": rel(u64, ux)}
    for s in mixed["kept"] + (plain["kept"] if plain else []):
        s.close()
    progress(f"errors: {errors}")

    # ---- the 48^3 Gaussian problem on a seeded sample spread over the mesh
    large = None
    if not args.no_large and fits("large_48cubed", 60.0):
        big = Problem(nlq, ctx, torch, LARGE)
        large = {"workload": "3D [0,1]^3 Kuhn 48^3 x 6 (663,552 P1 tets), truncated Gaussian kernel, "
                             "delta=3h, eps=delta/32, depth<=6, 15-pt rule"}
        lo, hi = W.stratified_ranges(big.host.n_elems, args.large_fraction, 32, seed=5)
        for precision, key in ((nlq.NLQ_FP32_MIXED, "fp32_mixed"), (nlq.NLQ_FP64_PLAIN, "fp64_plain")):
            if precision == nlq.NLQ_FP64_PLAIN and (args.skip_fp64 or not fits("large_48cubed_fp64", 60.0)):
                continue
            t0 = time.perf_counter()
            s = nlq.System.prepare(ctx, big.mesh, big.params(nlq, precision))
            torch.cuda.synchronize()
            t_prep = time.perf_counter() - t0
            off, _ = s.pairs()
            t, leaves, nzero = s.integrate_ranges(lo, hi)
            sample_pairs = int(sum(off[b] - off[a] for a, b in zip(lo, hi)))
            total_pairs = int(off[-1])
            evals = int(np.sum(leaves)) * 225
            large[key] = {"sample_outer_elements": int(np.sum(hi - lo)), "sample_pairs": sample_pairs,
                          "kernel_s": t, "pairs_per_s": sample_pairs / t,
                          "alg1_kernel_evals": evals, "evaluated_kernel_evals": evals - nzero * 225,
                          "whole_mesh_kernel_s_extrapolated": t * total_pairs / sample_pairs,
                          "prepare_s": t_prep, "pairs": total_pairs}
            s.close()
            progress(f"48^3 {key}: {large[key]}")
        big.mesh.close()
        large["sample"] = (f"seeded {args.large_fraction:.6f} of the outer elements in 32 strata, one launch; "
                           "whole-mesh time = sample time x total pairs / sample pairs")

    # ---- 2D 128^2 problems
    two_d = None
    if not args.no_2d and fits("2d_128", 20.0):
        probs = [Problem(nlq, ctx, torch, n) for n in WORKLOADS_2D]
        m2 = run_steps(nlq, ctx, torch, probs, nlq.NLQ_FP32_MIXED, 3, 1, "2d fp32")
        p2 = None if args.skip_fp64 else run_steps(nlq, ctx, torch, probs, nlq.NLQ_FP64_PLAIN, 3, 1, "2d fp64")
        kt = sum(t for t, _ in m2["kernel"])
        ke = sum(e for _, e in m2["kernel"])
        two_d = {"workload": "2D [0,1]^2 Kuhn 128x128 (32768 P1 triangles), delta in {2h,4h}, eps=delta/32, "
                             "depth<=5, 7-pt rule, constant kernel; a step assembles + solves both",
                 "value": m2["value"], "ms_per_step": m2["ms"], "pairs_per_step": m2["pairs"],
                 "kernel_ms_per_step": 1e3 * kt / 3,
                 "kernel_tflops": ke * flops_per_eval(2) / kt / 1e12,
                 "fp64_plain": None if p2 is None else {"value": p2["value"], "ms_per_step": p2["ms"]}}
        for p in probs:
            p.mesh.close()

    # ---- other element types (FP64)
    elements = {}
    if not args.no_elements and fits("element_types", 60.0):
        for name, rows in ELEMENT_WORKLOADS:
            elements[name] = element_case(nlq, ctx, torch, name, rows)
            progress(f"{name}: {elements[name]}")
        elements["what"] = ("FP64 whole assembly + load + solve of one step after a warm one; kernel_tflops = "
                            "evaluated kernel evaluations x (distance + 2 x rows) flops / integration time; "
                            f"frac_of_fp64_peak against {FP64_PEAK_TFLOPS} TFLOP/s")

    # ---- serving: capacity at 20/s, then 0.8 of it for both precisions
    serving = {}
    if args.serve_requests > 0 and fits("serving", 150.0):
        base = stream(20.0)[:args.serve_requests]
        over = serve_replay(nlq, ctx, nlq.NLQ_FP32_MIXED, base, "fp32 at 20/s", 400.0)
        capacity = over["requests_per_s"]
        lam = 0.8 * capacity
        serving["overload_fp32_mixed"] = dict(over, what="offered at 20/s, beyond capacity: p99 is backlog drain")
        serving["capacity_requests_per_s"] = capacity
        if fits("serving_at_0.8_capacity", over["wall_s"] * 1.3 + 10):
            reqs = stream(lam)[:args.serve_requests]
            at = serve_replay(nlq, ctx, nlq.NLQ_FP32_MIXED, reqs, f"fp32 at {lam:.2f}/s", 400.0)
            serving["fp32_mixed"] = at
            if not args.skip_fp64 and fits("serving_fp64_plain", over["wall_s"] * 2.6 + 10):
                serving["fp64_plain"] = serve_replay(nlq, ctx, nlq.NLQ_FP64_PLAIN, reqs, f"fp64 at {lam:.2f}/s",
                                                     400.0)
        serving["workload"] = (f"the first {len(base)} requests of the seeded stream (2D 8^2..96^2 / 3D 6^3..20^3, "
                               "delta 2h..4h, eps delta/16, depth 3, random quadratic u), open loop; the same "
                               "requests at Poisson rate 0.8 x capacity, capacity = requests/s of the 20/s run")
        serving["arrival_rate_per_s"] = lam

    # ---- line
    fpe = flops_per_eval(3)
    kt = sum(t for t, _ in mixed["kernel"])
    ke = sum(e for _, e in mixed["kernel"])
    achieved = ke * fpe / kt / 1e12
    lat = serving.get("fp32_mixed")
    out = {
        "metric": METRIC,
        "value": mixed["value"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "3D [0,1]^3 Kuhn 24^3 cubes x 6 (82944 P1 tets, 15625 nodes), delta=3h=0.125, "
                        "eps=delta/16, depth<=4, 15-pt rule, constant kernel C_{delta,eps}, u=x1^2, f=-2; "
                        "per step: tables + pair list + pattern + Algorithm 1 integration + FP64 CSR + "
                        "load/lift + CG",
            "pairs_per_step": mixed["pairs"],
            "alg1_kernel_evals_per_step": mixed["evals"],
            "evaluated_kernel_evals_per_step": mixed["evals"] - mixed["zero_evals"],
            "precision": "fp32 kernel evaluation + fp32 matrix-core contraction, fp64 blocks/CSR/CG",
        },
        "latency_ms": ({"p50": lat["p50_ms"], "p99": lat["p99_ms"],
                        "source": f"serving stream at 0.8 x capacity ({serving['arrival_rate_per_s']:.2f}/s)"}
                       if lat else {"p50": 1e3 * percentile(mixed["lat"], 50),
                                    "p99": 1e3 * percentile(mixed["lat"], 99), "source": "headline steps"}),
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": measured_traffic("hbm_traffic_k_integrate_3d24_c3.md"),
            "kernel": "k_integrate<3,1>",
            "flops_per_eval": fpe,
            "evals": "kernel evaluations performed (Algorithm 1's less the all-zero leaves not evaluated)",
            "kernel_ms_per_step": 1e3 * kt / args.steps,
        },
        "errors": errors,
    }
    if plain is not None:
        pkt = sum(t for t, _ in plain["kernel"])
        out["fp64_plain"] = {"value": plain["value"], "ms_per_step": plain["ms"], "steps": args.fp64_steps,
                             "kernel_ms_per_step": 1e3 * pkt / args.fp64_steps}
        out["speedup_vs_fp64_plain"] = out["value"] / plain["value"]
    if serving:
        out["serving"] = serving
        if "fp64_plain" in serving and "fp32_mixed" in serving:
            out["fp64_plain_latency_ms"] = {"p50": serving["fp64_plain"]["p50_ms"],
                                            "p99": serving["fp64_plain"]["p99_ms"]}
            out["p99_speedup_vs_fp64_plain"] = serving["fp64_plain"]["p99_ms"] / serving["fp32_mixed"]["p99_ms"]
    if large:
        out["large_48cubed_gauss"] = large
    if two_d:
        out["2d_128"] = two_d
    if elements:
        out["element_types"] = elements
    if tuned:
        out["autotune"] = tuned
    head.mesh.close()
    ctx.close()
    if not args.no_cpu_baseline and fits("cpu_baseline", 45.0):
        out["cpu_baseline"] = cpu_baseline()
    if skipped:
        out["skipped"] = skipped
    out["wall_s"] = elapsed()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
