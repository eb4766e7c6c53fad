"""Benchmark of the hot path on one MI355X.

Throughput: a step is one pass of the whole path (element tables, pair list,
CSR pattern, Algorithm 1 + leaf integration, FP64 CSR accumulation, load vector
+ lifting, CG solve) for each of the two 2D 128x128 problems (delta = 2h and
4h, eps = delta/32, depth <= 5, constant kernel, u = x1^2 + x2^2).  Mesh and
data are resident in HBM before the timed region.  The value is element-pair
integrals per second of the FP32-mixed path; the FP64 plain path is timed on
the same steps.

Latency: the seeded serving stream (Poisson arrivals at 20/s; 2D meshes 8^2 ..
96^2 and 3D 6^3 .. 20^3, sizes uniform in log; delta in {2h, 3h, 4h},
eps = delta/16, depth 3; random quadratic u) replayed open loop against the
library's serving loop, once per precision; p50 / p99 of submit -> solution.
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
WORKLOADS = ("c2a_2d128_d2h", "c2b_2d128_d4h")
FP32_VECTOR_PEAK_TFLOPS = 157.3


def flops_per_eval(dim: int) -> int:
    """Algorithmic flops of one kernel evaluation: distance (dim subtractions,
    dim multiply-adds) plus the contraction into the N+1 + N(N+1)/2 rows of
    the per-pair accumulators (one multiply-add each)."""
    nv = dim + 1
    rows = nv + nv * (nv - 1) // 2
    return dim + 2 * dim + 2 * rows - 1


T0 = time.perf_counter()


def progress(msg):
    print(f"[bench {time.perf_counter() - T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per integration launch from the committed counter profile
    (FETCH_SIZE, WRITE_SIZE scaled by a plain copy), or None when the kernel
    sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_k_integrate_2d128.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_source_sha256_16"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    h = hashlib.sha256()
    for f in ("nlq_integrate.hip", "nlq_device.hpp", "nlq_refine.hpp"):
        with open(os.path.join(ROOT, "paper_2101_08825_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if fields.get("kernel_source_sha256_16") != h.hexdigest()[:16]:
        return None
    return float(fields["traffic_bytes_per_launch"])


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else float("nan")


def run_steps(nlq, ctx, setups, precision, steps, warmup, torch, min_l2=0):
    lat = []
    step_times = []
    kernel = []
    pairs_per_step = 0
    evals_per_step = 0
    for it in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pairs = evals = 0
        kt = []
        for (mesh, wl, f_t, g_t) in setups:
            r0 = time.perf_counter()
            s = nlq.System(ctx, mesh, nlq.params(2, wl.delta, wl.eps, wl.lmax, precision=precision,
                                                 min_dist_l2=min_l2))
            s.set_data_device(f_t.data_ptr(), g_t.data_ptr())
            _, inf = s.solve(rtol=1e-10, copy=False)
            info = s.info()
            s.close()
            lat.append(time.perf_counter() - r0)
            pairs += info.n_pairs
            evals += info.n_evals
            kt.append((info.t_kernel, info.n_evals))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if it >= warmup:
            step_times.append(dt)
            kernel.extend(kt)
        else:
            lat.clear()
        pairs_per_step, evals_per_step = pairs, evals
        progress(f"precision {precision}{f' (refine test {min_l2})' if min_l2 else ''} step {it + 1}/{warmup + steps} "
                 f"{1e3 * dt:.1f} ms")
    return dict(step_times=step_times, lat=lat, kernel=kernel, pairs=pairs_per_step,
                evals=evals_per_step)


def serve_replay(nlq, ctx, precision, n_requests, cache):
    """Open-loop replay of the first n_requests of the seeded serving stream."""
    reqs = W.serving_stream()[:n_requests]
    srv = nlq.Server(ctx, cache_systems=cache)
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
    progress(f"serving precision {precision}: {len(tickets)} requests submitted")
    res = []
    deadline = time.perf_counter() + 420.0
    for k, t in enumerate(tickets):
        while True:
            x = srv.wait(t, timeout_ms=5000)
            if x is not None:
                break
            st = srv.stats()
            progress(f"serving precision {precision}: waiting for request {k}: {st}")
            if time.perf_counter() > deadline:
                progress("serving did not finish within 420 s; exiting without stopping the server")
                os._exit(3)
        res.append(x)
        progress(f"serving precision {precision}: request {k} done in {1e3 * x['latency_s']:.1f} ms "
                 f"(dim {reqs[k].dim}, n {reqs[k].n}, {x['n_pairs']} pairs, {x['launches']} launches; "
                 f"queue {1e3 * x['queue_s']:.1f} setup {1e3 * x['setup_s']:.1f} "
                 f"integrate {1e3 * (x['assemble_s'] - x['setup_s']):.1f} solve {1e3 * x['solve_s']:.1f} ms, "
                 f"{x['cg_iterations']} CG iterations)")
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.stop()
    bad = [x for x in res if x["status"] != 0]
    if bad:
        raise RuntimeError(f"serving: {len(bad)} requests failed: {bad[0]['error']}")
    lat = [x["latency_s"] for x in res]
    pairs = sum(x["n_pairs"] for x in res)
    phases = {"queue": [x["queue_s"] for x in res], "setup": [x["setup_s"] for x in res],
              "integrate": [x["assemble_s"] - x["setup_s"] for x in res], "solve": [x["solve_s"] for x in res]}
    return {"requests": len(res), "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
            "phase_p50_ms": {k: 1e3 * percentile(v, 50) for k, v in phases.items()},
            "mean_ms": 1e3 * float(np.mean(lat)), "wall_s": wall, "pairs": pairs,
            "launches": st["launches"], "mean_requests_per_launch": st["launch_segments"] / max(st["launches"], 1),
            "max_requests_per_launch": st["max_per_launch"], "max_admitted": st["max_admitted"],
            "cache_hits": st["cache_hits"], "peak_hbm_gib": st["peak_bytes"] / 2**30}


def cpu_baseline(sample_frac=0.10, seed=0):
    """The oracle on a seeded sample of outer elements of both problems."""
    import oracle
    nt = max(1, min(16, os.cpu_count() or 1))
    pairs = 0
    secs = 0.0
    nsel = 0
    for name in WORKLOADS:
        wl = W.WORKLOADS[name]
        mesh = wl.mesh()
        m = oracle.OracleMesh(mesh.coords, mesh.conn)
        prm = oracle.params(wl.delta, wl.eps, wl.lmax)
        off, pm = oracle.pairs(m, wl.delta + wl.eps, nt)
        rp, col = oracle.pattern(m, off, pm)
        rng = np.random.default_rng(seed)
        k = max(1, int(sample_frac * mesh.n_elems))
        sel = np.sort(rng.choice(mesh.n_elems, k, replace=False))
        t0 = time.perf_counter()
        oracle.assemble(m, prm, off, pm, rp, col, sel=sel, nthreads=nt)
        secs += time.perf_counter() - t0
        progress(f"cpu baseline {name} done")
        pairs += int(np.sum(off[sel + 1] - off[sel]))
        nsel += k
    return {"value": pairs / secs, "unit": "pairs/s", "cores": nt, "kind": "oracle",
            "sample": f"{nsel} seeded outer elements ({100 * sample_frac:.0f}% of each 128^2 "
                      f"problem, {pairs} pairs, Algorithm 1 + integration + CSR scatter), "
                      f"{secs:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-cache", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-ablation", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU only (the path has no cross-GPU sharding); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    progress("importing torch")
    import torch
    from paper_2101_08825_amd import nlq
    assert torch.cuda.is_available(), "bench needs the GPU"
    progress("torch ready")
    torch.cuda.init()
    ctx = nlq.Context(0)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    setups = []
    for name in WORKLOADS:
        wl = W.WORKLOADS[name]
        mesh = wl.mesh()
        _, f, g = W.nodal_data(mesh, wl.u)
        m = nlq.Mesh.create(ctx, mesh.coords, mesh.conn, mesh.constrained)
        f_t = torch.as_tensor(f, dtype=torch.float64, device="cuda")
        g_t = torch.as_tensor(g, dtype=torch.float64, device="cuda")
        setups.append((m, wl, f_t, g_t))
    torch.cuda.synchronize()

    # autotune the integration launch of each problem and precision (kept in the
    # context, so the timed steps' assemblies use it); not timed
    tuned = {}
    if not args.no_autotune:
        for precision in (nlq.NLQ_FP32_MIXED, nlq.NLQ_FP64_PLAIN):
            for (mesh, wl, f_t, g_t) in setups:
                s = nlq.System(ctx, mesh, nlq.params(2, wl.delta, wl.eps, wl.lmax, precision=precision))
                tuned[f"{wl.name}/{'fp32' if precision else 'fp64'}"] = s.autotune(budget_s=3.0)
                s.close()
        progress(f"autotuned: {tuned}")

    mixed = run_steps(nlq, ctx, setups, nlq.NLQ_FP32_MIXED, args.steps, args.warmup, torch)
    plain = None
    if not args.skip_fp64:
        plain = run_steps(nlq, ctx, setups, nlq.NLQ_FP64_PLAIN, args.steps, args.warmup, torch)

    # ablations of Algorithm 1's refine test, the Euclidean gap to the inner
    # element's box (1) or to its quadrature points' box (2): both drop only zero
    # contributions (the same matrices to round-off, fewer leaves)
    ablations = {}
    if not args.no_ablation:
        mesh, wl, _, _ = setups[-1]
        ref = nlq.System(ctx, mesh, nlq.params(2, wl.delta, wl.eps, wl.lmax, precision=nlq.NLQ_FP32_MIXED))
        ref_val = ref.csr()[2]
        ref.close()
        what = {1: "the Euclidean gap between the sub-element's box and the inner element's box",
                2: "the Euclidean gap between the sub-element's box and the box of the inner element's "
                   "quadrature points (a tighter test of our own)"}
        for mode, key in ((1, "ablation_l2_box_gap"), (2, "ablation_quad_point_box")):
            r = run_steps(nlq, ctx, setups, nlq.NLQ_FP32_MIXED, args.steps, args.warmup, torch, min_l2=mode)
            s = nlq.System(ctx, mesh, nlq.params(2, wl.delta, wl.eps, wl.lmax, precision=nlq.NLQ_FP32_MIXED,
                                                 min_dist_l2=mode))
            val = s.csr()[2]
            s.close()
            ms_r = 1e3 * float(np.mean(r["step_times"]))
            ablations[key] = {
                "value": r["pairs"] / (ms_r * 1e-3), "unit": "pairs/s", "ms_per_step": ms_r,
                "kernel_ms_per_step": 1e3 * sum(t for t, _ in r["kernel"]) / args.steps,
                "kernel_evals_per_step": r["evals"],
                "rel_frobenius_vs_paper_test": float(np.linalg.norm(val - ref_val) / np.linalg.norm(ref_val)),
                "what": f"FP32-mixed steps with Algorithm 1's refine test on {what[mode]} instead of the "
                        "L_inf gap of Sec. 5.1 (same pair lists and J^int test; drops sub-elements whose "
                        "every point pair is beyond delta+eps); matrix difference measured on delta = 4h",
            }

    serve = serve64 = None
    if args.serve_requests > 0:
        serve = serve_replay(nlq, ctx, nlq.NLQ_FP32_MIXED, args.serve_requests, bool(args.serve_cache))
        if not args.skip_fp64:
            serve64 = serve_replay(nlq, ctx, nlq.NLQ_FP64_PLAIN, args.serve_requests, bool(args.serve_cache))

    ms = 1e3 * float(np.mean(mixed["step_times"]))
    value = mixed["pairs"] / (ms * 1e-3)
    # dominant kernel: the integration launch, timed with HIP events on its stream
    fpe = flops_per_eval(2)
    kt = sum(t for t, _ in mixed["kernel"])
    ke = sum(e for _, e in mixed["kernel"])
    achieved = ke * fpe / kt / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "2D [0,1]^2 Kuhn 128x128 (32768 P1 triangles), delta in {2h,4h}, "
                        "eps=delta/32, depth<=5, 7-pt rule, constant gamma, u=x1^2+x2^2, "
                        "f=-4; per step: assemble + load/lift + CG for both horizons",
            "pairs_per_step": mixed["pairs"],
            "kernel_evals_per_step": mixed["evals"],
            "precision": "fp32 kernel evaluation + fp32 matrix-core contraction, fp64 blocks/CSR/CG",
        },
        "latency_ms": ({"p50": serve["p50_ms"], "p99": serve["p99_ms"], "source": "serving stream"}
                       if serve else {"p50": 1e3 * percentile(mixed["lat"], 50),
                                      "p99": 1e3 * percentile(mixed["lat"], 99), "source": "128^2 steps"}),
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": measured_traffic(),
            "kernel": "k_integrate<2,1>",
            "flops_per_eval": fpe,
            "kernel_ms_per_step": 1e3 * kt / args.steps,
        },
    }
    if serve:
        which = "all" if serve["requests"] >= 256 else f"first {serve['requests']} of the"
        out["serving"] = dict(serve, workload=f"{which} 256 requests of the seeded stream "
                              "(Poisson 20/s, 2D 8^2..96^2 / 3D 6^3..20^3, delta 2h..4h, eps delta/16, "
                              "depth 3), open loop", matrix_cache=bool(args.serve_cache))
    if serve64:
        out["serving_fp64_plain"] = serve64
    if tuned:
        out["autotune"] = tuned
    for key, ab in ablations.items():
        ab["speedup_vs_paper_test"] = ab["value"] / value
        out[key] = ab
    out["c2_request_ms"] = {"p50": 1e3 * percentile(mixed["lat"], 50), "p99": 1e3 * percentile(mixed["lat"], 99)}
    if plain is not None:
        pms = 1e3 * float(np.mean(plain["step_times"]))
        pkt = sum(t for t, _ in plain["kernel"])
        out["fp64_plain"] = {
            "value": plain["pairs"] / (pms * 1e-3),
            "ms_per_step": pms,
            "latency_ms": ({"p50": serve64["p50_ms"], "p99": serve64["p99_ms"], "source": "serving stream"}
                           if serve64 else {"p50": 1e3 * percentile(plain["lat"], 50),
                                            "p99": 1e3 * percentile(plain["lat"], 99), "source": "128^2 steps"}),
            "kernel_ms_per_step": 1e3 * pkt / args.steps,
        }
        out["speedup_vs_fp64_plain"] = out["value"] / out["fp64_plain"]["value"]
        if serve and serve64:
            out["p99_speedup_vs_fp64_plain"] = serve64["p99_ms"] / serve["p99_ms"]
    for (m, *_rest) in setups:
        m.close()
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
