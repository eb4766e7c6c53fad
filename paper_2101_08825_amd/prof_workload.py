"""Profiling driver: integration launches of one workload, plus an optional
plain device copy of known size (the reference for HBM byte counters).

    python -m paper_2101_08825_amd.prof_workload --workload c2b_2d128_d4h --precision 1 --reps 2
    python -m paper_2101_08825_amd.prof_workload --copy-mib 1024

Run it under rocprofv3 (kernel trace or counters); it prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2101_08825_amd import workloads as W  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="")
    ap.add_argument("--precision", type=int, default=1)
    ap.add_argument("--reps", type=int, default=1)
    ap.add_argument("--copy-mib", type=int, default=0)
    a = ap.parse_args()
    import torch
    from paper_2101_08825_amd import nlq
    assert torch.cuda.is_available()
    out = {}
    if a.copy_mib > 0:
        n = a.copy_mib << 18   # float32 elements
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        out["copy_bytes_read"] = out["copy_bytes_written"] = 4 * n
    if a.workload:
        wl = W.WORKLOADS[a.workload]
        mesh = wl.mesh()
        ctx = nlq.Context(0)
        m = nlq.Mesh.create(ctx, mesh.coords, mesh.conn, mesh.constrained, order=wl.order, shape=wl.shape)
        precision = a.precision if (wl.order == 1 and wl.shape == 0) else nlq.NLQ_FP64_PLAIN
        s = nlq.System(ctx, m, nlq.params(mesh.dim, wl.delta, wl.eps, wl.lmax, precision=precision,
                                          kernel=wl.kernel))
        times = [s.info().t_kernel]
        for _ in range(a.reps - 1):
            s.reassemble()
            times.append(s.info().t_kernel)
        inf = s.info()
        out.update(workload=a.workload, precision=precision, t_kernel_ms=[1e3 * t for t in times],
                   n_pairs=inf.n_pairs, n_evals=inf.n_evals, n_leaf_zero=inf.n_leaf_zero, nnz=inf.nnz,
                   n_leaf=list(inf.n_leaf))
        s.close()
        m.close()
        ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
