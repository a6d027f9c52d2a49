"""The paper's own experiment shape: fields of 3x3 to 6x6 cells (including the
non-square 3x4, 4x5 and 5x6), the start cell fixed at (0, 0), no obstacles,
one annealing run per field.  Reports the cost of the best tour in seconds and
the solve time against the grid size (the two results of Sec. IV-D, Figs. 2
and 3; the conclusion, Sec. V, states optimal paths in under 320 ms), for the
open path of eq. (1a) and for the closed tour.

Driver only: every numeric step runs in libuavq (QUBO build, annealing,
decode).  Costs are integers in tenths of a second: a cell of 5 m flown at
5 m/s takes one second (Sec. IV-C), so w = round(10 d) is in deciseconds and the
energy of a feasible state is the tour time in deciseconds.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2608_25376_amd import uavq  # noqa: E402

SIZES = [(3, 3), (3, 4), (4, 4), (4, 5), (5, 5), (5, 6), (6, 6)]


def solve(rows, cols, closed, replicas=1024, sweeps=1000, T0=100.0, T1=0.5, seed=1):
    """One field: build, upload, anneal (timed with HIP events), decode.
    Returns a dict with the best tour, its cost and the times."""
    import torch
    t_host = time.perf_counter()
    q = uavq.qubo_build(rows, cols, closed=closed)
    plan = uavq.Plan([q], [rows * 100 + cols], replicas, sweeps, T0, T1, seed)
    plan.upload()
    out = plan.alloc_outputs()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plan.anneal(out=out)
    e1.record()
    torch.cuda.synchronize()
    anneal_ms = e0.elapsed_time(e1)
    best_E = int(out.inst_best_E.cpu().numpy()[0])
    state = out.inst_best_state.cpu().numpy().view(np.uint32)[: q.state_words]
    path, cost = uavq.decode_path(q, state)
    total_ms = (time.perf_counter() - t_host) * 1e3
    return {"rows": rows, "cols": cols, "closed": closed, "m": q.m, "n_vars": q.n_vars, "replicas": replicas,
            "sweeps": sweeps, "best_E": best_E, "feasible": path is not None,
            "cost_s": cost / 10.0 if path is not None else None,
            "path": [int(v) for v in path[: q.m + (2 if closed else 1)]] if path is not None else None,
            "anneal_ms": anneal_ms, "total_ms": total_ms,
            "best_replica": int(out.inst_best_replica.cpu().numpy()[0]),
            "best_sweep": int(out.inst_best_sweep.cpu().numpy()[0])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--replicas", type=int, default=1024)
    ap.add_argument("--sweeps", type=int, default=1000)
    ap.add_argument("--T0", type=float, default=100.0)
    ap.add_argument("--T1", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available()
    rows_out = []
    solve(3, 3, True, 64, 10)   # warm the library and the runtime
    for closed in (False, True):
        for r, c in SIZES:
            res = solve(r, c, closed, args.replicas, args.sweeps, args.T0, args.T1, args.seed)
            print(json.dumps(res), flush=True)
            rows_out.append(res)
    if args.out:
        with open(args.out, "w") as f:
            for res in rows_out:
                f.write(json.dumps(res) + "\n")


if __name__ == "__main__":
    main()
