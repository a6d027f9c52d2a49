"""Exact optimal tours of small fields, from the oracle alone (test infrastructure).

Writes tests/golden/optima_small_fields.json: the Held-Karp optimum (oracle
`orc_held_karp`, the textbook dynamic programme over subsets; m <= 24 free
cells) of

* the paper's fields of Sec. IV-C (3x3, 3x4, 4x4, 4x5, 5x5; start cell (0, 0), no
  obstacles), as open paths (eq. (1a)) and closed tours, and
* every instance of the 256-field batch workload with m <= 24 (closed tours).

Costs are the integer travel costs of eq. (3) at the default scale
(deciseconds at 5 m cells flown at 5 m/s).  Nothing here touches the GPU path.

    python -m oracle.paper_optima [--out PATH] [--jobs 8]
"""
import argparse
import json
import os
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PAPER_FIELDS = [(3, 3), (3, 4), (4, 4), (4, 5), (5, 5)]


def _paper(task):
    import oracle
    rows, cols, closed = task
    o = oracle.OracleQubo(rows, cols, closed=closed, dense=False)
    return f"{rows}x{cols}_{'closed' if closed else 'open'}", o.m, o.held_karp()


def _batch(task):
    import oracle
    from paper_2608_25376_amd import inputs
    inst = task
    g = inputs.workload("batch256").grids[inst]
    o = oracle.OracleQubo(g.rows, g.cols, nofly=g.nofly, dense=False)
    return str(g.inst_id), o.m, o.held_karp()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(ROOT, "tests", "golden", "optima_small_fields.json"))
    ap.add_argument("--jobs", type=int, default=8)
    args = ap.parse_args()
    from paper_2608_25376_amd import inputs
    grids = inputs.workload("batch256").grids
    small = [i for i, g in enumerate(grids) if g.n_free <= 24]
    # the largest fields first, so the pool's tail is short
    small.sort(key=lambda i: -grids[i].n_free)
    paper_tasks = [(r, c, closed) for (r, c) in PAPER_FIELDS for closed in (False, True)]
    paper_tasks.sort(key=lambda t: -(t[0] * t[1]))
    with Pool(args.jobs) as pool:
        paper = pool.map(_paper, paper_tasks, chunksize=1)
        batch = pool.map(_batch, small, chunksize=1)
    out = {
        "about": "Held-Karp optima (oracle orc_held_karp) of the paper's fields (Sec. IV-C) as open paths and "
                 "closed tours, and of the 256-field batch workload's instances with m <= 24 (closed tours); "
                 "integer costs at the default scale (deciseconds). Written by oracle/paper_optima.py.",
        "paper_fields": {k: {"m": m, "optimum": v} for k, m, v in sorted(paper)},
        "batch256": {k: {"m": m, "optimum": v} for k, m, v in sorted(batch, key=lambda t: int(t[0]))},
    }
    for k, v in out["paper_fields"].items():
        assert v["optimum"] > 0, k
    for k, v in out["batch256"].items():
        assert v["optimum"] > 0, k
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"wrote {args.out}: {len(paper)} paper fields, {len(batch)} batch instances")


if __name__ == "__main__":
    main()
