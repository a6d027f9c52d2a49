"""Parallel tempering against the plain annealer at the same work.

The paper runs many independent replicas through one geometric schedule
(Sec. III-C, Alg. 1).  Parallel tempering spends the same replica-sweeps on K
slots of R chains at the fixed temperatures of a ladder, neighbouring slots
trading states between segments.  This driver runs both on the same fields
(the paper's sizes of Sec. IV-D as open paths, and an 8x8 field with no-fly
cells, 54 cells to visit, as a closed tour), and the plain annealer once more
with several times the sweeps for a comparison at about equal GPU time; it
reports the best tour, its cost in seconds and the GPU time of each.

Driver only: every numeric step runs in libuavq (QUBO build, sweeps,
exchange rounds, decode).  Costs are in tenths of a second (a 5 m cell flown
at 5 m/s takes one second, Sec. IV-C).
"""
import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2608_25376_amd import inputs, uavq  # noqa: E402

FIELDS = [  # name, rows, cols, no-fly density, closed
    ("3x4", 3, 4, 0.0, False), ("4x4", 4, 4, 0.0, False), ("4x5", 4, 5, 0.0, False),
    ("5x6", 5, 6, 0.0, False), ("6x6", 6, 6, 0.0, False), ("8x8_nofly0.1", 8, 8, 0.1, True),
]


def _cost(q, state_words):
    path, cost = uavq.decode_path(q, state_words)
    return None if path is None else cost / 10.0


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    r = fn()
    e1.record()
    torch.cuda.synchronize()
    return r, e0.elapsed_time(e1)


def plain(q, inst, replicas, sweeps, T0, T1, seed):
    plan = uavq.Plan([q], [inst], replicas, sweeps, T0, T1, seed)
    plan.upload()
    out = plan.alloc_outputs()
    _, ms = _timed(lambda: plan.anneal(out=out))
    best = int(out.inst_best_E.cpu()[0])
    st = out.inst_best_state.cpu().numpy().view(np.uint32)[:q.state_words]
    return {"best_E": best, "cost_s": _cost(q, st), "ms": ms}


def tempering(q, inst, K, R, sweeps, T_hot, T_cold, seed, interval):
    pt = uavq.ParallelTempering(q, inst, K, R, sweeps, T_hot, T_cold, seed=seed, interval=interval)
    res, ms = _timed(pt.run)
    rounds = res["rounds"]
    bests = [int(v) for v in res["inst_best_E"].cpu().numpy()]
    k = int(np.argmin(bests))
    st = res["inst_best_state"][k].cpu().numpy().view(np.uint32)
    sw = res["swaps"].cpu().numpy()
    # attempts per pair: rounds whose parity matches the pair, times R chains
    att = np.array([sum(1 for e in range(rounds) if e % 2 == j % 2) * R for j in range(K - 1)], np.float64)
    return {"best_E": bests[k], "best_slot": k, "cost_s": _cost(q, st), "ms": ms, "rounds": rounds,
            "swap_rate": [float(a) for a in np.where(att > 0, sw / np.maximum(att, 1), 0.0)],
            "slot_best_E": bests, "T": [float(t) for t in pt.T]}


def batch_study(n, K, R, sweeps, T_hot, T_cold, seed, interval):
    """n fields of sides 4..10 (no-fly density up to 0.2) tempered as one plan
    with one batched exchange launch per round, against one tempering run per
    field; the outputs are identical, only the time differs."""
    import torch
    grids = inputs.batch(n, seed=seed)
    qs = [uavq.qubo_build(g.rows, g.cols, nofly=g.nofly) for g in grids]
    ids = [g.inst_id * K for g in grids]          # disjoint id ranges of K slots
    bt = uavq.ParallelTemperingBatch(qs, ids, K, R, sweeps, T_hot, T_cold, seed=seed, interval=interval)
    res, batch_ms = _timed(bt.run)
    singles = [uavq.ParallelTempering(q, i, K, R, sweeps, T_hot, T_cold, seed=seed, interval=interval)
               for q, i in zip(qs, ids)]
    outs, single_ms = _timed(lambda: [p.run() for p in singles])
    same = all(torch.equal(a["best_E"], b["best_E"]) and torch.equal(a["states"], b["states"])
               for a, b in zip(res, outs))
    return {"fields": n, "m": [q.m for q in qs], "K": K, "R": R, "sweeps": sweeps, "interval": interval,
            "batch_ms": batch_ms, "per_field_ms": single_ms, "identical": bool(same)}


def ttt_study(n, K, R, ladder, T_hot, T_cold, seed, interval, ref_sweeps, T_const=0.0):
    """Time to target on the warm-start study's held-out fields (n fields of
    10x10, ids from 20000): for each sweep budget S of the ladder, the plain
    annealer (K*R replicas per field, T_hot -> T_cold, one persistent launch for
    all fields) and batched tempering (K slots x R chains per field, exchanges
    every `interval` sweeps); a field is at target when its best energy is
    within 1% of the best any run found (a plain reference run of ref_sweeps
    included).  With T_const > 0 the plain annealer also runs at that constant
    temperature.  Reports the fraction at target per budget and the time of
    the ladder up to the largest first budget at target."""
    from paper_2608_25376_amd import warmstart
    grids = warmstart.make_instances(n, 20000)
    qs = [uavq.qubo_build(g.rows, g.cols, nofly=g.nofly) for g in grids]
    _, ref, _ = warmstart._anneal(qs, grids, K * R, ref_sweeps, T_hot, T_cold, seed + 1000)
    best = ref.inst_best_E.cpu().numpy().copy()
    runs = {}
    for S in ladder:
        _, out, ms = warmstart._anneal(qs, grids, K * R, S, T_hot, T_cold, seed)
        runs[("plain", S)] = (out.inst_best_E.cpu().numpy().copy(), ms)
        bt = _tempering_batch_best(qs, grids, K, R, S, T_hot, T_cold, seed, interval)
        runs[("tempering", S)] = bt
        if T_const > 0:
            _, out, ms = warmstart._anneal(qs, grids, K * R, S, T_const, T_const, seed)
            runs[("constant", S)] = (out.inst_best_E.cpu().numpy().copy(), ms)
    for v in runs.values():
        best = np.minimum(best, v[0])
    stop = None
    if T_const > 0:
        # the constant-temperature runs freeze early: the same anneal with UAVQ_STOP_FROZEN at the largest budget
        S = ladder[-1]
        plan = uavq.Plan(qs, [g.inst_id for g in grids], K * R, S, T_const, T_const, seed, persistent=True,
                         stop_frozen=True)
        plan.upload()
        out = plan.alloc_outputs()
        _, ms = _timed(lambda: plan.anneal(out=out))
        stop = {"sweeps": S, "ms": ms,
                "identical": bool(np.array_equal(out.inst_best_E.cpu().numpy(), runs[("constant", S)][0]))}
    hit = lambda E: 100 * E <= 101 * best
    rep = {"fields": n, "K": K, "R": R, "ladder": list(ladder), "T_hot": T_hot, "T_cold": T_cold,
           "interval": interval, "ref_sweeps": ref_sweeps, "T_const": T_const, "constant_stop_frozen": stop,
           "modes": {}}
    for mode in ("plain", "tempering") + (("constant",) if T_const > 0 else ()):
        frac = {S: float(hit(runs[(mode, S)][0]).mean()) for S in ladder}
        gap = {S: float(np.mean(runs[(mode, S)][0] / best - 1.0)) for S in ladder}
        firsts = [next((S for S in ladder if hit(runs[(mode, S)][0])[i]), None) for i in range(n)]
        reached = [S for S in firsts if S is not None]
        s_last = max(reached) if reached else None
        ladder_ms = sum(runs[(mode, S)][1] for S in ladder if s_last is not None and S <= s_last)
        rep["modes"][mode] = {"fraction_at_target": frac, "mean_gap": gap, "solved": len(reached),
                              "ladder_ms_to_all_first_hits": ladder_ms,
                              "ms_per_S": {S: runs[(mode, S)][1] for S in ladder}}
    return rep


def _tempering_batch_best(qs, grids, K, R, S, T_hot, T_cold, seed, interval):
    """(per-field best energy over all slots, ms) of one batched tempering run."""
    ids = [g.inst_id * K for g in grids]          # disjoint id ranges of K slots
    bt = uavq.ParallelTemperingBatch(qs, ids, K, R, S, T_hot, T_cold, seed=seed, interval=interval)
    res, ms = _timed(bt.run)
    return np.array([int(r["inst_best_E"].min().cpu()) for r in res], np.int64), ms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--K", type=int, default=16)
    ap.add_argument("--R", type=int, default=64, help="chains per slot (the plain run gets K*R replicas)")
    ap.add_argument("--sweeps", type=int, default=1000)
    ap.add_argument("--T-hot", type=float, default=100.0)
    ap.add_argument("--T-cold", type=float, default=0.5)
    ap.add_argument("--intervals", default="1,10")
    ap.add_argument("--seeds", default="1,2,3,4,5", help="annealing seeds (medians reported)")
    ap.add_argument("--long-factor", type=int, default=3,
                    help="also run the plain annealer with this many times the sweeps (about the GPU time of "
                         "tempering with an exchange every 10 sweeps); 0 = skip")
    ap.add_argument("--fields", default="")
    ap.add_argument("--batch", type=int, default=0, help="only the batch study: this many fields in one plan")
    ap.add_argument("--ttt", type=int, default=0, help="only the time-to-target study on this many held-out fields")
    ap.add_argument("--ladder", default="50,100,200,400,800,1600,3200")
    ap.add_argument("--T-const", type=float, default=0.0, help="time-to-target study: also a plain run at this "
                    "constant temperature")
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available()
    if args.ttt:
        ladder = [int(v) for v in args.ladder.split(",")]
        iv = int(args.intervals.split(",")[-1])
        rep = ttt_study(args.ttt, args.K, args.R, ladder, args.T_hot, args.T_cold, 1, iv, 8000, args.T_const)
        print(json.dumps(rep), flush=True)
        if args.out:
            with open(args.out, "w") as f:
                f.write(json.dumps(rep) + "\n")
        return
    if args.batch:
        q0 = uavq.qubo_build(3, 3)
        tempering(q0, 0, 2, 8, 4, 10.0, 1.0, 1, 1)     # load the kernels before timing
        rows = [batch_study(args.batch, args.K, args.R, args.sweeps, args.T_hot, args.T_cold, 1, iv)
                for iv in [int(v) for v in args.intervals.split(",")]]
        for r in rows:
            print(json.dumps(r), flush=True)
        if args.out:
            with open(args.out, "w") as f:
                for r in rows:
                    f.write(json.dumps(r) + "\n")
        return
    names = set(args.fields.split(",")) if args.fields else None
    seeds = [int(v) for v in args.seeds.split(",")]
    rows = []
    q0 = uavq.qubo_build(3, 3)
    tempering(q0, 0, 2, 8, 4, 10.0, 1.0, 1, 1)     # load the kernels before timing
    for name, r, c, dens, closed in FIELDS:
        if names and name not in names:
            continue
        g = inputs.grid(r, c, dens, seed=1, inst=0)
        q = uavq.qubo_build(g.rows, g.cols, nofly=g.nofly, closed=closed)
        res = {"field": name, "m": q.m, "closed": closed, "K": args.K, "R": args.R, "sweeps": args.sweeps,
               "T_hot": args.T_hot, "T_cold": args.T_cold, "seeds": seeds, "per_seed": {}}
        ivs = [int(v) for v in args.intervals.split(",")]
        for sd in seeds:
            one = {"plain": plain(q, g.inst_id, args.K * args.R, args.sweeps, args.T_hot, args.T_cold, sd)}
            if args.long_factor > 0:
                one[f"plain_x{args.long_factor}"] = plain(q, g.inst_id, args.K * args.R, args.long_factor * args.sweeps,
                                                          args.T_hot, args.T_cold, sd)
            for iv in ivs:
                one[f"pt_interval{iv}"] = tempering(q, g.inst_id, args.K, args.R, args.sweeps, args.T_hot,
                                                    args.T_cold, sd, iv)
            res["per_seed"][str(sd)] = one
        # a feasible state's energy is its tour time in deciseconds
        res["median"] = {mode: {"best_E": float(np.median([res["per_seed"][str(sd)][mode]["best_E"] for sd in seeds])),
                                "ms": float(np.median([res["per_seed"][str(sd)][mode]["ms"] for sd in seeds])),
                                "feasible": sum(res["per_seed"][str(sd)][mode]["cost_s"] is not None for sd in seeds)}
                         for mode in res["per_seed"][str(seeds[0])]}
        print(json.dumps(res), flush=True)
        rows.append(res)
    if args.out:
        with open(args.out, "w") as f:
            for res in rows:
                f.write(json.dumps(res) + "\n")


if __name__ == "__main__":
    main()
