"""Learned warm start: labelling, training and the time-to-target protocol.

Driver only: every numeric step (annealing, features aside, network
forward/backward/Adam, quantisation, sampling) runs in libuavq's kernels;
this module moves tensors between those calls.

Protocol (all inputs synthetic, 10x10 fields, no-fly density U[0, 0.2]):
  0. schedule: the annealing schedule of the whole study (labels and
     evaluation) is chosen on training instances only, among geometric
     schedules and constant temperatures, by the mean gap of their best
     energies at a fixed budget;
  1. label: anneal the training instances (ids from 10000) and take each
     instance's best tour, oriented so that its first visited cell has the
     smaller free-list index (a tour and its reversal cost the same);
  2. train the per-cell network to predict the visiting step of every cell;
  3. time-to-target on held-out instances (ids from 20000): the smallest
     sweep budget S of a ladder at which the best energy is within 1% of the
     best known energy (100 E <= 101 E_best_known; best known = the minimum
     over every run made, reference runs of several schedules included), for
       plain   - one launch per instance, all replicas random,
       batched - all instances in one persistent launch,
       warm    - half of the replicas seeded with tours sampled from the
                 network and started at the first sweep with T_s <= T_warm,
       batched+warm.
     Warm times include feature, inference and sampling time.
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

from paper_2608_25376_amd import inputs, uavq  # noqa: E402


def make_instances(n, first_id, seed=1, side=10, density_hi=0.2):
    return inputs.batch(n, seed=seed, side=side, density_hi=density_hi, first_id=first_id)


def _qubos(grids):
    return [uavq.qubo_build(g.rows, g.cols, nofly=g.nofly) for g in grids]


def _anneal(qs, grids, R, S, T0, T1, seed, init=None, stream=None, out=None, plan=None):
    """One persistent launch; returns (plan, out, elapsed ms)."""
    import torch
    if plan is None:
        plan = uavq.Plan(qs, [g.inst_id for g in grids], R, S, T0, T1, seed, persistent=True)
        plan.upload()
    if out is None:
        out = plan.alloc_outputs()
    torch.cuda.synchronize()
    s = stream or torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    plan.anneal(out=out, stream=s, **(init or {}))
    e1.record(s)
    torch.cuda.synchronize()
    return plan, out, e0.elapsed_time(e1)


def best_tours(plan, qs, out):
    """Per instance: best energy and the visiting order (free-list indices) or None."""
    E = out.inst_best_E.cpu().numpy()
    words = out.inst_best_state.cpu().numpy().view(np.uint32)
    res, off = [], 0
    for i, q in enumerate(qs):
        x = uavq.unpack_states(words[off:off + q.state_words], q.m).reshape(q.m, q.m)
        off += q.state_words
        order = None
        if (x.sum(0) == 1).all() and (x.sum(1) == 1).all():
            order = np.argmax(x, 1)
        res.append((int(E[i]), order))
    return res


def canonical(order):
    return order if order[0] < order[-1] else order[::-1]


def label_data(grids, R, S, T0, T1, seed, chunk=200, log=None):
    """Best tours of plain annealing, in launches of ``chunk`` instances (an
    instance's result does not depend on the batch it runs in)."""
    data, ms = [], 0.0
    for c0 in range(0, len(grids), chunk):
        part = grids[c0:c0 + chunk]
        qs = _qubos(part)
        plan, out, dt = _anneal(qs, part, R, S, T0, T1, seed)
        ms += dt
        for (E, order), q, g in zip(best_tours(plan, qs, out), qs, part):
            if order is None:
                continue
            order = canonical(order)
            labels = np.empty(q.m, np.int32)
            labels[order] = np.arange(q.m, dtype=np.int32)     # cell -> step (0-based)
            data.append((uavq.mlp_features(q), labels, q.m, g))
        del plan, out
        if log:
            log(f"labelled {min(c0 + chunk, len(grids))}/{len(grids)} ({ms / 1e3:.1f} s of annealing)")
    return data, ms


# Candidate schedules of step 0: (T0, T1); equal ends are a constant temperature.
SCHEDULE_CANDIDATES = [(200.0, 0.5), (100.0, 1.0), (50.0, 5.0), (30.0, 10.0), (25.0, 12.0), (8.0, 8.0), (10.0, 10.0),
                       (12.0, 12.0), (14.0, 14.0), (16.0, 16.0), (18.0, 18.0), (20.0, 20.0), (25.0, 25.0)]


def choose_schedule(grids, R, S, seed, candidates=SCHEDULE_CANDIDATES, log=None):
    """Step 0, on training instances only: every candidate anneals the same
    fields at budget S; the one with the smallest mean gap to the per-field
    best over all candidates wins.  Returns ((T0, T1), table)."""
    qs = _qubos(grids)
    res = {}
    for T0, T1 in candidates:
        _, out, ms = _anneal(qs, grids, R, S, T0, T1, seed)
        res[(T0, T1)] = (out.inst_best_E.cpu().numpy().astype(np.float64), ms)
    best = np.min(np.stack([v[0] for v in res.values()]), 0)
    table = []
    for (T0, T1), (E, ms) in res.items():
        gap = float(np.mean(E / best - 1.0))
        hit = float(np.mean(100 * E <= 101 * best))
        table.append({"T0": T0, "T1": T1, "mean_gap": gap, "fraction_within_1pct": hit, "ms": ms})
        if log:
            log(f"schedule {T0} -> {T1}: mean gap {gap:.4f}, within 1% {hit:.2f}, {ms:.0f} ms")
    win = min(table, key=lambda r: r["mean_gap"])
    return (win["T0"], win["T1"]), table


def init_params(seed):
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, (16, 128)) * np.sqrt(6 / (16 + 128)), np.zeros(128),
             rng.uniform(-1, 1, (128, 128)) * np.sqrt(6 / 256), np.zeros(128),
             rng.uniform(-1, 1, (128, 128)) * np.sqrt(6 / 256), np.zeros(128)]
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


def train(data, epochs=30, batch=64, lr=1e-3, seed=1, log=None):
    import torch
    net = uavq.Mlp(init_params(seed))
    rng = np.random.default_rng(seed)
    curve = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        idx = rng.permutation(len(data))
        tot, rows = 0.0, 0
        for b in range(0, len(idx), batch):
            sel = [data[i] for i in idx[b:b + batch]]
            X = torch.from_numpy(np.concatenate([d[0] for d in sel])).cuda()
            lab = torch.from_numpy(np.concatenate([d[1] for d in sel])).cuda()
            msteps = torch.from_numpy(np.concatenate([np.full(d[2], d[2], np.int32) for d in sel])).cuda()
            loss = net.train_step(X, msteps, lab, lr=lr)
            tot += float(loss.cpu()[0])
            rows += X.shape[0]
        curve.append(tot / rows)
        if log:
            log(f"epoch {ep}: mean CE {curve[-1]:.4f}")
    torch.cuda.synchronize()
    return net, curve, time.perf_counter() - t0


def first_sweep_below(T0, T1, S, T_warm):
    """First s with T_s <= T_warm on the geometric schedule (the library's)."""
    if S <= 1 or T_warm >= T0:
        return 0
    for s in range(S):
        if T0 * (T1 / T0) ** (s / (S - 1)) <= T_warm:
            return s
    return S - 1


def warm_init(net, plan, qs, frac, s0, stream=None):
    """Seed states (first frac of each instance's replicas), seeded mask and
    start sweeps; returns the init dict and the elapsed time (ms)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X = torch.from_numpy(np.concatenate([uavq.mlp_features(q) for q in qs])).cuda()
    msteps = torch.from_numpy(np.concatenate([np.full(q.m, q.m, np.int32) for q in qs])).cuda()
    probs = net.forward(X, msteps)
    qm = uavq.quantize_marginals(probs, msteps)
    offs = np.cumsum([0] + [q.m for q in qs])[:-1]
    R = plan.replicas
    ns = [int(round(frac * R))] * len(qs)
    states = torch.zeros(plan.total_state_words, dtype=torch.int32, device="cuda")
    uavq.sample_seeds(plan, qm, offs, ns, states)
    seeded = np.zeros(plan.total_replicas, np.uint8)
    start = np.zeros(plan.total_replicas, np.int32)
    for i in range(len(qs)):
        r0 = plan.rep_offset[i]
        seeded[r0:r0 + ns[i]] = 1
        start[r0:r0 + ns[i]] = s0
    init = {"init_states": states, "seeded": torch.from_numpy(seeded).cuda(),
            "start_sweep": torch.from_numpy(start).cuda()}
    torch.cuda.synchronize()
    return init, (time.perf_counter() - t0) * 1e3


def bits_init(plan, qs, probs, density, frac, seed, uniform=False):
    """Seeds for the density study, drawn on the host: in each instance the
    first frac of the replicas start from independent bits, x_{t,c} = 1 with
    probability min(1, density p(t|c)), p the network's marginal of cell c over
    the steps (or 1/m with ``uniform``), so about density ones per step."""
    import torch
    rng = np.random.default_rng(seed)
    words = np.zeros(plan.total_state_words, np.uint32)
    seeded = np.zeros(plan.total_replicas, np.uint8)
    n = int(round(frac * plan.replicas))
    row = 0
    for i, q in enumerate(qs):
        m = q.m
        p = np.full((m, m), 1.0 / m) if uniform else probs[row:row + m, :m]
        row += m
        pr = np.minimum(1.0, density * p.T)          # [step][cell]
        x = (rng.random((n, m, m)) < pr[None]).astype(np.uint8)
        base = plan.state_offset[i]
        words[base:base + n * q.state_words] = uavq.pack_states(x.reshape(n, -1), m).reshape(-1)
        seeded[plan.rep_offset[i]:plan.rep_offset[i] + n] = 1
    return {"init_states": torch.from_numpy(words.view(np.int32)).cuda(), "seeded": torch.from_numpy(seeded).cuda()}


def density_study(grids, net, R, S, T0, T1, seed, densities=(3.0, 4.0, 5.0, 6.0, 8.0, 12.0), log=None):
    """The annealer at one budget from: random bits (Bernoulli 1/2), tours
    sampled from the network (half of the replicas), and sparse bits at
    several densities biased by the network's marginals or uniform (every
    replica); the best energies are compared with the best of all these runs."""
    import torch
    qs = _qubos(grids)
    X = torch.from_numpy(np.concatenate([uavq.mlp_features(q) for q in qs])).cuda()
    msteps = torch.from_numpy(np.concatenate([np.full(q.m, q.m, np.int32) for q in qs])).cuda()
    probs = net.forward(X, msteps).cpu().numpy()
    runs = {}
    plan, out, _ = _anneal(qs, grids, R, S, T0, T1, seed)
    runs["random bits"] = out.inst_best_E.cpu().numpy().copy()
    init, _ = warm_init(net, plan, qs, 0.5, 0)
    _, out, _ = _anneal(qs, grids, R, S, T0, T1, seed, init=init, plan=plan)
    runs["sampled tours (half)"] = out.inst_best_E.cpu().numpy().copy()
    for uniform in (False, True):
        for dens in densities:
            init = bits_init(plan, qs, probs, dens, 1.0, seed + 17, uniform=uniform)
            _, out, _ = _anneal(qs, grids, R, S, T0, T1, seed, init=init, plan=plan)
            runs[f"{'uniform' if uniform else 'network'} bits, {dens:g} per step"] = out.inst_best_E.cpu().numpy().copy()
            if log:
                log(f"density study: {'uniform' if uniform else 'network'} {dens}")
    best = np.min(np.stack(list(runs.values())), 0)
    return {k: {"fraction_within_1pct": float(np.mean(100 * E <= 101 * best)),
                "mean_gap": float(np.mean(E / best - 1.0))} for k, E in runs.items()}


def ttt(grids, net, R, ladder, T0, T1, seed, T_warm, frac=0.5, ref_sweeps=8000, single=True, log=None,
        refs=()):
    """``refs``: further reference runs (T0, T1, sweeps) whose energies enter the best known."""
    qs = _qubos(grids)
    n = len(qs)
    runs = {}            # (mode, S) -> (per-instance best E, ms)
    # reference runs (best known): this schedule at ref_sweeps, and the extra ones
    _, out, ms = _anneal(qs, grids, R, ref_sweeps, T0, T1, seed + 1000)
    best_known = out.inst_best_E.cpu().numpy().copy()
    for (rT0, rT1, rS) in refs:
        _, out, ms = _anneal(qs, grids, R, rS, rT0, rT1, seed + 2000)
        best_known = np.minimum(best_known, out.inst_best_E.cpu().numpy())
    for S in ladder:
        s0 = first_sweep_below(T0, T1, S, T_warm)
        plan, out, ms = _anneal(qs, grids, R, S, T0, T1, seed)
        runs[("batched", S)] = (out.inst_best_E.cpu().numpy().copy(), ms)
        init, inf_ms = warm_init(net, plan, qs, frac, s0)
        plan, out, ms = _anneal(qs, grids, R, S, T0, T1, seed, init=init, plan=plan)
        runs[("batched+warm", S)] = (out.inst_best_E.cpu().numpy().copy(), ms + inf_ms)
        if single:
            Ep, tp, Ew, tw = np.zeros(n, np.int64), np.zeros(n), np.zeros(n, np.int64), np.zeros(n)
            for i in range(n):
                p1, o1, m1 = _anneal([qs[i]], [grids[i]], R, S, T0, T1, seed)
                Ep[i], tp[i] = int(o1.inst_best_E.cpu()[0]), m1
                init, inf_ms = warm_init(net, p1, [qs[i]], frac, s0)
                p1, o1, m1 = _anneal([qs[i]], [grids[i]], R, S, T0, T1, seed, init=init, plan=p1)
                Ew[i], tw[i] = int(o1.inst_best_E.cpu()[0]), m1 + inf_ms
            runs[("plain", S)] = (Ep, tp)
            runs[("warm", S)] = (Ew, tw)
        if log:
            log(f"S={S}: " + ", ".join(f"{k[0]} {np.mean(100 * v[0] <= 101 * np.minimum(best_known, v[0])):.2f}"
                                       for k, v in runs.items() if k[1] == S))
    for v in runs.values():
        best_known = np.minimum(best_known, v[0])
    hit = lambda E: 100 * E <= 101 * best_known
    report = {"instances": n, "replicas": R, "ladder": list(ladder), "T_warm": T_warm, "seeded_fraction": frac,
              "modes": {}}
    for mode in ("plain", "warm", "batched", "batched+warm"):
        if (mode, ladder[0]) not in runs:
            continue
        frac_hit = {S: float(hit(runs[(mode, S)][0]).mean()) for S in ladder}
        gap = {S: float(np.mean(runs[(mode, S)][0] / best_known - 1.0)) for S in ladder}
        if mode in ("plain", "warm"):
            # each instance stops at its own first budget at target (unsolved: the largest budget)
            per = []
            for i in range(n):
                S_i = next((S for S in ladder if hit(runs[(mode, S)][0])[i]), None)
                per.append((S_i is not None, float(runs[(mode, S_i if S_i is not None else ladder[-1])][1][i])))
            solved = sum(ok for ok, _ in per)
            report["modes"][mode] = {"ttt_ms": sum(t for _, t in per), "solved": solved,
                                     "fraction_at_target": frac_hit, "mean_gap": gap}
        else:
            q = {}
            for level in (0.5, 0.9, 1.0):
                S_q = next((S for S in ladder if hit(runs[(mode, S)][0]).mean() >= level - 1e-12), None)
                q[str(level)] = {"sweeps": S_q, "ms": runs[(mode, S_q)][1] if S_q is not None else None}
            # the batched ladder yields every instance's first budget at target once it has run up to
            # the largest such budget (the energies equal the per-instance launches: same instance ids)
            firsts = [next((S for S in ladder if hit(runs[(mode, S)][0])[i]), None) for i in range(n)]
            reached = [S for S in firsts if S is not None]
            s_last = max(reached) if reached else None
            ladder_ms = sum(runs[(mode, S)][1] for S in ladder if s_last is not None and S <= s_last)
            report["modes"][mode] = {"ttt_ms": q["1.0"]["ms"], "ttt_quantiles": q, "fraction_at_target": frac_hit,
                                     "mean_gap": gap, "ms_per_S": {S: runs[(mode, S)][1] for S in ladder},
                                     "ladder_ms_to_all_first_hits": ladder_ms, "solved": len(reached)}
    return report


SEED_KEYS = ("ttt_ms", "ladder_ms_to_all_first_hits", "solved", "fraction_at_target", "mean_gap")


def per_seed_fields(report):
    """The per-mode figures of one seed's report that the medians are taken over."""
    return {m: {k: v[k] for k in SEED_KEYS if k in v} for m, v in report["modes"].items()}


def seed_medians(per_seed):
    """Median over seeds of every figure (per budget for the per-budget ones);
    a scalar with a missing value on some seed gets no median."""
    seeds = list(per_seed)
    med = {}
    for m in per_seed[seeds[0]]:
        med[m] = {}
        for k in per_seed[seeds[0]][m]:
            vals = [per_seed[sd][m].get(k) for sd in seeds]
            if isinstance(vals[0], dict):
                med[m][k] = {S: float(np.median([v[S] for v in vals])) for S in vals[0]}
            elif all(v is not None for v in vals):
                med[m][k] = float(np.median(vals))
    return med


def merge_reports(paths):
    """Combine the per-seed figures of several reports (one per set of seeds)."""
    reps = [json.load(open(p)) for p in paths]
    per = {}
    for r in reps:
        per.update(r["per_seed"])
    out = dict(reps[0])
    out["seeds"] = sorted(int(k) for k in per)
    out["per_seed"] = {str(k): per[str(k)] for k in out["seeds"]}
    out["median"] = seed_medians(out["per_seed"])
    out["merged_from"] = [os.path.basename(p) for p in paths]
    return out


def mean_ce(net, data, batch=64):
    """Mean cross-entropy per cell of the network on labelled fields, and of
    the uniform distribution over each field's steps (log m)."""
    import torch
    tot, rows, uni = 0.0, 0, 0.0
    for b in range(0, len(data), batch):
        sel = data[b:b + batch]
        X = torch.from_numpy(np.concatenate([d[0] for d in sel])).cuda()
        lab = torch.from_numpy(np.concatenate([d[1] for d in sel])).cuda()
        msteps = torch.from_numpy(np.concatenate([np.full(d[2], d[2], np.int32) for d in sel])).cuda()
        tot += float(net.loss_grad(X, msteps, lab)[0].cpu()[0])
        rows += X.shape[0]
        uni += float(sum(d[2] * np.log(d[2]) for d in sel))
    return tot / rows, uni / rows


def save_labels(path, data):
    """Labels for an independent fit: per labelled instance its id, side and
    no-fly mask (which fix its features) and the step (0-based) of every free
    cell, concatenated in instance order."""
    np.savez(path, ids=np.asarray([d[3].inst_id for d in data], np.int64),
             m=np.asarray([d[2] for d in data], np.int32),
             side=np.asarray([d[3].rows for d in data], np.int32),
             nofly=np.stack([d[3].nofly for d in data]).astype(np.uint8),
             labels=np.concatenate([d[1] for d in data]).astype(np.int32))


CONFIG = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs", "warmstart_grid10x10.json")


def main():
    with open(CONFIG) as f:
        cfg = json.load(f)    # the study's shape: field counts, replicas, sweeps, ladder
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-n", type=int, default=cfg["train"]["n"])
    ap.add_argument("--heldout-n", type=int, default=cfg["heldout"]["n"])
    ap.add_argument("--schedule", default="auto",
                    help="'auto' (chosen on training instances among SCHEDULE_CANDIDATES) or T0,T1")
    ap.add_argument("--choose-n", type=int, default=100, help="training instances that choose the schedule")
    ap.add_argument("--choose-sweeps", type=int, default=100)
    ap.add_argument("--label-replicas", type=int, default=cfg["label_replicas"])
    ap.add_argument("--label-sweeps", type=int, default=cfg["label_sweeps"])
    ap.add_argument("--replicas", type=int, default=cfg["replicas"])
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--ladder", default=",".join(str(v) for v in cfg["ladder"]))
    ap.add_argument("--ref-sweeps", type=int, default=3200)
    ap.add_argument("--T-warm", type=float, default=0.0, help="0 = choose on training instances")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--seeds", default="1", help="annealing seeds of the held-out evaluation (medians reported)")
    ap.add_argument("--params", default="", help="network parameters saved by an earlier run (.npy): "
                    "skip labelling and training (needs --schedule T0,T1)")
    ap.add_argument("--save-labels", default="", help="write the training labels to this .npz")
    ap.add_argument("--labels-only", action="store_true", help="stop after labelling (with --save-labels)")
    ap.add_argument("--density-study", type=int, default=0, metavar="S",
                    help="also run the initial-density study on the held-out set at S sweeps")
    ap.add_argument("--merge", default="", help="comma-separated reports of earlier runs: combine their seeds "
                    "and write the medians to --out (no GPU work)")
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    if args.merge:
        txt = json.dumps(merge_reports(args.merge.split(",")))
        print(txt, flush=True)
        if args.out:
            with open(args.out, "w") as f:
                f.write(txt + "\n")
        return
    import torch
    assert torch.cuda.is_available()
    t_start = time.perf_counter()
    log = lambda s: print(f"[{time.perf_counter() - t_start:7.1f} s] {s}", flush=True)
    seed = 1
    sched_table = None
    if args.schedule == "auto":
        if args.params:
            raise SystemExit("--params needs the schedule it was trained with (--schedule T0,T1)")
        (T0, T1), sched_table = choose_schedule(make_instances(args.choose_n, 10000), args.replicas,
                                                args.choose_sweeps, seed + 11, log=log)
    else:
        T0, T1 = (float(v) for v in args.schedule.split(","))
    log(f"schedule {T0} -> {T1}")
    if args.params:
        net = uavq.Mlp(np.load(args.params).astype(np.float32))
        data, label_ms, curve, train_s = None, None, None, None
        log(f"network loaded from {args.params}")
    else:
        train_grids = make_instances(args.train_n, 10000)
        data, label_ms = label_data(train_grids, args.label_replicas, args.label_sweeps, T0, T1, seed, log=log)
        log(f"labelled {len(data)}/{len(train_grids)} training instances in {label_ms / 1e3:.1f} s")
        if args.save_labels:
            save_labels(args.save_labels, data)
        if args.labels_only:
            return
        net, curve, train_s = train(data, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    ladder = [int(v) for v in args.ladder.split(",")]
    constant = T0 == T1
    T_warm = args.T_warm
    if constant:
        T_warm = T0            # seeded replicas start at sweep 0: a constant schedule has no colder part
    elif T_warm <= 0:
        # choose on a slice of the training instances only
        tune = make_instances(24, 10000)
        best = None
        for cand in (0.05 * T0, 0.125 * T0, 0.25 * T0, 0.5 * T0):
            r = ttt(tune, net, args.replicas, [ladder[len(ladder) // 2]], T0, T1, seed + 7, cand,
                    ref_sweeps=args.ref_sweeps // 2, single=False)
            g = r["modes"]["batched+warm"]["mean_gap"][ladder[len(ladder) // 2]]
            log(f"T_warm {cand}: mean gap {g:.4f}")
            if best is None or g < best[0]:
                best = (g, cand)
        T_warm = best[1]
    held = make_instances(args.heldout_n, 20000)
    # held-out labels (best tours of a long reference run) measure what the network learned
    held_data, _ = label_data(held, args.label_replicas, args.label_sweeps, T0, T1, seed + 3000)
    ce_held, ce_uniform = mean_ce(net, held_data)
    log(f"held-out cross-entropy {ce_held:.4f} (uniform {ce_uniform:.4f})")
    refs = [(200.0, 0.5, 8000), (15.4, 15.4, 3200)]
    seeds = [int(v) for v in args.seeds.split(",")]
    reps = {}
    for sd in seeds:
        log(f"held-out evaluation, seed {sd}")
        reps[sd] = ttt(held, net, args.replicas, ladder, T0, T1, sd, T_warm, ref_sweeps=args.ref_sweeps,
                       single=not args.no_single, log=log, refs=refs)
    rep = dict(reps[seeds[0]])
    rep["seeds"] = seeds
    rep["per_seed"] = {str(sd): per_seed_fields(r) for sd, r in reps.items()}
    rep["median"] = seed_medians(rep["per_seed"])
    rep.update({"schedule": [T0, T1], "schedule_table": sched_table, "references": refs,
                "heldout_ce": ce_held, "heldout_ce_uniform": ce_uniform})
    if args.density_study:
        rep["density_study"] = {"sweeps": args.density_study, "replicas": args.replicas,
                                "runs": density_study(held, net, args.replicas, args.density_study, T0, T1, seed,
                                                      log=log)}
    if args.params:
        rep.update({"params": os.path.basename(args.params)})
    else:
        ce_train, ce_train_uniform = mean_ce(net, data)
        rep.update({"train_instances": len(data), "label_replicas": args.label_replicas,
                    "label_sweeps": args.label_sweeps, "label_s": label_ms / 1e3, "train_s": train_s,
                    "train_curve": curve, "epochs": args.epochs, "train_ce": ce_train,
                    "train_ce_uniform": ce_train_uniform})
    txt = json.dumps(rep)
    print(txt, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(txt + "\n")
        if not args.params:
            np.save(os.path.splitext(args.out)[0] + "_params.npy", net.params.cpu().numpy())


if __name__ == "__main__":
    main()
