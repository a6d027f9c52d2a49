"""Benchmark: spin-flip attempts per second of the MI355X annealer.

One step = one full anneal_batch of the workload (replica initialisation,
all sweeps, per-instance reduction) with the plan's static data already
resident in HBM.  Prints one JSON line.

Default workload: 12x12 field, no obstacles (143 free cells, 20449
variables), 4096 replicas, 4000 sweeps, geometric T 200 -> 0.5, seed 1 --
the largest single-GPU configuration of the hot path.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published figures and the integer-VALU peak derived from unit counts:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 int32 lane-ops/s.
PEAK_ALU_OPS = 256 * 4 * 16 * 2.4e9
# Algorithmic integer operations of the structured Metropolis step: per
# attempted flip (form h from R_t, C_c, x and two travel rows; sign; two
# compares), per random draw (a quarter of a Philox4x32-10 call, a table read,
# a compare) and per accepted flip (plus m for the O(m) travel-row update).
OPS_PER_ATTEMPT = 11
OPS_PER_DRAW = 27
OPS_PER_ACCEPT_BASE = 5


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="grid12x12",
                    help="a named workload (paper_2608_25376_amd/configs/<name>.json)")
    ap.add_argument("--config", default="", help="a workload config JSON file (instead of --workload)")
    ap.add_argument("--kernel", default="factored", choices=["factored", "dense"])
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--rowmask", action="store_true", help="m <= 64: rebuild travel rows from step masks")
    ap.add_argument("--no-producer", action="store_true",
                    help="m <= 64 at one wave per SIMD: no cut-producing wave beside each replica")
    ap.add_argument("--generic-chunk", action="store_true",
                    help="64 < m <= 192: the generic chunked walk instead of the block-tested kernel")
    ap.add_argument("--persistent", action="store_true", help="persistent work-queue sweep kernels")
    ap.add_argument("--graph", action="store_true", help="replay anneal_batch as a captured HIP graph")
    ap.add_argument("--autotune", action="store_true", help="choose the launch shape with uavq_autotune")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-replicas", type=int, default=0, help="oracle sample size (0 = auto)")
    ap.add_argument("--concurrent", action="store_true",
                    help="run the chunk classes' sweep kernels at the same time (UAVQ_CONCURRENT_CLASSES)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES of device memory once (reference run for the HBM byte counters)")
    ap.add_argument("--aux", action="store_true",
                    help="instead: time the MFMA energy refresh and the warm-start network step (one JSON line each)")
    ap.add_argument("--mfma-only", action="store_true",
                    help="with --aux: only the two MFMA users (for counter runs)")
    ap.add_argument("--segments", default="",
                    help="instead: one anneal of the workload cut at these sweeps (e.g. 0,500,1000,4000), one "
                         "JSON line per piece with its sweep-kernel time and counts (the schedule's regimes)")
    return ap.parse_args()


PEAK_INT8_OPS = 5.0e15      # MI355X dense int8 MFMA
PEAK_BF16_FLOPS = 2.5e15    # MI355X dense bf16 MFMA


def _time_ms(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def aux_measurements(args):
    """The two MFMA users besides the sweep: the int8 energy refresh (Z = X D
    per state, two byte limbs, int32 accumulation) at the 12x12 and 8x8 sizes,
    and one forward+backward step of the warm-start network (bf16 operands,
    fp32 accumulation) on a batch of 32 fields of 10x10, eager and replayed
    from a captured HIP graph; the time to result with UAVQ_STOP_FROZEN; and
    parallel tempering against the plain anneal of the same replica-sweeps."""
    import numpy as np
    import torch
    from paper_2608_25376_amd import inputs, uavq
    for name in ("grid12x12", "grid8x8_nofly0.1"):
        w = inputs.workload(name)
        g = w.grids[0]
        q = uavq.qubo_build(g.rows, g.cols, nofly=g.nofly)
        rng = np.random.default_rng(7)
        X = np.zeros((w.replicas, q.m, q.m), np.uint8)
        for r in range(w.replicas):
            X[r, np.arange(q.m), rng.permutation(q.m)] = 1
        d_states = torch.from_numpy(uavq.pack_states(X.reshape(w.replicas, -1), q.m).view(np.int32)).cuda()
        d_E = torch.empty(w.replicas, dtype=torch.int64, device="cuda")
        ms = _time_ms(lambda: uavq.energy_eval_dev(q, d_states, d_E), 20)
        ops = 4.0 * q.m ** 3 * w.replicas   # 2 limbs x m^3 MACs x 2 ops per state
        print(json.dumps({"metric": "int8 MFMA ops/s (energy refresh)", "value": ops / (ms * 1e-3), "unit": "ops/s",
                          "kernel": "k_energy_refresh", "config": {"workload": name, "m": q.m, "states": w.replicas},
                          "ms_per_call": ms, "ops_per_call": ops, "peak": PEAK_INT8_OPS,
                          "frac": ops / (ms * 1e-3) / PEAK_INT8_OPS}), flush=True)
    if not args.mfma_only:
        extra_measurements()
    mlp_measurement()


def extra_measurements():
    """Time to result with UAVQ_STOP_FROZEN, and parallel tempering beside the
    plain anneal of the same replica-sweeps."""
    import numpy as np
    from paper_2608_25376_amd import inputs, uavq
    # time to result with UAVQ_STOP_FROZEN: the same anneals, identical outputs, frozen sweeps skipped
    # (a wall time, not a throughput: the skipped sweeps are not evaluated)
    for name in ("grid8x8_nofly0.1", "grid12x12"):
        w = inputs.workload(name)
        qs = [uavq.qubo_build(g.rows, g.cols, nofly=g.nofly) for g in w.grids]
        row = {"metric": "ms per anneal, replicas stop once frozen", "unit": "ms", "higher_is_better": False,
               "config": {"workload": name, "replicas": w.replicas, "sweeps": w.sweeps}}
        outs = {}
        for stop in (False, True):
            plan = uavq.Plan(qs, [g.inst_id for g in w.grids], w.replicas, w.sweeps, w.T0, w.T1, w.seed,
                             stop_frozen=stop)
            plan.upload()
            out = plan.alloc_outputs()
            row["stop" if stop else "all_sweeps"] = _time_ms(lambda: plan.anneal(out=out), 3)
            outs[stop] = [getattr(out, f).cpu().numpy() for f in ("final_states", "best_E", "best_sweep",
                                                                 "accepts", "draws", "inst_best_E")]
        row["identical_outputs"] = all(np.array_equal(x, y) for x, y in zip(outs[False], outs[True]))
        row["value"] = row["stop"]
        print(json.dumps(row), flush=True)
    # parallel tempering on the bench field: 16 slots x 64 chains, 1000 sweeps, one launch per
    # exchange round; attempts/s counts every slot's sweeps (the same count as the plain anneal of
    # 1024 replicas x 1000 sweeps, timed beside it)
    w = inputs.workload("grid8x8_nofly0.1")
    g = w.grids[0]
    q = uavq.qubo_build(g.rows, g.cols, nofly=g.nofly)
    K, R, S = 16, 64, 1000
    attempts = float(K * R * S * q.n_vars)
    plain = uavq.Plan([q], [g.inst_id], K * R, S, 100.0, 0.5, 1)
    plain.upload()
    pout = plain.alloc_outputs()
    row = {"metric": "spin-flip attempts/s, parallel tempering", "unit": "attempts/s",
           "config": {"workload": w.name, "slots": K, "chains": R, "sweeps": S, "T_hot": 100.0, "T_cold": 0.5},
           "plain_ms": _time_ms(lambda: plain.anneal(out=pout), 3)}
    for iv in (1, 10):
        pt = uavq.ParallelTempering(q, g.inst_id, K, R, S, 100.0, 0.5, seed=1, interval=iv)
        row[f"interval{iv}_ms"] = _time_ms(pt.run, 2)
    row["value"] = attempts / (row["interval10_ms"] * 1e-3)
    row["plain_value"] = attempts / (row["plain_ms"] * 1e-3)
    print(json.dumps(row), flush=True)


def mlp_measurement():
    """One forward+backward step of the warm-start network on 32 fields of
    10x10 (about 85 free cells each), eager and replayed from a HIP graph."""
    import numpy as np
    import torch
    from paper_2608_25376_amd import inputs, uavq
    from paper_2608_25376_amd import warmstart
    grids = inputs.batch(32, seed=1, side=10, density_hi=0.2, first_id=10000)
    feats, steps, labels = [], [], []
    for gr in grids:
        qq = uavq.qubo_build(gr.rows, gr.cols, nofly=gr.nofly)
        feats.append(uavq.mlp_features(qq))
        steps.append(np.full(qq.m, qq.m, np.int32))
        labels.append(np.random.default_rng(gr.inst_id).permutation(qq.m).astype(np.int32))
    Xf = torch.from_numpy(np.concatenate(feats)).cuda()
    Ms = torch.from_numpy(np.concatenate(steps)).cuda()
    Lb = torch.from_numpy(np.concatenate(labels)).cuda()
    rows = Xf.shape[0]
    net = uavq.Mlp(warmstart.init_params(1))
    eager_ms = _time_ms(lambda: net.loss_grad(Xf, Ms, Lb), 50)
    g_eager = net.grad.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        net.loss_grad(Xf, Ms, Lb, stream=side)   # workspace allocated outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        net.loss_grad(Xf, Ms, Lb, stream=torch.cuda.current_stream())
    same = True
    for _ in range(3):                            # every replay equals the eager step
        net.grad.zero_()
        graph.replay()
        torch.cuda.synchronize()
        same &= bool(torch.equal(net.grad, g_eager))
    graph_ms = _time_ms(graph.replay, 50)
    flops = 3 * 2.0 * rows * (16 * 128 + 128 * 128 + 128 * 128)   # forward + two backward products per layer
    print(json.dumps({"metric": "bf16 MFMA FLOP/s (warm-start network forward+backward)",
                      "value": flops / (graph_ms * 1e-3), "unit": "FLOP/s", "kernel": "k_gemm_bf16 + k_softmax_ce",
                      "config": {"rows": rows, "fields": 32, "params": uavq.mlp_param_count()},
                      "eager_ms": eager_ms, "graph_ms": graph_ms, "graph_equals_eager": same,
                      "flops_per_step": flops, "peak": PEAK_BF16_FLOPS,
                      "frac": flops / (graph_ms * 1e-3) / PEAK_BF16_FLOPS}), flush=True)


# Sources of each sweep kernel's translation unit; an HBM-traffic record
# applies only to the build whose sources hash to the value stored with it.
_CSRC = "paper_2608_25376_amd/csrc/"
_COMMON = [_CSRC + "uavq_device.h", _CSRC + "uavq_kargs.h"]
KERNEL_SOURCES = {
    "k_sweep_chunk": [_CSRC + "uavq_sweep_chunk.hip", _CSRC + "uavq_chunk.h"] + _COMMON,
    "k_sweep_chunk<5>": [_CSRC + "uavq_sweep_chunk_wide.hip", _CSRC + "uavq_chunk.h"] + _COMMON,
    "k_sweep_chunk<6>": [_CSRC + "uavq_sweep_chunk_wide.hip", _CSRC + "uavq_chunk.h"] + _COMMON,
    "k_sweep_chunk_big": [_CSRC + "uavq_sweep_chunk_big.hip", _CSRC + "uavq_chunk.h"] + _COMMON,
    "k_sweep_factored_big": [_CSRC + "uavq_sweep_big.hip", _CSRC + "uavq_factored.h"] + _COMMON,
    "k_sweep_dense": [_CSRC + "uavq_refresh.hip", _CSRC + "uavq_internal.h"] + _COMMON,
    "k_sweep": [_CSRC + "uavq_kernels.hip", _CSRC + "uavq_factored.h", _CSRC + "uavq_internal.h"] + _COMMON,
}


def segment_measurements(args):
    """One anneal of the workload run as consecutive segments of its schedule
    (uavq_anneal_segment, resumed): per piece, the sweep kernels' time (HIP
    events on their stream) and the attempts, accepts and draws it added."""
    import numpy as np
    import torch
    from paper_2608_25376_amd import inputs, uavq
    w = inputs.load_config(args.config) if args.config else inputs.workload(args.workload)
    cuts = [int(v) for v in args.segments.split(",")]
    assert cuts[0] == 0 and cuts[-1] == w.sweeps and cuts == sorted(cuts), "cuts must run from 0 to the sweeps"
    qs = [uavq.qubo_build(g.rows, g.cols, nofly=g.nofly) for g in w.grids]
    plan = uavq.Plan(qs, [g.inst_id for g in w.grids], w.replicas, w.sweeps, w.T0, w.T1, w.seed,
                     generic_chunk=args.generic_chunk)
    plan.upload()
    out = plan.alloc_outputs()
    plan.set_timing(True)
    torch.cuda.synchronize()
    n_vars = sum(q.n_vars for q in qs)
    acc0 = drw0 = 0
    for a, b in zip(cuts[:-1], cuts[1:]):
        plan.anneal(out=out, s_begin=a, s_end=b, resume=a > 0)
        torch.cuda.synchronize()
        ms = plan.sweep_ms()
        acc, drw = int(out.accepts.sum()), int(out.draws.sum())
        att = float(n_vars * w.replicas * (b - a))
        T_a = w.T0 * (w.T1 / w.T0) ** (a / max(w.sweeps - 1, 1))
        print(json.dumps({"workload": w.name, "sweeps": [a, b], "T_first": T_a, "kernel_ms": ms,
                          "ms_per_sweep": ms / max(b - a, 1), "attempts": att, "attempts_per_s": att / (ms * 1e-3),
                          "accepts": acc - acc0, "draws": drw - drw0,
                          "kernel": "+".join(k for k in (plan.kernel_name(c) for c in range(1, uavq.CHUNK_CLASSES + 1)) if k)}),
              flush=True)
        acc0, drw0 = acc, drw


def kernel_source_sha256(kernel):
    """sha256 over the sources that build `kernel` (longest matching name prefix)."""
    key = max((k for k in KERNEL_SOURCES if kernel.startswith(k)), key=len)
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[key]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary of this kernel
    and workload (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size), or
    None if there is none or the kernel sources changed since it was taken."""
    name = re.sub(r"[^A-Za-z0-9.]+", "_", f"{kernel}_{workload}_traffic").strip("_") + ".md"
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    sha = re.search(r"^source_sha256:\s*([0-9a-f]{64})\s*$", txt, re.M)
    val = re.search(r"^hbm_bytes_per_launch:\s*([0-9.eE+]+)\s*$", txt, re.M)
    if not sha or not val or sha.group(1) != kernel_source_sha256(kernel):
        return None
    return float(val.group(1))


def copy_calibration(nbytes):
    """One device-to-device copy of nbytes (the reference for the byte counters)."""
    import torch
    x = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "read_bytes": nbytes, "write_bytes": nbytes}), flush=True)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the platform string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(w, q_gpu_m, args):
    """The oracle as it stands, on a bounded sample of the same workload: one
    replica on one thread (the single-thread rate), then a sample sized for
    about 15 s on all threads."""
    import oracle
    g = w.grids[0]
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    # large fields: the oracle evaluates each coefficient of J from its definition
    o = oracle.OracleQubo(g.rows, g.cols, nofly=g.nofly, dense=len(g.nofly) <= 100)
    table = oracle.thresholds(w.T0, w.T1, w.sweeps)
    t0 = time.perf_counter()
    oracle.anneal(o, w.sweeps, w.T0, w.T1, w.seed, g.inst_id, [0], table=table, threads=1)
    one = time.perf_counter() - t0
    reps = args.cpu_replicas
    if reps <= 0:
        reps = int(max(threads, min(w.replicas, round(15.0 * threads / max(one, 1e-3)))))
    t0 = time.perf_counter()
    oracle.anneal(o, w.sweeps, w.T0, w.T1, w.seed, g.inst_id, list(range(reps)), table=table, threads=threads)
    dt = time.perf_counter() - t0
    attempts = reps * w.sweeps * o.N
    return {"value": attempts / dt, "unit": "attempts/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
            "single_thread_value": w.sweeps * o.N / one,
            "sample": f"{reps} of {w.replicas} replicas x {w.sweeps} sweeps of the same instance "
                      f"({attempts:.3g} attempts, {dt:.1f} s on {threads} threads; single thread: replica 0, "
                      f"{w.sweeps * o.N:.3g} attempts, {one:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the annealer runs on one GPU; --gpus {args.gpus} is not supported "
              f"(it would shard by instance and replica, with one reduction of per-instance bests at the end)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2608_25376_amd import inputs, uavq

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return
    if args.aux:
        aux_measurements(args)
        return
    if args.segments:
        segment_measurements(args)
        return
    w = inputs.load_config(args.config) if args.config else inputs.workload(args.workload)
    dense = args.kernel == "dense"
    qs = [uavq.qubo_build(g.rows, g.cols, nofly=g.nofly, dense=dense) for g in w.grids]
    ids = [g.inst_id for g in w.grids]
    tune = None
    if args.autotune:
        tune = uavq.autotune(qs, ids, w.replicas, w.sweeps, w.T0, w.T1, w.seed, persistent=args.persistent,
                             trial_sweeps=max(16, w.sweeps // 32),
                             cache=os.path.join(ROOT, "paper_2608_25376_amd", "tune_cache.json"))
    stream = torch.cuda.Stream() if args.graph else torch.cuda.current_stream()
    plan = uavq.Plan(qs, ids, w.replicas, w.sweeps, w.T0, w.T1, w.seed, dense=dense,
                     waves_per_block=args.waves_per_block, rowmask=args.rowmask, persistent=args.persistent,
                     no_producer=args.no_producer, generic_chunk=args.generic_chunk,
                     graph=args.graph, tune=tune, concurrent=args.concurrent)
    plan.upload(stream=stream if args.graph else None)
    out = plan.alloc_outputs()
    torch.cuda.synchronize()
    if not args.graph:
        plan.set_timing(True)

    for _ in range(args.warmup):
        plan.anneal(out=out, stream=stream)
    torch.cuda.synchronize()

    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sweep_ms = []
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        plan.anneal(out=out, stream=stream)
        # the library's events bracket the sweep kernels of this call (in graph
        # mode the whole replayed graph is timed instead)
        stream.synchronize()
        if not args.graph:
            sweep_ms.append(plan.sweep_ms())
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    ms_per_step = total_ms / args.steps

    n_vars = sum(q.n_vars for q in qs)
    attempts = float(sum(q.n_vars for q in qs) * w.replicas * w.sweeps)
    counted = int(out.attempts.cpu().numpy().astype(np.uint64).sum())
    assert counted == int(attempts), f"attempts counter {counted} != replicas x sweeps x N = {int(attempts)}"
    acc = out.accepts.cpu().numpy().astype(np.float64)
    drw = out.draws.cpu().numpy().astype(np.float64)
    m_per_rep = np.concatenate([np.full(w.replicas, q.m) for q in qs]).astype(np.float64)
    ops = OPS_PER_ATTEMPT * attempts + OPS_PER_DRAW * drw.sum() + ((m_per_rep + OPS_PER_ACCEPT_BASE) * acc).sum()
    sweep_avg = float(np.mean(sweep_ms)) if sweep_ms else ms_per_step
    achieved = ops / (sweep_avg * 1e-3)
    value = attempts / (ms_per_step * 1e-3)
    kernels = [k for k in (plan.kernel_name(c) for c in range(1, uavq.CHUNK_CLASSES + 1)) if k]
    kernel = "+".join(kernels)

    res = {
        "metric": "spin-flip attempts/s",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": w.name, "instances": len(qs), "m": int(qs[0].m) if len(qs) == 1 else None,
                   "n_vars": n_vars, "replicas": w.replicas, "sweeps": w.sweeps, "T0": w.T0, "T1": w.T1,
                   "seed": w.seed, "kernel": args.kernel, "persistent": args.persistent, "graph": args.graph,
                   "no_producer": args.no_producer, "generic_chunk": args.generic_chunk,
                   "concurrent": args.concurrent,
                   "tune": repr(tune) if tune is not None else None, "attempts_per_step": attempts,
                   "accept_rate": float(acc.sum() / attempts), "draw_rate": float(drw.sum() / attempts),
                   "best_E": [int(v) for v in out.inst_best_E.cpu().numpy()[:4]]},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_ALU_OPS / 1e12,
                     "unit": "Tops/s (int32 lane-ops)", "frac": achieved / PEAK_ALU_OPS,
                     "traffic": recorded_traffic(kernel, w.name),
                     "kernel": kernel, "kernel_ms": sweep_avg, "ops_per_launch": ops},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, qs[0].m, args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
