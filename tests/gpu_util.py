"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
run the oracle on the same seeded inputs."""
import sys

import numpy as np


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_anneal(U, grids, R, S, T0, T1, seed=1, dense=False, wpb=0, closed=True, init_x=None, seeded=None,
               start_sweep=None, check_E=False, rowmask=False, persistent=False, graph=False, tune=None,
               stream=None, replays=1, no_producer=False, stop_frozen=False, penalty=0, generic_chunk=False,
               concurrent=False):
    """Anneal ``grids`` (inputs.Grid list) on cuda:0; returns (qubos, plan, numpy results)."""
    import torch
    qs = [U.qubo_build(g.rows, g.cols, nofly=g.nofly, closed=closed, dense=dense, penalty=penalty) for g in grids]
    plan = U.Plan(qs, [g.inst_id for g in grids], R, S, T0, T1, seed, dense=dense, waves_per_block=wpb,
                  rowmask=rowmask, persistent=persistent, graph=graph, tune=tune, no_producer=no_producer,
                  stop_frozen=stop_frozen, generic_chunk=generic_chunk, concurrent=concurrent)
    plan.upload(stream=stream)
    kw = {}
    if init_x is not None:
        packed = np.concatenate([U.pack_states(init_x[i], q.m).reshape(-1) for i, q in enumerate(qs)])
        kw["init_states"] = torch.from_numpy(packed.view(np.int32)).cuda()
        kw["seeded"] = torch.from_numpy(np.ascontiguousarray(seeded, dtype=np.uint8).reshape(-1)).cuda()
    if start_sweep is not None:
        kw["start_sweep"] = torch.from_numpy(np.ascontiguousarray(start_sweep, dtype=np.int32).reshape(-1)).cuda()
    if check_E:
        kw["check_E"] = torch.zeros(plan.total_replicas, dtype=torch.int64, device="cuda")
    if stream is not None:
        torch.cuda.synchronize()
    out = plan.anneal(stream=stream, **kw)
    for _ in range(replays - 1):
        out = plan.anneal(out=out, stream=stream, **kw)
    torch.cuda.synchronize()
    res = {k: getattr(out, k).cpu().numpy() for k in out.__dataclass_fields__}
    if check_E:
        res["check_E"] = kw["check_E"].cpu().numpy()
    return qs, plan, res


def split(U, qs, plan, res):
    """Per-instance numpy views: states unpacked to uint8 [R, N]."""
    out = []
    inst_off = 0
    for i, q in enumerate(qs):
        r0, r1 = plan.rep_offset[i], plan.rep_offset[i + 1]
        s0, s1 = plan.state_offset[i], plan.state_offset[i + 1]
        R = r1 - r0
        d = dict(
            final_x=U.unpack_states(res["final_states"][s0:s1].view(np.uint32).reshape(R, q.state_words), q.m),
            best_x=U.unpack_states(res["best_states"][s0:s1].view(np.uint32).reshape(R, q.state_words), q.m),
            final_E=res["final_E"][r0:r1], best_E=res["best_E"][r0:r1], best_sweep=res["best_sweep"][r0:r1],
            accepts=res["accepts"][r0:r1].view(np.uint64), draws=res["draws"][r0:r1].view(np.uint64),
            inst_best_E=int(res["inst_best_E"][i]), inst_best_replica=int(res["inst_best_replica"][i]),
            inst_best_sweep=int(res["inst_best_sweep"][i]),
            inst_best_x=U.unpack_states(res["inst_best_state"][inst_off:inst_off + q.state_words].view(np.uint32),
                                        q.m))
        if "check_E" in res:
            d["check_E"] = res["check_E"][r0:r1]
        inst_off += q.state_words
        out.append(d)
    return out


FIELDS = ("final_x", "final_E", "best_E", "best_sweep", "best_x", "accepts", "draws")


def compare_replicas(gpu, orc, reps, label=""):
    """Bit-exact comparison of the GPU replicas ``reps`` against oracle output rows."""
    for f in FIELDS:
        g = np.asarray(gpu[f])[reps]
        o = np.asarray(orc[f])
        if g.dtype != o.dtype:
            g = g.astype(o.dtype)
        if not np.array_equal(g, o):
            bad = np.nonzero((g != o).reshape(len(reps), -1).any(1))[0]
            raise AssertionError(f"{label}: field {f} differs for replicas {[reps[i] for i in bad[:8]]}: "
                                 f"gpu {g.reshape(len(reps), -1)[bad[0]][:12]} oracle {o.reshape(len(reps), -1)[bad[0]][:12]}")


def check_reduce(oracle, gi, R, label=""):
    """The per-instance outputs equal the oracle's lexicographic minimum of
    (best_E, replica) taken over the GPU's own per-replica results (every
    replica, whether or not the oracle re-ran it)."""
    best = oracle.instance_best(gi, list(range(R)))
    assert gi["inst_best_E"] == best["best_E"], label
    assert gi["inst_best_replica"] == best["best_replica"], label
    assert gi["inst_best_sweep"] == best["best_sweep"], label
    assert (gi["inst_best_x"] == best["best_x"]).all(), label
