"""Segmented annealing, checkpoint/resume and the time-limit mode on the GPU.

Every random draw is addressed by (instance, replica, sweep, site), so a run
cut at sweep boundaries, or stopped, copied out and restored, must give the
outputs of one straight run bit for bit; a run stopped early (time-limit mode)
must equal the oracle on the completed prefix of the schedule."""
import numpy as np
import pytest

from paper_2608_25376_amd import inputs
from tests.gpu_util import compare_replicas, say, split

pytestmark = pytest.mark.gpu

OUT_FIELDS = ("final_states", "final_E", "best_E", "best_sweep", "best_states", "accepts", "draws",
              "inst_best_E", "inst_best_replica", "inst_best_sweep", "inst_best_state")


@pytest.fixture(scope="module")
def U():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_25376_amd import uavq
    uavq.lib()
    return uavq


def _plan(U, grids, R, S, T0, T1, seed, dense=False, rowmask=False, graph=False, stream=None, wpb=0):
    qs = [U.qubo_build(g.rows, g.cols, nofly=g.nofly, dense=dense) for g in grids]
    plan = U.Plan(qs, [g.inst_id for g in grids], R, S, T0, T1, seed, dense=dense, rowmask=rowmask, graph=graph,
                  waves_per_block=wpb)
    plan.upload(stream=stream)
    return qs, plan


def _init_kw(U, qs, plan, R, S, rng):
    """Half the replicas seeded with random bit states, start sweeps spread over [0, S]."""
    import torch
    xs = [rng.integers(0, 2, size=(R, q.m * q.m), dtype=np.uint8) for q in qs]
    packed = np.concatenate([U.pack_states(x, q.m).reshape(-1) for x, q in zip(xs, qs)])
    seeded = (rng.random(plan.total_replicas) < 0.5).astype(np.uint8)
    start = rng.integers(0, S + 1, size=plan.total_replicas).astype(np.int32)
    return dict(init_states=torch.from_numpy(packed.view(np.int32)).cuda(),
                seeded=torch.from_numpy(seeded).cuda(), start_sweep=torch.from_numpy(start).cuda())


def _np(out):
    return {f: getattr(out, f).cpu().numpy() for f in OUT_FIELDS}


def _run(plan, cuts, kw=None, stream=None, check_E=None):
    """Anneal through the sweep boundaries ``cuts`` (0 = c_0 < ... < c_k = S), one call per piece."""
    import torch
    kw = dict(kw or {})
    out = plan.alloc_outputs()
    if stream is not None:
        torch.cuda.synchronize()
    for i in range(len(cuts) - 1):
        piece = dict(kw) if i == 0 else {k: v for k, v in kw.items() if k == "start_sweep"}
        plan.anneal(out=out, s_begin=cuts[i], s_end=cuts[i + 1], resume=i > 0, stream=stream,
                    check_E=check_E, **piece)
    torch.cuda.synchronize()
    return out


def _assert_same(a, b, label):
    for f in OUT_FIELDS:
        if not np.array_equal(a[f], b[f]):
            bad = np.nonzero(a[f].reshape(-1) != b[f].reshape(-1))[0]
            raise AssertionError(f"{label}: {f} differs at {bad[:8]}")


@pytest.mark.parametrize("case", ["ylds", "factored", "rowmask", "mixed", "dense", "wpb1"])
def test_segments_equal_straight_run(U, case):
    """Cut at several sweep boundaries (one empty piece) == one anneal_batch."""
    S, R = 90, 96
    grids = {"ylds": [inputs.grid(6, 7, 0.1, seed=3, inst=1)],
             "factored": [inputs.grid(9, 9, 0.1, seed=3, inst=2)],
             "rowmask": [inputs.grid(5, 6, 0.0, seed=3, inst=3)],
             "mixed": [inputs.grid(4, 4, 0.0, seed=3, inst=4), inputs.grid(12, 12, 0.05, seed=3, inst=5),
                       inputs.grid(8, 8, 0.2, seed=3, inst=6)],
             "dense": [inputs.grid(4, 5, 0.0, seed=3, inst=7)],
             "wpb1": [inputs.grid(7, 7, 0.0, seed=3, inst=8)]}[case]
    say(f"case: segments {case} R={R} S={S}")
    qs, plan = _plan(U, grids, R, S, 150.0, 0.5, 9, dense=case == "dense", rowmask=case == "rowmask",
                     wpb=1 if case == "wpb1" else 0)
    straight = _np(_run(plan, [0, S]))
    for cuts in ([0, 1, S], [0, 37, 37, 64, S], [0, S - 1, S]):
        _assert_same(_np(_run(plan, cuts)), straight, f"{case} cuts={cuts}")


@pytest.mark.parametrize("case", ["ylds", "factored"])
def test_segments_seeded_and_start_sweeps(U, case):
    """Seeded replicas and per-replica start sweeps inside and across the pieces."""
    S, R = 70, 80
    g = inputs.grid(6, 6, 0.0, seed=4, inst=2) if case == "ylds" else inputs.grid(10, 10, 0.1, seed=4, inst=3)
    say(f"case: seeded segments {case} R={R} S={S}")
    qs, plan = _plan(U, [g], R, S, 120.0, 0.5, 5)
    kw = _init_kw(U, qs, plan, R, S, np.random.default_rng(11))
    straight = _np(_run(plan, [0, S], kw))
    _assert_same(_np(_run(plan, [0, 20, 41, S], kw)), straight, f"{case} seeded")


def test_segments_graph_mode(U):
    """Graph mode captures each distinct piece; replays equal the eager straight run."""
    import torch
    S, R = 60, 64
    g = inputs.grid(6, 6, 0.1, seed=6, inst=1)
    say(f"case: graph segments R={R} S={S}")
    st = torch.cuda.Stream()
    qs, plan = _plan(U, [g], R, S, 100.0, 0.5, 2)
    straight = _np(_run(plan, [0, S]))
    qs, gplan = _plan(U, [g], R, S, 100.0, 0.5, 2, graph=True, stream=st)
    for _ in range(2):
        _assert_same(_np(_run(gplan, [0, 25, S], stream=st)), straight, "graph")


def test_checkpoint_restore_resume(U, oracle_lib):
    """Stop after S1 sweeps, copy the replica state out, keep annealing the
    live buffers (so the copy must be independent), restore the copy into
    fresh buffers and resume: equal to the straight run, and the MFMA energy
    check of the final states agrees."""
    import torch
    S, R, S1 = 80, 128, 33
    g = inputs.grid(7, 8, 0.1, seed=8, inst=4)
    say(f"case: checkpoint R={R} S={S} S1={S1}")
    qs, plan = _plan(U, [g], R, S, 90.0, 0.5, 13)
    straight = _np(_run(plan, [0, S]))
    live = plan.alloc_outputs()
    plan.anneal(out=live, s_begin=0, s_end=S1)
    ck = plan.checkpoint(live)
    plan.anneal(out=live, s_begin=S1, s_end=S, resume=True)
    # host round trip of the checkpoint, as a file would hold it
    host = {k: v.cpu().numpy().copy() for k, v in ck.items()}
    del ck
    restored = plan.restore({k: torch.from_numpy(v).cuda() for k, v in host.items()})
    check = torch.zeros(plan.total_replicas, dtype=torch.int64, device="cuda")
    plan.anneal(out=restored, s_begin=S1, s_end=S, resume=True, check_E=check)
    torch.cuda.synchronize()
    _assert_same(_np(restored), straight, "restored")
    _assert_same(_np(live), straight, "live")
    assert np.array_equal(check.cpu().numpy(), straight["final_E"])


def test_prefix_equals_oracle(U, oracle_lib):
    """A run stopped after S' < S sweeps of an S-sweep schedule equals the
    oracle run over the first S' rows of the same table."""
    S, Sp, R = 100, 41, 48
    g = inputs.grid(5, 6, 0.1, seed=9, inst=6)
    say(f"case: prefix R={R} S={S} S'={Sp}")
    qs, plan = _plan(U, [g], R, S, 70.0, 0.5, 21)
    out = _run(plan, [0, 17, Sp])
    res = {k: getattr(out, k).cpu().numpy() for k in out.__dataclass_fields__}
    gi = split(U, qs, plan, res)[0]
    o = oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly)
    dmax, thr = oracle_lib.thresholds(70.0, 0.5, S)
    orc = oracle_lib.anneal(o, Sp, 70.0, 0.5, 21, g.inst_id, list(range(R)), table=(dmax, thr[:Sp].copy()),
                            threads=8)
    compare_replicas(gi, orc, list(range(R)), "prefix")


def test_time_limited_mode(U, oracle_lib):
    """The time-limit mode stops at a piece boundary; whatever the stop, the
    outputs equal a run with s_end = sweeps completed and the oracle on that
    prefix (sampled replicas)."""
    import torch
    S, R = 4000, 2048
    g = inputs.grid(8, 8, 0.1, seed=10, inst=0)
    say(f"case: time limit R={R} S={S}")
    qs, plan = _plan(U, [g], R, S, 100.0, 0.5, 1)
    plan.anneal(s_end=10)          # warm the kernels before timing
    torch.cuda.synchronize()
    out, done = plan.anneal_time_limited(15.0, segment_sweeps=200)
    say(f"time limit: {done} of {S} sweeps in the budget")
    assert 200 <= done <= S and done % 200 == 0
    ref = _np(_run(plan, [0, done]))
    _assert_same(_np(out), ref, "time-limited")
    full, done_all = plan.anneal_time_limited(1e9, segment_sweeps=1000)
    assert done_all == S
    _assert_same(_np(full), _np(_run(plan, [0, S])), "unlimited")
    res = {k: getattr(out, k).cpu().numpy() for k in out.__dataclass_fields__}
    gi = split(U, qs, plan, res)[0]
    reps = [0, 777, R - 1]
    o = oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly)
    dmax, thr = oracle_lib.thresholds(100.0, 0.5, S)
    orc = oracle_lib.anneal(o, done, 100.0, 0.5, 1, g.inst_id, reps, table=(dmax, thr[:done].copy()), threads=3)
    compare_replicas(gi, orc, reps, "time-limited prefix")


def test_energy_check_flags_a_corrupted_state(U):
    """The invariant check (MFMA energy of the final states against the
    incrementally kept energies) is sensitive: after one bit of one replica's
    state is flipped, exactly that replica disagrees."""
    import torch
    g = inputs.grid(6, 6, 0.1, seed=3, inst=2)
    R, S = 32, 50
    say(f"case: invariant check R={R} S={S}")
    qs, plan = _plan(U, [g], R, S, 80.0, 0.5, 3)
    check = torch.zeros(plan.total_replicas, dtype=torch.int64, device="cuda")
    out = _run(plan, [0, S], check_E=check)
    final_E = out.final_E.cpu().numpy()
    assert np.array_equal(check.cpu().numpy(), final_E)
    q = qs[0]
    states = out.final_states.clone()
    states[5 * q.state_words + 2] ^= 1          # one bit of replica 5's state
    E2 = torch.empty(R, dtype=torch.int64, device="cuda")
    U.energy_eval_dev(q, states, E2)
    torch.cuda.synchronize()
    assert list(np.nonzero(E2.cpu().numpy() != final_E)[0]) == [5]


def test_reduce_at_end(U):
    """UAVQ_REDUCE_AT_END: segments before the last leave the per-instance
    outputs untouched; the last one fills them, and every output equals the
    straight run's."""
    import torch
    gs = [inputs.grid(6, 7, 0.1, seed=3, inst=21), inputs.grid(9, 9, 0.1, seed=3, inst=22)]
    S, R = 80, 40
    say(f"case: reduce at end R={R} S={S}")
    qs = [U.qubo_build(g.rows, g.cols, nofly=g.nofly) for g in gs]
    ref_plan = U.Plan(qs, [g.inst_id for g in gs], R, S, 120.0, 0.5, 5)
    ref_plan.upload()
    straight = _np(_run(ref_plan, [0, S]))
    plan = U.Plan(qs, [g.inst_id for g in gs], R, S, 120.0, 0.5, 5, reduce_at_end=True)
    plan.upload()
    out = plan.alloc_outputs()
    out.inst_best_E.fill_(-7)
    plan.anneal(out=out, s_begin=0, s_end=37)
    plan.anneal(out=out, s_begin=37, s_end=64, resume=True)
    torch.cuda.synchronize()
    assert (out.inst_best_E.cpu().numpy() == -7).all()
    plan.anneal(out=out, s_begin=64, s_end=S, resume=True)
    torch.cuda.synchronize()
    _assert_same(_np(out), straight, "reduce at end")
