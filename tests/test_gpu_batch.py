"""Batched annealing of many uneven instances: the persistent work-queue
launch, its HIP-graph capture and the autotuner's launch shapes all give the
oracle's results bit for bit (the random streams are addressed by instance
id, replica, sweep and site, so no launch shape can change a trajectory)."""
import json
import os

import numpy as np
import pytest

from paper_2608_25376_amd import inputs
from tests.gpu_util import check_reduce, compare_replicas, gpu_anneal, say, split

pytestmark = pytest.mark.gpu

FIELDS = ("final_states", "best_states", "final_E", "best_E", "best_sweep", "accepts", "draws", "inst_best_E",
          "inst_best_replica", "inst_best_sweep", "inst_best_state")


@pytest.fixture(scope="module")
def U():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_25376_amd import uavq
    uavq.lib()
    return uavq


def test_batch256_full_size_persistent_graph(U, oracle_lib):
    """256 instances (side 4..10, no-fly density 0..0.2), 256 replicas, 2000
    sweeps, persistent kernels captured in a HIP graph.  Per instance the
    oracle re-runs a sampled replica, and the per-instance reduce over all 256
    replicas is checked for every instance; for three instances the oracle
    runs all 256 replicas and the per-instance best (energy, replica, sweep,
    state) must match exactly."""
    import torch
    w = inputs.workload("batch256")
    stream = torch.cuda.Stream()
    say("case: batch256 full size, persistent + graph")
    qs, plan, res = gpu_anneal(U, w.grids, w.replicas, w.sweeps, w.T0, w.T1, w.seed, persistent=True, graph=True,
                               stream=stream)
    per = split(U, qs, plan, res)
    rng = np.random.default_rng(0)
    for i, g in enumerate(w.grids):
        o = oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly)
        r = int(rng.integers(0, w.replicas))
        orc = oracle_lib.anneal(o, w.sweeps, w.T0, w.T1, w.seed, g.inst_id, [r], threads=16)
        compare_replicas(per[i], orc, [r], f"batch256 instance {i} replica {r}")
        check_reduce(oracle_lib, per[i], w.replicas, f"batch256 instance {i} reduce")
    ms = [q.m for q in qs]
    for i in (int(np.argmin(ms)), 17, 101):
        g = w.grids[i]
        say(f"case: batch256 instance {i} (m={qs[i].m}) all replicas")
        o = oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly)
        reps = list(range(w.replicas))
        orc = oracle_lib.anneal(o, w.sweeps, w.T0, w.T1, w.seed, g.inst_id, reps, threads=16)
        best = oracle_lib.instance_best(orc, reps)
        assert per[i]["inst_best_E"] == best["best_E"]
        assert per[i]["inst_best_replica"] == best["best_replica"]
        assert per[i]["inst_best_sweep"] == best["best_sweep"]
        assert (per[i]["inst_best_x"] == best["best_x"]).all()
        assert np.array_equal(per[i]["best_E"], orc["best_E"])


def test_graph_replays_equal_eager(U):
    """Graph replays (with eager work and synchronisations in between) give
    the eager launch's bytes every time."""
    import torch
    grids = inputs.batch(24, seed=5, side_lo=3, side_hi=10)
    stream = torch.cuda.Stream()
    say("case: graph replays")
    qe, pe, eager = gpu_anneal(U, grids, 32, 60, 150.0, 0.5, 2, persistent=True, stream=stream)
    qg, pg, _ = gpu_anneal(U, grids, 32, 60, 150.0, 0.5, 2, persistent=True, graph=True, stream=stream)
    out = pg.alloc_outputs()
    torch.cuda.synchronize()
    for rep in range(4):
        pg.anneal(out=out, stream=stream)
        stream.synchronize()
        got = {k: getattr(out, k).cpu().numpy() for k in out.__dataclass_fields__}
        for k in FIELDS:
            assert np.array_equal(got[k], eager[k]), (rep, k)
        torch.zeros(1 << 20, device="cuda").sum().item()   # unrelated eager work between replays
        for f in out.__dataclass_fields__:
            getattr(out, f).zero_()
        torch.cuda.synchronize()


def test_launch_shapes_identical(U):
    """Every shape the autotuner may choose (replicas per block, m <= 64
    variant, persistent or not) gives identical bytes on an uneven batch."""
    grids = inputs.batch(12, seed=9, side_lo=3, side_hi=12)
    base = None
    for wpb, rowmask, persistent in ((4, False, False), (1, False, True), (2, True, True), (8, False, True),
                                     (16, True, False), (3, False, True)):
        say(f"case: shape wpb={wpb} rowmask={rowmask} persistent={persistent}")
        _, _, res = gpu_anneal(U, grids, 20, 40, 120.0, 0.5, 8, wpb=wpb, rowmask=rowmask, persistent=persistent)
        if base is None:
            base = res
        else:
            for k in FIELDS:
                assert np.array_equal(res[k], base[k]), (wpb, rowmask, persistent, k)


def test_concurrent_classes_identical(U):
    """UAVQ_CONCURRENT_CLASSES (the classes' kernels forked onto the plan's
    streams and joined back) gives the serial launch's bytes: plain, persistent,
    and captured in a graph over several replays, on a batch spanning classes
    1 to 3."""
    import torch
    grids = inputs.batch(20, seed=13, side_lo=3, side_hi=14)
    qs = [U.qubo_build(g.rows, g.cols, nofly=g.nofly) for g in grids]
    assert len({(q.m + 63) // 64 for q in qs}) >= 3
    say("case: concurrent classes")
    _, _, base = gpu_anneal(U, grids, 24, 50, 150.0, 0.5, 4)
    for persistent in (False, True):
        _, _, res = gpu_anneal(U, grids, 24, 50, 150.0, 0.5, 4, persistent=persistent, concurrent=True)
        for k in FIELDS:
            assert np.array_equal(res[k], base[k]), (persistent, k)
    stream = torch.cuda.Stream()
    _, _, res = gpu_anneal(U, grids, 24, 50, 150.0, 0.5, 4, persistent=True, graph=True, concurrent=True,
                           stream=stream, replays=3)
    for k in FIELDS:
        assert np.array_equal(res[k], base[k]), ("graph", k)


def test_autotune_cache_roundtrip(U, tmp_path):
    grids = inputs.batch(16, seed=2)
    qs = [U.qubo_build(g.rows, g.cols, nofly=g.nofly) for g in grids]
    ids = [g.inst_id for g in grids]
    cache = str(tmp_path / "tune.json")
    say("case: autotune")
    t1 = U.autotune(qs, ids, 64, 500, 200.0, 0.5, persistent=True, trial_sweeps=20, cache=cache)
    assert os.path.exists(cache)
    data = json.load(open(cache))
    assert len(data) == 1
    t2 = U.autotune(qs, ids, 64, 500, 200.0, 0.5, persistent=True, trial_sweeps=20, cache=cache)
    assert list(t2.waves_per_block) == list(t1.waves_per_block) and t2.variant_flags == t1.variant_flags
    # the tuned shape reproduces the default shape's results
    _, _, a = gpu_anneal(U, grids, 64, 30, 200.0, 0.5, 1, persistent=True, tune=t1)
    _, _, b = gpu_anneal(U, grids, 64, 30, 200.0, 0.5, 1)
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k
