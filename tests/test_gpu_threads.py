"""One plan used from several host threads at once (the plan's first-use
cache and its captured graph sit behind a per-plan lock; each thread brings
its own workspace, outputs and stream): every thread's outputs equal those of
a run on one thread."""
import threading

import numpy as np
import pytest

from paper_2608_25376_amd import inputs
from tests.gpu_util import say

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


@pytest.mark.parametrize("persistent,graph", [(False, False), (True, False), (True, True)])
def test_plan_shared_by_threads(U, persistent, graph):
    import torch
    grids = inputs.batch(10, seed=4, side_lo=3, side_hi=12)
    qs = [U.qubo_build(g.rows, g.cols, nofly=g.nofly) for g in grids]
    ids = [g.inst_id for g in grids]
    say(f"case: shared plan persistent={persistent} graph={graph}")
    ref_plan = U.Plan(qs, ids, 24, 60, 150.0, 0.5, 3, persistent=persistent)
    ref_plan.upload()
    ref = ref_plan.anneal()
    torch.cuda.synchronize()
    ref = {k: getattr(ref, k).cpu().numpy() for k in FIELDS}

    plan = U.Plan(qs, ids, 24, 60, 150.0, 0.5, 3, persistent=persistent, graph=graph)
    n = 4
    streams = [torch.cuda.Stream() for _ in range(n)]
    wss, outs = [], []
    for st in streams:
        with torch.cuda.stream(st):
            plan.upload(stream=st)          # a workspace per thread (persistent launches write their queue)
            wss.append(plan.ws)
            outs.append(plan.alloc_outputs())
    torch.cuda.synchronize()
    errors = []

    def work(i):
        try:
            for _ in range(3):
                plan.anneal(out=outs[i], stream=streams[i], ws=wss[i])
            streams[i].synchronize()
        except Exception as ex:   # noqa: BLE001 - reported below
            errors.append(repr(ex))

    ts = [threading.Thread(target=work, args=(i,)) for i in range(n)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for i in range(n):
        for k in FIELDS:
            assert np.array_equal(getattr(outs[i], k).cpu().numpy(), ref[k]), (i, k)
