"""Periodic invariant checks (uavq_anneal_checked) and the attempts counter on the GPU.

anneal_checked runs the schedule in resumed pieces and, after each, compares
the energy every replica carried by adding the dE of its accepted flips with
the MFMA recomputation of eqs. (3)-(6) from its state bits.  Its outputs must
equal one anneal_batch call bit for bit with no mismatch.  The attempts
counter is N per sweep a replica ran (sweeps max(start_sweep, s_begin) ..
s_end-1), carried across resumed segments."""
import numpy as np
import pytest

from paper_2608_25376_amd import inputs
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

FIELDS = ("final_states", "final_E", "best_E", "best_sweep", "best_states", "accepts", "draws",
          "inst_best_E", "inst_best_replica", "inst_best_sweep", "inst_best_state", "attempts")


@pytest.fixture(scope="module")
def U():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_25376_amd import uavq
    uavq.lib()
    return uavq


def _np(out):
    return {f: getattr(out, f).cpu().numpy() for f in FIELDS}


def _start_sweeps(U, plan, S, rng):
    import torch
    start = rng.integers(0, S + 1, size=plan.total_replicas).astype(np.int32)
    return start, torch.from_numpy(start).cuda()


CASES = {
    # name: (grids, replicas, sweeps, T0, dense)
    "m<=64": ([inputs.grid(8, 8, 0.1, seed=2, inst=3)], 48, 90, 100.0, False),
    "chunk2": ([inputs.grid(10, 10, 0.1, seed=4, inst=5)], 24, 70, 150.0, False),
    "chunk3": ([inputs.grid(12, 12, 0.0, seed=1, inst=0)], 12, 60, 200.0, False),
    "mixed": ([inputs.grid(5, 6, 0.1, seed=6, inst=1), inputs.grid(11, 11, 0.1, seed=7, inst=2)], 16, 64, 120.0,
              False),
    "dense": ([inputs.grid(5, 5, 0.0, seed=1, inst=4)], 32, 80, 60.0, True),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("every", [7, 1000])
def test_checked_equals_plain_run(U, case, every):
    """Pieces of `every` sweeps (a ragged last piece; 1000 = one piece), checked
    after each: no mismatch, and every output equals the plain run's."""
    import torch
    grids, R, S, T0, dense = CASES[case]
    say(f"case: anneal_checked {case} every={every} R={R} S={S}")
    qs = [U.qubo_build(g.rows, g.cols, nofly=g.nofly, dense=dense) for g in grids]
    plan = U.Plan(qs, [g.inst_id for g in grids], R, S, T0, 0.5, 3, dense=dense)
    plan.upload()
    rng = np.random.default_rng(11)
    start, d_start = _start_sweeps(U, plan, S, rng)
    plain = _np(plan.anneal(start_sweep=d_start))
    torch.cuda.synchronize()
    out, viol, n = plan.anneal_checked(every, start_sweep=d_start)
    torch.cuda.synchronize()
    assert n == 0 and int(viol.sum()) == 0
    got = _np(out)
    for f in FIELDS:
        assert np.array_equal(got[f], plain[f]), f"{case}: {f} differs"
    # the attempts counter: N per sweep each replica ran
    N = np.concatenate([np.full(R, q.n_vars, np.int64) for q in qs])
    assert np.array_equal(got["attempts"], N * (S - start)), case


def test_attempts_across_segments(U):
    """attempts after resumed pieces equal a straight run's, and a replica that
    starts after a piece's end adds nothing in it."""
    import torch
    g = inputs.grid(7, 7, 0.1, seed=5, inst=9)
    R, S = 40, 60
    say(f"case: attempts across segments R={R} S={S}")
    q = U.qubo_build(g.rows, g.cols, nofly=g.nofly)
    plan = U.Plan([q], [g.inst_id], R, S, 90.0, 0.5, 2)
    plan.upload()
    start, d_start = _start_sweeps(U, plan, S, np.random.default_rng(5))
    straight = plan.anneal(start_sweep=d_start).attempts.cpu().numpy()
    out = plan.alloc_outputs()
    seen = []
    for a, b in [(0, 13), (13, 13), (13, 41), (41, S)]:
        plan.anneal(out=out, s_begin=a, s_end=b, resume=a > 0, start_sweep=d_start)
        torch.cuda.synchronize()
        seen.append(out.attempts.cpu().numpy().copy())
        assert np.array_equal(seen[-1], q.n_vars * np.maximum(0, b - start)), (a, b)
    assert np.array_equal(seen[-1], straight)
