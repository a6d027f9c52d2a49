"""UAVQ_STOP_FROZEN: a replica whose sweep had neither an accept nor a draw
stops sweeping.  Every later sweep would have left it unchanged (each of its
dE is at or above the draw cutoff, which never grows along the schedule), so
every output must equal the run that sweeps to the end, bit for bit."""
import numpy as np
import pytest

from paper_2608_25376_amd import inputs
from tests.gpu_util import gpu_anneal, say

pytestmark = pytest.mark.gpu

FIELDS = ("final_states", "final_E", "best_E", "best_sweep", "best_states", "accepts", "draws",
          "inst_best_E", "inst_best_replica", "inst_best_sweep", "inst_best_state")


@pytest.fixture(scope="module")
def U():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_25376_amd import uavq
    uavq.lib()
    return uavq


@pytest.mark.parametrize("case,grids,R,S,kw,cls,kernel", [
    ("pc", [(8, 8, 0.1, 0)], 96, 400, {}, 1, "k_sweep_ylds_pc"),
    ("w1", [(7, 7, 0.0, 1)], 64, 400, {"no_producer": True}, 1, "k_sweep_ylds_w1"),
    ("ylds", [(6, 6, 0.1, 2)], 64, 300, {"wpb": 8}, 1, "k_sweep_ylds"),
    ("chunk2", [(9, 9, 0.1, 3)], 32, 300, {}, 2, "k_sweep_chunk<2>"),
    ("chunk3", [(12, 12, 0.0, 4)], 16, 200, {}, 3, "k_sweep_chunk<3>"),
    ("chunk4", [(15, 15, 0.05, 8)], 8, 200, {}, 4, "k_sweep_chunk<4>"),
    ("chunk5", [(18, 18, 0.1, 9)], 4, 150, {}, 5, "k_sweep_chunk<5>"),
    ("factored2", [(9, 9, 0.1, 3)], 32, 300, {"generic_chunk": True}, 2, "k_sweep_factored<2>"),
    ("factored3", [(12, 12, 0.0, 4)], 16, 200, {"generic_chunk": True}, 3, "k_sweep_factored<3>"),
    ("persistent_batch", [(4, 4, 0.0, 5), (10, 10, 0.1, 6), (5, 6, 0.2, 7)], 24, 300, {"persistent": True}, 2,
     "k_sweep_chunk<2>"),
])
def test_stop_frozen_identical(U, case, grids, R, S, kw, cls, kernel):
    gs = [inputs.grid(r, c, d, seed=3, inst=i) for r, c, d, i in grids]
    say(f"case: stop_frozen {case} R={R} S={S}")
    rng = np.random.default_rng(5)
    start = rng.integers(0, S // 2, size=R * len(gs)).astype(np.int32)   # replicas that start late
    qa, pa, ra = gpu_anneal(U, gs, R, S, 120.0, 0.5, 9, start_sweep=start, **kw)
    qb, pb, rb = gpu_anneal(U, gs, R, S, 120.0, 0.5, 9, start_sweep=start, stop_frozen=True, **kw)
    assert pb.kernel_name(cls) == kernel
    for f in FIELDS:
        assert np.array_equal(ra[f], rb[f]), f"{case}: {f} differs"


def test_stop_frozen_with_segments(U):
    """Segments restart the freeze detection (one sweep later); the result is
    still the straight run's."""
    import torch
    g = inputs.grid(7, 8, 0.1, seed=4, inst=8)
    R, S = 64, 300
    say(f"case: stop_frozen segments R={R} S={S}")
    qs, plan, ref = gpu_anneal(U, [g], R, S, 100.0, 0.5, 2)
    q = U.qubo_build(g.rows, g.cols, nofly=g.nofly)
    p2 = U.Plan([q], [g.inst_id], R, S, 100.0, 0.5, 2, stop_frozen=True)
    p2.upload()
    out = p2.alloc_outputs()
    for i, (b, e) in enumerate([(0, 120), (120, 121), (121, 260), (260, S)]):
        p2.anneal(out=out, s_begin=b, s_end=e, resume=i > 0)
    torch.cuda.synchronize()
    for f in FIELDS:
        assert np.array_equal(getattr(out, f).cpu().numpy(), ref[f]), f
