"""End-to-end warm start on the GPU at a small scale: label instances with
the annealer, train the network with the library's kernels, sample seed
tours, anneal with half of the replicas seeded, and run the time-to-target
protocol.  The first test checks that every piece is wired as specified; the
second records what the trained network gains over random starts at a fixed
budget (the full study is the protocol's run) and checks that it learned
something: its cross-entropy on held-out labels is below the uniform level."""
import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_25376_amd import uavq, warmstart
    uavq.lib()
    return warmstart


def test_warm_start_pipeline(W):
    import torch
    from paper_2608_25376_amd import uavq
    say("case: warm start end to end (small)")
    train = W.make_instances(40, 10000)
    data, _ = W.label_data(train, 64, 300, 200.0, 0.5, 1)
    assert len(data) >= 35                         # best states are tours (penalty 2 w_max)
    for X, lab, m, _ in data:
        assert X.shape == (m, 16) and sorted(lab.tolist()) == list(range(m))
    net, curve, _ = W.train(data, epochs=6, batch=8, lr=3e-3)
    assert np.isfinite(curve).all() and curve[-1] <= curve[0] + 1e-3

    held = W.make_instances(6, 20000)
    qs = W._qubos(held)
    R, S = 32, 60
    plan = uavq.Plan(qs, [g.inst_id for g in held], R, S, 200.0, 0.5, 1, persistent=True)
    plan.upload()
    # seeded replicas started at sweep S run no sweep: their final state is the sampled tour
    init, _ = W.warm_init(net, plan, qs, 0.5, S)
    out = plan.anneal(**init)
    torch.cuda.synchronize()
    seeds = init["init_states"].cpu().numpy().view(np.uint32)
    fin = out.final_states.cpu().numpy().view(np.uint32)
    for i, q in enumerate(qs):
        for r in range(R // 2):
            w0 = plan.state_offset[i] + r * q.state_words
            x = uavq.unpack_states(seeds[w0:w0 + q.state_words], q.m).reshape(q.m, q.m)
            assert (x.sum(0) == 1).all() and (x.sum(1) == 1).all()
            assert np.array_equal(fin[w0:w0 + q.state_words], seeds[w0:w0 + q.state_words])
    rep = W.ttt(held, net, R, [25, 100], 200.0, 0.5, 1, 50.0, ref_sweeps=400, single=True)
    for mode in ("plain", "warm", "batched", "batched+warm"):
        fr = rep["modes"][mode]["fraction_at_target"]
        assert all(0.0 <= v <= 1.0 for v in fr.values())
    # plain and batched share instance ids, hence identical energies
    assert rep["modes"]["plain"]["fraction_at_target"] == rep["modes"]["batched"]["fraction_at_target"]
    say(f"ttt: {rep['modes']['batched']['fraction_at_target']} vs warm {rep['modes']['batched+warm']['fraction_at_target']}")


def test_warm_against_random_at_fixed_budget(W):
    """Schedule of the study (a constant T = 12, chosen on training fields
    only); 160 training fields labelled by 1024-replica annealing; 16
    held-out fields, 128 replicas, 50 sweeps: the fraction of fields within 1%
    of the best energy any of the runs found, with half of the replicas
    seeded from the network's tours against all random, is recorded."""
    T = 12.0
    say("case: warm vs random, 160 training / 16 held-out fields")
    train = W.make_instances(160, 10000)
    data, _ = W.label_data(train, 1024, 200, T, T, 1)
    assert len(data) == len(train)
    net, curve, _ = W.train(data, epochs=20, batch=16, lr=3e-3)
    held = W.make_instances(16, 20000)
    held_data, _ = W.label_data(held, 1024, 200, T, T, 4)
    ce, uni = W.mean_ce(net, held_data)
    say(f"held-out cross-entropy {ce:.4f}, uniform {uni:.4f}")
    assert ce < uni - 0.05                          # the network learned per-cell signal
    rep = W.ttt(held, net, 128, [50], T, T, 1, T, ref_sweeps=400, single=False, refs=[(15.4, 15.4, 400)])
    rnd = rep["modes"]["batched"]["fraction_at_target"][50]
    warm = rep["modes"]["batched+warm"]["fraction_at_target"][50]
    say(f"fraction at target at 50 sweeps: random {rnd:.3f}, warm {warm:.3f}; mean gap random "
        f"{rep['modes']['batched']['mean_gap'][50]:.4f}, warm {rep['modes']['batched+warm']['mean_gap'][50]:.4f}")
    assert 0.0 <= rnd <= 1.0 and 0.0 <= warm <= 1.0
