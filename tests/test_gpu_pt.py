"""Parallel tempering on the GPU against the oracle, bit for bit.

The exchange kernel alone is compared with the oracle's exchange on random
states and energies (ragged chain counts, several rounds, both parities); the
whole tempering run (constant-temperature slot plans in segments plus exchange
rounds) is compared slot by slot and chain by chain: final and best states,
energies, best sweeps, counters and the number of swaps per pair."""
import numpy as np
import pytest

from paper_2608_25376_amd import inputs
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def U():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_25376_amd import uavq
    uavq.lib()
    return uavq


@pytest.mark.parametrize("K,R,W,T_hot,T_cold", [(5, 301, 3, 100.0, 2.0), (2, 64, 1, 50.0, 5.0),
                                                 (8, 129, 130, 200.0, 0.5), (1, 10, 2, 10.0, 1.0)])
def test_exchange_kernel_equals_oracle(U, oracle_lib, K, R, W, T_hot, T_cold):
    import torch
    say(f"case: pt_exchange K={K} R={R} W={W}")
    rng = np.random.default_rng(K * 1000 + R)
    states = rng.integers(-2 ** 31, 2 ** 31, (K, R, W), dtype=np.int64).astype(np.int32)
    E = rng.integers(-200, 1500, (K, R)).astype(np.int64)
    T, DX, xthr = U.pt_ladder(T_hot, T_cold, K)
    d_DX = torch.from_numpy(DX if K > 1 else np.zeros(1, np.int32)).cuda()
    d_xthr = torch.from_numpy(np.ascontiguousarray(xthr if K > 1 else np.zeros((1, 2), np.uint32)).view(np.int32)).cuda()
    ds, dE = torch.from_numpy(states.copy()).cuda(), torch.from_numpy(E.copy()).cuda()
    sw = torch.zeros(max(K - 1, 1), dtype=torch.int64, device="cuda")
    x = states.view(np.uint8).reshape(K, R, 4 * W).copy()
    Eo = E.copy()
    swo = np.zeros(max(K - 1, 1), np.uint64)
    for rnd in range(7):
        U.pt_exchange(rnd, 9, 4, d_DX, d_xthr, ds, dE, sw)
        if K > 1:
            oracle_lib.pt_exchange(x, Eo, rnd, 9, 4, DX, xthr, swo)
    torch.cuda.synchronize()
    assert np.array_equal(ds.cpu().numpy().view(np.uint8).reshape(K, R, 4 * W), x)
    assert np.array_equal(dE.cpu().numpy(), Eo)
    assert np.array_equal(sw.cpu().numpy()[:K - 1].astype(np.uint64), swo[:K - 1])
    if K > 1:
        assert swo.sum() > 0


CASES = [
    # name, grid (rows, cols, density, inst), closed, K, R, S, T_hot, T_cold, interval, plan options
    ("3x4_open", (3, 4, 0.0, 1), False, 4, 40, 60, 80.0, 2.0, 1, {}),
    ("6x6_nofly", (6, 6, 0.1, 2), True, 5, 33, 50, 150.0, 3.0, 3, {}),
    ("8x8_pc", (8, 8, 0.1, 3), True, 3, 64, 24, 200.0, 5.0, 2, {}),
    ("7x7_w1", (7, 7, 0.0, 5), True, 4, 20, 30, 100.0, 2.0, 4, {"no_producer": True}),
    ("9x9_class2", (9, 9, 0.1, 4), True, 3, 6, 12, 120.0, 4.0, 5, {}),
]


@pytest.mark.parametrize("name,grid,closed,K,R,S,T_hot,T_cold,interval,kw", CASES)
def test_tempering_equals_oracle(U, oracle_lib, name, grid, closed, K, R, S, T_hot, T_cold, interval, kw):
    import torch
    rows, cols, dens, inst = grid
    g = inputs.grid(rows, cols, dens, seed=5, inst=inst)
    say(f"case: tempering {name} K={K} R={R} S={S} interval={interval}")
    q = U.qubo_build(g.rows, g.cols, nofly=g.nofly, closed=closed)
    pt = U.ParallelTempering(q, g.inst_id, K, R, S, T_hot, T_cold, seed=11, interval=interval, **kw)
    res = pt.run()
    torch.cuda.synchronize()
    o = oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly, closed=closed)
    ref = oracle_lib.pt_anneal(o, K, R, S, T_hot, T_cold, 11, g.inst_id, interval=interval, threads=8)
    assert res["rounds"] == ref["rounds"]
    assert np.array_equal(pt.T, ref["T"])
    assert np.array_equal(res["swaps"].cpu().numpy().astype(np.uint64), ref["swaps"])
    W = q.state_words
    h = {f: res[f].cpu().numpy() for f in ("states", "E", "best_E", "best_sweep", "best_states", "accepts", "draws",
                                          "inst_best_E")}
    for k in range(K):
        fx = U.unpack_states(h["states"][k].view(np.uint32), q.m)
        bx = U.unpack_states(h["best_states"][k].view(np.uint32), q.m)
        assert np.array_equal(fx, ref["final_x"][k]), (name, k, "final_x")
        assert np.array_equal(h["E"][k], ref["final_E"][k]), (name, k, "final_E")
        assert np.array_equal(h["best_E"][k], ref["best_E"][k]), (name, k, "best_E")
        assert np.array_equal(h["best_sweep"][k], ref["best_sweep"][k]), (name, k, "best_sweep")
        assert np.array_equal(bx, ref["best_x"][k]), (name, k, "best_x")
        assert np.array_equal(h["accepts"][k].view(np.uint64), ref["accepts"][k]), (name, k)
        assert np.array_equal(h["draws"][k].view(np.uint64), ref["draws"][k]), (name, k)
        assert h["inst_best_E"][k] == ref["best_E"][k].min()
    # the MFMA energy of every slot's states equals the energy carried with it
    chk = torch.empty(K * R, dtype=torch.int64, device="cuda")
    U.energy_eval_dev(q, res["states"].reshape(-1), chk)
    torch.cuda.synchronize()
    assert np.array_equal(chk.cpu().numpy(), h["E"].reshape(-1))


def test_instance_schedules_equal_separate_plans(U, oracle_lib):
    """A plan whose instances carry their own schedules (cooling and constant,
    a repeated one among them) gives each instance exactly what a plan of that
    instance alone with that schedule gives."""
    import torch
    gs = [inputs.grid(6, 6, 0.1, seed=2, inst=40), inputs.grid(9, 9, 0.1, seed=2, inst=41),
          inputs.grid(5, 7, 0.0, seed=2, inst=42), inputs.grid(6, 6, 0.1, seed=2, inst=43)]
    sch = [(150.0, 0.5), (60.0, 60.0), (90.0, 2.0), (150.0, 0.5)]
    R, S = 24, 40
    say(f"case: per-instance schedules R={R} S={S}")
    qs = [U.qubo_build(g.rows, g.cols, nofly=g.nofly) for g in gs]
    plan = U.Plan(qs, [g.inst_id for g in gs], R, S, 200.0, 0.5, 7, inst_T=sch)
    plan.upload()
    out = plan.anneal()
    torch.cuda.synchronize()
    for i, (q, g, (T0, T1)) in enumerate(zip(qs, gs, sch)):
        p1 = U.Plan([q], [g.inst_id], R, S, T0, T1, 7)
        p1.upload()
        o1 = p1.anneal()
        torch.cuda.synchronize()
        r0, r1 = plan.rep_offset[i], plan.rep_offset[i + 1]
        s0, s1 = plan.state_offset[i], plan.state_offset[i + 1]
        for f in ("final_E", "best_E", "best_sweep", "accepts", "draws"):
            assert np.array_equal(getattr(out, f)[r0:r1].cpu().numpy(), getattr(o1, f).cpu().numpy()), (i, f)
        for f in ("final_states", "best_states"):
            assert np.array_equal(getattr(out, f)[s0:s1].cpu().numpy(), getattr(o1, f).cpu().numpy()), (i, f)
        assert int(out.inst_best_E[i].cpu()) == int(o1.inst_best_E[0].cpu())
    # and one of them against the oracle
    o = oracle_lib.OracleQubo(gs[1].rows, gs[1].cols, nofly=gs[1].nofly)
    ref = oracle_lib.anneal(o, S, 60.0, 60.0, 7, gs[1].inst_id, list(range(R)), threads=8)
    r0 = plan.rep_offset[1]
    assert np.array_equal(out.final_E[r0:r0 + R].cpu().numpy(), ref["final_E"])
    assert np.array_equal(out.best_E[r0:r0 + R].cpu().numpy(), ref["best_E"])


@pytest.mark.parametrize("interval", [1, 10])
def test_tempering_full_size_sampled_chains(U, oracle_lib, interval):
    """The tempering study's configuration at full size (8x8 field with no-fly
    cells, K = 16 slots x R = 64 chains, 1000 sweeps, ladder 100 -> 0.5):
    sampled chains, every slot, bit-exact with the oracle's per-chain loop."""
    import torch
    g = inputs.grid(8, 8, 0.1, seed=1, inst=0)
    K, R, S = 16, 64, 1000
    chains = [0, 1, 13, 31, 32, 47, 62, 63]
    say(f"case: tempering full size K={K} R={R} S={S} interval={interval}")
    q = U.qubo_build(g.rows, g.cols, nofly=g.nofly)
    pt = U.ParallelTempering(q, g.inst_id, K, R, S, 100.0, 0.5, seed=1, interval=interval)
    res = pt.run()
    torch.cuda.synchronize()
    o = oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly)
    ref = oracle_lib.pt_anneal_chains(o, K, chains, S, 100.0, 0.5, 1, g.inst_id, interval=interval, threads=8)
    W = q.state_words
    h = {f: res[f].cpu().numpy() for f in ("states", "E", "best_E", "best_sweep", "best_states", "accepts", "draws")}
    for i, r in enumerate(chains):
        for k in range(K):
            assert np.array_equal(U.unpack_states(h["states"][k, r].view(np.uint32)[None], q.m)[0],
                                  ref["final_x"][i, k]), (r, k, "final_x")
            assert h["E"][k, r] == ref["final_E"][i, k], (r, k)
            assert h["best_E"][k, r] == ref["best_E"][i, k], (r, k)
            assert h["best_sweep"][k, r] == ref["best_sweep"][i, k], (r, k)
            assert np.array_equal(U.unpack_states(h["best_states"][k, r].view(np.uint32)[None], q.m)[0],
                                  ref["best_x"][i, k]), (r, k, "best_x")
            assert int(h["accepts"][k, r]) == int(ref["accepts"][i, k]), (r, k)
            assert int(h["draws"][k, r]) == int(ref["draws"][i, k]), (r, k)
    assert ref["swaps"].sum() > 0


@pytest.mark.parametrize("kw", [{"stop_frozen": True}, {"persistent": True}, {"no_producer": True}])
def test_tempering_plan_options_equal_default(U, kw):
    """Plan options that never change results (stopping frozen replicas, whose
    constant schedules never raise the cutoff; the persistent work queue; the
    one-wave kernel) give the default tempering run's outputs bit for bit."""
    import torch
    g = inputs.grid(7, 8, 0.1, seed=6, inst=3)
    K, R, S = 6, 48, 60
    say(f"case: tempering options {kw} K={K} R={R} S={S}")
    q = U.qubo_build(g.rows, g.cols, nofly=g.nofly)
    ref = U.ParallelTempering(q, g.inst_id, K, R, S, 90.0, 1.0, seed=4, interval=3).run()
    got = U.ParallelTempering(q, g.inst_id, K, R, S, 90.0, 1.0, seed=4, interval=3, **kw).run()
    torch.cuda.synchronize()
    for f in ("states", "E", "best_E", "best_sweep", "best_states", "accepts", "draws", "inst_best_E", "swaps"):
        assert torch.equal(got[f], ref[f]), (kw, f)
    assert got["rounds"] == ref["rounds"]


def test_batch_equals_single_fields(U, oracle_lib):
    """A batch of fields of different sizes in one plan, one batched exchange
    launch per round: every field's outputs equal its own tempering run bit
    for bit, and one of them equals the oracle's per-chain loop."""
    import torch
    gs = [inputs.grid(5, 6, 0.0, seed=7, inst=100), inputs.grid(8, 8, 0.1, seed=7, inst=200),
          inputs.grid(9, 9, 0.1, seed=7, inst=300)]
    K, R, S, iv = 4, 24, 30, 2
    say(f"case: tempering batch of {len(gs)} fields K={K} R={R} S={S}")
    qs = [U.qubo_build(g.rows, g.cols, nofly=g.nofly) for g in gs]
    batch = U.ParallelTemperingBatch(qs, [g.inst_id for g in gs], K, R, S, 90.0, 1.5, seed=3, interval=iv).run()
    torch.cuda.synchronize()
    for i, (g, q) in enumerate(zip(gs, qs)):
        one = U.ParallelTempering(q, g.inst_id, K, R, S, 90.0, 1.5, seed=3, interval=iv).run()
        torch.cuda.synchronize()
        for f in ("states", "E", "best_E", "best_sweep", "best_states", "accepts", "draws", "inst_best_E", "swaps"):
            assert torch.equal(batch[i][f], one[f]), (i, f)
        assert batch[i]["rounds"] == one["rounds"]
    g, q = gs[1], qs[1]
    o = oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly)
    ref = oracle_lib.pt_anneal_chains(o, K, list(range(R)), S, 90.0, 1.5, 3, g.inst_id, interval=iv, threads=8)
    assert np.array_equal(batch[1]["E"].cpu().numpy(), ref["final_E"].T)
    assert np.array_equal(batch[1]["best_E"].cpu().numpy(), ref["best_E"].T)
    assert np.array_equal(batch[1]["swaps"].cpu().numpy().astype(np.uint64), ref["swaps"].sum(0))
