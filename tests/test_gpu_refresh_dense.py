"""GPU tests of the MFMA refresh and the dense-field kernel.

- energy_eval_dev (int8-limb MFMA, int32 accumulation) equals the oracle's
  QUBO energy on random, sparse and permutation states of several sizes;
- check_E (the final states re-evaluated by the refresh) equals the energies
  the sweep kernels maintained incrementally;
- the dense kernel (h = b + J x from the MFMA GEMM, O(N) row updates) follows
  the oracle's trajectories bit for bit, and equals the factored kernel."""
import numpy as np
import pytest

from paper_2608_25376_amd import inputs
from tests.gpu_util import check_reduce, compare_replicas, gpu_anneal, say, split

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def U():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_25376_amd import uavq
    uavq.lib()
    return uavq


def _states(o, rng, n):
    xs = [(rng.random(o.N) < p).astype(np.uint8) for p in np.linspace(0.0, 0.7, n - 4)]
    for _ in range(4):
        X = np.zeros((o.m, o.m), np.uint8)
        X[np.arange(o.m), rng.permutation(o.m)] = 1
        xs.append(X.reshape(-1))
    return np.array(xs)


@pytest.mark.parametrize("rows,cols,dens,closed", [(1, 2, 0.0, True), (3, 3, 0.0, True), (5, 6, 0.1, False),
                                                   (8, 8, 0.1, True), (10, 10, 0.0, True), (12, 12, 0.0, True)])
def test_energy_eval_dev_matches_oracle(U, oracle_lib, rows, cols, dens, closed):
    import torch
    g = inputs.grid(rows, cols, dens, seed=12, inst=rows)
    say(f"case: energy refresh {rows}x{cols} closed={closed}")
    q = U.qubo_build(rows, cols, nofly=g.nofly, closed=closed)
    o = oracle_lib.OracleQubo(rows, cols, nofly=g.nofly, closed=closed, dense=q.n_vars <= 4096)
    rng = np.random.default_rng(rows * 7 + cols)
    xs = _states(o, rng, 24)
    packed = U.pack_states(xs, o.m)
    d = torch.from_numpy(packed.view(np.int32).reshape(-1)).cuda()
    E = U.energy_eval_dev(q, d).cpu().numpy()
    torch.cuda.synchronize()
    if o.J is not None:
        ref = [o.energy(x) for x in xs]
    else:
        ref = [o.literal_energy(x) for x in xs]
    assert [int(e) for e in E] == ref


def test_check_E_equals_incremental_energy(U):
    grids = [inputs.grid(3, 3), inputs.grid(8, 8, 0.1, 1, 0), inputs.grid(10, 10, 0.1, 1, 5)]
    say("case: check_E batch of 3")
    qs, plan, res = gpu_anneal(U, grids, 24, 80, 150.0, 0.5, 9, check_E=True)
    assert np.array_equal(res["check_E"], res["final_E"])


@pytest.mark.parametrize("rows,cols,dens,inst,closed", [(1, 2, 0.0, 0, True), (3, 3, 0.0, 1, True),
                                                        (4, 5, 0.2, 2, True), (5, 5, 0.0, 3, False),
                                                        (7, 7, 0.1, 4, True)])
def test_dense_kernel_matches_oracle(U, oracle_lib, rows, cols, dens, inst, closed):
    g = inputs.grid(rows, cols, dens, seed=5, inst=inst)
    say(f"case: dense {rows}x{cols} inst={inst} closed={closed}")
    qs, plan, res = gpu_anneal(U, [g], 13, 50, 80.0, 0.5, 21, dense=True, closed=closed, check_E=True)
    gi = split(U, qs, plan, res)[0]
    o = oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly, closed=closed)
    orc = oracle_lib.anneal(o, 50, 80.0, 0.5, 21, g.inst_id, list(range(13)), threads=8)
    compare_replicas(gi, orc, list(range(13)), f"dense {rows}x{cols}")
    assert np.array_equal(res["check_E"], res["final_E"])
    best = oracle_lib.instance_best(orc, list(range(13)))
    assert gi["inst_best_E"] == best["best_E"] and gi["inst_best_replica"] == best["best_replica"]


def test_dense_equals_factored_grid8x8(U, oracle_lib):
    """The 8x8 workload at full size (dense J int16, 2916 variables, 1024
    replicas x 2000 sweeps): dense kernel == factored kernel on every
    replica, == oracle on sampled replicas, and its per-instance reduce over
    all replicas == the oracle's over the same per-replica results."""
    w = inputs.workload("grid8x8_nofly0.1")
    g = w.grids[0]
    R, S = w.replicas, w.sweeps
    say(f"case: dense vs factored 8x8 R={R} S={S}")
    qd, pd, rd = gpu_anneal(U, [g], R, S, w.T0, w.T1, w.seed, dense=True, check_E=True)
    qf, pf, rf = gpu_anneal(U, [g], R, S, w.T0, w.T1, w.seed)
    for k in ("final_states", "best_states", "final_E", "best_E", "best_sweep", "accepts", "draws", "inst_best_E",
              "inst_best_replica", "inst_best_state"):
        assert np.array_equal(rd[k], rf[k]), k
    assert np.array_equal(rd["check_E"], rd["final_E"])
    gi = split(U, qd, pd, rd)[0]
    o = oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly)
    reps = [0, 1, 77, 255, 256, 511, 640, 1023]
    orc = oracle_lib.anneal(o, S, w.T0, w.T1, w.seed, g.inst_id, reps, threads=8)
    compare_replicas(gi, orc, reps, "dense 8x8")
    check_reduce(oracle_lib, gi, R, "dense 8x8 reduce")


def test_dense_largest_penalty(U, oracle_lib):
    """The largest penalty the dense J accepts (2P + w_max = 16383, so the high
    int8 limb of J is 127): the MFMA field refresh and the dense sweep follow
    the oracle bit for bit, and one more unit of penalty is refused."""
    g = inputs.grid(7, 7, 0.1, seed=5, inst=70)
    wmax = U.qubo_build(g.rows, g.cols, nofly=g.nofly).w_max
    P = (16383 - wmax) // 2
    say(f"case: dense 7x7 P={P}")
    R, S, T0, T1 = 16, 40, 200.0, 0.5
    qs, plan, res = gpu_anneal(U, [g], R, S, T0, T1, 23, dense=True, check_E=True, penalty=P)
    gi = split(U, qs, plan, res)[0]
    assert np.array_equal(res["check_E"], res["final_E"])
    o = oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly, penalty=P)
    orc = oracle_lib.anneal(o, S, T0, T1, 23, g.inst_id, list(range(R)), threads=8)
    compare_replicas(gi, orc, list(range(R)), "dense largest penalty")
    check_reduce(oracle_lib, gi, R, "dense largest penalty reduce")
    with pytest.raises(U.UavqError):
        U.qubo_build(g.rows, g.cols, nofly=g.nofly, penalty=P + 1, dense=True)
