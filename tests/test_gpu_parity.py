"""GPU parity: the HIP annealer, called through the C ABI, against the CPU
oracle on the same seeded inputs.  All annealing arithmetic is integer, so
the bar is bit-exact equality of every trajectory output (final and best
states, energies, best sweep, accept and draw counts)."""
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


def _oracle_for(oracle_lib, g, closed=True, penalty=0):
    return oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly, closed=closed, penalty=penalty,
                                 dense=g.rows * g.cols <= 100)


def _check_instance(U, oracle_lib, g, R, S, T0, T1, seed, reps=None, closed=True, wpb=0, dense=False,
                    rowmask=False, penalty=0, check_E=False, threads=8):
    say(f"case: {g.rows}x{g.cols} n_free={g.n_free} inst={g.inst_id} R={R} S={S} T={T0}->{T1} seed={seed} "
        f"closed={closed} wpb={wpb} dense={dense} rowmask={rowmask} penalty={penalty}")
    qs, plan, res = gpu_anneal(U, [g], R, S, T0, T1, seed, dense=dense, wpb=wpb, closed=closed, rowmask=rowmask,
                               penalty=penalty, check_E=check_E)
    gi = split(U, qs, plan, res)[0]
    if check_E:
        assert np.array_equal(gi["check_E"], gi["final_E"])
    o = _oracle_for(oracle_lib, g, closed, penalty)
    reps = list(range(R)) if reps is None else list(reps)
    orc = oracle_lib.anneal(o, S, T0, T1, seed, g.inst_id, reps, threads=threads)
    compare_replicas(gi, orc, reps, f"{g.rows}x{g.cols}")
    # the reduce over every replica (those the oracle did not re-run included)
    check_reduce(oracle_lib, gi, R, f"{g.rows}x{g.cols} reduce")
    if len(reps) == R:
        best = oracle_lib.instance_best(orc, reps)
        assert gi["inst_best_E"] == best["best_E"]
        assert gi["inst_best_replica"] == best["best_replica"]
        assert gi["inst_best_sweep"] == best["best_sweep"]
        assert (gi["inst_best_x"] == best["best_x"]).all()
    return gi, o


def test_grid3x3_full(U, oracle_lib):
    """3x3, 64 replicas, 1000 sweeps, T 100 -> 0.5, seed 1: every replica."""
    w = inputs.workload("grid3x3")
    gi, o = _check_instance(U, oracle_lib, w.grids[0], w.replicas, w.sweeps, w.T0, w.T1, w.seed)
    # the returned best state decodes to a tour whose cost is its energy
    path, cost = U.decode_path(U.qubo_build(3, 3), U.pack_states(gi["inst_best_x"], o.m))
    assert path is not None and cost == gi["inst_best_E"]


@pytest.mark.parametrize("rows,cols,dens,inst,closed", [
    (1, 2, 0.0, 0, True),        # m = 1
    (2, 2, 0.0, 1, True),
    (4, 5, 0.2, 2, True),
    (5, 5, 0.0, 3, False),       # open path
    (6, 7, 0.1, 4, True),
])
def test_small_fields_all_replicas(U, oracle_lib, rows, cols, dens, inst, closed):
    g = inputs.grid(rows, cols, dens, seed=5, inst=inst)
    _check_instance(U, oracle_lib, g, 37, 60, 60.0, 0.5, 11, closed=closed)


@pytest.mark.parametrize("side,dens,inst", [(9, 0.15, 7), (11, 0.0, 8), (12, 0.0, 9)])
def test_multi_chunk_rows(U, oracle_lib, side, dens, inst):
    """m > 64: a step spans two or three 64-cell chunks (m = 65..143)."""
    g = inputs.grid(side, side, dens, seed=2, inst=inst)
    assert g.n_free > 64
    _check_instance(U, oracle_lib, g, 9, 12, 200.0, 0.5, 3)


@pytest.mark.parametrize("rows,cols,m", [(8, 9, 63), (8, 9, 64), (8, 9, 65), (12, 12, 127), (12, 12, 128),
                                         (12, 12, 129), (14, 14, 191), (14, 14, 192), (14, 14, 193)])
def test_chunk_class_boundaries(U, oracle_lib, rows, cols, m):
    """Fields whose free-cell count sits on either side of a 64-cell chunk
    boundary (the kernel changes there), against the oracle on two replicas
    started from random tours over a short hot schedule."""
    from paper_2608_25376_amd.inputs import Grid
    rng = np.random.default_rng(m)
    nofly = np.zeros(rows * cols, np.uint8)
    nofly[1 + rng.choice(rows * cols - 1, rows * cols - 1 - m, replace=False)] = 1
    g = Grid(rows, cols, nofly, inst_id=50 + m)
    assert g.n_free == m
    R, S, T0, T1 = 8, 4, 150.0, 50.0
    x0 = np.zeros((R, m * m), np.uint8)
    for r in range(R):
        X = np.zeros((m, m), np.uint8)
        X[np.arange(m), rng.permutation(m)] = 1
        x0[r] = X.reshape(-1)
    seeded = np.ones(R, np.uint8)
    say(f"case: class boundary {rows}x{cols} m={m} R={R} S={S}")
    qs, plan, res = gpu_anneal(U, [g], R, S, T0, T1, 4, init_x=[x0], seeded=seeded, check_E=True)
    gi = split(U, qs, plan, res)[0]
    assert np.array_equal(gi["check_E"], gi["final_E"])
    o = oracle_lib.OracleQubo(rows, cols, nofly=nofly, dense=m <= 80)
    reps = [0, R - 1]
    orc = oracle_lib.anneal(o, S, T0, T1, 4, g.inst_id, reps, init_x=x0[reps], threads=2)
    compare_replicas(gi, orc, reps, f"m={m}")


@pytest.mark.parametrize("side,dens,inst", [(14, 0.0, 12), (16, 0.05, 13)])
def test_fourth_class_fields(U, oracle_lib, side, dens, inst):
    """192 < m <= 256 (up to 65,025 variables): the fourth chunk class's kernel
    against the oracle, which evaluates every coefficient from its definition
    (a stored J would take gigabytes), on two replicas over a short hot
    schedule; every replica's energy agrees with the MFMA recomputation."""
    g = inputs.grid(side, side, dens, seed=2, inst=inst)
    assert 192 < g.n_free <= 256
    m = g.n_free
    R, S, T0, T1 = 6, 5, 150.0, 50.0
    # the compared replicas start from random tours (the oracle's cost is then its
    # O(N) field updates per accepted flip, not the clean-up of random bits)
    rng = np.random.default_rng(inst)
    x0 = np.zeros((R, m * m), np.uint8)
    for r in range(R):
        X = np.zeros((m, m), np.uint8)
        X[np.arange(m), rng.permutation(m)] = 1
        x0[r] = X.reshape(-1)
    seeded = np.array([1, 0, 0, 1, 0, 1], np.uint8)
    say(f"case: fourth class {side}x{side} m={m} R={R} S={S}")
    qs, plan, res = gpu_anneal(U, [g], R, S, T0, T1, 3, init_x=[x0], seeded=seeded, check_E=True)
    assert plan.kernel_name(4) == "k_sweep_chunk<4>"
    gi = split(U, qs, plan, res)[0]
    assert np.array_equal(gi["check_E"], gi["final_E"])
    o = oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly, dense=False)
    reps = [0, R - 1]
    orc = oracle_lib.anneal(o, S, T0, T1, 3, g.inst_id, reps, init_x=x0[reps], threads=2)
    compare_replicas(gi, orc, reps, f"{side}x{side}")


@pytest.mark.parametrize("side,dens,inst,cls", [(18, 0.1, 14, 5), (19, 0.05, 15, 6)])
def test_fifth_and_sixth_class_fields(U, oracle_lib, side, dens, inst, cls):
    """256 < m <= 384 (up to 19x19 fields, 121,801 variables at m = 349): the
    one-wave-per-SIMD chunked kernels against the oracle (coefficients from
    their definition) on two replicas started from random tours over a short
    hot schedule; every replica's energy agrees with the host evaluation of
    its final state (the MFMA check's LDS does not reach these sizes)."""
    g = inputs.grid(side, side, dens, seed=2, inst=inst)
    m = g.n_free
    assert (m + 63) // 64 == cls
    R, S, T0, T1 = 6, 3, 150.0, 50.0
    rng = np.random.default_rng(inst)
    x0 = np.zeros((R, m * m), np.uint8)
    for r in range(R):
        X = np.zeros((m, m), np.uint8)
        X[np.arange(m), rng.permutation(m)] = 1
        x0[r] = X.reshape(-1)
    seeded = np.array([1, 0, 0, 1, 0, 1], np.uint8)
    say(f"case: class {cls} {side}x{side} m={m} R={R} S={S}")
    qs, plan, res = gpu_anneal(U, [g], R, S, T0, T1, 3, init_x=[x0], seeded=seeded)
    assert plan.kernel_name(cls) == f"k_sweep_chunk<{cls}>"
    gi = split(U, qs, plan, res)[0]
    q = qs[0]
    E_host = U.energy_eval(q, res["final_states"].view(np.uint32).reshape(R, q.state_words))
    assert np.array_equal(E_host, gi["final_E"])
    o = oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly, dense=False)
    reps = [0, R - 1]
    orc = oracle_lib.anneal(o, S, T0, T1, 3, g.inst_id, reps, init_x=x0[reps], threads=2)
    compare_replicas(gi, orc, reps, f"{side}x{side}")


@pytest.mark.parametrize("rows,cols,dens,inst,closed", [
    (1, 2, 0.0, 0, True), (3, 3, 0.0, 1, True), (5, 5, 0.0, 3, False), (8, 8, 0.1, 0, True)])
def test_rowmask_variant(U, oracle_lib, rows, cols, dens, inst, closed):
    """The m <= 64 kernel that rebuilds travel rows from step masks (instead
    of keeping them in LDS) follows the same trajectories."""
    g = inputs.grid(rows, cols, dens, seed=5, inst=inst)
    _check_instance(U, oracle_lib, g, 21, 50, 100.0, 0.5, 13, closed=closed, rowmask=True)


def test_ragged_replicas_and_block_shapes(U, oracle_lib):
    """Replica counts that do not fill the last block, several
    replicas-per-block choices and both m <= 64 kernels give identical bytes."""
    g = inputs.grid(5, 6, 0.1, seed=4, inst=21)
    base = None
    for wpb, rm in ((1, False), (3, False), (4, False), (16, False), (4, True), (7, True)):
        gi, _ = _check_instance(U, oracle_lib, g, 19, 40, 80.0, 0.5, 6, wpb=wpb, rowmask=rm)
        if base is None:
            base = gi
        else:
            for f in ("final_x", "best_x", "final_E", "best_E", "accepts", "draws"):
                assert np.array_equal(gi[f], base[f])


@pytest.mark.parametrize("variant,kw,kernel", [
    ("pc", {}, "k_sweep_ylds_pc"),
    ("pc_persistent", {"persistent": True}, "k_sweep_ylds_pc"),
    ("pc_wpb2", {"wpb": 2}, "k_sweep_ylds_pc"),
    ("w1", {"no_producer": True}, "k_sweep_ylds_w1"),
    ("ylds", {"wpb": 8}, "k_sweep_ylds"),
])
def test_m64_kernel_variants(U, oracle_lib, variant, kw, kernel):
    """The three m <= 64 sweeps (with a cut-producing wave per replica, one
    wave per SIMD, several waves per SIMD) against the oracle on every replica,
    with seeded replicas starting at different sweeps (so producers start and
    stop at different points of the run), through the hot, middle and frozen
    parts of a schedule."""
    g = inputs.grid(7, 7, 0.1, seed=12, inst=40)
    o = _oracle_for(oracle_lib, g)
    R, S, T0, T1 = 24, 160, 150.0, 0.5
    rng = np.random.default_rng(3)
    x0 = rng.integers(0, 2, size=(R, o.N), dtype=np.uint8)
    seeded = (np.arange(R) % 3 == 0).astype(np.uint8)
    start = np.where(seeded == 1, rng.integers(0, S + 1, size=R), 0).astype(np.int32)
    start[3] = S            # a replica that never sweeps
    start[6] = S - 1        # and one that sweeps once
    say(f"case: m<=64 variant {variant} 7x7 R={R} S={S}")
    qs, plan, res = gpu_anneal(U, [g], R, S, T0, T1, 5, init_x=[x0], seeded=seeded, start_sweep=start, **kw)
    assert plan.kernel_name(1) == kernel
    gi = split(U, qs, plan, res)[0]
    table = oracle_lib.thresholds(T0, T1, S)
    for r in range(R):
        ix = x0[[r]] if seeded[r] else None
        o_r = oracle_lib.anneal(o, S, T0, T1, 5, g.inst_id, [r], init_x=ix, start_sweep=int(start[r]), table=table)
        compare_replicas(gi, o_r, [r], f"{variant} replica {r}")


def test_single_sweep_and_constant_temperature(U, oracle_lib):
    g = inputs.grid(4, 4, 0.0, seed=1, inst=5)
    _check_instance(U, oracle_lib, g, 8, 1, 30.0, 30.0, 2)
    _check_instance(U, oracle_lib, g, 8, 25, 5.0, 5.0, 2)


def test_seeded_states_and_start_sweep(U, oracle_lib):
    """Replicas started from given states at a later sweep (the warm-start
    interface) follow the oracle's trajectory from the same start."""
    g = inputs.grid(6, 6, 0.1, seed=8, inst=33)
    o = _oracle_for(oracle_lib, g)
    R, S = 12, 50
    rng = np.random.default_rng(1)
    x0 = np.zeros((R, o.N), np.uint8)
    for r in range(R):
        X = np.zeros((o.m, o.m), np.uint8)
        X[np.arange(o.m), rng.permutation(o.m)] = 1
        x0[r] = X.reshape(-1)
    seeded = (np.arange(R) % 2 == 0).astype(np.uint8)
    start = np.where(seeded == 1, 20, 0).astype(np.int32)
    say("case: seeded 6x6 R=12 S=50 start 20")
    qs, plan, res = gpu_anneal(U, [g], R, S, 60.0, 0.5, 7, init_x=[x0], seeded=seeded, start_sweep=start)
    gi = split(U, qs, plan, res)[0]
    # oracle: seeded replicas from x0 at sweep 20, the others from random bits at 0
    table = oracle_lib.thresholds(60.0, 0.5, S)
    sr = [r for r in range(R) if seeded[r]]
    ur = [r for r in range(R) if not seeded[r]]
    o_s = oracle_lib.anneal(o, S, 60.0, 0.5, 7, g.inst_id, sr, init_x=x0[sr], start_sweep=20, table=table)
    o_u = oracle_lib.anneal(o, S, 60.0, 0.5, 7, g.inst_id, ur, table=table)
    compare_replicas(gi, o_s, sr, "seeded")
    compare_replicas(gi, o_u, ur, "random")


def test_batched_equals_single(U, oracle_lib):
    """An instance gives the same bytes alone and inside a batch of uneven
    instances (the random streams are addressed by instance id)."""
    grids = inputs.batch(9, seed=3, side_lo=3, side_hi=10)
    say("case: batch of 9, sides 3..10")
    qs, plan, res = gpu_anneal(U, grids, 10, 30, 100.0, 0.5, 4)
    per = split(U, qs, plan, res)
    for i in (0, 4, 8):
        g = grids[i]
        q1, p1, r1 = gpu_anneal(U, [g], 10, 30, 100.0, 0.5, 4)
        one = split(U, q1, p1, r1)[0]
        for f in ("final_x", "best_x", "final_E", "best_E", "best_sweep", "accepts", "draws"):
            assert np.array_equal(per[i][f], one[f]), (i, f)
    for i, g in enumerate(grids):
        o = _oracle_for(oracle_lib, g)
        orc = oracle_lib.anneal(o, 30, 100.0, 0.5, 4, g.inst_id, [0, 9], threads=8)
        compare_replicas(per[i], orc, [0, 9], f"batch inst {i}")


def test_determinism(U):
    g = inputs.grid(8, 8, 0.1, seed=1, inst=0)
    say("case: determinism 8x8")
    a = gpu_anneal(U, [g], 64, 100, 200.0, 0.5, 1)[2]
    b = gpu_anneal(U, [g], 64, 100, 200.0, 0.5, 1)[2]
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_grid8x8_full_size_all_replicas(U, oracle_lib):
    """The 8x8 workload (no-fly 0.1, 1024 replicas, 2000 sweeps, T 200 ->
    0.5) in its default launch configuration: every replica against the
    oracle, the per-instance best against the oracle's, and the MFMA energy of
    every final state against the incrementally kept one."""
    w = inputs.workload("grid8x8_nofly0.1")
    g = w.grids[0]
    _check_instance(U, oracle_lib, g, w.replicas, w.sweeps, w.T0, w.T1, w.seed, check_E=True, threads=16)


def test_grid12x12_full_size_sampled(U, oracle_lib):
    """The 12x12 configuration (143 free cells, 20449 variables, 4096
    replicas, 4000 sweeps, T 200 -> 0.5) at full size, in the launch the
    benchmark times: sixteen replicas spread over the grid of workgroups are
    recomputed by the oracle one by one, the per-instance reduce over all 4096
    replicas is checked, and every final state's MFMA energy equals the
    incrementally kept one."""
    w = inputs.workload("grid12x12")
    g = w.grids[0]
    assert g.n_free == 143 and w.replicas == 4096 and w.sweeps == 4000
    reps = [0, 1, 2, 3, 255, 256, 1023, 1024, 2047, 2049, 3000, 3071, 3333, 4092, 4094, 4095]
    _check_instance(U, oracle_lib, g, w.replicas, w.sweeps, w.T0, w.T1, w.seed, reps=reps, check_E=True,
                    threads=16)


@pytest.mark.parametrize("rows,cols,dens,inst,R", [(6, 6, 0.1, 60, 24), (8, 8, 0.1, 0, 64), (10, 10, 0.1, 61, 16),
                                                   (12, 12, 0.0, 62, 8)])
def test_largest_penalty(U, oracle_lib, rows, cols, dens, inst, R):
    """The largest penalty qubo_build accepts for these fields (P = 2^20):
    energy changes far beyond 24 bits in the first sweeps (random states
    break hundreds of one-hot constraints) follow the oracle bit for bit, on
    the m <= 64 kernel and on the two- and three-chunk kernels."""
    g = inputs.grid(rows, cols, dens, seed=3, inst=inst)
    P = 1 << 20
    gi, o = _check_instance(U, oracle_lib, g, R, 30, 200.0, 0.5, 17, penalty=P, check_E=True)
    assert o.P == P
    with pytest.raises(U.UavqError):
        U.qubo_build(rows, cols, nofly=g.nofly, penalty=P + 1)


@pytest.mark.parametrize("T", [5.0, 20.0])
def test_permutation_quiet_loop_against_oracle(U, oracle_lib, T):
    """12x12 field (m = 143) at a constant temperature, every replica against
    the oracle.  Half the replicas start from tours: at T = 5 the cut (about
    111) is below 2P - 2 w_max (312), so from the first sweep their quiet
    blocks take the permutation state's min test and its loop; at T = 20 (cut
    about 444) they take the general block test, where only a step's set site
    can fall below the cut.  The other half start random and reach tours
    during the run."""
    g = inputs.grid(12, 12, 0.0, seed=9, inst=12)
    m = g.n_free
    R, S = 16, 200
    rng = np.random.default_rng(12)
    x0 = np.zeros((R, m * m), np.uint8)
    for r in range(R):
        X = np.zeros((m, m), np.uint8)
        X[np.arange(m), rng.permutation(m)] = 1
        x0[r] = X.reshape(-1)
    seeded = (np.arange(R) < R // 2).astype(np.uint8)
    say(f"case: permutation quiet loop 12x12 m={m} R={R} S={S} T={T}")
    qs, plan, res = gpu_anneal(U, [g], R, S, T, T, 8, init_x=[x0], seeded=seeded, check_E=True)
    gi = split(U, qs, plan, res)[0]
    assert np.array_equal(gi["check_E"], gi["final_E"])
    o = _oracle_for(oracle_lib, g)
    reps = list(range(R))
    seeded_reps = [r for r in reps if seeded[r]]
    random_reps = [r for r in reps if not seeded[r]]
    orc_s = oracle_lib.anneal(o, S, T, T, 8, g.inst_id, seeded_reps, init_x=x0[seeded_reps], threads=8)
    compare_replicas(gi, orc_s, seeded_reps, f"12x12 T={T} seeded")
    orc_r = oracle_lib.anneal(o, S, T, T, 8, g.inst_id, random_reps, threads=8)
    compare_replicas(gi, orc_r, random_reps, f"12x12 T={T} random")
    check_reduce(oracle_lib, gi, R, f"12x12 T={T} reduce")


@pytest.mark.parametrize("side", [10, 12])
def test_block_tested_shapes_and_packed_words(U, side):
    """Two and three chunks (m = 99, 143): four, eight and sixteen replicas
    per workgroup give identical bytes in every output, and equal the generic
    walk.  The last chunk's packed draw words sit in LDS only where that
    leaves the resident workgroups per CU unchanged (on the 12x12 field: off
    at four replicas per workgroup, on at eight), so both paths are compared.
    A quarter of the replicas start from tours (the quiet loop of a
    permutation state runs once the cut is low enough), over a whole schedule."""
    g = inputs.grid(side, side, 0.0, seed=9, inst=side)
    m = g.n_free
    R, S = 64, 600
    rng = np.random.default_rng(side)
    x0 = np.zeros((R, m * m), np.uint8)
    for r in range(R):
        X = np.zeros((m, m), np.uint8)
        X[np.arange(m), rng.permutation(m)] = 1
        x0[r] = X.reshape(-1)
    seeded = (np.arange(R) % 4 == 0).astype(np.uint8)
    runs = {}
    for wpb in (4, 8, 16):
        say(f"case: block-tested {side}x{side} m={m} R={R} S={S} wpb={wpb}")
        _, pa, runs[wpb] = gpu_anneal(U, [g], R, S, 200.0, 0.5, 3, wpb=wpb, init_x=[x0], seeded=seeded)
        assert pa.kernel_name((m + 63) // 64) == f"k_sweep_chunk<{(m + 63) // 64}>"
    say(f"case: generic walk {side}x{side} m={m}")
    _, _, rg = gpu_anneal(U, [g], R, S, 200.0, 0.5, 3, init_x=[x0], seeded=seeded, generic_chunk=True)
    for wpb in (4, 16):
        for k in runs[8]:
            assert np.array_equal(runs[wpb][k], runs[8][k]), (wpb, k)
    for k in runs[8]:
        assert np.array_equal(runs[8][k], rg[k]), k


@pytest.mark.parametrize("side,dens,inst", [(9, 0.1, 80), (10, 0.0, 81), (12, 0.0, 82), (13, 0.1, 83), (14, 0.05, 84),
                                           (15, 0.05, 85), (16, 0.0, 86), (18, 0.05, 88), (19, 0.0, 89),
                                           (20, 0.0, 91), (22, 0.0, 92), (24, 0.0, 93)])
def test_block_tested_kernel_equals_generic(U, side, dens, inst):
    """64 < m <= 576: the kernel that first tests blocks of four one-cell steps
    gives the generic chunked walk's bytes in every output, over a whole
    schedule (hot, middle and frozen sweeps), with seeded tours and late
    starts among the replicas."""
    g = inputs.grid(side, side, dens, seed=9, inst=inst)
    m = g.n_free
    assert 64 < m <= 576
    R, S = 48, 400
    rng = np.random.default_rng(inst)
    x0 = np.zeros((R, m * m), np.uint8)
    for r in range(R):
        X = np.zeros((m, m), np.uint8)
        X[np.arange(m), rng.permutation(m)] = 1
        x0[r] = X.reshape(-1)
    seeded = (np.arange(R) % 4 == 1).astype(np.uint8)
    start = np.where(seeded == 1, rng.integers(0, S, size=R), 0).astype(np.int32)
    say(f"case: block-tested vs generic {side}x{side} m={m} R={R} S={S}")
    ce = m <= 256   # the MFMA energy check's reach; beyond it the host evaluates the final states
    qa, pa, ra = gpu_anneal(U, [g], R, S, 200.0, 0.5, 6, init_x=[x0], seeded=seeded, start_sweep=start,
                            check_E=ce)
    cls = (m + 63) // 64
    blk = {7: "k_sweep_chunk_big<7>", 8: "k_sweep_chunk_big<9>", 9: "k_sweep_chunk_big<9>"}
    assert pa.kernel_name(cls) == blk.get(cls, f"k_sweep_chunk<{cls}>")
    qs = [U.qubo_build(g.rows, g.cols, nofly=g.nofly)]
    plan = U.Plan(qs, [g.inst_id], R, S, 200.0, 0.5, 6, generic_chunk=True)
    generic = {4: "k_sweep_factored4", 5: "k_sweep_factored_wide<5>", 6: "k_sweep_factored_wide<6>",
               7: "k_sweep_factored_big<7>", 8: "k_sweep_factored_big<9>", 9: "k_sweep_factored_big<9>"}
    assert plan.kernel_name(cls) == generic.get(cls, f"k_sweep_factored<{cls}>")
    _, _, rb = gpu_anneal(U, [g], R, S, 200.0, 0.5, 6, init_x=[x0], seeded=seeded, start_sweep=start,
                          check_E=ce, generic_chunk=True)
    for k in ra:
        assert np.array_equal(ra[k], rb[k]), k
    if ce:
        assert np.array_equal(ra["check_E"], ra["final_E"])
    else:
        q = qa[0]
        E_host = U.energy_eval(q, ra["final_states"].view(np.uint32).reshape(R, q.state_words))
        assert np.array_equal(E_host, ra["final_E"])


@pytest.mark.parametrize("rows,cols,dens,inst,scale,cls,kernel", [
    (20, 20, 0.0, 90, 10, 7, "k_sweep_chunk_big<7>"),     # m = 399, w_max = 269: 16-bit costs
    (20, 20, 0.0, 91, 5, 7, "k_sweep_chunk_big<7>"),      # m = 399, w_max = 134: class 7 by size alone
    (22, 22, 0.0, 92, 10, 8, "k_sweep_chunk_big<9>"),     # m = 483: class 8 runs in the nine-chunk build
    (24, 24, 0.0, 93, 10, 9, "k_sweep_chunk_big<9>"),     # m = 575, 330,625 variables
    (1, 30, 0.0, 94, 10, 7, "k_sweep_chunk_big<7>"),      # m = 29 but w_max = 290: 16-bit costs
])
def test_sixteen_bit_cost_fields(U, oracle_lib, rows, cols, dens, inst, scale, cls, kernel):
    """Fields past 19x19 and fields whose travel costs exceed a byte: the
    kernels of classes 7..9 (16-bit costs read from global memory) against the
    oracle (coefficients from their definition) on two replicas started from
    random tours over a short hot schedule; every replica's energy equals the
    host evaluation of its final state."""
    g = inputs.grid(rows, cols, dens, seed=2, inst=inst)
    q0 = U.qubo_build(rows, cols, nofly=g.nofly, cost_scale=scale)
    m = q0.m
    R, S, T0, T1 = 6, 3, 150.0, 50.0
    rng = np.random.default_rng(inst)
    x0 = np.zeros((R, m * m), np.uint8)
    for r in range(R):
        X = np.zeros((m, m), np.uint8)
        X[np.arange(m), rng.permutation(m)] = 1
        x0[r] = X.reshape(-1)
    seeded = np.ones(R, np.uint8)
    say(f"case: 16-bit costs {rows}x{cols} scale={scale} m={m} w_max={q0.w_max} R={R} S={S}")
    import torch
    q = q0
    plan = U.Plan([q], [g.inst_id], R, S, T0, T1, 3)
    assert plan.kernel_name(cls) == kernel
    plan.upload()
    packed = U.pack_states(x0, m).reshape(-1)
    out = plan.anneal(init_states=torch.from_numpy(packed.view(np.int32)).cuda(),
                      seeded=torch.from_numpy(seeded).cuda())
    torch.cuda.synchronize()
    res = {k: getattr(out, k).cpu().numpy() for k in out.__dataclass_fields__}
    gi = split(U, [q], plan, res)[0]
    E_host = U.energy_eval(q, res["final_states"].view(np.uint32).reshape(R, q.state_words))
    assert np.array_equal(E_host, gi["final_E"])
    check_reduce(oracle_lib, gi, R, f"{rows}x{cols} reduce")
    o = oracle_lib.OracleQubo(rows, cols, nofly=g.nofly, scale=scale, dense=False)
    assert o.wmax == q.w_max and o.P == q.P
    reps = [0, R - 1] if m > 100 else list(range(R))
    orc = oracle_lib.anneal(o, S, T0, T1, 3, g.inst_id, reps, init_x=x0[reps], threads=2)
    compare_replicas(gi, orc, reps, f"{rows}x{cols}")


@pytest.mark.parametrize("name,kernel", [("grid20x20", "k_sweep_chunk_big<7>"),
                                         ("grid24x24", "k_sweep_chunk_big<9>")])
def test_sixteen_bit_cost_workloads(U, oracle_lib, name, kernel):
    """The 20x20 and 24x24 workloads in the launch the benchmark times (4096
    replicas, 1024 workgroups), over three sweeps of a hot schedule from random
    tours: four replicas spread over the grid against the oracle (coefficients
    from their definition), the per-instance reduce over all 4096 replicas,
    and the host energy of every final state against the kept one."""
    import torch
    w = inputs.workload(name)
    g = w.grids[0]
    q = U.qubo_build(g.rows, g.cols, nofly=g.nofly)
    m, R, S, T0, T1 = q.m, w.replicas, 3, 150.0, 50.0
    rng = np.random.default_rng(m)
    perms = np.stack([rng.permutation(m) for _ in range(R)])      # step t visits cell perms[r, t]
    W = q.row_words
    packed = np.zeros((R, m, W), np.uint32)                       # one set bit per step row
    packed[np.arange(R)[:, None], np.arange(m)[None, :], perms // 32] = np.left_shift(1, perms % 32).astype(np.uint32)
    reps = [0, 1025, 2049, R - 1]
    x0 = np.zeros((len(reps), m, m), np.uint8)                    # the sampled replicas, unpacked
    x0[np.arange(len(reps))[:, None], np.arange(m)[None, :], perms[reps]] = 1
    x0 = x0.reshape(len(reps), m * m)
    assert np.array_equal(U.pack_states(x0, m), packed[reps].reshape(len(reps), -1))
    say(f"case: {name} m={m} w_max={q.w_max} R={R} S={S}")
    plan = U.Plan([q], [g.inst_id], R, S, T0, T1, w.seed)
    assert plan.kernel_name((m + 63) // 64) == kernel
    plan.upload()
    packed = packed.reshape(-1)
    out = plan.anneal(init_states=torch.from_numpy(packed.view(np.int32)).cuda(),
                      seeded=torch.ones(R, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    res = {k: getattr(out, k).cpu().numpy() for k in out.__dataclass_fields__}
    gi = split(U, [q], plan, res)[0]
    E_host = U.energy_eval(q, res["final_states"].view(np.uint32).reshape(R, q.state_words))
    assert np.array_equal(E_host, gi["final_E"])
    check_reduce(oracle_lib, gi, R, f"{name} reduce")
    o = oracle_lib.OracleQubo(g.rows, g.cols, nofly=g.nofly, dense=False)
    orc = oracle_lib.anneal(o, S, T0, T1, w.seed, g.inst_id, reps, init_x=x0, threads=4)
    compare_replicas(gi, orc, reps, name)
