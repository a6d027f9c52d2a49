"""Pins of the replica-exchange (parallel tempering) oracle, on the CPU.

The exchange rule is the Metropolis rule on the product of the Boltzmann
weights of two neighbouring temperatures.  Pinned here by what that rule and
the ladder fix independently of the oracle's code: the ladder's end points and
constant ratio, the table entries in 40-digit arithmetic, the stationary
distribution of the exchange step alone over permutations of fixed states
(computed by enumeration), the conservation of each chain's energies, the
reductions to the plain annealer, and the Boltzmann distribution of every
slot of a long tempering run on a 9-variable field."""
import itertools
from decimal import Decimal, getcontext

import numpy as np
import pytest


def _all_states(N):
    return ((np.arange(1 << N)[:, None] >> np.arange(N)) & 1).astype(np.uint8)


def test_ladder_geometric(oracle_lib):
    T, DX, xthr = oracle_lib.pt_ladder(200.0, 2.0, 8)
    assert T[0] == 200.0 and abs(T[-1] - 2.0) < 1e-12
    ratio = T[1:] / T[:-1]
    assert np.allclose(ratio, (2.0 / 200.0) ** (1 / 7), rtol=1e-13, atol=0)
    assert DX.shape == (7,) and xthr.shape[0] == 7 and xthr.shape[1] == DX.max() + 1
    # colder pairs have a larger 1/T gap, so shorter tables
    assert (np.diff(DX) < 0).all()
    T1, DX1, _ = oracle_lib.pt_ladder(50.0, 1.0, 1)
    assert list(T1) == [50.0] and DX1.size == 0
    with pytest.raises(ValueError):
        oracle_lib.pt_ladder(5.0, 5.0, 3)          # no 1/T gap: no finite table


def test_exchange_table_exact(oracle_lib):
    """xthr[k][a] = min(2^32-1, floor(2^32 exp(-a (1/T_{k+1} - 1/T_k)))), checked
    in 40-digit decimal arithmetic away from integer boundaries; DX_k is the
    first zero entry."""
    getcontext().prec = 40
    T, DX, xthr = oracle_lib.pt_ladder(120.0, 3.0, 6)
    rng = np.random.default_rng(0)
    checked = 0
    for k in range(5):
        db = Decimal(repr(float(1.0 / T[k + 1] - 1.0 / T[k])))
        for a in sorted(set(rng.integers(1, DX[k] + 1, 40).tolist()) | {1, int(DX[k]) - 1, int(DX[k])}):
            exact = (Decimal(2) ** 32) * (-(Decimal(a) * db)).exp()
            frac = exact - int(exact)
            if Decimal("1e-9") < frac < 1 - Decimal("1e-9"):
                assert int(xthr[k, a]) == min(int(exact), 2 ** 32 - 1), (k, a)
                checked += 1
        assert xthr[k, DX[k]] == 0 and xthr[k, DX[k] - 1] > 0
        assert (xthr[k, DX[k]:] == 0).all()
        assert (np.diff(xthr[k, 1:DX[k] + 1].astype(np.int64)) <= 0).all()
    assert checked > 100


def test_exchange_stationary_over_permutations(oracle_lib):
    """The exchange step alone (no sweeps) moves three fixed states over three
    temperatures.  Each round satisfies detailed balance for
    pi(sigma) ~ prod_k exp(-E_sigma(k) / T_k), so after many rounds the
    assignment frequencies over many independent chains follow pi (computed
    by enumerating the 6 permutations).  A flipped sign, a wrong 1/T gap or a
    wrong pair index each give a different distribution."""
    K, R = 3, 200000
    Evals = np.array([0, 30, 75], np.int64)
    T, DX, xthr = oracle_lib.pt_ladder(90.0, 15.0, K)
    x = np.zeros((K, R, 1), np.uint8)
    E = np.zeros((K, R), np.int64)
    for k in range(K):
        x[k, :, 0] = k                       # state label k carries energy Evals[k]
        E[k] = Evals[k]
    for rnd in range(60):
        oracle_lib.pt_exchange(x, E, rnd, 7, 3, DX, xthr)
    # energies travel with their states
    assert (E == Evals[x[:, :, 0]]).all()
    perms = list(itertools.permutations(range(K)))
    w = np.array([np.exp(-sum(Evals[p[k]] / T[k] for k in range(K))) for p in perms])
    pi = w / w.sum()
    code = {p: i for i, p in enumerate(perms)}
    idx = np.array([code[tuple(x[:, r, 0])] for r in range(R)])
    emp = np.bincount(idx, minlength=len(perms)) / R
    se = np.sqrt(pi * (1 - pi) / R)
    assert (np.abs(emp - pi) < 5 * se + 1e-4).all(), (emp, pi)


def test_exchange_conserves_chain_energies(oracle_lib):
    rng = np.random.default_rng(1)
    K, R, N = 5, 300, 12
    T, DX, xthr = oracle_lib.pt_ladder(100.0, 2.0, K)
    x = rng.integers(0, 2, (K, R, N)).astype(np.uint8)
    E = rng.integers(-50, 400, (K, R)).astype(np.int64)
    tag = {(k, r): (E[k, r], x[k, r].tobytes()) for k in range(K) for r in range(R)}
    E0 = np.sort(E, axis=0).copy()
    sw = np.zeros(K - 1, np.uint64)
    for rnd in range(9):
        oracle_lib.pt_exchange(x, E, rnd, 11, 0, DX, xthr, sw)
    assert (np.sort(E, axis=0) == E0).all()
    # every (energy, state) pair is one of the chain's original pairs
    for r in range(R):
        orig = {tag[(k, r)] for k in range(K)}
        assert {(E[k, r], x[k, r].tobytes()) for k in range(K)} == orig
    assert sw.sum() > 0
    # pairs (k, k+1) with k = round mod 2: round 0 never touches pair 1
    x2, E2 = x.copy(), E.copy()
    sw2 = np.zeros(K - 1, np.uint64)
    oracle_lib.pt_exchange(x2, E2, 0, 12, 0, DX, xthr, sw2)
    assert sw2[1] == 0 and sw2[3] == 0


def test_pt_reduces_to_plain_anneal(oracle_lib):
    """K = 1, or no exchange round (interval >= sweeps): every slot is the plain
    annealer at its constant temperature with instance id inst + k."""
    q = oracle_lib.OracleQubo(3, 3)
    R, S = 12, 40
    pt = oracle_lib.pt_anneal(q, 1, R, S, 30.0, 1.0, 5, 2, interval=7)
    ref = oracle_lib.anneal(q, S, 30.0, 30.0, 5, 2, list(range(R)))
    assert pt["rounds"] == 0
    for f in ("final_x", "final_E", "best_E", "best_sweep", "best_x", "accepts", "draws"):
        assert np.array_equal(pt[f][0], ref[f]), f
    K = 3
    pt = oracle_lib.pt_anneal(q, K, R, S, 30.0, 1.0, 5, 2, interval=S)
    for k in range(K):
        ref = oracle_lib.anneal(q, S, pt["T"][k], pt["T"][k], 5, 2 + k, list(range(R)))
        for f in ("final_x", "final_E", "best_E", "best_sweep", "accepts"):
            assert np.array_equal(pt[f][k], ref[f]), (k, f)


def test_pt_states_carry_their_energies(oracle_lib):
    q = oracle_lib.OracleQubo(3, 4, closed=False)
    K, R, S = 4, 16, 60
    pt = oracle_lib.pt_anneal(q, K, R, S, 80.0, 2.0, 3, 1, interval=2)
    assert pt["rounds"] == S // 2 - 1 and pt["swaps"].sum() > 0
    for k in range(K):
        for r in range(R):
            assert q.energy(pt["final_x"][k, r]) == pt["final_E"][k, r]
            assert q.energy(pt["best_x"][k, r]) == pt["best_E"][k, r]
            assert 0 <= pt["best_sweep"][k, r] < S


@pytest.mark.slow
def test_pt_slots_sample_boltzmann(oracle_lib):
    """A long tempering run on the 2x2 field (9 variables): every slot's final
    states over independent chains follow exp(-E/T_k)/Z (enumeration); the
    hottest and coldest slots differ, so states must travel with their
    temperatures' statistics, not their origin's."""
    q = oracle_lib.OracleQubo(2, 2)
    K, R, S = 4, 6000, 40
    pt = oracle_lib.pt_anneal(q, K, R, S, 80.0, 8.0, 21, 0, interval=1, threads=8)
    Eall = np.array([q.energy(x) for x in _all_states(q.N)], np.float64)
    for k in range(K):
        p = np.exp(-(Eall - Eall.min()) / pt["T"][k])
        p /= p.sum()
        mean, var = (p * Eall).sum(), (p * Eall ** 2).sum() - ((p * Eall).sum()) ** 2
        emp = pt["final_E"][k].astype(np.float64)
        assert abs(emp.mean() - mean) < 5 * np.sqrt(var / R) + 1e-9, (k, emp.mean(), mean)


@pytest.mark.parametrize("K,interval,closed", [(4, 1, True), (5, 3, False), (1, 2, True)])
def test_chain_loop_equals_composition(oracle_lib, K, interval, closed):
    """The one-loop-per-chain tempering (fields kept across rounds) equals the
    composition of plain anneals and exchange rounds, for all chains and for
    a subset of chain ids."""
    q = oracle_lib.OracleQubo(3, 4, closed=closed)
    R, S = 9, 25
    ref = oracle_lib.pt_anneal(q, K, R, S, 60.0, 2.0, 4, 6, interval=interval)
    for chains in (list(range(R)), [7, 2]):
        got = oracle_lib.pt_anneal_chains(q, K, chains, S, 60.0, 2.0, 4, 6, interval=interval)
        for f in ("final_x", "final_E", "best_E", "best_sweep", "best_x", "accepts", "draws"):
            assert np.array_equal(got[f], np.swapaxes(ref[f], 0, 1)[chains]), (f, chains)
        if K > 1 and len(chains) == R:
            assert np.array_equal(got["swaps"].sum(0), ref["swaps"])
