"""Pins for the warm-start part of the oracle: the network gradient against
central finite differences (float64, no rounding), bfloat16 rounding against
hand-worked values, softmax/cross-entropy special cases, Adam against its
closed form after one step, features against hand-computed values, and the
seed sampler's outputs (always permutations; uniform when the marginals are)."""
import math

import numpy as np
import pytest

from paper_2608_25376_amd import inputs


@pytest.fixture(scope="module")
def M(oracle_lib):
    from oracle import mlp
    return mlp


def _rand_problem(M, rows=24, seed=0):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.2, M.N_PARAMS)
    X = rng.normal(0, 1, (rows, 16))
    ms = rng.integers(3, 128, rows)
    labels = np.array([rng.integers(0, m) for m in ms])
    return theta, X, ms, labels


def test_bf16_rounding_hand_values(M):
    # 1 + 2^-8 lies halfway between bf16 neighbours 1 and 1 + 2^-7: ties go to even (1.0)
    assert M.bf16(1.0) == 1.0
    assert M.bf16(1 + 2 ** -8) == 1.0
    assert M.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6      # halfway to odd neighbour -> rounds up to even
    assert M.bf16(1 + 2 ** -7) == 1 + 2 ** -7           # exactly representable
    assert M.bf16(-2.5) == -2.5
    assert abs(M.bf16(math.pi) - math.pi) < 2 ** -7 * 4


def test_gradient_matches_finite_differences(M):
    theta, X, ms, labels = _rand_problem(M)
    loss, g = M.loss_grad(theta, X, ms, labels, bf16_ops=False)
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(M.N_PARAMS, 60, replace=False),
                          [0, 16 * 128 + 5, 16 * 128 + 128 + 77, M.N_PARAMS - 1]])
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        lp = M.loss_grad(tp, X, ms, labels, bf16_ops=False)[0] / len(X)
        lm = M.loss_grad(tm, X, ms, labels, bf16_ops=False)[0] / len(X)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_softmax_cross_entropy_special_cases(M):
    theta = np.zeros(M.N_PARAMS)          # all logits equal -> uniform over the first m steps
    X = np.ones((5, 16))
    ms = np.array([1, 2, 7, 99, 128])
    labels = np.array([0, 1, 3, 50, 127])
    _, _, _, P = M.forward(theta, X, ms)
    for r, m in enumerate(ms):
        assert np.allclose(P[r, :m], 1.0 / m) and (P[r, m:] == 0).all()
    loss, _ = M.loss_grad(theta, X, ms, labels)
    assert abs(loss - sum(math.log(m) for m in ms)) < 1e-9


def test_adam_first_step_closed_form(M):
    rng = np.random.default_rng(1)
    th, g = rng.normal(size=50), rng.normal(size=50)
    new, m1, m2 = M.adam(th, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    # after one step the bias-corrected moments are g and g^2: update = lr * sign(g) (up to eps)
    assert np.allclose(new, th - 1e-3 * g / (np.abs(g) + 1e-8))


def test_features_hand_values(M):
    # 3x3 field, start cell 0, cell 4 (centre) no-fly: free cells 1,2,3,5,6,7,8
    nf = np.zeros(9, np.uint8)
    nf[4] = 1
    X = M.features(3, 3, 0, nf)
    assert X.shape == (7, 16)
    f = X[6]                                 # cell 8 = (2, 2)
    assert np.allclose(f[:5], [1.0, 1.0, 1.0, 1.0, 1.0])
    assert abs(f[5] - 1 / 8) < 1e-7          # ring 1 of (2,2): (1,1) no-fly, (1,2), (2,1) free -> 1 no-fly
    assert abs(f[6] - 1 / 24) < 1e-7
    assert abs(f[7] - 2 / 3) < 1e-7          # ring 1: 3 in-grid cells, 2 free
    assert abs(f[8] - 5 / 5) < 1e-7          # ring 2: (0,0),(0,1),(0,2),(1,0),(2,0) all free
    assert (f[9:15] == 0).all()
    assert abs(f[15] - 7 / 99) < 1e-7
    f = X[0]                                 # cell 1 = (0, 1)
    assert np.allclose(f[:5], [0.0, 0.5, 0.0, 0.5, 0.5 / math.sqrt(2)], atol=1e-7)


def test_sampler_outputs_permutations_and_is_uniform_on_flat_marginals(M):
    m = 3
    q = np.ones((m, 128), np.uint16)
    counts = {}
    for r in range(6000):
        x = M.sample_seed(q, m, 7, 0, r).reshape(m, m)
        assert (x.sum(0) == 1).all() and (x.sum(1) == 1).all()
        key = tuple(np.argmax(x, 1))
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 6
    freq = np.array(list(counts.values())) / 6000
    assert np.abs(freq - 1 / 6).max() < 0.02


def test_sampler_follows_peaked_marginals(M):
    m = 12
    rng = np.random.default_rng(2)
    perm = rng.permutation(m)                 # step t -> cell perm[t]
    q = np.ones((m, 128), np.uint16)
    q[perm, np.arange(m)] = 65535
    hits = 0
    for r in range(200):
        x = M.sample_seed(q, m, 3, 9, r).reshape(m, m)
        assert (x.sum(0) == 1).all() and (x.sum(1) == 1).all()
        hits += (np.argmax(x, 1) == perm).all()
    assert hits >= 190


def test_quantize(M):
    P = np.array([[0.0, 1e-9, 0.5, 1.0] + [0.25] * 124])
    q = M.quantize(P, np.array([4]))
    assert q[0, :4].tolist() == [1, 1, 32768, 65535]      # never 0 inside the mask, never wraps
    assert (q[0, 4:] == 0).all()
