"""The allocation-free energy evaluation (uavq_energy_eval_dev_noalloc,
staging in the library's static device buffer) against the workspace entry
point uavq_energy_eval_dev, through the C ABI: bit-exact energies on two
calls in a row, the second on a smaller field with fewer states (the buffer
keeps the first call's bytes beyond what the second writes), and the size
limit refused with ETOOBIG."""
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


def _states(m, n, rng):
    xs = []
    for i in range(n):
        if i % 3 == 0:
            X = np.zeros((m, m), np.uint8)
            X[np.arange(m), rng.permutation(m)] = 1
            xs.append(X.reshape(-1))
        else:
            xs.append((rng.random(m * m) < 0.05 + 0.6 * (i % 7) / 7).astype(np.uint8))
    return np.array(xs)


def test_noalloc_energy_equals_workspace_entry_point(U):
    import torch
    rng = np.random.default_rng(11)
    # a large field first, then a smaller one with fewer states
    for rows, cols, dens, n in ((16, 16, 0.0, 300), (12, 12, 0.0, 129), (5, 6, 0.2, 7)):
        g = inputs.grid(rows, cols, dens, seed=3, inst=rows)
        q = U.qubo_build(rows, cols, nofly=g.nofly)
        say(f"case: noalloc energy {rows}x{cols} m={q.m} n={n}")
        xs = _states(q.m, n, rng)
        d = torch.from_numpy(U.pack_states(xs, q.m).view(np.int32).reshape(-1)).cuda()
        ref = U.energy_eval_dev(q, d).cpu().numpy()
        out = torch.full((n,), -1, dtype=torch.int64, device="cuda")
        U.energy_eval_dev_noalloc(q, d, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref)
        assert np.array_equal(got, U.energy_eval(q, U.pack_states(xs, q.m)))


def test_noalloc_energy_refuses_staging_beyond_the_buffer(U):
    import torch
    q = U.qubo_build(30, 30, cost_scale=1)      # m = 899: 808 KB of staging
    d = torch.zeros(q.state_words, dtype=torch.int32, device="cuda")
    E = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(U.UavqError) as e:
        U.energy_eval_dev_noalloc(q, d, E)
    assert e.value.code == U.ETOOBIG
    # and a valid call right after still works
    q2 = U.qubo_build(4, 4)
    X = np.zeros((q2.m, q2.m), np.uint8)
    X[np.arange(q2.m), np.arange(q2.m)] = 1
    d2 = torch.from_numpy(U.pack_states(X.reshape(1, -1), q2.m).view(np.int32).reshape(-1)).cuda()
    E2 = torch.zeros(1, dtype=torch.int64, device="cuda")
    U.energy_eval_dev_noalloc(q2, d2, E2)
    torch.cuda.synchronize()
    assert int(E2.cpu()[0]) == int(U.energy_eval(q2, U.pack_states(X.reshape(1, -1), q2.m))[0])
