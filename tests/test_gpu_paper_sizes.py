"""The paper's field sizes (Sec. IV-D) with the annealer's defaults for them
(1024 replicas x 1000 sweeps, T 100 -> 0.5): the returned state is a tour
(feasible, a permutation of the free cells) whose cost is the returned energy,
for the open path of eq. (1a) and for the closed tour; it is never below the
exact optimum (Held-Karp in the oracle, stored in tests/golden by
oracle/paper_optima.py) and, on 3x3, equals it.  Single-flip
Metropolis on the one-hot encoding does not always reach the optimum on the
larger fields; each case prints its gap."""
import json
import os

import pytest

from tests.gpu_util import say

OPTIMA = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "optima_small_fields.json")))

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def PS():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_25376_amd import paper_sizes, uavq
    uavq.lib()
    return paper_sizes


@pytest.mark.parametrize("closed", [False, True])
@pytest.mark.parametrize("rows,cols", [(3, 3), (3, 4), (4, 4), (4, 5), (5, 5)])
def test_tours_on_paper_fields(PS, oracle_lib, rows, cols, closed):
    say(f"case: paper field {rows}x{cols} closed={closed}")
    res = PS.solve(rows, cols, closed, replicas=1024, sweeps=1000)
    o = oracle_lib.OracleQubo(rows, cols, closed=closed, dense=False)
    opt = OPTIMA["paper_fields"][f"{rows}x{cols}_{'closed' if closed else 'open'}"]["optimum"]
    if o.m <= 15:
        assert o.held_karp() == opt
    say(f"  {rows}x{cols} {'closed' if closed else 'open'}: best {res['best_E']} optimum {opt} "
        f"gap {100.0 * (res['best_E'] - opt) / opt:.1f}% anneal {res['anneal_ms']:.2f} ms")
    assert res["feasible"]
    path = res["path"]
    assert path[0] == 0 and (path[-1] == 0) == closed
    assert len(path) == o.m + (2 if closed else 1)
    cells = path[1:-1] if closed else path[1:]
    assert sorted(cells) == sorted(int(f) for f in o.F)
    assert o.path_cost(path) == res["best_E"]
    # never below the optimum; the gap grows with the field (about 1.6x on 5x5, see the module docstring)
    assert opt <= res["best_E"] <= 2 * opt
    if (rows, cols) == (3, 3):
        assert res["best_E"] == opt
