"""Host-side bookkeeping of the warm-start protocol: the schedule start of a
seeded replica and the medians over annealing seeds (no GPU work)."""
import json

import numpy as np

from paper_2608_25376_amd import warmstart


def test_first_sweep_below_matches_geometric_schedule():
    T0, T1, S = 200.0, 0.5, 400
    for Tw in (100.0, 25.0, 0.5, 1e-3, 250.0):
        s0 = warmstart.first_sweep_below(T0, T1, S, Tw)
        T = T0 * (T1 / T0) ** (np.arange(S) / (S - 1))
        below = np.nonzero(T <= Tw)[0]
        assert s0 == (0 if Tw >= T0 else (below[0] if len(below) else S - 1))


def _report(ttt, frac):
    return {"modes": {"plain": {"ttt_ms": ttt, "solved": 3, "fraction_at_target": frac,
                                "mean_gap": {k: 0.01 for k in frac}},
                      "batched": {"ttt_ms": None, "ladder_ms_to_all_first_hits": ttt / 2, "solved": 2,
                                  "fraction_at_target": frac, "mean_gap": {k: 0.02 for k in frac}}}}


def test_seed_medians_and_merge(tmp_path):
    per = {"1": warmstart.per_seed_fields(_report(10.0, {"50": 0.1, "100": 0.4})),
           "2": warmstart.per_seed_fields(_report(30.0, {"50": 0.3, "100": 0.2})),
           "3": warmstart.per_seed_fields(_report(20.0, {"50": 0.2, "100": 0.3}))}
    med = warmstart.seed_medians(per)
    assert med["plain"]["ttt_ms"] == 20.0
    assert med["plain"]["fraction_at_target"] == {"50": 0.2, "100": 0.3}
    assert "ttt_ms" not in med["batched"]            # None on some seed: no median
    assert med["batched"]["ladder_ms_to_all_first_hits"] == 10.0
    # two runs (seeds 1,2 and 3) merged give the same medians
    a = dict(_report(10.0, {}), seeds=[1, 2], per_seed={"1": per["1"], "2": per["2"]})
    b = dict(_report(20.0, {}), seeds=[3], per_seed={"3": per["3"]})
    pa, pb = tmp_path / "a.json", tmp_path / "b.json"
    pa.write_text(json.dumps(a))
    pb.write_text(json.dumps(b))
    m = warmstart.merge_reports([str(pb), str(pa)])
    assert m["seeds"] == [1, 2, 3]
    assert m["median"] == med
