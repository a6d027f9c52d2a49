"""Workload configs (one JSON file per configuration under
paper_2608_25376_amd/configs/): every file loads, the fields have the sizes
their notes state, and a config written elsewhere loads the same way."""
import json
import os

from paper_2608_25376_amd import inputs

SIZES = {   # name: (instances, free cells of the first field, replicas, sweeps, T0, T1)
    "grid3x3": (1, 8, 64, 1000, 100.0, 0.5),
    "grid8x8_nofly0.1": (1, 54, 1024, 2000, 200.0, 0.5),
    "grid12x12": (1, 143, 4096, 4000, 200.0, 0.5),
    "grid16x16": (1, 255, 4096, 1000, 200.0, 0.5),
    "grid19x19": (1, 360, 4096, 1000, 200.0, 0.5),
    "grid20x20": (1, 399, 4096, 1000, 200.0, 0.5),
    "grid24x24": (1, 575, 4096, 1000, 200.0, 0.5),
    "batch256": (256, None, 256, 2000, 200.0, 0.5),
}


def test_every_config_loads():
    assert sorted(inputs.workload_names()) == sorted(SIZES)
    for name, (n, m, R, S, T0, T1) in SIZES.items():
        w = inputs.workload(name)
        assert w.name == name and len(w.grids) == n
        assert (w.replicas, w.sweeps, w.T0, w.T1) == (R, S, T0, T1)
        if m is not None:
            assert w.grids[0].n_free == m
    b = inputs.workload("batch256").grids
    assert [g.inst_id for g in b] == list(range(256))
    assert all(4 <= g.rows <= 10 and g.rows == g.cols for g in b)


def test_config_file_roundtrip(tmp_path):
    spec = {"name": "mine", "fields": {"kind": "grid", "rows": 5, "cols": 7, "density": 0.1, "seed": 3, "inst": 9},
            "replicas": 32, "sweeps": 50, "T0": 40.0, "T1": 1.0, "seed": 2}
    p = tmp_path / "mine.json"
    p.write_text(json.dumps(spec))
    w = inputs.load_config(str(p))
    g = inputs.grid(5, 7, 0.1, 3, 9)
    assert w.grids[0].inst_id == 9 and (w.grids[0].nofly == g.nofly).all()
    assert (w.replicas, w.sweeps, w.T0, w.T1, w.seed) == (32, 50, 40.0, 1.0, 2)


def test_warm_start_config_matches_the_driver_defaults():
    c = json.load(open(os.path.join(inputs.CONFIG_DIR, "warmstart_grid10x10.json")))
    tr, ho = inputs.fields_from_spec(c["train"]), inputs.fields_from_spec(c["heldout"])
    assert len(tr) == 2000 and len(ho) == 200
    assert tr[0].inst_id == 10000 and ho[0].inst_id == 20000
    assert all(g.rows == 10 == g.cols for g in tr[:50] + ho[:50])
