"""The split-K cache of paper_1007_3753_amd.tuning: keys, lookup, install and
record, with a stand-in plan (no GPU)."""
import json

from paper_1007_3753_amd import tuning


class _FakePlan:
    structure, problem, m, n_dict, max_batch, precision = "cab", "p1", 1200, 700, 512, "bf16_refine"

    def __init__(self):
        self.installed = None

    def set_ksplit(self, table):
        self.installed = list(table)

    def tune_ksplit(self, iters):
        return [0, 3, 2, 1, 1, 1, 1, 1]


def test_key_lookup_apply_and_tune(tmp_path, monkeypatch):
    monkeypatch.setattr(tuning, "_arch", lambda: "gfx950")
    path = str(tmp_path / "cache.json")
    pl = _FakePlan()
    assert tuning.key(pl) == "gfx950|cab|p1|m1200|n700|batch512|bf16_refine"
    assert tuning.lookup(pl, path) is None and tuning.apply(pl, path) is None and pl.installed is None
    table = tuning.tune(pl, iters=64, path=path)
    assert table == [0, 3, 2, 1, 1, 1, 1, 1]
    rec = json.load(open(path))
    assert rec[tuning.key(pl)] == {"ksplit": table, "iters": 64}
    other = _FakePlan()
    other.m = 4800
    assert tuning.lookup(other, path) is None           # another shape, another key
    assert tuning.apply(pl, path) == table and pl.installed == table


def test_committed_cache_is_well_formed():
    rec = json.load(open(tuning.CACHE))
    assert rec, "the package ships tuned tables"
    for key, entry in rec.items():
        arch, structure, problem, m, n, batch, prec = key.split("|")
        assert arch.startswith("gfx") and m.startswith("m") and n.startswith("n") and batch.startswith("batch")
        t = entry["ksplit"]
        # entry 1 is tuned only for operators too large for the tail kernel
        assert len(t) == 8 and all(0 <= v <= 4 for v in t)
