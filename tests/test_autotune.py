"""Tile autotuner (paper_2110_00967_amd/autotune.py): the cache logic, on the
CPU with a fake timer.  The GPU side -- a tuned tile gives the default tile's
results bit for bit -- is in tests/test_gpu_autotune.py."""
import json
import os

import pytest

from paper_2110_00967_amd import autotune as AT


def fake_measure(table, calls=None):
    def m(t):
        if calls is not None:
            calls.append(t)
        return table[t]
    return m


def test_record_and_lookup_persist_per_arch(tmp_path):
    path = str(tmp_path / "tiles.json")
    t = AT.TileTuner(path=path, arch="gfx950", defaults=None)
    assert t.lookup("batch/f32/AB/pop8192MiB/n9-64") is None
    best = AT.tune(AT.BATCH_TILES, fake_measure({(64, 4): 1000.7, (128, 2): 998.2, (256, 1): 1003.6}), t,
                   "batch/f32/AB/pop8192MiB/n9-64")
    assert best == (128, 2)
    # a new tuner on the same file sees it; another architecture does not
    again = AT.TileTuner(path=path, arch="gfx950", defaults=None)
    assert again.lookup("batch/f32/AB/pop8192MiB/n9-64") == (128, 2)
    assert again.timings("batch/f32/AB/pop8192MiB/n9-64") == {"64x4": 1000.7, "128x2": 998.2, "256x1": 1003.6}
    other = AT.TileTuner(path=path, arch="gfx942", defaults=None)
    assert other.lookup("batch/f32/AB/pop8192MiB/n9-64") is None
    # recording for the other architecture keeps the first one's entry
    AT.tune(AT.BATCH_TILES, fake_measure({(64, 4): 1.0, (128, 2): 2.0, (256, 1): 3.0}), other, "k")
    assert AT.TileTuner(path=path, arch="gfx950", defaults=None).lookup("batch/f32/AB/pop8192MiB/n9-64") == (128, 2)
    assert AT.TileTuner(path=path, arch="gfx942", defaults=None).lookup("k") == (64, 4)


def test_tune_times_each_candidate_per_round_and_keeps_the_best(tmp_path):
    t = AT.TileTuner(path=str(tmp_path / "c.json"), arch="a")
    seq = {(64, 4): [5.0, 3.0], (128, 2): [4.0, 4.5]}
    calls = []

    def m(tile):
        calls.append(tile)
        return seq[tile][sum(1 for c in calls if c == tile) - 1]

    assert AT.tune([(64, 4), (128, 2)], m, t, "k", rounds=2) == (64, 4)  # 3.0 < 4.0
    assert calls == [(64, 4), (128, 2), (64, 4), (128, 2)]  # interleaved rounds
    assert t.timings("k") == {"64x4": 3.0, "128x2": 4.0}


def test_ties_go_to_the_first_candidate(tmp_path):
    t = AT.TileTuner(path=str(tmp_path / "c.json"), arch="a")
    assert AT.tune([(128, 2), (64, 4)], fake_measure({(64, 4): 7.0, (128, 2): 7.0}), t, "k", rounds=1) == (128, 2)


def test_corrupt_or_foreign_cache_starts_empty(tmp_path):
    path = tmp_path / "tiles.json"
    path.write_text("{not json")
    t = AT.TileTuner(path=str(path), arch="gfx950", defaults=None)
    assert t.lookup("x") is None
    path.write_text(json.dumps({"version": 99, "arch": {"gfx950": {"x": {"tile": [64, 4]}}}}))
    assert AT.TileTuner(path=str(path), arch="gfx950", defaults=None).lookup("x") is None
    # and it is rewritten in the current format on the next record
    AT.tune([(64, 4)], fake_measure({(64, 4): 1.0}), t, "x", rounds=1)
    d = json.loads(path.read_text())
    assert d["version"] == AT.TileTuner.VERSION and d["arch"]["gfx950"]["x"]["tile"] == [64, 4]


def test_unwritable_cache_keeps_the_choice_in_memory(tmp_path):
    # the cache directory cannot be created (a plain file is in the way)
    blocker = tmp_path / "file"
    blocker.write_text("x")
    t = AT.TileTuner(path=str(blocker / "sub" / "tiles.json"), arch="a")
    assert AT.tune([(64, 4), (128, 2)], fake_measure({(64, 4): 2.0, (128, 2): 1.0}), t, "k") == (128, 2)
    assert t.lookup("k") == (128, 2)


def test_class_keys():
    # population bytes rounded up to a power of two MiB; two buffers or one
    assert AT.size_bucket(2 ** 20) == "pop1MiB"
    assert AT.size_bucket(2 ** 20 + 1) == "pop2MiB"
    assert AT.size_bucket(146e6) == "pop256MiB"
    assert AT.population_bytes(2000, 1000, "f32") == 2 * 9 * 2048 * 1000 * 4
    assert AT.population_bytes(2000, 1000, "f32", "AA") == 9 * 2048 * 1000 * 4
    assert AT.lattice_key("f32", "AB", 2000, 1000) == "lattice/f32/AB/pop256MiB/wide"
    assert AT.lattice_key(2, "AB", 400, 2000) == "lattice/f16dev/AB/pop32MiB/narrow"
    assert AT.lattice_key("f64", "AB", 8192, 8192) == "lattice/f64/AB/pop16384MiB/wide"

    class L:
        def __init__(self, nx, ny):
            self.nx, self.ny = nx, ny

    class B:
        lattices = [L(1000, 500), L(1500, 750), L(2000, 1000)] * 21 + [L(1000, 500)]

    assert AT.batch_key("f32", "AB", B) == "batch/f32/AB/pop8192MiB/n9-64"
    assert AT.parse_tile(AT.tile_name((128, 2))) == (128, 2)


def test_default_cache_path_follows_the_environment(monkeypatch, tmp_path):
    monkeypatch.setenv("VPLBM_TILE_CACHE", str(tmp_path / "x.json"))
    assert AT.default_cache_path() == str(tmp_path / "x.json")
    monkeypatch.delenv("VPLBM_TILE_CACHE")
    monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path))
    assert AT.default_cache_path() == os.path.join(str(tmp_path), "vplbm", "tiles.json")


def test_shipped_defaults_are_the_fallback(tmp_path):
    # classes missing from the user cache come from the shipped table; a
    # user entry of the same class wins
    t = AT.TileTuner(path=str(tmp_path / "tiles.json"), arch="gfx950")
    shipped = t.shipped["arch"]["gfx950"]
    assert "batch/f32/AB/pop8192MiB/n9-64" in shipped
    for key, e in shipped.items():
        assert tuple(e["tile"]) in AT.LATTICE_TILES
        assert AT.tile_name(e["tile"]) in e["us"] and min(e["us"].values()) == e["us"][AT.tile_name(e["tile"])]
        if key.startswith("batch/"):
            assert tuple(e["tile"]) in AT.BATCH_TILES
    key = "batch/f32/AB/pop8192MiB/n9-64"
    assert t.lookup(key) == tuple(shipped[key]["tile"]) and t.entry(key)["source"] == "shipped"
    AT.tune([(256, 1)], fake_measure({(256, 1): 1.0}), t, key, rounds=1)
    assert t.lookup(key) == (256, 1) and t.entry(key)["source"] == "cache"
    # another architecture sees none of the shipped gfx950 choices
    assert AT.TileTuner(path=str(tmp_path / "tiles.json"), arch="gfx942").lookup(key) is None
