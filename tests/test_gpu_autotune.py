"""Tile autotuner on the GPU: a tuned tile (lattice and batch) gives exactly
the default tile's results -- populations, force histories, body state --
and the tuner times every candidate and records the fastest."""
import numpy as np
import pytest

from gpu_cases import build_gpu, say
from test_gpu_batch import mixed_specs, state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["f32", "f16dev"])
def test_tuned_lattice_tile_gives_default_bits(tmp_path, precision):
    from paper_2110_00967_amd import autotune as AT
    s = mixed_specs()[4]  # 300 x 130, disk with SI points, random fields
    tuner = AT.TileTuner(path=str(tmp_path / "tiles.json"))
    scratch = build_gpu(s, precision)
    say("tune lattice tile", precision)
    best = AT.tune_lattice(scratch, tuner, steps=20, warmup=2)
    key = AT.lattice_key(scratch.params.precision, "AB", scratch.nx, scratch.ny)
    assert best in AT.LATTICE_TILES and tuner.lookup(key) == best
    assert set(tuner.timings(key)) == {AT.tile_name(t) for t in AT.LATTICE_TILES}
    scratch.close()
    a, b = build_gpu(s, precision), build_gpu(s, precision)
    # the cached choice, from a new tuner on the same file
    assert AT.apply_lattice(a, AT.TileTuner(path=tuner.path)) == best and a.tile == best
    assert b.tile == (64, 4)
    a.step(37)
    b.step(37)
    for x, y in zip(state(a), state(b)):
        assert np.array_equal(x, y)
    a.close()
    b.close()


def test_tuned_batch_tile_gives_default_bits(tmp_path):
    from paper_2110_00967_amd import autotune as AT
    from paper_2110_00967_amd import vplbm as V
    specs = mixed_specs()
    tuner = AT.TileTuner(path=str(tmp_path / "tiles.json"))
    say("tune batch tile f32")
    lats = [build_gpu(s, "f32") for s in specs]
    bt = V.Batch(lats)
    best = AT.tune_batch(bt, tuner, steps=12, warmup=2)
    assert best in AT.BATCH_TILES and bt.tile == best
    bt.close()
    for g in lats:
        g.close()
    runs = []
    for tuned in (True, False):
        lats = [build_gpu(s, "f32") for s in specs]
        bt = V.Batch(lats)
        if tuned:
            assert AT.apply_batch(bt, tuner) == best
        bt.step([40, 17, 33, 5, 26, 35])
        runs.append([state(g) for g in lats])
        bt.close()
        for g in lats:
            g.close()
    for a, r in zip(*runs):
        for x, y in zip(a, r):
            assert np.array_equal(x, y)


def test_tuning_a_lattice_with_moving_disks_times_its_one_tile(tmp_path):
    # a lattice with moving disks runs 64x4 only: the tuner times that tile
    # alone and records it
    from paper_2110_00967_amd import autotune as AT
    from paper_2110_00967_amd import vplbm as V
    import workloads as W
    say("tune a lattice with a moving disk")
    g = V.Lattice.from_case(W.case_sedimentation(), precision="f32")
    tuner = AT.TileTuner(path=str(tmp_path / "tiles.json"))
    assert AT.tune_lattice(g, tuner, steps=10, warmup=2) == (64, 4)
    key = AT.lattice_key(g.params.precision, "AB", g.nx, g.ny)
    assert set(tuner.timings(key)) == {"64x4"} and g.tile == (64, 4)
    g.close()
