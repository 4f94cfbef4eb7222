"""Batched stepping (vplbm_batch_*): every lattice in a batch must compute
exactly what it computes alone -- bitwise, populations and force histories --
whatever else is in the batch and however many steps each one takes.  The
long runs go through the captured-graph path (pairs of launches replayed).
One lattice is also checked against the oracle."""
import numpy as np
import pytest

import workloads as W
from gpu_cases import CV, F, OUT, P, V_, build_gpu, build_oracle, oracle_pops, random_fields, say, small_naca, spec

pytestmark = pytest.mark.gpu



def step_eager(g, n):
    """n steps, one call each: the plain per-step launches, never a graph."""
    for _ in range(n):
        g.step(1)

def mixed_specs():
    poly, ref, si = small_naca(nx=150, ny=75, chord=30.0, aoa=8.0)
    return [
        spec(150, 75, tau=0.56, edges=((V_, 0.05, 0), (OUT, 0, 0), (F, 0, 0), (F, 0, 0)), polygon=poly, ref=ref,
             si=si, init=("uniform", 1.0, 0.05, 0.0)),
        spec(128, 64, tau=0.62, edges=((V_, 0.05, 0), (OUT, 0, 0), (P, 0, 0), (P, 0, 0)), disk=(32.0, 32.0, 8.0),
             si=W.disk_si_points(32.0, 32.0, 8.0, 64), init=("uniform", 1.0, 0.05, 0.0)),
        spec(80, 200, tau=0.6, edges=((V_, 0, 0), (V_, 0, 0), (OUT, 0, 0), (V_, 0, 0)), disk=(40.0, 150.0, 6.0),
             si=W.disk_si_points(40.0, 150.0, 6.0, 40), dynamics=(1.5, 0.0, -2e-4, 1)),
        spec(131, 37, tau=0.7, eta=1e-3, edges=((P, 0, 0), (P, 0, 0), (V_, 0, 0), (V_, 0.02, 0)),
             gx=1e-6, disk=(40.0, 18.0, 6.0), init=("fields",) + random_fields(131, 37, 5, amp=0.01)),
        spec(300, 130, tau=0.65, disk=(150.3, 64.6, 20.2), si=W.disk_si_points(150.3, 64.6, 20.2, 128),
             init=("fields",) + random_fields(300, 130, 3)),
        spec(96, 40, tau=0.6, edges=((V_, 0.04, 0), (CV, 0.04, 0), (F, 0, 0), (V_, 0, 0)), disk=(30.0, 20.0, 5.0),
             init=("uniform", 1.0, 0.04, 0.0)),
    ]


def state(g):
    return g.populations(), g.history(0), g.history(1), g.body_state()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_equals_alone_bitwise(precision):
    from paper_2110_00967_amd import vplbm as V
    specs = mixed_specs()
    nsteps = [40, 17, 33, 0, 26, 35]
    say("batch of", len(specs), "lattices,", precision, "steps", nsteps)
    solo = [build_gpu(s, precision) for s in specs]
    for g, n in zip(solo, nsteps):
        step_eager(g, n)
    lats = [build_gpu(s, precision) for s in specs]
    b = V.Batch(lats)
    b.step(nsteps)
    for k, (g, ref) in enumerate(zip(lats, solo)):
        assert g.step_count == nsteps[k]
        if nsteps[k] == 0:
            continue
        for a, r in zip(state(g), state(ref)):
            assert np.array_equal(a, r), (precision, k)
    # the batched lattices go on with direct steps (buffer parity and pending
    # forces handed over by the batch) and still match the direct runs
    for g, ref in zip(lats, solo):
        step_eager(g, 3)
        step_eager(ref, 3)
        for a, r in zip(state(g), state(ref)):
            assert np.array_equal(a, r), precision
    # a second round with the roles changed (chunks of different shapes)
    b.step([5, 0, 12, 9, 1, 3])
    assert [g.step_count for g in lats] == [48, 20, 48, 12, 30, 41]
    b.close()
    for g in solo + lats:
        g.close()


def test_trt_batch_equals_alone_bitwise():
    from paper_2110_00967_amd import vplbm as V
    poly, ref, si = small_naca(nx=150, ny=75, chord=30.0, aoa=12.0)
    specs = [
        spec(150, 75, tau=0.55, trt=1.0 / 6.0, edges=((V_, 0.05, 0), (OUT, 0, 0), (F, 0, 0), (F, 0, 0)),
             polygon=poly, ref=ref, si=si, init=("uniform", 1.0, 0.05, 0.0)),
        spec(131, 37, tau=0.7, eta=1e-3, trt=3.0 / 16.0, edges=((P, 0, 0), (P, 0, 0), (V_, 0, 0), (V_, 0.02, 0)),
             gx=1e-6, disk=(40.0, 18.0, 6.0), init=("fields",) + random_fields(131, 37, 5, amp=0.01)),
        spec(80, 200, tau=0.6, trt=1.0 / 6.0, edges=((V_, 0, 0), (V_, 0, 0), (OUT, 0, 0), (V_, 0, 0)),
             disk=(40.0, 150.0, 6.0), si=W.disk_si_points(40.0, 150.0, 6.0, 40), dynamics=(1.5, 0.0, -2e-4, 0)),
    ]
    nsteps = [37, 52, 20]
    say("TRT batch of", len(specs), "lattices, steps", nsteps)
    alone = []
    for s, n in zip(specs, nsteps):
        g = build_gpu(s, "f64")
        step_eager(g, n)
        alone.append(state(g))
        g.close()
    lats = [build_gpu(s, "f64") for s in specs]
    b = V.Batch(lats)
    b.step(nsteps)
    for g, ref in zip(lats, alone):
        for a, r in zip(state(g), ref):
            assert np.array_equal(a, r)
    # BGK and TRT lattices cannot share a launch
    bgk = build_gpu(mixed_specs()[1], "f64")
    with pytest.raises(V.VplbmError):
        V.Batch([lats[0], bgk])
    b.close()


def test_batch_long_run_graph_replay_vs_oracle():
    # a long uneven run: most steps come from replays of the captured pair
    from paper_2110_00967_amd import vplbm as V
    specs = mixed_specs()[:3]
    say("batch graph replay, 3 lattices x up to 301 steps fp64")
    lats = [build_gpu(s, "f64") for s in specs]
    b = V.Batch(lats)
    b.step([301, 250, 120])
    orc = build_oracle(specs[1])
    orc.step(250)
    assert np.abs(lats[1].populations() - oracle_pops(orc)).max() <= 1e-12
    h = lats[1].history(0)
    assert np.abs(h - orc.me()).max() <= 1e-10 * np.abs(orc.me()).max()
    # the same run alone, eager launches, must match bitwise
    g = build_gpu(specs[0], "f64")
    for _ in range(301):
        g.step(1)
    assert np.array_equal(g.populations(), lats[0].populations())
    assert np.array_equal(g.history(1), lats[0].history(1))
    b.close()


def test_batch_rejects_mixed_precision():
    from paper_2110_00967_amd import vplbm as V
    specs = mixed_specs()
    a = build_gpu(specs[1], "f64")
    c = build_gpu(specs[1], "f32")
    with pytest.raises(V.VplbmError):
        V.Batch([a, c])
    with pytest.raises(V.VplbmError):
        V.Batch([a, a])


@pytest.mark.parametrize("name", ["periodic_disk_random", "convective_trt_naca", "couette_walls_force"])
def test_one_lattice_batch_equals_eager_steps(name):
    # 57 steps: one eager launch, one captured group of 16 step pairs, then
    # 12 pairs launched directly -- bitwise the same as one call per step
    from paper_2110_00967_amd import vplbm as V
    from test_gpu_parity import RAGGED
    s = RAGGED[name]
    say("one-lattice batch vs eager steps", name)
    a, b = build_gpu(s, "f32"), build_gpu(s, "f32")
    bt = V.Batch([a])
    bt.step([57])
    step_eager(b, 57)
    for x, y in zip(state(a), state(b)):
        assert np.array_equal(x, y), name
    bt.close()
    a.close()
    b.close()


def test_one_lattice_batch_moving_disk_equals_eager_steps():
    from paper_2110_00967_amd import vplbm as V
    case = W.case_sedimentation(nx=96, ny=320, d=16.0, rho_r=1.5, g=2e-4, npts=48, force_source=1)
    say("one-lattice batch vs eager steps, free disk")
    a = V.Lattice.from_case(case, precision="f32")
    b = V.Lattice.from_case(case, precision="f32")
    bt = V.Batch([a])
    bt.step([75])
    step_eager(b, 75)
    assert np.array_equal(a.body_state(), b.body_state())
    assert np.array_equal(a.populations(), b.populations())
    assert np.array_equal(a.history(1), b.history(1))
    bt.close()
    a.close()
    b.close()


def test_lattice_beyond_the_cache_default_tile_and_batch():
    # two FP64 buffers of 2048 x 2048 (604 MB) exceed 256 MB: the lattice
    # steps with 128x2 tiles by default, and a batch still takes it (batched
    # launches use 64x4 tiles); all three runs give the same bits
    from paper_2110_00967_amd import vplbm as V
    nx = ny = 2048
    # random fields: every cell changes at every step, so a tile left out
    # anywhere shows in the comparison
    s = spec(nx, ny, tau=0.6, edges=((V_, 0.05, 0), (OUT, 0, 0), (F, 0, 0), (F, 0, 0)), disk=(1500.3, 1024.6, 40.2),
             si=W.disk_si_points(1500.3, 1024.6, 40.2, 256), init=("fields",) + random_fields(nx, ny, 7, amp=0.03))
    say("2048x2048 fp64: default tile, 64x4 tile, batch")
    runs = []
    for mode in ("default", "64x4", "batch"):
        g = build_gpu(s, "f64")
        assert g.tile == (128, 2)  # 604 MB of FP64 populations
        if mode == "64x4":
            g.set_tile(64, 4)
            assert g.tile == (64, 4)
        if mode == "batch":
            b = V.Batch([g])
            b.step([12])
            b.close()
        else:
            g.step(12)
        g.step(1, macro=True)
        runs.append([g.populations(), *g.macro(), g.history(0), g.history(1)])
        g.close()
    for r in runs[1:]:
        for a, b_ in zip(r, runs[0]):
            assert np.array_equal(a, b_)
    # and the run moved every cell away from its initial state
    g = build_gpu(s, "f64")
    first = g.populations()
    g.close()
    assert (runs[0][0] != first).any(axis=0).mean() > 0.99


@pytest.mark.parametrize("precision", ["f64", "f32", "f16dev"])
def test_aa_batch_equals_alone_bitwise(precision):
    # lattices in the AA pattern, batched: odd and even launches per lattice
    # by its own step parity, perimeter copies alternating; chunks long
    # enough for the captured-graph path, odd and even step counts
    from paper_2110_00967_amd import vplbm as V
    specs = mixed_specs()
    nsteps = [41, 17, 36, 0, 26, 35]
    say("AA batch of", len(specs), "lattices,", precision, "steps", nsteps)
    solo = [build_gpu(s, precision, streaming=V.STREAM_AA) for s in specs]
    for g, n in zip(solo, nsteps):
        step_eager(g, n)
    lats = [build_gpu(s, precision, streaming=V.STREAM_AA) for s in specs]
    b = V.Batch(lats)
    b.step(nsteps)
    for k, (g, ref) in enumerate(zip(lats, solo)):
        assert g.step_count == nsteps[k]
        if nsteps[k] == 0:
            continue
        for a, r in zip(state(g), state(ref)):
            assert np.array_equal(a, r), (precision, k)
    # the batched lattices go on with direct steps (perimeter copies and
    # layout handed over by the batch) and still match the direct runs
    for g, ref in zip(lats, solo):
        step_eager(g, 3)
        step_eager(ref, 3)
        for a, r in zip(state(g), state(ref)):
            assert np.array_equal(a, r), precision
    # a second round that starts every lattice on the other parity
    b.step([3, 1, 2, 7, 0, 4])
    for g, n in zip(lats, [47, 21, 41, 10, 29, 42]):
        assert g.step_count == n
    b.close()
    for g in solo + lats:
        g.close()


def test_aa_batch_with_a_moving_disk_above_the_rotation_limit():
    # AA lattices with a moving disk batched with a static lattice of 8320
    # tiles (64x4): the launches exceed the band rotation's 8192 tiles and
    # run the moving-disk kernel without it until the static lattice is
    # done, then with it; every lattice as alone, bit for bit
    from paper_2110_00967_amd import vplbm as V
    specs = [mixed_specs()[2],
             spec(2048, 1040, tau=0.6, edges=((V_, 0.03, 0), (OUT, 0, 0), (F, 0, 0), (F, 0, 0)),
                  init=("fields",) + random_fields(2048, 1040, 11, amp=0.01))]
    assert specs[0]["dynamics"] is not None
    nsteps = [23, 14]
    say("AA batch, a moving disk and a 2048x1040 lattice, f32, steps", nsteps)
    solo = [build_gpu(s, "f32", streaming=V.STREAM_AA) for s in specs]
    for g, n in zip(solo, nsteps):
        step_eager(g, n)
    lats = [build_gpu(s, "f32", streaming=V.STREAM_AA) for s in specs]
    b = V.Batch(lats)
    b.step(nsteps)
    for k, (g, ref) in enumerate(zip(lats, solo)):
        assert g.step_count == nsteps[k]
        for a, r in zip(state(g), state(ref)):
            assert np.array_equal(a, r), k
    b.close()
    for g in solo + lats:
        g.close()


def test_batch_rejects_mixed_storage():
    from paper_2110_00967_amd import vplbm as V
    specs = mixed_specs()[:2]
    say("AA and AB lattices in one batch")
    a = build_gpu(specs[0], "f32", streaming=V.STREAM_AA)
    c = build_gpu(specs[1], "f32")
    with pytest.raises(V.VplbmError) as e:
        V.Batch([a, c])
    assert e.value.code == V.EINVAL
    a.close()
    c.close()


@pytest.mark.parametrize("precision", ["f32", "f16dev"])
def test_batch_of_many_tiny_lattices_equals_alone(precision):
    # 70 lattices of one to three 64x4 tiles each: a block of the lattice
    # table (64 global tiles) spans dozens of lattices, the last ones only
    # partly; some hold a disk (their tile 0 sums the forces), the step counts
    # differ, so the active set and the table change from chunk to chunk
    from paper_2110_00967_amd import vplbm as V
    rng = np.random.default_rng(11)
    specs = []
    for k in range(70):
        nx, ny = int(rng.integers(8, 150)), int(rng.integers(4, 9))
        if k % 7 == 3:
            ny = 12
            specs.append(spec(nx, ny, tau=0.7, disk=(nx / 2.0, 6.0, 2.5), init=("fields",) + random_fields(nx, ny, k)))
        else:
            specs.append(spec(nx, ny, tau=0.6 + 0.003 * k, init=("fields",) + random_fields(nx, ny, k)))
    nsteps = [int(v) for v in rng.integers(0, 12, len(specs))]
    say("batch of", len(specs), "tiny lattices,", precision, "steps", nsteps[:10], "...")
    solo = [build_gpu(s, precision) for s in specs]
    for g, n in zip(solo, nsteps):
        step_eager(g, n)
    lats = [build_gpu(s, precision) for s in specs]
    b = V.Batch(lats)
    b.step(nsteps)
    for k, (g, ref) in enumerate(zip(lats, solo)):
        got, want = (state(g), state(ref)) if specs[k]["disk"] else ((g.populations(),), (ref.populations(),))
        for x, y in zip(got, want):
            assert np.array_equal(x, y), k
    b.close()
    for g in lats + solo:
        g.close()


@pytest.mark.parametrize("precision", ["f64", "f32", "f16dev"])
def test_batch_tiles_give_the_same_bits(precision):
    # the tile of the batched launches (vplbm_batch_set_tile) changes the
    # workgroup shape only: every tile gives the 64x4 result bit for bit,
    # through the captured-graph path (40 steps) and a short chunk
    from paper_2110_00967_amd import vplbm as V
    specs = mixed_specs()
    nsteps = [40, 17, 33, 5, 26, 35]
    runs = {}
    for tile in ((64, 4), (128, 2), (256, 1)):
        say("batch tile", tile, precision)
        lats = [build_gpu(s, precision) for s in specs]
        b = V.Batch(lats)
        b.set_tile(*tile)
        assert b.tile == tile
        b.step(nsteps)
        runs[tile] = [state(g) for g in lats]
        b.close()
        for g in lats:
            g.close()
    for tile in ((128, 2), (256, 1)):
        for k, (a, r) in enumerate(zip(runs[tile], runs[(64, 4)])):
            for x, y in zip(a, r):
                assert np.array_equal(x, y), (tile, k)


def test_batch_tile_rules():
    from paper_2110_00967_amd import vplbm as V
    specs = mixed_specs()[:2]
    say("batch tile rules")
    lats = [build_gpu(s, "f32") for s in specs]
    b = V.Batch(lats)
    assert b.tile == (64, 4)
    for bad in ((64, 2), (32, 8), (128, 4), (64, 8)):
        with pytest.raises(V.VplbmError) as e:
            b.set_tile(*bad)
        assert e.value.code == V.EINVAL
    assert b.tile == (64, 4)
    b.close()
    aa = [build_gpu(s, "f32", streaming=V.STREAM_AA) for s in specs]
    b = V.Batch(aa)
    with pytest.raises(V.VplbmError):
        b.set_tile(128, 2)
    b.close()
    for g in lats + aa:
        g.close()
