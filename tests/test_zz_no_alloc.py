"""The allocation-free batched step (vplbm_batch_step_noalloc, for callers
that cannot allocate device memory) against the batch handle's step
(vplbm_batch_step), bit for bit: populations, both force histories, body
state and mask, on two calls in a row, the second with a smaller input
(fewer and smaller lattices, one call after the first has left its tables in
the library's static array)."""
import numpy as np
import pytest

import workloads as W
from gpu_cases import F, OUT, P, V_, build_gpu, random_fields, say, small_naca, spec

pytestmark = pytest.mark.gpu


def first_specs():
    poly, ref, si = small_naca(nx=150, ny=75, chord=30.0, aoa=8.0)
    return [
        spec(150, 75, tau=0.56, edges=((V_, 0.05, 0), (OUT, 0, 0), (F, 0, 0), (F, 0, 0)), polygon=poly, ref=ref,
             si=si, init=("uniform", 1.0, 0.05, 0.0)),
        spec(80, 200, tau=0.6, edges=((V_, 0, 0), (V_, 0, 0), (OUT, 0, 0), (V_, 0, 0)), disk=(40.0, 150.0, 6.0),
             si=W.disk_si_points(40.0, 150.0, 6.0, 40), dynamics=(1.5, 0.0, -2e-4, 1)),
        spec(300, 130, tau=0.65, disk=(150.3, 64.6, 20.2), si=W.disk_si_points(150.3, 64.6, 20.2, 128),
             init=("fields",) + random_fields(300, 130, 3)),
    ]


def second_specs():
    return [
        spec(128, 64, tau=0.62, edges=((V_, 0.05, 0), (OUT, 0, 0), (P, 0, 0), (P, 0, 0)), disk=(32.0, 32.0, 8.0),
             si=W.disk_si_points(32.0, 32.0, 8.0, 64), init=("uniform", 1.0, 0.05, 0.0)),
        spec(70, 37, tau=0.7, eta=1e-3, edges=((P, 0, 0), (P, 0, 0), (V_, 0, 0), (V_, 0.02, 0)),
             gx=1e-6, disk=(30.0, 18.0, 6.0), init=("fields",) + random_fields(70, 37, 5, amp=0.01)),
    ]


def state(g):
    return g.populations(), g.history(0), g.history(1), g.body_state(), g.mask()


def compare(specs, nsteps, precision):
    from paper_2110_00967_amd import vplbm as V
    ref = [build_gpu(s, precision) for s in specs]
    b = V.Batch(ref)
    b.step(nsteps)
    b.close()
    lats = [build_gpu(s, precision) for s in specs]
    V.batch_step_noalloc(lats, nsteps)
    for k, (g, r) in enumerate(zip(lats, ref)):
        assert g.step_count == r.step_count == nsteps[k]
        for a, c in zip(state(g), state(r)):
            assert np.array_equal(a, c), (precision, k)
    for g in ref + lats:
        g.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_batch_step_equals_batch_step(precision):
    say("no-alloc batched step vs vplbm_batch_step,", precision, ": 3 lattices, then 2 smaller ones")
    compare(first_specs(), [41, 36, 40], precision)
    compare(second_specs(), [23, 9], precision)


def test_noalloc_rejects_too_many_tiles():
    from paper_2110_00967_amd import vplbm as V
    # 2^20 tiles of 64 x 4 cells: a lattice of 4100 x 1024 cells has
    # 65 x 256 = 16,640 tiles, so 64 of them are too many for one call
    say("no-alloc batched step: tile limit")
    p = V.make_params(4100, 1024, 0.6, 1e-4, 1.0, "f16dev", max_si_points=16)
    lats = [V.Lattice(p) for _ in range(64)]
    with pytest.raises(V.VplbmError) as e:
        V.batch_step_noalloc(lats, [1] * 64)
    assert e.value.code == V.EINVAL
    assert all(g.step_count == 0 for g in lats)
    for g in lats:
        g.close()
