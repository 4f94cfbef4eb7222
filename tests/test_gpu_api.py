"""Boundary calls not covered by the parity tests: device-side macro readout
and divergence detection."""
import numpy as np
import pytest

import workloads as W
from gpu_cases import build_gpu, say
from test_gpu_parity import RAGGED

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["f64", "f32", "f16dev"])
def test_macro_device_equals_host_readout(precision):
    say("macro on the device", precision)
    s = RAGGED["inlet_outlet_freeslip_naca"]
    g = build_gpu(s, precision)
    g.step(17, macro=True)
    host = g.macro()
    dev = [t.cpu().numpy() for t in g.macro_device()]
    for h, d in zip(host, dev):
        assert d.shape == h.shape
        assert np.array_equal(d.astype(np.float64), h)  # the same stored values
    g.step(1)  # no macro on this step
    from paper_2110_00967_amd import vplbm as V
    with pytest.raises(V.VplbmError) as e:
        g.macro_device()
    assert e.value.code == V.ESTATE
    g.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_divergence_is_reported(precision):
    from paper_2110_00967_amd import vplbm as V
    say("diverging run reported as EUNSTABLE", precision)
    P = (V.PERIODIC, 0, 0)
    p = V.make_params(64, 32, 0.5001, 1e-4, 1.0, precision, P, P, P, P)
    g = V.Lattice(p)
    ux, uy = W.smooth_random_velocity(64, 32, seed=3, amp=0.35)
    g.set_fields(W.random_density(64, 32, seed=4, amp=0.05), ux, uy)
    g.step(700)  # the FP64 oracle reaches non-finite values by step 500
    with pytest.raises(V.VplbmError) as e:
        g.sync()
    assert e.value.code == V.EUNSTABLE
    # re-initialization clears it; a stable run reports nothing
    g.init_uniform(1.0, 0.01, 0.0)
    g.step(50)
    g.sync()
    g.close()


def test_default_tile_follows_the_footprint():
    # 64x4 unless the two population buffers exceed 1 GiB (FP64: 256 MB);
    # the AA pattern always runs 64x4
    from paper_2110_00967_amd import vplbm as V
    say("default step tile by footprint")
    cases = [((2000, 1000, "f32", 0), (64, 4)),    # 146 MB
             ((2000, 1000, "f64", 0), (128, 2)),   # 292 MB
             ((1600, 1000, "f64", 0), (64, 4)),    # 234 MB
             ((6000, 6000, "f32", 0), (128, 2)),   # 2.6 GB
             ((6000, 6000, "f32", 1), (64, 4))]    # AA
    for (nx, ny, prec, aa), tile in cases:
        g = V.Lattice(V.make_params(nx, ny, 0.6, 1e-3, 1.0, prec, streaming=aa))
        assert g.tile == tile, (nx, ny, prec, aa, g.tile)
        g.close()


def test_degenerate_calls():
    # zero steps (alone and batched) change nothing; a negative count is
    # rejected; removing every stress-integration point leaves SI forces of
    # exactly zero while ME goes on
    import numpy as np
    from paper_2110_00967_amd import vplbm as V
    say("degenerate calls: zero steps, empty point set")
    g = build_gpu(RAGGED["periodic_disk_random"], "f32")
    g.step(5)
    pops, h_me, h_si = g.populations(), g.history(0), g.history(1)
    g.step(0)
    b = V.Batch([g])
    b.step([0])
    b.close()
    assert g.step_count == 5
    assert np.array_equal(g.populations(), pops)
    assert np.array_equal(g.history(0), h_me) and np.array_equal(g.history(1), h_si)
    with pytest.raises(V.VplbmError) as e:
        g.step(-1)
    assert e.value.code == V.EINVAL
    g.set_si_points(np.zeros((0, 2)), np.zeros((0, 2)), np.zeros(0))
    g.step(2)
    assert np.all(g.forces_si() == 0.0)
    assert np.abs(g.forces_me()).max() > 0.0
    g.close()
