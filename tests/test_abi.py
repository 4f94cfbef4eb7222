"""C-ABI contract checks that run without a GPU: the library loads, exports
every entry point include/vplbm.h declares, and its parameter validation
(vplbm_required_bytes, pure host logic) accepts and rejects what the header
says."""
import math
import os
import re
import subprocess

import pytest

from paper_2110_00967_amd import vplbm as V

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vplbm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vplbm_[a-z_]+)\s*\(", src)))


def test_header_declares_what_the_binding_wraps():
    assert declared_functions() == sorted(V.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = V.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", V.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (vplbm_[a-z_]+)", out))
    assert set(declared_functions()) <= exported


def test_library_has_no_oracle_dependency():
    out = subprocess.run(["ldd", V.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle" not in out
    syms = subprocess.run(["nm", "-D", V.LIB_PATH], capture_output=True, text=True).stdout
    assert "orc_" not in syms


def base(**kw):
    args = dict(nx=128, ny=64, tau=0.62, eta=1e-4, precision="f32", west=(V.VELOCITY, 0.05, 0),
                east=(V.OUTFLOW, 0, 0), south=(V.PERIODIC, 0, 0), north=(V.PERIODIC, 0, 0))
    args.update(kw)
    return V.make_params(**args)


def test_required_bytes_valid():
    n32 = V.required_bytes(base())
    n64 = V.required_bytes(base(precision="f64"))
    n16 = V.required_bytes(base(precision="f16dev"))
    assert 0 < n16 < n32 < n64
    # A and B dominate: 2 * 9 planes of the padded lattice
    assert n32 >= 2 * 9 * 64 * 128 * 4
    assert V.required_bytes(base(nx=2000, ny=1000)) > 2 * 9 * 2000 * 1000 * 4


@pytest.mark.parametrize("kw", [
    dict(nx=3), dict(ny=2), dict(tau=0.5), dict(tau=0.3), dict(tau=float("nan")), dict(eta=0.0),
    dict(eta=-1.0), dict(eta=float("nan")), dict(precision=7), dict(west=(V.PERIODIC, 0, 0)),
    dict(south=(V.VELOCITY, 0, 0)), dict(north=(9, 0, 0)), dict(east=(V.VELOCITY, float("inf"), 0)),
    dict(nx=200000, ny=200000), dict(max_si_points=5000), dict(hist_capacity=-1),
    dict(trt_lambda=-0.1), dict(trt_lambda=float("nan")), dict(si_rule=2), dict(si_rule=-1),
    dict(si_rule=1, max_si_points=1025), dict(si_rule=1, max_si_points=0),
    dict(east=(V.CONVECTIVE, -0.01, 0)), dict(east=(V.CONVECTIVE, float("nan"), 0)), dict(east=(5, 0, 0)),
    dict(max_bodies=64), dict(max_bodies=-1), dict(max_interface_cells=-1), dict(streaming=2), dict(streaming=-1),
])
def test_required_bytes_rejects(kw):
    assert V.required_bytes(base(**kw)) == 0


def test_size_limit_is_cells_below_2e31():
    # populations are indexed in 64 bits, cells (ny * pitch) in 32: a lattice
    # of 32768 x 65535 (2^31 - 32768 cells, 1.9e10 elements) is accepted, one
    # more row is not; nx has no limit of its own
    n = V.required_bytes(base(nx=32768, ny=65535))
    assert n >= 2 * 9 * 32768 * 65535 * 4
    assert V.required_bytes(base(nx=32768, ny=65536)) == 0
    assert V.required_bytes(base(nx=100000, ny=64)) > 0


def test_si_rule_interpolated_accepts_up_to_1024_points():
    n1 = V.required_bytes(base(si_rule=1, max_si_points=1024))
    n0 = V.required_bytes(base(si_rule=0, max_si_points=1024))
    # room for 4 sample records (48 bytes each) per point instead of 1
    assert n1 - n0 >= 3 * 1024 * 48


def test_more_bodies_take_more_history_room():
    n1 = V.required_bytes(base(max_bodies=1, hist_capacity=1000))
    n63 = V.required_bytes(base(max_bodies=63, hist_capacity=1000))
    assert V.required_bytes(base(hist_capacity=1000)) == n1
    # one (steps x 6) FP64 history per body
    assert n63 - n1 >= 62 * 6 * 8 * 1000


def test_interface_slots_are_sized_by_the_caller():
    a = V.required_bytes(base(max_interface_cells=100))
    b = V.required_bytes(base(max_interface_cells=100000))
    assert 0 < a < b


def test_aa_storage_keeps_one_population_buffer():
    for prec, es in (("f64", 8), ("f32", 4), ("f16dev", 2)):
        ab = V.required_bytes(base(precision=prec, nx=2000, ny=1000))
        aa = V.required_bytes(base(precision=prec, nx=2000, ny=1000, streaming=V.STREAM_AA))
        pop = 9 * 1000 * 2048 * es  # one [9][ny][pitch] buffer
        # one buffer less, plus the two perimeter copies (9 x 5996 cells each)
        assert ab - aa >= pop - 2 * 9 * 6000 * es - 4096
        assert ab - aa <= pop


def test_convective_edge_accepted():
    assert V.required_bytes(base(east=(V.CONVECTIVE, 0.05, 0))) > 0
    assert V.required_bytes(base(east=(V.CONVECTIVE, 0.0, 0))) > 0


def test_eta_infinite_is_allowed():
    assert V.required_bytes(base(eta=math.inf)) > 0
