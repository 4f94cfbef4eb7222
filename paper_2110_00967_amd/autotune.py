"""Workgroup-tile autotuner for the fused step kernel.

The step kernel runs one cell per thread on tiles of 64x4, 128x2 or 256x1
cells (single lattices also 64x2, 128x1, 64x1); which one is fastest depends
on the device, the storage precision, the storage scheme and how far the
populations exceed the Infinity Cache.  Results never depend on the tile
(forces are summed in an order fixed at geometry set-up), so the choice is
pure performance.

``TileTuner`` keeps, per device architecture, the fastest tile of each
class -- launch kind (one lattice or a batch), precision, storage scheme and
population size rounded up to a power of two -- with the timings it was
chosen from, in a JSON file (``$VPLBM_TILE_CACHE``, else
``$XDG_CACHE_HOME/vplbm/tiles.json``, else ``~/.cache/vplbm/tiles.json``).
Classes not in that file fall back to the choices shipped with the package
(``tile_defaults.json``, written by ``python -m
paper_2110_00967_amd.autotune --write-defaults`` on the target GPU).
``tune_lattice`` times the candidates on a lattice with per-launch HIP events
(``vplbm_step_timed``); ``tune_batch`` times a batch's launches with events
around each run; both record the winner and apply it (``vplbm_set_tile``,
``vplbm_batch_set_tile``).  ``apply_lattice`` / ``apply_batch`` take a cached
choice without timing anything.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
import time
from typing import Callable, Dict, Iterable, Optional, Tuple

Tile = Tuple[int, int]

LATTICE_TILES: Tuple[Tile, ...] = ((64, 4), (128, 2), (256, 1), (64, 2), (128, 1), (64, 1))
BATCH_TILES: Tuple[Tile, ...] = ((64, 4), (128, 2), (256, 1))
AA_TILES: Tuple[Tile, ...] = ((64, 4),)
ELEM_BYTES = {"f64": 8, "f32": 4, "f16dev": 2, 0: 8, 1: 4, 2: 2}
PREC_NAME = {0: "f64", 1: "f32", 2: "f16dev", "f64": "f64", "f32": "f32", "f16dev": "f16dev"}


def default_cache_path() -> str:
    env = os.environ.get("VPLBM_TILE_CACHE")
    if env:
        return env
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "vplbm", "tiles.json")


def detect_arch() -> str:
    """The GPU architecture name (gfx950 on MI355X), 'unknown' without a GPU."""
    try:
        import torch

        if torch.cuda.is_available():
            return str(torch.cuda.get_device_properties(0).gcnArchName).split(":")[0]
    except Exception:
        pass
    return "unknown"


def size_bucket(pop_bytes: float) -> str:
    """Population bytes rounded up to a power of two MiB ('pop256MiB')."""
    mib = max(float(pop_bytes) / 2 ** 20, 1.0)
    return f"pop{2 ** math.ceil(math.log2(mib) - 1e-12):d}MiB"


def population_bytes(nx: int, ny: int, precision, streaming: str = "AB") -> int:
    """Bytes of the population buffers of one lattice (two, or one for AA)."""
    pitch = -(-int(nx) // 64) * 64
    nbuf = 1 if streaming == "AA" else 2
    return nbuf * 9 * pitch * int(ny) * ELEM_BYTES[precision]


def lattice_key(precision, streaming: str, nx: int, ny: int) -> str:
    shape = "narrow" if nx < 512 else "wide"
    return f"lattice/{PREC_NAME[precision]}/{streaming}/{size_bucket(population_bytes(nx, ny, precision, streaming))}/{shape}"


def batch_key(precision, streaming: str, batch) -> str:
    """Class of a batch: precision, storage, total population bytes, lattices."""
    total = sum(population_bytes(l.nx, l.ny, precision, streaming) for l in batch.lattices)
    n = len(batch.lattices)
    count = "n1" if n == 1 else ("n2-8" if n <= 8 else ("n9-64" if n <= 64 else "n65+"))
    return f"batch/{PREC_NAME[precision]}/{streaming}/{size_bucket(total)}/{count}"


def tile_name(t: Tile) -> str:
    return f"{int(t[0])}x{int(t[1])}"


def parse_tile(name: str) -> Tile:
    a, b = name.split("x")
    return int(a), int(b)


SHIPPED_DEFAULTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile_defaults.json")


class TileTuner:
    """Cache of the fastest tile per class, keyed by device architecture;
    classes missing from it fall back to the shipped defaults (read-only)."""

    VERSION = 1

    def __init__(self, path: Optional[str] = None, arch: Optional[str] = None,
                 defaults: Optional[str] = SHIPPED_DEFAULTS):
        self.path = path or default_cache_path()
        self.arch = arch or detect_arch()
        self.data = self._load(self.path)
        self.shipped = self._load(defaults) if defaults else {"version": self.VERSION, "arch": {}}

    @classmethod
    def _load(cls, path) -> dict:
        try:
            with open(path) as fh:
                d = json.load(fh)
            if isinstance(d, dict) and d.get("version") == cls.VERSION and isinstance(d.get("arch"), dict):
                return d
        except (OSError, ValueError):
            pass
        return {"version": cls.VERSION, "arch": {}}

    def _entries(self) -> dict:
        return self.data["arch"].setdefault(self.arch, {})

    def entry(self, key: str) -> Optional[dict]:
        """The cached entry of a class (the user cache first, then the shipped
        defaults), with "source" set to "cache" or "shipped"."""
        for src, d in (("cache", self.data), ("shipped", self.shipped)):
            e = d["arch"].get(self.arch, {}).get(key)
            if e:
                return dict(e, source=src)
        return None

    def lookup(self, key: str) -> Optional[Tile]:
        e = self.entry(key)
        if not e:
            return None
        try:
            return tuple(int(v) for v in e["tile"])  # type: ignore[return-value]
        except (KeyError, TypeError, ValueError):
            return None

    def timings(self, key: str) -> Dict[str, float]:
        e = self.entry(key)
        return dict(e.get("us", {})) if e else {}

    def record(self, key: str, timings: Dict[Tile, float]) -> Tile:
        """Store the timings of one class and its fastest tile (ties: the first
        candidate, in the order given); returns that tile."""
        if not timings:
            raise ValueError("no timings to choose from")
        best = min(timings, key=lambda t: (timings[t], list(timings).index(t)))
        self._entries()[key] = {"tile": list(best), "us": {tile_name(t): round(float(v), 3) for t, v in timings.items()},
                                "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
        try:
            self.save()
        except OSError:
            pass  # a read-only cache location: the choice holds for this process only
        return best

    def save(self) -> None:
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".tiles.", suffix=".json")
        with os.fdopen(fd, "w") as fh:
            json.dump(self.data, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def tune(candidates: Iterable[Tile], measure: Callable[[Tile], float], tuner: TileTuner, key: str,
         rounds: int = 2) -> Tile:
    """Time every candidate `rounds` times (interleaved, the best of each kept),
    record the class's winner and return it."""
    cands = list(candidates)
    best: Dict[Tile, float] = {}
    for _ in range(rounds):
        for t in cands:
            us = float(measure(t))
            best[t] = min(best.get(t, math.inf), us)
    return tuner.record(key, best)


def _runs(lat, t: Tile) -> bool:
    """Whether the lattice accepts tile t (a lattice with moving disks or in
    the AA pattern runs 64x4 only)."""
    from . import vplbm as V

    try:
        lat.set_tile(*t)
    except V.VplbmError as e:
        if e.code != V.EINVAL:
            raise
        return False
    return True


def tune_lattice(lat, tuner: TileTuner, key: Optional[str] = None, candidates: Optional[Iterable[Tile]] = None,
                 steps: int = 50, warmup: int = 5) -> Tile:
    """Time the tiles on a lattice (it advances by the steps timed) with
    per-launch HIP events of the step kernel; applies and returns the winner."""
    from . import vplbm as V

    aa = lat.params.streaming == V.STREAM_AA
    key = key or lattice_key(lat.params.precision, "AA" if aa else "AB", lat.nx, lat.ny)
    cands = [t for t in (candidates or (AA_TILES if aa else LATTICE_TILES)) if _runs(lat, t)]

    def measure(t: Tile) -> float:
        lat.set_tile(*t)
        lat.step(warmup)
        return lat.step_timed(steps) / steps * 1e3

    best = tune(cands, measure, tuner, key)
    lat.set_tile(*best)
    return best


def tune_batch(batch, tuner: TileTuner, key: Optional[str] = None, candidates: Optional[Iterable[Tile]] = None,
               steps: int = 40, warmup: int = 4) -> Tile:
    """Time the batch tiles with events around runs of `steps` batched steps
    (the lattices advance); applies and returns the winner."""
    import torch

    from . import vplbm as V

    aa = batch.lattices[0].params.streaming == V.STREAM_AA
    prec = batch.lattices[0].params.precision
    key = key or batch_key(prec, "AA" if aa else "AB", batch)
    cands = list(candidates or (AA_TILES if aa else BATCH_TILES))
    n = len(batch.lattices)

    def measure(t: Tile) -> float:
        batch.set_tile(*t)
        batch.step([warmup] * n)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        batch.step([steps] * n)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps * 1e3

    best = tune(cands, measure, tuner, key)
    batch.set_tile(*best)
    return best


def apply_lattice(lat, tuner: Optional[TileTuner] = None) -> Optional[Tile]:
    """Set the cached tile of the lattice's class, if one is cached."""
    from . import vplbm as V

    tuner = tuner or TileTuner()
    aa = lat.params.streaming == V.STREAM_AA
    t = tuner.lookup(lattice_key(lat.params.precision, "AA" if aa else "AB", lat.nx, lat.ny))
    if t is not None:
        lat.set_tile(*t)
    return t


def apply_batch(batch, tuner: Optional[TileTuner] = None) -> Optional[Tile]:
    """Set the cached tile of the batch's class, if one is cached."""
    from . import vplbm as V

    tuner = tuner or TileTuner()
    aa = batch.lattices[0].params.streaming == V.STREAM_AA
    t = tuner.lookup(batch_key(batch.lattices[0].params.precision, "AA" if aa else "AB", batch))
    if t is not None:
        batch.set_tile(*t)
    return t


def write_defaults(path: str = SHIPPED_DEFAULTS) -> dict:
    """Tune the standard classes on this GPU and write them as the shipped
    defaults: the 64-case airfoil sweep as one batch (FP32 and FP16
    deviations), and single airfoil lattices of 2000 x 1000 and 8192 x 8192
    and the 400 x 2000 sedimentation channel in FP64, FP32 and FP16."""
    import torch

    import workloads as W

    from . import vplbm as V

    tuner = TileTuner(path=path, defaults=None)
    for prec in ("f32", "f16dev"):
        lats = [V.Lattice.from_case(c, precision=prec) for c in W.sweep_cases()]
        b = V.Batch(lats)
        print(prec, "sweep", tune_batch(b, tuner, steps=60), flush=True)
        b.close()
        for g in lats:
            g.close()
        torch.cuda.empty_cache()
    singles = [W.case_naca(chord=200, aoa_deg=10.0), W.case_sedimentation()]
    big = W.case_naca(chord=819, aoa_deg=10.0)
    big.nx = big.ny = 8192
    singles.append(big)
    for prec in ("f64", "f32", "f16dev"):
        for case in singles:
            g = V.Lattice.from_case(case, precision=prec)
            steps = 20 if case.nx * case.ny > 1e7 else 200
            print(prec, case.name, tune_lattice(g, tuner, steps=steps), flush=True)
            g.close()
            torch.cuda.empty_cache()
    return tuner.data


if __name__ == "__main__":
    import sys

    if "--write-defaults" in sys.argv:
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        if root not in sys.path:
            sys.path.insert(0, root)
        out = sys.argv[sys.argv.index("--out") + 1] if "--out" in sys.argv else SHIPPED_DEFAULTS
        write_defaults(out)
    else:
        print("usage: python -m paper_2110_00967_amd.autotune --write-defaults [--out PATH]", file=sys.stderr)
