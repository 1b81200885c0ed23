"""Launch-layout autotuner for pr_solve.

For a sample of the caller's workload it times every candidate layout on
the GPU (HIP events, the best over three passes of the median of repeats,
after three seconds of warm-up launches) and keeps the fastest:

  * tile         -- polynomials per degree-sorted tile (mixed degrees only),
  * grid_blocks  -- the mixed-degree launch's shape: 0 for one wave per 64
                    consecutive polynomials of a degree-sorted tile, or the
                    number of persistent one-wave blocks walking the tiles
                    (tried at several per compute unit),
  * paired       -- FP32 form, index order: one or two polynomials per lane
                    (PR_FLAG_PAIRED_LANES),
  * ahead        -- one-per-lane launches: lock-step levels, or lanes one
                    level below the wave's running ahead (PR_FLAG_RUN_AHEAD),
  * cap          -- QR steps per level before NOT_CONVERGED; a cap is only
                    eligible if it flags no polynomial of the sample that the
                    default cap of 30 does not flag, and a smaller cap is only
                    taken if it is faster than the default's best layout by
                    more than CAP_MARGIN (a cap that no lane reaches changes
                    nothing but the result on harder inputs, and timing noise
                    alone would otherwise pick it half of the time).

Results go to a JSON cache keyed by architecture, form, dmax and degree mix
(``PROOTS_TUNE_CACHE`` overrides the path); uniform batches small enough to
leave the GPU latency-bound (at most ``SMALL_WAVES_PER_SIMD`` one-wave blocks
per SIMD) have keys of their own, tuned on a sample of that size, since
their best layout differs from a large batch's.  ``tuned_options`` reads the
cache; ``paper_2507_02164_amd.solve`` consults it when the caller leaves the
layout options unset.

    python -m paper_2507_02164_amd.autotune [uniform|uniform_small|mixed ...]
                                                # tunes the standard workloads
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import _capi

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(_HERE, "tuning", "tune_cache.json")

TILES = (512, 1024, 2048, 4096)
BLOCKS_PER_CU = (8, 16, 32, 64, 128)
SLICED_TILES = (128, 256, 512, 1024, 2048, 4096)
CAPS = (20, 24, 30)
DEFAULT_CAP = 30
CAP_MARGIN = 0.03
WARMUP_S = 3.0
ROUNDS = 3
# a uniform batch of at most this many one-wave blocks per SIMD (64
# polynomials each, 4 SIMDs per compute unit) is looked up under its own key
SMALL_WAVES_PER_SIMD = 2

_cache = None


def cache_path() -> str:
    return os.environ.get("PROOTS_TUNE_CACHE", DEFAULT_CACHE)


_arch = {}
_cus = {}


def arch_name(device=None) -> str:
    idx = torch.device(device).index if device is not None else 0
    idx = 0 if idx is None else idx
    if idx not in _arch:
        props = torch.cuda.get_device_properties(idx)
        _arch[idx] = getattr(props, "gcnArchName", "unknown").split(":")[0]
    return _arch[idx]


def key(arch, precision, dmax, mixed, small=False) -> str:
    kind = "mixed" if mixed else ("uniform_small" if small else "uniform")
    return f"{arch}/{precision}/dmax{dmax}/{kind}"


def small_limit(compute_units) -> int:
    """Largest uniform batch looked up under the small-batch key."""
    return compute_units * 4 * 64 * SMALL_WAVES_PER_SIMD


def lookup(cache, arch, precision, dmax, mixed, n=None, compute_units=None) -> dict:
    """Options for a batch of n polynomials from a cache dict: a small
    uniform batch takes its own key when that was tuned, every other batch
    (and a small one without it) the key of its form, dmax and degree mix."""
    if not mixed and n is not None and compute_units and n <= small_limit(compute_units):
        rec = cache.get(key(arch, precision, dmax, False, small=True))
        if rec is not None:
            return dict(rec.get("options", {}))
    return dict(cache.get(key(arch, precision, dmax, mixed), {}).get("options", {}))


def load_cache() -> dict:
    global _cache
    if _cache is None:
        p = cache_path()
        _cache = json.load(open(p)) if os.path.exists(p) else {}
    return _cache


def tuned_options(precision, dmax, mixed, device=None, n=None) -> dict:
    """Options recorded for this configuration and batch size ({} when none
    were tuned)."""
    if not torch.cuda.is_available():
        return {}
    idx = torch.device(device).index if device is not None else 0
    idx = 0 if idx is None else idx
    if idx not in _cus:
        _cus[idx] = torch.cuda.get_device_properties(idx).multi_processor_count
    return lookup(load_cache(), arch_name(device), precision, dmax, mixed, n, _cus[idx])


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def tune(coeffs, degrees=None, precision="fp32_polish", reps=5, log=print) -> dict:
    """Time the candidate layouts on this sample; returns the record
    {"options": {...}, "ms": best, "trials": [...]}."""
    dmax = coeffs.shape[0] - 1
    n = coeffs.shape[1]
    dev = coeffs.device
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    roots = torch.empty((dmax, n), dtype=torch.complex128, device=dev)
    status = torch.empty((n,), dtype=torch.int32, device=dev)

    def run(paired=0, ahead=0, **o):
        flags = (_capi.FLAG_PAIRED_LANES if paired else 0) | (_capi.FLAG_RUN_AHEAD if ahead else 0)
        _capi.solve(coeffs, degrees, precision, roots=roots, status=status, flags=flags, **o)

    # warm the GPU up first (clocks ramp over the first launches; without
    # this the first trials time slower than the same layout later)
    t_end = time.perf_counter() + WARMUP_S
    while time.perf_counter() < t_end:
        run(max_iter_per_level=30, tile=-1)
        torch.cuda.synchronize()
    # caps that flag nothing extra
    run(max_iter_per_level=30, tile=-1)
    torch.cuda.synchronize()
    base_flags = int(((status & _capi.ST_NOT_CONVERGED) != 0).sum())
    caps = []
    for cap in CAPS:
        run(max_iter_per_level=cap, tile=-1)
        torch.cuda.synchronize()
        if int(((status & _capi.ST_NOT_CONVERGED) != 0).sum()) <= base_flags:
            caps.append(cap)
    layouts = [dict(tile=-1), dict(tile=-1, ahead=1)]
    if precision == "fp32_polish":
        layouts.append(dict(tile=-1, paired=1))   # two polynomials per lane
    if degrees is not None:
        layouts += [dict(tile=t, grid_blocks=0, ahead=a) for t in SLICED_TILES for a in (0, 1)]
        layouts += [dict(tile=t, grid_blocks=b * cus) for t in TILES for b in BLOCKS_PER_CU]
    # every candidate is timed in ROUNDS passes over the whole list, every
    # other pass in reverse order, and keeps its best median: a drift of the
    # GPU's clock over the run then favours no position in the list (warm-up
    # alone does not settle it: after three seconds of it the first pass's
    # first trials still timed up to 20% slower than the same layouts later)
    cands = [dict(lay, max_iter_per_level=cap) for cap in caps for lay in layouts]
    best_ms = [float("inf")] * len(cands)
    for rnd in range(ROUNDS):
        order = range(len(cands)) if rnd % 2 == 0 else reversed(range(len(cands)))
        for k in order:
            o = cands[k]
            ms = _time(lambda: run(**o), reps)
            best_ms[k] = min(best_ms[k], ms)
            log(f"  {precision} {o}: {ms:.3f} ms")
    trials = [{"options": o, "ms": ms} for o, ms in zip(cands, best_ms)]
    best = min(trials, key=lambda t: t["ms"])
    at_default = [t for t in trials if t["options"]["max_iter_per_level"] == DEFAULT_CAP]
    if at_default:
        best_default = min(at_default, key=lambda t: t["ms"])
        if best_default["ms"] <= best["ms"] * (1 + CAP_MARGIN):
            best = best_default
    return {"options": best["options"], "ms": best["ms"], "n": n, "trials": trials,
            "eligible_caps": caps, "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S")}


def save(k, record):
    c = load_cache()
    c[k] = record
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def main():
    import sys
    root = os.path.dirname(_HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import workloads
    dev = torch.device("cuda:0")
    arch = arch_name(dev)
    # (mixed, small): sample
    samples = {
        (False, False): (torch.from_numpy(workloads.parametric(2048, seed=0)).to(dev), None),
        # one wave per SIMD: the 65,536-polynomial Gaussian batch
        (False, True): (torch.from_numpy(workloads.gaussian(65536, seed=0)).to(dev), None),
    }
    # the persistent grid's best size depends on the batch (work per block):
    # the mixed-degree layouts are tuned at the size of the 64 Mi workload
    a, d = workloads.mixed(64 * 2 ** 20, seed=0)
    samples[(True, False)] = (torch.from_numpy(a).to(dev), torch.from_numpy(d).to(dev))
    only = set(sys.argv[1:])  # optional: tune only these kinds (uniform, uniform_small, mixed)
    for (mixed, small), (c, deg) in samples.items():
        kind = key("", "", 0, mixed, small).rsplit("/", 1)[1]
        if only and kind not in only:
            continue
        for precision in ("fp32_polish", "fp64"):
            print(f"tuning {precision} {kind} on n={c.shape[1]}", flush=True)
            rec = tune(c, deg, precision)
            save(key(arch, precision, c.shape[0] - 1, mixed, small), rec)
            print(f"  -> {rec['options']} {rec['ms']:.3f} ms", flush=True)


if __name__ == "__main__":
    main()
