"""Autotuner of pass schedules.

For one instance shape it enumerates the schedules the library can run (``ps_schedule_candidates``: the
N = N1 x N2 split of the four-step transform, the column-pass tile width, the row-pass frames per batch, the
column-pass frame grouping and the number of accumulator slots), times a whole integration with each of
them on the device, and keeps the fastest in a JSON cache.  The cache is keyed by the instance's shape and
format, the GPU architecture and the HIP version, and lives at $POLARIS_TUNE_CACHE (default
~/.cache/paper_1412_1256_amd/tune.json).

Every schedule computes the same spectra up to rounding; only speed differs.
"""
from __future__ import annotations

import json
import os
import tempfile
from dataclasses import asdict

from . import Instance, Plan, Schedule, schedule_candidates

CACHE_ENV = "POLARIS_TUNE_CACHE"


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "paper_1412_1256_amd",
                                                     "tune.json")


def cache_key(instance: Instance, device) -> str:
    import torch
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", props.name)
    pairs = ",".join(f"{x}{y}" for x, y in instance.pairs)
    return "|".join([arch, f"hip{torch.version.hip}", f"N{instance.fft_len}", f"bits{instance.bits}",
                     f"S{instance.n_streams}", f"pairs{pairs}", str(instance.window), str(instance.precision),
                     str(instance.accum), f"chunk{instance.chunk_frames}"])


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def _save_cache(d: dict, path: str | None = None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _synthetic_input(instance: Instance, frames: int, device):
    """Packed input of the instance's format (values do not change the timing of these kernels)."""
    import torch
    n = frames * instance.fft_len * instance.n_streams
    g = torch.Generator(device=device)
    g.manual_seed(1412)
    if instance.bits == 32:
        return torch.randint(-8, 8, (n,), generator=g, device=device).to(torch.float32).view(torch.uint8)
    return torch.randint(0, 256, (n * instance.bits // 8,), generator=g, device=device, dtype=torch.uint8)


RING_BYTES = 768 << 20  # inputs cycled through while timing: three times the 256 MB last-level cache


def _input_ring(instance: Instance, frames: int, device) -> list:
    """Distinct input buffers, so each timed integration streams its input from HBM as in real use."""
    first = _synthetic_input(instance, frames, device)
    n = max(1, min(24, -(-RING_BYTES // first.numel())))
    return [first] + [first.clone() for _ in range(n - 1)]


def time_schedule(instance: Instance, sched: Schedule, device, frames: int, reps: int = 5, warmup: int = 2,
                  ring: list | None = None, inner: int = 8) -> float:
    """Time (ms) of one whole integration: reset, accumulate `frames` frames from the next buffer of the input
    ring, Stokes (the Stokes pass sums the accumulator slots, so its cost depends on the schedule too).  Each
    of the `reps` samples times `inner` consecutive integrations (single integrations of some 70 us are too
    short to rank schedules a few percent apart); the median sample is returned."""
    import torch
    plan = Plan([instance], device=device, schedules=[sched])
    ring = ring if ring is not None else _input_ring(instance, frames, device)
    out = torch.empty((instance.n_pairs, 4, instance.channels), dtype=torch.float32, device=device)
    k = [0]

    def step():
        buf = ring[k[0] % len(ring)]
        k[0] += 1
        plan.reset()
        plan.accumulate(buf)
        plan.stokes(out=out)

    for _ in range(warmup):
        step()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(plan.stream)
        for _ in range(inner):
            step()
        b.record(plan.stream)
        b.synchronize()
        times.append(a.elapsed_time(b) / inner)
    times.sort()
    return times[len(times) // 2]


def default_frames(instance: Instance) -> int:
    """About 16 M samples per stream, between 4 and 64 frames."""
    return max(4, min(64, (1 << 24) // instance.fft_len))


def tune(instance: Instance, device=None, frames: int | None = None, reps: int = 5, cache: str | None = None,
         force: bool = False) -> tuple[Schedule, dict]:
    """Time every candidate schedule of the instance; return the fastest and the timings, and record the
    winner in the cache (unless it is already there and force is False)."""
    import torch
    device = torch.device(device if device is not None else "cuda")
    key = cache_key(instance, device)
    d = load_cache(cache)
    if key in d and not force:
        return Schedule(**d[key]["schedule"]), d[key].get("timings_ms", {})
    frames = frames or default_frames(instance)
    ring = _input_ring(instance, frames, device)
    # the first hundred or so integrations after start-up run several percent slow (clocks, first touches of
    # the input ring): run them before the first candidate is timed
    time_schedule(instance, Schedule(), device, frames, reps=1, warmup=0, ring=ring, inner=max(32, 2 * len(ring)))
    timings = {}
    best, best_ms = None, float("inf")
    for s in schedule_candidates(instance):
        ms = time_schedule(instance, s, device, frames, reps, ring=ring)
        timings[json.dumps(asdict(s), sort_keys=True)] = ms
        if ms < best_ms:
            best, best_ms = s, ms
    d = load_cache(cache)
    d[key] = {"schedule": asdict(best), "ms": best_ms, "frames": frames, "timings_ms": timings}
    _save_cache(d, cache)
    return best, timings


def best_schedule(instance: Instance, device=None, cache: str | None = None) -> Schedule:
    """The cached schedule of the instance's shape, tuning it first on a cache miss."""
    return tune(instance, device=device, cache=cache)[0]
