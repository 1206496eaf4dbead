"""FIR / IIR crossover tuner for the AUTO spatial mode.

The two spatial modes are two different spatial filters for the Gaussian
filtering step of the method (eq. (8)): the FIR mode convolves with the
sampled Gaussian truncated at the window radius ceil(3 sigma_s) (its cost
grows with the radius), the recursive mode with Deriche's untruncated
recursive Gaussian (the same cost at every sigma_s, but five launches and two
passes through a channel stack: a fixed cost that matters on small images).
Their outputs differ slightly (about 0.1 gray levels on 8-bit data, from the
truncation and the fit of the recursive kernel), so the table this tuner
installs decides which of the two filters AUTO computes, not only how fast.
Which is faster for a given radius depends on the image size and the device.

`tune()` times both on this device for a ladder of image sizes, finds for
each size the largest radius at which FIR is still faster (the FIR time rises
with the radius, so a bisection over radii suffices), installs the result in
the library as its size-dependent crossover table and stores it in a JSON
cache keyed by device architecture, compute-unit count and degree.  `ensure()` loads the cached table, or
tunes once when there is none.  Timing uses synthetic images on the device;
the filter's cost does not depend on the pixel values.

`plan_batch()` chooses the launch shape of a batch plan's recursive images
(band height, channel groups of the column and of the row passes; every
recursive image of a plan shares it) by timing one plan per candidate shape
on the batch itself, and caches the choice under the batch's composition
(the sizes, and for each image the spatial mode AUTO resolves), so that later
plans of the same composition are built directly.  The launch shape decides
the rounding of the recursive images (at the 1e-5 level on 0..255 data), so
the chosen shape is returned with the plan: single calls made under the same
tuning override give the same bits.
"""
import hashlib
import json
import os

import torch

from . import (FIR_MAX_RADIUS, BatchPlan, get_fir_crossover_table, gp_forward, resolve_spatial,
               set_fir_crossover_table, set_iir_tuning, workspace)

# (H, W) ladder; each entry covers images up to its pixel count
SIZES = ((256, 256), (512, 512), (1024, 1024), (2048, 2048), (4096, 4096))
CACHE_ENV = "BFGP_TUNE_CACHE"


def cache_path():
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "bfgp", "crossover.json")


def _key(device, N):
    # architecture and compute-unit count identify the device class (the
    # marketing name is not always reported, e.g. under a profiler)
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", "") or props.name
    return f"{arch}|{props.multi_processor_count}CU|N={N}"


def _time_ms(fn, reps, warmup=2):
    for _ in range(warmup):
        fn()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        start.record()
        fn()
        end.record()
        end.synchronize()
        times.append(start.elapsed_time(end))
    times.sort()
    return times[len(times) // 2]


def crossover_for_size(H, W, N=20, sigma_r=30.0, reps=7, device="cuda"):
    """Largest FIR radius (0..FIR_MAX_RADIUS) whose forward is faster than the
    recursive forward on an H x W image, with both timings."""
    gen = torch.Generator(device=device).manual_seed(H * 7919 + W)
    img = torch.rand((H, W), generator=gen, device=device) * 255.0
    out = torch.empty_like(img)
    ws_iir = workspace(H, W, N, 10.0, "iir", device=device)
    t_iir = _time_ms(lambda: gp_forward(img, 10.0, sigma_r, N, spatial="iir", out=out, ws=ws_iir), reps)
    ws_fir = workspace(H, W, N, 1.0, "fir", device=device)
    timed = {}

    def fir_ms(r):
        if r not in timed:
            ss = r / 3.0  # ceil(3 sigma_s) = r
            timed[r] = _time_ms(lambda: gp_forward(img, ss, sigma_r, N, spatial="fir", out=out, ws=ws_fir), reps)
        return timed[r]

    lo, hi = 0, FIR_MAX_RADIUS  # invariant: FIR faster at lo (radius 0 = never FIR), not known at hi
    if fir_ms(hi) < t_iir:
        lo = hi
    else:
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if fir_ms(mid) < t_iir:
                lo = mid
            else:
                hi = mid
    return lo, t_iir, dict(sorted(timed.items()))


def tune(N=20, sizes=SIZES, sigma_r=30.0, reps=7, device="cuda", save=True, log=None):
    """Measures the crossover for every size, installs the table, caches it,
    and returns {"table": [(max_pixels, radius), ...], "detail": {...}}."""
    table, detail = [], {}
    for H, W in sizes:
        r, t_iir, fir = crossover_for_size(H, W, N, sigma_r, reps, device)
        table.append((H * W, r))
        detail[f"{H}x{W}"] = {"radius": r, "iir_ms": t_iir, "fir_ms": {str(k): v for k, v in fir.items()}}
        if log:
            log(f"crossover {H}x{W}: FIR up to radius {r} (IIR {t_iir:.3f} ms)")
    set_fir_crossover_table(table)
    result = {"table": table, "detail": detail}
    if save:
        path = cache_path()
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            cache = {}
            if os.path.exists(path):
                with open(path) as f:
                    cache = json.load(f)
            cache[_key(device, N)] = result
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return result


def load(N=20, device="cuda"):
    """Installs the cached table for this device and degree; returns it, or
    None when there is none."""
    path = cache_path()
    try:
        with open(path) as f:
            entry = json.load(f).get(_key(device, N))
    except (OSError, ValueError):
        return None
    if not entry:
        return None
    table = [(int(a), int(b)) for a, b in entry["table"]]
    set_fir_crossover_table(table)
    return table


def ensure(N=20, device="cuda", log=None):
    """The cached table, or a fresh tuning run when there is none."""
    table = load(N, device)
    if table is None:
        table = tune(N, device=device, log=log)["table"]
    return get_fir_crossover_table() if table is not None else None


# candidate launch shapes of a batch plan's recursive images: (band rows,
# column channel groups, row channel groups), as set_iir_tuning takes them
BATCH_SHAPES = ((32, 1, 1), (64, 1, 1), (32, 2, 2))


def _batch_key(device, imgs, sigmas_s, N, spatial):
    comp = sorted((int(x.shape[0]), int(x.shape[1]), resolve_spatial(float(s), spatial, shape=tuple(x.shape)))
                  for x, s in zip(imgs, sigmas_s))
    digest = hashlib.sha1(json.dumps(comp).encode()).hexdigest()[:16]
    return f"{_key(device, N)}|batch|{digest}"


def _plan_with(shape, imgs, sigmas_s, sigmas_r, N, spatial):
    # the plan takes its launch shapes when it is made; the process-wide
    # tuning override is cleared afterwards
    set_iir_tuning(*shape)
    try:
        return BatchPlan(imgs, sigmas_s, sigmas_r, N, spatial=spatial)
    finally:
        set_iir_tuning(0, 0, 0)


def tune_batch(imgs, sigmas_s, sigmas_r, N=20, spatial="auto", shapes=BATCH_SHAPES, reps=5, save=True, log=None):
    """Times one plan of the batch per candidate shape (graph replays, median
    of `reps`), caches the fastest and returns (plan, shape, {shape: ms})."""
    device = imgs[0].device
    best, timings = None, {}
    for shape in shapes:
        plan = _plan_with(shape, imgs, sigmas_s, sigmas_r, N, spatial)
        plan.run()
        g = plan.graph()
        timings[tuple(shape)] = _time_ms(g.replay, reps)
        if log:
            log(f"batch plan shape {tuple(shape)}: {timings[tuple(shape)]:.3f} ms")
        if best is None or timings[tuple(shape)] < timings[best[1]]:
            best = (plan, tuple(shape))
        del g
    if save:
        path = cache_path()
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            cache = {}
            if os.path.exists(path):
                with open(path) as f:
                    cache = json.load(f)
            cache[_batch_key(device, imgs, sigmas_s, N, spatial)] = {
                "shape": list(best[1]), "ms": {",".join(map(str, k)): v for k, v in timings.items()}}
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return best[0], best[1], timings


def plan_batch(imgs, sigmas_s, sigmas_r, N=20, spatial="auto", log=None):
    """A BatchPlan built with the cached launch shape for this batch's
    composition, tuned (tune_batch) when there is none; returns (plan,
    shape)."""
    device = imgs[0].device
    try:
        with open(cache_path()) as f:
            entry = json.load(f).get(_batch_key(device, imgs, sigmas_s, N, spatial))
    except (OSError, ValueError):
        entry = None
    if entry:
        shape = tuple(int(v) for v in entry["shape"])
        return _plan_with(shape, imgs, sigmas_s, sigmas_r, N, spatial), shape
    plan, shape, _ = tune_batch(imgs, sigmas_s, sigmas_r, N, spatial, log=log)
    return plan, shape
