"""Autotuner for the launch-shape knobs of a context.

Every knob setting computes bit-identical results (the knobs change how
many residues a thread holds and how work items map to XCDs, never the
arithmetic), so tuning is a pure timing search: each candidate setting runs
the caller's workload a few times, timed with HIP events on the context's
stream, and the fastest setting is kept. Results are cached in a JSON file
keyed by device name, ring degree, chain shape and workload name, so a
server tunes once per configuration.
"""
import itertools
import json
import os

import torch

DEFAULT_SPACE = {"ntt_wide": (0, 1), "ew_log": (1, 2, 3), "xcd_remap": (0, 1), "fuse_tail": (0, 1), "ip_cts": (2, 4, 16),
                 "ntt_fp": (0, 1)}


def _key(ctx, workload):
    props = torch.cuda.get_device_properties(ctx.device)
    dev = getattr(props, "gcnArchName", "") or props.name or "device"
    dev = dev.split(":")[0]
    return "%s|N=2^%d|q=%d|p=%d|dnum=%d|%s" % (dev, ctx.log_n, len(ctx.q), len(ctx.p), ctx.dnum, workload)


def candidates(ctx, space=None):
    space = dict(space or DEFAULT_SPACE)
    if ctx.log_n < 11 or ctx.log_n > 14:
        space["ntt_wide"] = (0,)
    names = sorted(space)
    for vals in itertools.product(*(space[n] for n in names)):
        yield dict(zip(names, vals))


def time_setting(ctx, fn, setting, reps=5, warmup=1):
    """Mean milliseconds of ``fn()`` under ``setting`` (HIP events on the context's stream)."""
    old = ctx.tuning()
    ctx.set_tuning(**setting)
    try:
        for _ in range(warmup):
            fn()
        s = torch.cuda.current_stream(ctx.device)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps
    finally:
        ctx.set_tuning(**old)


def autotune(ctx, fn, workload, cache=None, space=None, reps=5):
    """Pick the fastest knob setting for ``fn`` on ``ctx`` and apply it.

    Returns ``(setting, {setting_string: ms})``; the timings dict is empty
    when the setting came from the cache."""
    key = _key(ctx, workload)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            ctx.set_tuning(**table[key]["setting"])
            return table[key]["setting"], {}
    times = {}
    best, best_ms = None, float("inf")
    for st in candidates(ctx, space):
        ms = time_setting(ctx, fn, st, reps=reps)
        times[json.dumps(st, sort_keys=True)] = ms
        if ms < best_ms:
            best, best_ms = st, ms
    ctx.set_tuning(**best)
    if cache:
        table[key] = {"setting": best, "ms": best_ms}
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return best, times
