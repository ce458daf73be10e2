"""Autotuner of the pass launch shapes.

For each pass kind (x rows, y columns, z columns) every launch-shape
candidate that holds the handle's longest transform is timed with the
library's per-launch HIP-event profiler, one kind at a time with the other
two held at their current choice; the fastest stays selected.  A handle of
several blocks then times whole runs (`runs` iterations) with that choice
against the per-length plans for all three kinds under each schedule (pass
major, block major, run major: with the per-length plans each block lane
runs its blocks without joining the other lanes after every pass, and the
block-major schedules keep a few blocks in the memory-side cache from pass
to pass, gains the per-pass profile cannot see), and keeps the fastest.
The estimates are restored afterwards.  Results are cached in a JSON file keyed by GPU
architecture, volume dims, view count and variant.
"""
from __future__ import annotations

import json
import os
import sys

import torch

from . import mvd

KIND_PASSES = {0: ("x_ratio", "x_update"), 1: ("y_forward", "y_inverse"), 2: ("z_product",)}
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mvd_tiles.json")


def _key(d, variant):
    arch = torch.cuda.get_device_properties(d.device).gcnArchName.split(":")[0]
    return f"{arch}|{sorted(d.dims)}|{d.n_views}|{mvd._variant(variant)}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def autotune(d, variant="eff", iters=1, cache_path=DEFAULT_CACHE, use_cache=True, verbose=False, runs=1):
    """Select the fastest launch shapes (and, for several blocks, schedule)
    for handle d; returns (x, y, z) and the per-candidate timings (ms per
    launch of the kind's passes; ms per run of `runs` iterations)."""
    key = _key(d, variant)
    cache = _load(cache_path) if cache_path else {}
    if use_cache and key in cache:
        d.set_tiles(*cache[key]["tiles"])
        d.set_schedule(cache[key].get("schedule", "pass"))
        return tuple(cache[key]["tiles"]), cache[key].get("timings", {})
    d.set_schedule("pass")
    lens = d.max_lengths()
    best = list(d.tiles())
    timings = {}
    saved = [d.estimate(b).clone() for b in range(len(d.dims))]
    d.profile(1, variant)  # warm: compound spectra, first touch
    for kind in (2, 1, 0):
        res = {}
        for c in mvd.tile_candidates(kind, lens[kind]):
            cfg = list(best)
            cfg[kind] = c
            try:
                d.set_tiles(*cfg)
            except mvd.MVDError:
                continue  # a compile-time plan whose length not every block has
            prof = d.profile(iters, variant)
            res[c] = sum(prof[p][0] for p in KIND_PASSES[kind])
            if verbose:
                print(f"[tune] kind {kind} candidate {c} {mvd.tile_shape(kind, c)}: {res[c]:.4f} ms", file=sys.stderr,
                      flush=True)
        best[kind] = min(res, key=res.get)
        timings[str(kind)] = {str(c): t for c, t in res.items()}
    schedule = "pass"
    if len(d.dims) > 1:
        exact = [_per_length_candidate(k, lens[k]) for k in range(3)]
        if None not in exact:
            trials = [(best, "pass")] if exact != best else []
            trials += [(exact, sch) for sch in ("pass", "block", "run")]
            res = {}
            for tiles, sch in trials:
                res[(tuple(tiles), sch)] = _run_ms(d, tiles, sch, variant, runs)
                if verbose:
                    print(f"[tune] whole run of {runs}: tiles {tiles} schedule {sch}: "
                          f"{res[(tuple(tiles), sch)]:.4f} ms", file=sys.stderr, flush=True)
            (tiles, schedule) = min(res, key=res.get)
            best = list(tiles)
            timings["run"] = {f"{list(t)}/{sch}": ms for (t, sch), ms in res.items()}
    d.set_tiles(*best)
    d.set_schedule(schedule)
    for b, e in enumerate(saved):
        d.set_estimate(e, b)
    if cache_path:
        cache[key] = {"tiles": best, "schedule": schedule, "timings": timings}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return tuple(best), timings


def _per_length_candidate(kind, max_len):
    for c in mvd.tile_candidates(kind, max_len):
        if mvd.tile_shape(kind, c)["exact_len"] < 0:
            return c
    return None


def _run_ms(d, tiles, schedule, variant, runs, reps=2):
    """Device time of a run of `runs` iterations (graph replay) with the
    given shapes and schedule."""
    d.set_tiles(*tiles)
    d.set_schedule(schedule)
    d.iterate(runs, variant)  # builds the graphs
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(d.stream)
    for _ in range(reps):
        d.iterate(runs, variant)
    e1.record(d.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps
