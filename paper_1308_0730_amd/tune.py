"""Autotuner of the pass launch shapes.

For each pass kind (x rows, y columns, z columns) every launch-shape
candidate that holds the handle's longest transform is timed with the
library's per-launch HIP-event profiler, one kind at a time with the other
two held at their current choice; the fastest stays selected.  A handle of
several blocks then times whole iterations with that choice against the
per-length plans for all three kinds, which alone let each block lane run
its view-updates without joining the other lanes after every pass (a gain
the per-pass profile cannot see), and keeps the faster.  The estimates are
restored afterwards.  Results are cached in a JSON file keyed by GPU
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


def autotune(d, variant="eff", iters=1, cache_path=DEFAULT_CACHE, use_cache=True, verbose=False):
    """Select the fastest launch shapes for handle d; returns (x, y, z) and
    the per-candidate timings (ms per launch of the kind's passes)."""
    key = _key(d, variant)
    cache = _load(cache_path) if cache_path else {}
    if use_cache and key in cache:
        d.set_tiles(*cache[key]["tiles"])
        return tuple(cache[key]["tiles"]), cache[key].get("timings", {})
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
    if len(d.dims) > 1:
        exact = [_per_length_candidate(k, lens[k]) for k in range(3)]
        if None not in exact and exact != best:
            t_best = _iteration_ms(d, best, variant)
            t_exact = _iteration_ms(d, exact, variant)
            timings["iteration"] = {"tuned": t_best, "per_length": t_exact}
            if verbose:
                print(f"[tune] whole iteration: {best} {t_best:.4f} ms, per-length {exact} {t_exact:.4f} ms",
                      file=sys.stderr, flush=True)
            if t_exact < t_best:
                best = exact
    d.set_tiles(*best)
    for b, e in enumerate(saved):
        d.set_estimate(e, b)
    if cache_path:
        cache[key] = {"tiles": best, "timings": timings}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return tuple(best), timings


def _per_length_candidate(kind, max_len):
    for c in mvd.tile_candidates(kind, max_len):
        if mvd.tile_shape(kind, c)["exact_len"] < 0:
            return c
    return None


def _iteration_ms(d, tiles, variant, reps=2):
    """Device time of one iteration (graph replay) with the given shapes."""
    d.set_tiles(*tiles)
    d.iterate(1, variant)  # builds the graph
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(d.stream)
    d.iterate(reps, variant)
    e1.record(d.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps
