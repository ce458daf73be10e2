"""Autotuner of the pass launch shapes.

For each pass kind (x rows, y columns, z columns) every launch-shape
candidate that holds the handle's longest transform is timed with the
library's per-launch HIP-event profiler, one kind at a time with the other
two held at their current choice; the fastest stays selected.  Results are
cached in a JSON file keyed by GPU architecture, volume dims, view count and
variant.
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
    d.set_tiles(*best)
    if cache_path:
        cache[key] = {"tiles": best, "timings": timings}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return tuple(best), timings
