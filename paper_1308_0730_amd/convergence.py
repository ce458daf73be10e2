"""Convergence of the update schemes and variants against a known ground truth.

The paper compares how fast the derivations reach the same reconstruction
quality: the classic multi-view methods with combined updates (ML-EM with the
arithmetic mean, the Bayesian-based derivation of eq. 50/51 with the
geometric mean), the efficient variant and Optimizations I and II (eq. 220,
230, 240), each with combined or sequential (OS-EM) updates (main figure 1d-f,
the section on benchmarks).  This module measures the same on a synthetic
problem with its ground truth: every method runs one iteration at a time on
the GPU until its estimate is within a target distance of the truth.

Reported per method: iterations, updates of psi (one per iteration for the
combined schemes, one per view for the sequential one) and the device time of
those iterations (events on the stream the library launches on; the distance
evaluation between iterations is outside the timed spans).

The distance is the relative L2 error ||psi - truth|| / ||truth||.  Unless a
target is given, it is the distance that classic ML-EM (combined, arithmetic
mean, mirrored PSFs) reaches after `ref_iters` iterations, i.e. "the quality
ML-EM reaches in that many iterations", which every faster method reaches
first.
"""
from __future__ import annotations

import numpy as np
import torch

from . import mvd

# (scheme, variant); scheme "sequential" or "combined-<mean>"
METHODS = (
    ("combined-arithmetic", "rl"),   # ML-EM
    ("combined-geometric", "rl"),    # Bayesian-based, eq. 50/51
    ("combined-geometric", "eff"),
    ("combined-geometric", "opt1"),
    ("combined-geometric", "opt2"),
    ("sequential", "rl"),            # OS-EM
    ("sequential", "eff"),
    ("sequential", "opt1"),
    ("sequential", "opt2"),
)


def _distance(psi, truth, tnorm):
    return float(torch.linalg.vector_norm(psi - truth) / tnorm)


def _step(d, scheme, variant):
    if scheme == "sequential":
        d.iterate(1, variant)
    else:
        d.iterate_combined(1, variant, scheme.split("-", 1)[1])


def trace(d, truth, scheme, variant, n_iter, stop_at=None):
    """Run up to n_iter iterations from the flat start; return the distance
    after every iteration and the device time of each iteration (ms).  Stops
    after the first iteration within stop_at when it is given."""
    t = torch.as_tensor(truth, device=d.device, dtype=torch.float32)
    tnorm = torch.linalg.vector_norm(t)
    flat = torch.full_like(t, float(d.stats()["scale"]))
    d.set_estimate(flat)
    dist, ms = [], []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(n_iter):
        e0.record(d.stream)
        _step(d, scheme, variant)
        e1.record(d.stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
        dist.append(_distance(d.estimate(), t, tnorm))
        if stop_at is not None and dist[-1] <= stop_at:
            break
    return dist, ms


def compare(problem, methods=METHODS, target=None, ref_iters=100, max_iter=400, lam=0.0):
    """Iterations, updates and device time each method needs to come within
    `target` of the ground truth (see the module docstring for the default)."""
    s = problem
    n = len(s.views)
    with mvd.Deconvolver(s.views, s.psfs, lam=lam) as d:
        for scheme, variant in methods:  # build every kernel set and graph outside the timing
            _step(d, scheme, variant)
        if target is None:
            dist, _ = trace(d, s.truth, "combined-arithmetic", "rl", ref_iters)
            target = dist[-1]
        rows = []
        for scheme, variant in methods:
            dist, ms = trace(d, s.truth, scheme, variant, max_iter, stop_at=target)
            hit = dist[-1] <= target
            it = len(dist) if hit else None
            rows.append({
                "scheme": scheme, "variant": variant, "iterations": it,
                "updates": None if it is None else (it * n if scheme == "sequential" else it),
                "ms": None if it is None else round(sum(ms), 3),
                "best_distance": round(min(dist), 5),
            })
    return {"target_distance": round(target, 5), "views": n, "dims": list(s.dims), "methods": rows}


def sweep(make, lams=(0.0, 0.0006, 0.006, 0.06), noises=("none", "photons"), scheme="sequential",
          variant="opt1", n_iter=60):
    """Best distance to the truth and the iteration where it is reached, per
    noise model and Tikhonov weight (the paper's noise and regularisation
    study).  `make(noise)` returns a synthetic problem."""
    out = []
    for noise in noises:
        s = make(noise)
        for lam in lams:
            with mvd.Deconvolver(s.views, s.psfs, lam=lam) as d:
                dist, _ = trace(d, s.truth, scheme, variant, n_iter)
            k = int(np.argmin(dist))
            out.append({"noise": noise, "lambda": lam, "best_distance": round(dist[k], 5),
                        "at_iteration": k + 1, "final_distance": round(dist[-1], 5)})
    return out
