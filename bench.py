#!/usr/bin/env python3
"""Throughput of the sequential multi-view deconvolution on one MI355X.

A step is one whole deconvolution run of the workload (every iteration, every
view-update) on inputs already resident in HBM.  Default workload: the
embryo-scale volume, 512x512x256 float32, six views at 60-degree steps,
31x31x41 PSFs, per-view overlap weights, lambda = 0.0006, Optimization I,
10 iterations (60 view-updates).

Prints one JSON line: voxel-view updates/s over the timed steps, the
roofline position of the dominant pass (per-launch HIP-event durations,
algorithmic bytes; against the vendor peak and against the runtime's device
copy measured in the same run), and the FP64 CPU oracle timed on a bounded
sample on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
PASS_NAMES = ("y_forward", "y_inverse", "z_product", "x_ratio", "x_update")
KERNEL_SOURCES = tuple("paper_1308_0730_amd/csrc/" + f for f in (
    "mvd_kernels.hip", "mvd_kernels_ct.hip", "mvd_ct_passes.h", "mvd_exact_x.hip", "mvd_exact_x_comb.hip",
    "mvd_exact_x_win.hip",
    "mvd_exact_class.hip",
    "mvd_exact_y.hip", "mvd_exact_z.hip", "mvd_exact_lengths.h", "fft_engine.h", "fft_ct.h", "mvd_device.h",
    "mvd_gmem.h", "mvd_types.h", "fft_small_tw.h"))


def workload(cfg):
    from paper_1308_0730_amd import synth
    if cfg == 1:
        s = synth.config1()
        return [s], dict(workload="tiny 64^3, 2 views, 17^3 PSFs, efficient update, 5 iterations",
                         variant="eff", iterations=5, lam=0.0)
    if cfg == 2:
        s = synth.config2()
        return [s], dict(workload="128^3, 4 views, 25^3 PSFs, efficient update, 20 iterations",
                         variant="eff", iterations=20, lam=0.0)
    if cfg == 3:
        s = synth.config3()
        return [s], dict(workload="embryo 512x512x256, 6 views at 60 deg, 31x31x41 PSFs, overlap weights, "
                                  "lambda 0.0006, Optimization I, 10 iterations",
                         variant="opt1", iterations=10, lam=0.0006)
    if cfg == 4:
        blocks = synth.config4()
        return blocks, dict(workload="batched: 48 blocks (x,y in [96,256], z in [96,160]), 4 views, 17^3 PSFs, "
                                     "efficient update, 10 iterations",
                            variant="eff", iterations=10, lam=0.0)
    raise SystemExit(f"unknown config {cfg}")


def workload_shapes(cfg):
    """(dims, PSF shapes (kz, ky, kx), weighted) of every block of a
    workload, without rendering it."""
    from paper_1308_0730_amd import synth
    if cfg == 1:
        return [((64, 64, 64), [(17, 17, 17)] * 2)], False
    if cfg == 2:
        return [((128, 128, 128), [(25, 25, 25)] * 4)], False
    if cfg == 3:
        return [((512, 512, 256), [(41, 31, 31)] * 6)], True
    if cfg == 4:
        dims, _ = synth.config4_dims()
        return [(d, [(17, 17, 17)] * 4) for d in dims], False
    raise SystemExit(f"unknown config {cfg}")


def pass_bytes(blocks, weighted):
    """Algorithmic HBM bytes of one launch of each pass kind (all blocks);
    blocks: workload blocks, or (dims, PSF shapes) pairs."""
    out = dict.fromkeys(PASS_NAMES, 0.0)
    for b in blocks:
        dims, shapes = (b.dims, [p.shape for p in b.psfs]) if hasattr(b, "dims") else b
        nx, ny, nz = dims
        V = nx * ny * nz
        S = ((nx // 2) * ny * nz + ny * nz) * 8.0  # half spectrum, complex float32
        # kernel planes: x/y-stage spectrum on the common odd z window
        kz = max(sh[0] | 1 for sh in shapes)
        Hk = ((nx // 2) * ny * kz + ny * kz) * 8.0
        out["y_forward"] += 2 * S
        out["y_inverse"] += 2 * S
        out["z_product"] += 2 * S + Hk
        out["x_ratio"] += 2 * S + 4 * V
        out["x_update"] += 2 * S + (12 if weighted else 8) * V
    return out


def parse_tiles(d, spec):
    """Launch shapes from 'x,y,z': a candidate index per pass kind, or p for
    the per-length compile-time plans of that kind."""
    from paper_1308_0730_amd import mvd
    lens = d.max_lengths()
    out = []
    for kind, f in enumerate(spec.split(",")):
        if f.strip() == "p":
            c = [c for c in mvd.tile_candidates(kind, lens[kind]) if mvd.tile_shape(kind, c)["exact_len"] < 0]
            if not c:
                raise SystemExit(f"no per-length plan for pass kind {kind}")
            out.append(c[0])
        else:
            out.append(int(f))
    return out


def source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(name, kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{name}.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_hash:\s*(\w+)", txt)
    if not m or m.group(1) != source_hash():
        return None
    m = re.search(rf"^{kernel}:\s*([0-9.eE+]+)\s*bytes_per_launch", txt, re.M)
    return float(m.group(1)) if m else None


# ---- rocprofv3 summaries (the text files under profiles/) -----------------

def _csv_rows(d, suffix):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    return rows


def pass_of_kernel(name):
    """The pass kind a library kernel implements (None for other kernels)."""
    m = re.search(r"k_(ypass|zconv|xpass)(?:_ct|_class)?<(\w+)", name)
    if not m:
        return None
    kind, arg = m.group(1), m.group(2)
    if kind == "ypass":
        return "y_inverse" if arg == "true" else "y_forward"
    if kind == "zconv":
        return "z_product"
    # modes 8 and 10: the block-wise form's forward and update passes
    return {"0": "x_forward", "1": "x_ratio", "2": "x_update", "8": "x_forward", "10": "x_update"}.get(arg)


def _short(name, n=150):
    name = re.sub(r"\(.*\)$", "", name)
    name = re.sub(r"((?:mvdk::)?ColPlan<[^>]*>, )+(?:mvdk::)?ColPlan<[^>]*>", "ColPlan<L>...", name)
    return name if len(name) <= n else name[:n] + "..."


def summarize_kernel_trace(d, title, command, top=20):
    """Kernel statistics (name, calls, total, average, percent) and the
    launch resources of the listed kernels, from a --kernel-trace --stats
    run."""
    stats = _csv_rows(d, "kernel_stats.csv")
    trace = _csv_rows(d, "kernel_trace.csv")
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in stats) / 1e6
    lines = [f"# rocprofv3 kernel statistics: {title}", f"# command: {command}",
             f"# source_hash: {source_hash()}", "# name | calls | total_ms | average_us | percent"]
    for r in stats[:top]:
        lines.append(f"{_short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f}")
    if len(stats) > top:
        lines.append(f"# ... {len(stats) - top} more kernels; all kernels total {total:.2f} ms")
    lines.append("# resources of the kernels above: name | grid | workgroup | vgpr | lds_bytes | scratch_bytes")
    seen = set()
    names = {r["Name"] for r in stats[:top]}
    for r in trace:
        n = r["Kernel_Name"]
        if n in names and n not in seen:
            seen.add(n)
            lines.append(f"{_short(n)} | {r['Grid_Size_X']} | {r['Workgroup_Size_X']} | {r['VGPR_Count']} | "
                         f"{r['LDS_Block_Size']} | {r['Scratch_Size']}")
    return "\n".join(lines)


def summarize_sq_counters(d, title, command, top=20):
    """Per-launch averages of the SQ counters of a rocprofv3 --pmc run (CSV)
    for the kernels with the most vector instructions; issue shares against
    the chip's vector rate are left to the reader (one wave instruction
    covers 64 lanes; a SIMD issues one every 4 cycles)."""
    rows = _csv_rows(d, "counter_collection.csv")
    agg, n, names = {}, {}, []
    for r in rows:
        k, c = r["Kernel_Name"], r["Counter_Name"]
        if k not in agg:
            agg[k], n[k] = {}, {}
            names.append(k)
        agg[k][c] = agg[k].get(c, 0.0) + float(r["Counter_Value"])
        n[k][c] = n[k].get(c, 0) + 1
    counters = sorted({c for k in agg for c in agg[k]})
    key = "SQ_INSTS_VALU" if "SQ_INSTS_VALU" in counters else counters[0]
    names = [k for k in names if pass_of_kernel(k)]
    names.sort(key=lambda k: -agg[k].get(key, 0.0))
    lines = [f"# rocprofv3 SQ counters per launch: {title}", f"# command: {command}",
             f"# source_hash: {source_hash()}", "# name | launches | " + " | ".join(counters)]
    for k in names[:top]:
        m = max(n[k].values())
        lines.append(f"{_short(k)} | {m} | " + " | ".join(f"{agg[k].get(c, 0.0) / n[k].get(c, 1):.4e}"
                                                          for c in counters))
    return "\n".join(lines)


def summarize_counters(fetch_dir, write_dir, cfg, iterations, title, commands):
    """HBM bytes per pass launch (one pass over every block) from a
    FETCH_SIZE run and a WRITE_SIZE run, each scaled by what the counter
    reads for the 1 GiB device copy of --copy-calibration; iterations: the
    iterations the profiled command ran (a pass launch count per kind)."""
    shapes, weighted = workload_shapes(cfg)
    views = len(shapes[0][1])
    alg = pass_bytes(shapes, weighted)
    per_vu = {"y_forward": 2, "y_inverse": 2, "z_product": 2, "x_ratio": 1, "x_update": 1}
    tot, cal, kern = {}, {}, {}
    for cname, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _csv_rows(d, "counter_collection.csv") if r["Counter_Name"] == cname]
        cal[cname] = max(float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"])
        acc = dict.fromkeys(PASS_NAMES, 0.0)
        for r in rows:
            k = pass_of_kernel(r["Kernel_Name"])
            if k in acc:
                acc[k] += float(r["Counter_Value"])
                kern.setdefault(k, set()).add(_short(r["Kernel_Name"], 80))
        tot[cname] = acc
    f_fac = (1 << 20) / cal["FETCH_SIZE"]
    w_fac = (1 << 20) / cal["WRITE_SIZE"]
    lines = [f"# HBM traffic per launch from rocprofv3 counters: {title}",
             "# commands (two passes, one counter each):"] + [f"#   {c}" for c in commands] + [
             f"# calibration: a 1 GiB device copy reads FETCH_SIZE = {cal['FETCH_SIZE']:.0f} KiB and "
             f"WRITE_SIZE = {cal['WRITE_SIZE']:.0f} KiB,",
             f"#   so fetch bytes = FETCH_SIZE * 1024 * {f_fac:.4f} and write bytes = WRITE_SIZE * 1024 * {w_fac:.4f}",
             f"# a launch is one pass over every block; launches = {iterations} iterations x {views} views x "
             "passes of the kind per view-update",
             f"source_hash: {source_hash()}",
             "# pass: measured_bytes_per_launch | fetch_bytes | write_bytes | algorithmic_bytes | launches | kernels"]
    for k in PASS_NAMES:
        n = iterations * views * per_vu[k]
        fb = tot["FETCH_SIZE"][k] * 1024 * f_fac / n
        wb = tot["WRITE_SIZE"][k] * 1024 * w_fac / n
        ks = sorted(kern.get(k, ()))
        kdesc = ks[0] if len(ks) == 1 else f"{len(ks)} kernels"
        lines.append(f"{k}: {fb + wb:.4e} bytes_per_launch | {fb:.4e} | {wb:.4e} | {alg[k]:.4e} | {n} | {kdesc}")
    return "\n".join(lines)


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Read + write GB/s of the runtime's device-to-device copy of nbytes,
    best of reps (HIP events): the practical streaming ceiling measured on
    the same GPU in the same run, beside the vendor peak."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    st = torch.cuda.current_stream()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        b.copy_(a)
        e1.record(st)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (best / 1e3) / 1e9


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(blocks, meta, budget_s=60.0):
    """The FP64 oracle on this host: the view-updates of the same workload
    (the whole run, or as many as fit in about budget_s), scaled to
    voxel-view updates per second."""
    from oracle import mvd_oracle as O
    s = blocks[0]
    pb = O.Problem(s.views, s.psfs, s.weights, meta["lam"])
    variant = {"rl": O.RL, "eff": O.EFF, "opt1": O.OPT1, "opt2": O.OPT2}[meta["variant"]]
    K = pb.kernels(variant)
    psi = pb.psi0()
    V = int(np.prod(s.dims))
    n = 0
    t0 = time.perf_counter()
    while True:
        v = n % pb.n
        w = None if pb.weights is None else pb.weights[v]
        psi = O.view_update(psi, pb.views[v], pb.P[v], K[v], w, pb.lam_p, pb.eps)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= pb.n * meta["iterations"]:
            break
    return {"value": V * n / el / 1e9, "unit": "Gvox/s", "cores": os.cpu_count(), "cpu_model": cpu_model(),
            "kind": "oracle",
            "sample": f"{n} of the run's {pb.n * meta['iterations']} view-updates of block 0 of the same "
                      f"workload in FP64 (scipy.fft, all host cores), {el:.1f} s"}


def batched_form(steps, warmup):
    """The 48-block batched workload: one handle for all blocks (every pass of
    an iteration one launch over all blocks, one HIP graph per iteration)
    against the same blocks looped through one plain handle each."""
    import torch
    from paper_1308_0730_amd import mvd, tune
    t0 = time.time()
    blocks, meta = workload(4)
    print(f"[bench] batched workload generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    its, var = meta["iterations"], meta["variant"]
    vox = sum(int(np.prod(b.dims)) for b in blocks) * len(blocks[0].views) * its
    b = mvd.Deconvolver.batch([(x.views, x.psfs, x.weights) for x in blocks])
    b.iterate(1, var)
    tune.autotune(b, var, iters=1, cache_path=None, runs=its)
    for _ in range(warmup):
        b.iterate(its, var)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    for _ in range(steps):
        b.iterate(its, var)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1) / steps
    tiles = b.tiles()
    schedule = b.schedule()
    # per-pass timings of one pass-major iteration (HIP events around each
    # pass over all blocks)
    prof = b.profile(1, var)
    by = pass_bytes(blocks, False)
    run_bytes = sum(by[k] * prof[k][1] for k in PASS_NAMES) * its  # the profile ran one iteration
    # the timed run's roofline: with the run-major schedule the lanes run
    # different passes at once, so no pass has a launch time of its own; the
    # run's algorithmic bytes over its time instead, and the measured bytes
    # of every pass (counter summary) summed the same way
    ach = run_bytes / (ms_b / 1e3) / 1e9
    meas = [measured_traffic("batched48", k) for k in PASS_NAMES]
    traffic = (sum(m * prof[k][1] for m, k in zip(meas, PASS_NAMES)) * its
               if all(m is not None for m in meas) else None)
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "all passes",
            "bytes_per_run": run_bytes, "run_ms": round(ms_b, 3),
            "note": "the timed run's algorithmic bytes over its time (concurrent lanes)"}
    dom = max(PASS_NAMES, key=lambda k: prof[k][0] * prof[k][1])
    pass_major = {k: {"avg_ms": round(prof[k][0], 5), "GBps": round(by[k] / (prof[k][0] / 1e3) / 1e9, 1)}
                  for k in PASS_NAMES}
    b.close()
    del b
    plains = [mvd.Deconvolver(x.views, x.psfs, x.weights) for x in blocks]
    for d in plains:
        d.iterate(1, var)
    torch.cuda.synchronize()
    for _ in range(warmup):
        for d in plains:
            d.iterate(its, var)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        for d in plains:
            d.iterate(its, var)
    e1.record()
    torch.cuda.synchronize()
    ms_p = e0.elapsed_time(e1) / steps
    for d in plains:
        d.close()
    return {"workload": meta["workload"], "blocks": len(blocks), "voxel_view_updates_per_step": vox,
            "batched": {"ms_per_step": round(ms_b, 3), "value": round(vox / ms_b / 1e6, 3), "unit": "Gvox/s",
                        "tiles": list(tiles), "schedule": schedule,
                        "algorithmic_GBps": round(run_bytes / (ms_b / 1e3) / 1e9, 1)},
            "roofline": roof, "pass_major_profile": {"dominant": dom, "passes": pass_major},
            "plain_loop": {"ms_per_step": round(ms_p, 3), "value": round(vox / ms_p / 1e6, 3), "unit": "Gvox/s"},
            "batched_speedup": round(ms_p / ms_b, 3)}


def grad_form(steps, warmup):
    """The differentiated workload (128^3, four views, 25^3 PSFs, 8 RL
    iterations): forward (iterations + loss) against forward + backward
    (checkpointed recompute and adjoint passes, PSF and psi0 gradients)."""
    import torch
    from paper_1308_0730_amd import mvd
    s = synth_config5()
    its = 8
    vox = int(np.prod(s.dims)) * len(s.views) * its
    d = mvd.Deconvolver(s.views, s.psfs)
    res = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for name, grads in (("forward", False), ("forward_backward", True)):
        for _ in range(warmup):
            d.loss_grad(its, None, grad_psf=grads, grad_psi0=grads)
        e0.record(d.stream)
        for _ in range(steps):
            loss, _, _ = d.loss_grad(its, None, grad_psf=grads, grad_psi0=grads)
        e1.record(d.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[name] = {"ms_per_step": round(ms, 3), "value": round(vox / ms / 1e6, 3), "unit": "Gvox/s",
                     "loss": loss}
    # the layer form (autograd's MVDDeconvolve): a recorded forward returning
    # psi_n, then the vector-Jacobian product of a seed over that record
    seed = torch.ones(s.views[0].shape, dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        _, tok = d.forward_recorded(its)
        d.backward_recorded(tok, seed)
    e0.record(d.stream)
    for _ in range(steps):
        _, tok = d.forward_recorded(its)
        d.backward_recorded(tok, seed)
    e1.record(d.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    res["layer_forward_backward"] = {"ms_per_step": round(ms, 3), "value": round(vox / ms / 1e6, 3),
                                     "unit": "Gvox/s"}
    # the same loss and gradients through the efficient update (eq. 222):
    # the compound kernels' gradients go through their construction
    for _ in range(warmup):
        d.loss_grad(its, None, variant="eff")
    e0.record(d.stream)
    for _ in range(steps):
        loss, _, _ = d.loss_grad(its, None, variant="eff")
    e1.record(d.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    res["eff_forward_backward"] = {"ms_per_step": round(ms, 3), "value": round(vox / ms / 1e6, 3),
                                   "unit": "Gvox/s", "loss": loss}
    d.close()
    res["backward_over_forward"] = round(res["forward_backward"]["ms_per_step"] / res["forward"]["ms_per_step"], 3)
    res["workload"] = "128^3, 4 views, 25^3 PSFs, 8 RL iterations, loss sum_v |psi_8 (x) P_v - phi_v|^2"
    res["note"] = ("HIP events on the handle's stream around the calls (each call synchronises; the PSF "
                   "gradients' normalisation Jacobian runs on the host between device work)")
    return res


def convergence_form():
    """Iterations, updates and device time every scheme x variant needs to
    reach the same distance from the ground truth (the distance classic
    ML-EM has after 100 iterations) on the noise-free 128^3 four-view cube."""
    from paper_1308_0730_amd import convergence, synth
    s = synth.make_problem((128, 128, 128), 150, [0.0, 45.0, 90.0, 135.0], (25, 25, 25), 1.2, 4.0,
                           synth.SEED_BASE + 1, noise="none")
    r = convergence.compare(s, ref_iters=100, max_iter=400)
    r["workload"] = "128^3, 4 views at 45 deg, 25^3 PSFs, noise-free views, lambda 0, flat start"
    return r


def linear_form(steps, warmup):
    """The linear (padded) boundary at embryo scale: a 480x480x216 volume,
    six views, 31x31x41 PSFs, overlap weights, lambda 0.0006, OPT1, 10
    iterations, deconvolved on the volume plus the PSF radius on every side
    (a 512x512x256 grid, the plain workload's); value counts the volume's
    voxels, grid_value the grid's."""
    import torch
    from paper_1308_0730_amd import mvd, synth, tune
    t0 = time.time()
    s = synth.config3(dims=(480, 480, 216))
    print(f"[bench] linear workload generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    its, var, n = 10, "opt1", len(s.views)
    with mvd.Deconvolver(s.views, s.psfs, s.weights, lam=0.0006, boundary="linear") as d:
        d.iterate(1, var)  # compound kernels, graph
        tune.autotune(d, var, iters=1, cache_path=None)
        for _ in range(warmup):
            d.iterate(its, var)
        st = d.stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            d.iterate(its, var)
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / steps
        grid = d.grid_dims()
    vox = int(np.prod(s.dims)) * n * its
    gvox = int(np.prod(grid)) * n * its
    return {"workload": "linear boundary: 480x480x216, 6 views at 60 deg, 31x31x41 PSFs, overlap weights, "
                        "lambda 0.0006, Optimization I, 10 iterations",
            "grid": list(grid), "ms_per_step": round(ms, 3), "value": round(vox / (ms / 1e3) / 1e9, 3),
            "unit": "Gvox/s", "grid_value": round(gvox / (ms / 1e3) / 1e9, 3)}


def small_form(steps, warmup):
    """The two small plain workloads (cache-resident; the 64^3 one is
    launch-bound): 64^3 with two views, 5 iterations of the efficient update,
    and 128^3 with four views, 20 iterations."""
    import torch
    from paper_1308_0730_amd import mvd, tune
    out = {}
    for cfg, name in ((1, "tiny64"), (2, "cube128")):
        blocks, meta = workload(cfg)
        s = blocks[0]
        its, var = meta["iterations"], meta["variant"]
        with mvd.Deconvolver(s.views, s.psfs, s.weights, lam=meta["lam"]) as d:
            d.iterate(1, var)
            tune.autotune(d, var, iters=2, cache_path=None)
            for _ in range(warmup):
                d.iterate(its, var)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(d.stream)
            for _ in range(steps):
                d.iterate(its, var)
            e1.record(d.stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / steps
            vox = int(np.prod(s.dims)) * len(s.views) * its
            out[name] = {"workload": meta["workload"], "ms_per_step": round(ms, 4),
                         "value": round(vox / (ms / 1e3) / 1e9, 3), "unit": "Gvox/s",
                         "us_per_view_update": round(ms * 1e3 / (len(s.views) * its), 2), "tiles": list(d.tiles())}
    return out


def blocked_form(steps, warmup):
    """The block-wise form at the size of the paper's largest four-view
    dataset: 1640x1070x345 (an L1 larva), four views at 90 deg, 21x21x31
    PSFs, Optimization II, lambda 0, 10 iterations; the volume is not a
    transform length along any axis and y is beyond one, so it runs in
    blocks (the default blocking: 2x3x1 blocks on 864x400x405 grids) with a
    halo of twice the PSF radius.  value counts the volume's voxels,
    grid_value the block grids'."""
    import torch
    from paper_1308_0730_amd import mvd, synth, tune
    t0 = time.time()
    s = synth.larva()
    print(f"[bench] block-wise workload generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    its, var, n = 10, "opt2", len(s.views)
    dev = [torch.from_numpy(v).cuda() for v in s.views]
    with mvd.Deconvolver.blocked(dev, s.psfs) as d:
        del dev
        d.iterate(1, var)
        tune.autotune(d, var, iters=1, cache_path=None)
        for _ in range(warmup):
            d.iterate(its, var)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(d.stream)
        for _ in range(steps):
            d.iterate(its, var)
        e1.record(d.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / steps
        tiles, halo, dims = d.blocking()
        grid = d.grid_dims(0)
        nb = tiles[0] * tiles[1] * tiles[2]
        # the column passes and the ratio pass over every block grid (one
        # iteration, HIP events around each pass); the update pass reads and
        # writes psi of the own voxels only and is left out
        prof = d.profile(1, var)
    by = pass_bytes([(grid, [p.shape for p in s.psfs])] * nb, False)
    rates = {k: round(by[k] / (prof[k][0] / 1e3) / 1e9, 1) for k in PASS_NAMES if k != "x_update"}
    dom = max(rates, key=lambda k: prof[k][0] * prof[k][1])
    vox = int(np.prod(s.dims)) * n * its
    gvox = int(np.prod(grid)) * nb * n * its
    return {"workload": "block-wise: 1640x1070x345, 4 views at 90 deg, 21x21x31 PSFs, Optimization II, "
                        "lambda 0, 10 iterations",
            "blocks": list(tiles), "halo": list(halo), "grid": list(grid), "ms_per_step": round(ms, 3),
            "value": round(vox / (ms / 1e3) / 1e9, 3), "unit": "Gvox/s",
            "grid_value": round(gvox / (ms / 1e3) / 1e9, 3), "passes_GBps": rates,
            "roofline": {"bound": "hbm", "achieved": rates[dom], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(rates[dom] / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                         "bytes_per_launch": by[dom], "avg_launch_ms": round(prof[dom][0], 5),
                         "note": "one pass over every block grid timed as one launch"}}


def spim_form():
    """The simulated SPIM acquisition (sphere object, 15-degree offset,
    light-sheet attenuation, axial x3 sampling, Poisson counts,
    re-registration) of a 96^3 volume with four views, deconvolved with
    Optimization I (20 sequential iterations) using PSFs rotated 0, 10 and 20
    degrees off: the best correlation to the ground truth and where it is
    reached, next to the views' own correlation."""
    from paper_1308_0730_amd import spim_sim
    t0 = time.time()
    acq = spim_sim.simulate()
    t_sim = time.time() - t0
    t0 = time.time()
    r = spim_sim.psf_robustness(acq, errors=(0.0, 10.0, 20.0), variant="opt1", n_iter=20)
    r.update({"workload": "SPIM simulation 96^3, 4 views at 90 deg, 13x13x25 PSFs (1.0, 3.0), OPT1, 20 iterations",
              "simulate_s": round(t_sim, 2), "deconvolve_s": round(time.time() - t0, 2)})
    return r


def psf_refine_form():
    """PSF refinement through the differentiated form: the per-view Gaussian
    widths of a 64^3 four-view problem (17^3 PSFs, true widths (1.2, 4.0))
    fitted from a start perturbed by U[0.75, 1.25], 4 RL iterations per loss,
    up to 25 descent steps."""
    from paper_1308_0730_amd import psf_refine, synth
    angles = [0.0, 45.0, 90.0, 135.0]
    s = synth.make_problem((64, 64, 64), 40, angles, (17, 17, 17), 1.2, 4.0, 77, noise="none")
    true = np.array([[1.2, 4.0]] * 4)
    th0 = true * np.random.default_rng(5).uniform(0.75, 1.25, size=true.shape)
    t0 = time.time()
    th, hist = psf_refine.refine(s.views, angles, (17, 17, 17), th0, n_iter=4, steps=25)
    return {"workload": "64^3, 4 views, 17^3 PSFs, widths (1.2, 4.0) per view from a start x U[0.75, 1.25]",
            "steps": len(hist) - 1, "loss_start": hist[0][0], "loss_end": hist[-1][0],
            "max_rel_width_error_start": round(float(np.abs(th0 / true - 1).max()), 4),
            "max_rel_width_error_end": round(float(np.abs(th / true - 1).max()), 4),
            "wall_s": round(time.time() - t0, 2)}


def synth_config5():
    from paper_1308_0730_amd import synth
    return synth.config5()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=60.0)
    ap.add_argument("--profile-iters", type=int, default=2)
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--tiles", type=str, default=None,
                    help="force launch shapes 'x,y,z': candidate indices, or p for the per-length plans")
    ap.add_argument("--schedule", type=str, default=None, choices=("pass", "block", "run"),
                    help="force the schedule of a multi-block handle")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched (48 blocks, against the plain form looped over them), the small "
                         "plain workloads (64^3, 128^3), the block-wise (1640x1070x345), the "
                         "differentiated (forward against forward + backward), the convergence "
                         "(every scheme x variant to one distance from the ground truth), the "
                         "linear-boundary, the simulated-SPIM and the PSF-refinement measurements")
    ap.add_argument("--only-form", type=str, default=None,
                    choices=("batched", "small", "blocked", "grad", "convergence", "linear", "spim", "psf_refine"),
                    help="run one side measurement alone (--steps timed runs after --warmup) and print its JSON")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference kernel for HBM counters)")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("DIR", "TITLE", "COMMAND"),
                    help="print the kernel-statistics summary of a rocprofv3 --kernel-trace --stats run (CSV)")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "TITLE", "COMMANDS"),
                    help="print the HBM-traffic summary of a FETCH_SIZE and a WRITE_SIZE rocprofv3 run (CSV) of "
                         "--config; COMMANDS separated by ';;'")
    ap.add_argument("--summarize-sq", nargs=3, metavar=("DIR", "TITLE", "COMMAND"),
                    help="print the per-launch SQ counter summary of a rocprofv3 --pmc run (CSV)")
    ap.add_argument("--counted-iterations", type=int, default=12,
                    help="iterations the profiled command ran (1 at create + steps x iterations + profile iterations)")
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_kernel_trace(*args.summarize_trace))
        return
    if args.summarize_sq:
        print(summarize_sq_counters(*args.summarize_sq))
        return
    if args.summarize_counters:
        fd, wd, title, cmds = args.summarize_counters
        print(summarize_counters(fd, wd, args.config, args.counted_iterations, title, cmds.split(";;")))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path has no multi-GPU form",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1308_0730_amd import mvd

    form_fns = {"batched": lambda st, wu: batched_form(st, wu), "small": small_form, "blocked": blocked_form,
                "grad": grad_form, "convergence": lambda st, wu: convergence_form(),
                "linear": linear_form, "spim": lambda st, wu: spim_form(),
                "psf_refine": lambda st, wu: psf_refine_form()}
    if args.only_form:
        print(json.dumps({args.only_form: form_fns[args.only_form](args.steps, args.warmup)}), flush=True)
        return

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        print("[bench] copy calibration: 2 x 1 GiB device copies", file=sys.stderr, flush=True)

    t0 = time.time()
    blocks, meta = workload(args.config)
    print(f"[bench] generated workload in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    weighted = blocks[0].weights is not None
    t0 = time.time()
    if len(blocks) == 1:
        d = mvd.Deconvolver(blocks[0].views, blocks[0].psfs, blocks[0].weights, lam=meta["lam"])
    else:
        d = mvd.Deconvolver.batch([(b.views, b.psfs, b.weights) for b in blocks], lam=meta["lam"])
    d.synchronize()
    # create from host arrays: validation, the copies over PCIe, the kernel planes
    create_s = time.time() - t0
    t1 = time.time()
    d.iterate(1, meta["variant"])  # builds the compound spectra and the graph
    d.synchronize()
    first_s = time.time() - t1
    print(f"[bench] created handle in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    t0 = time.time()
    if args.tiles:
        d.set_tiles(*parse_tiles(d, args.tiles))
        if args.schedule:
            d.set_schedule(args.schedule)
    elif not args.no_tune:
        from paper_1308_0730_amd import tune
        tune.autotune(d, meta["variant"], iters=1, cache_path=None, verbose=True, runs=meta["iterations"])
    tiles = d.tiles()
    schedule = d.schedule()
    launch = {}
    for i, (k, c) in enumerate(zip(("x", "y", "z"), tiles)):
        sh = mvd.tile_shape(i, c)
        launch[k] = dict(plans="per-length", candidate=c) if sh["exact_len"] < 0 else dict(sh, candidate=c)
    print(f"[bench] launch shapes {tiles} ({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)

    its = meta["iterations"]
    for _ in range(args.warmup):
        d.iterate(its, meta["variant"])
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        d.iterate(its, meta["variant"])
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    st = d.stats()
    print(f"[bench] timed {args.steps} steps: {ms:.3f} ms/step", file=sys.stderr, flush=True)

    n_views = d.n_views
    vox_updates = sum(int(np.prod(b.dims)) for b in blocks) * n_views * its
    value = vox_updates / (ms / 1e3) / 1e9

    # per-pass timings right after the timed runs (the device still busy)
    prof = d.profile(args.profile_iters, meta["variant"])
    d.synchronize()
    # the estimate back to host memory (pageable), as a caller holding host
    # buffers would take it
    t1 = time.time()
    for b in range(len(blocks)):
        d.estimate(b).cpu()
    d2h_s = time.time() - t1
    # a one-shot run: create, the first iteration with its one-time builds
    # (compound kernels, graph capture), the other iterations, the estimate back
    one_shot = create_s + first_s + (its - 1) / its * ms / 1e3 + d2h_s
    pcie = {"create_s": round(create_s, 3), "first_iteration_s": round(first_s, 3), "d2h_ms": round(d2h_s * 1e3, 2),
            "value": round(vox_updates / one_shot / 1e9, 3), "unit": "Gvox/s",
            "note": "one run with its create from host arrays, its first iteration's one-time builds and the "
                    "estimate copied back (wall clock)"}
    by = pass_bytes(blocks, weighted)
    total = {k: prof[k][0] * prof[k][1] for k in PASS_NAMES}
    dom = max(total, key=total.get)
    avg = prof[dom][0]
    ach = by[dom] / (avg / 1e3) / 1e9
    name = {1: "tiny64", 2: "cube128", 3: "embryo512", 4: "batched48"}[args.config]
    tr = measured_traffic(name, dom)
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": tr, "kernel": dom,
            "bytes_per_launch": by[dom], "avg_launch_ms": round(avg, 5)}
    cbw = copy_bandwidth(torch)
    roof["copy_GBps"] = round(cbw, 1)
    roof["frac_of_copy"] = round(ach / cbw, 4)
    passes = {k: {"avg_ms": round(prof[k][0], 5), "launches": prof[k][1],
                  "GBps": round(by[k] / (prof[k][0] / 1e3) / 1e9, 1) if prof[k][0] > 0 else None}
              for k in PASS_NAMES}
    d.close()

    cpu = None
    if not args.no_cpu_baseline:
        del d
        torch.cuda.empty_cache()
        cpu = cpu_baseline(blocks, meta, args.cpu_budget)

    forms = None
    if not args.no_forms:
        forms = {}
        for name, fn in (("batched", lambda: form_fns["batched"](max(1, args.steps // 2), 1)),
                         ("small", lambda: form_fns["small"](max(3, args.steps), 1)),
                         ("blocked", lambda: form_fns["blocked"](max(1, args.steps // 2), 1)),
                         ("grad", lambda: form_fns["grad"](3, 1)),
                         ("convergence", lambda: form_fns["convergence"](0, 0)),
                         ("linear", lambda: form_fns["linear"](max(1, args.steps // 2), 1)),
                         ("spim", lambda: form_fns["spim"](0, 0)), ("psf_refine", lambda: form_fns["psf_refine"](0, 0))):
            try:
                forms[name] = fn()
            except Exception as e:  # a failing side measurement must not cost the main line
                print(f"[bench] form {name} failed: {e!r}", file=sys.stderr, flush=True)
                forms[name] = {"error": repr(e)}
            torch.cuda.empty_cache()

    dims = [list(b.dims) for b in blocks]
    out = {
        "metric": "voxel-view updates/s", "value": round(value, 3), "unit": "Gvox/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": meta["workload"], "dims": dims if len(dims) > 1 else dims[0],
                   "views": n_views, "iterations": its,
                   "variant": meta["variant"], "lambda": meta["lam"], "weights": weighted,
                   "voxel_view_updates_per_step": vox_updates},
        "roofline": roof, "passes": passes, "launch": launch, "schedule": schedule, "cpu_baseline": cpu,
        "pcie_inclusive": pcie,
        "forms": forms,
        "stats": {"flux_last_iteration": st["flux"], "ratio_clamps": st["ratio_clamps"],
                  "neg_clamps": st["neg_clamps"], "nonfinite": st["nonfinite"]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
