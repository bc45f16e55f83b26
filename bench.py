#!/usr/bin/env python3
"""Benchmark of the generalised-entropy MI hot path on one MI355X.

Workload (one "step"): the multi-modal sweep -- a 256x256x180 u16 T1-like
fixed phantom against a T2-like moving phantom, 1000 affine transforms
(10 x-translations x 10 z-rotations x 10 isotropic scales), 128-bin hard
joint histograms, Shannon MI and Tsallis MI for q in {0.5, 0.8, 1.2, 1.5, 2}
from each histogram.  One step = one mi_eval call over all 1000 transforms
(fixed binning, histogram sweep, MI reduction), inputs resident in HBM.

Prints one JSON line: throughput in voxel-transform evaluations per second
(fixed voxels x transforms / s), the histogram kernel's HBM roofline
fraction on algorithmic bytes (HIP-event timed), the one-transform-per-
launch path and the Parzen gradient path for comparison, and the CPU
oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-transform evals/s (warp+jointhist+MI) & MI-grad evals/s; % HBM roofline"
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 4 SIMD x 16 lanes per clock at 2.4 GHz
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "hist_hard_multimodal_traffic.txt")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


_SHAPE_FIELDS = {"gemi-tune": ("block", "slab_major", "chunks", "packed"),
                 "gemi-tune-parzen": ("fwd_block", "fwd_lds_kib", "bwd_block", "bwd_lds_kib", "chunk_shift"),
                 "gemi-tune-pairs": ("block", "slab_voxels", "packed", "transform_major")}


def tuned_shape(B, cache: str, kind: str, **key) -> dict | None:
    """The launch shape the tuner recorded last for the problem class whose
    key fields include ``key`` (None if it recorded none)."""
    hit = None
    for e in B.read_tune_cache(cache):
        if e["kind"] == kind and all(e.get(k) == v for k, v in key.items()):
            hit = e
    return None if hit is None else {f: hit[f] for f in _SHAPE_FIELDS[kind]}


def shape_source(args, shape) -> str:
    if shape is None:
        return "default (no tuned entry)"
    return "MI_TUNE_CACHE entry" if args.no_tune else "tuned in this run"


def algorithmic_bytes_per_voxel_xform(fixed, moving, mats, bins) -> float:
    """Fixed voxel read + moving voxels covered (|det| of the linear part)
    + the transform's histogram written once, per fixed voxel."""
    dets = np.abs(np.linalg.det(mats.reshape(-1, 3, 4)[:, :, :3]))
    return (fixed.itemsize + moving.itemsize * float(dets.mean()) +
            4.0 * bins * bins / fixed.size)


def read_profile(kernel_version: str, key: str):
    """A figure of the committed rocprofv3 counter summary of the sweep (HBM
    bytes per launch, VALU instructions per voxel-transform), if it was taken
    on the current kernel build."""
    try:
        text = open(PROFILE_TRAFFIC).read()
    except OSError:
        return None
    fields = dict(line.split("=", 1) for line in text.splitlines() if "=" in line and not line.startswith("#"))
    if fields.get("kernel_version", "").strip() != kernel_version:
        return None
    try:
        return float(fields[key])
    except (KeyError, ValueError):
        return None


def kernel_version() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("hard.hip", "sweep.h", "common.h", "plan.h"):
        h.update(open(os.path.join(ROOT, "paper_1909_10690_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _oracle_rate(oracle, F, M, c, order, threads: int, min_seconds: float):
    """Voxel-transforms per second of the oracle at `threads` threads over
    batches of `threads` transforms (taken in `order`) until ``min_seconds``
    of wall time have passed."""
    oracle.set_num_threads(threads)
    done, dt = 0, 0.0
    while dt < min_seconds and done < len(order):
        batch = c["transforms"][order[done:done + threads]]
        t0 = time.perf_counter()
        oracle.eval_hard(F, M, batch, c["bins"], c["q"])
        dt += time.perf_counter() - t0
        done += len(batch)
    return c["fixed"].size * done / dt, done, dt


def cpu_baseline(c, min_seconds: float) -> dict:
    """The oracle, as it stands, on random transforms of the same workload:
    at all host threads (the reported value) and at one thread."""
    import oracle
    F = oracle.volume(c["fixed"], *c["fixed_range"])
    M = oracle.volume(c["moving"], *c["moving_range"])
    threads = oracle.num_threads()
    order = np.random.default_rng(0).permutation(len(c["transforms"]))
    rate, done, dt = _oracle_rate(oracle, F, M, c, order, threads, min_seconds)
    rate1, done1, dt1 = _oracle_rate(oracle, F, M, c, order, 1, min_seconds)
    oracle.set_num_threads(threads)
    return {"value": rate, "unit": "voxel-transform evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} of the 1000 transforms (random order, seed 0), full 256x256x180 "
                      f"volume, all 6 entropies, {dt:.1f} s wall on {threads} threads",
            "single_thread": {"value": rate1, "unit": "voxel-transform evals/s", "cores": 1,
                              "sample": f"{done1} transforms of the same order, {dt1:.1f} s wall on 1 thread"}}


def plain_sweep_leg(ctx, B, inputs, dev, steps: int) -> dict:
    """The plain method: 64^3 u8 head phantom against itself translated by
    (3.5, -2, 1.25) voxels, 32 bins, Shannon MI over 21 x-translations in
    [-10, 10] voxels, one mi_eval call per sweep."""
    import torch
    c = inputs.plain_translation()
    F = B.Volume.from_numpy(c["fixed"], *c["fixed_range"], dev)
    Mv = B.Volume.from_numpy(c["moving"], *c["moving_range"], dev)
    tr = torch.from_numpy(c["transforms"]).to(dev)
    n = len(c["transforms"])
    ws = torch.empty(ctx.workspace_size(F, Mv, n, c["bins"], 1), dtype=torch.uint8, device=dev)
    out = torch.empty((n, 1), dtype=torch.float64, device=dev)
    for _ in range(3):
        ctx.eval(F, Mv, tr, c["bins"], c["q"], out=out, want_overlap=False, workspace=ws)
    torch.cuda.synchronize()
    ctx.timing_read(B.TIMER_HARD)
    ctx.timing(True)
    reps = max(50, steps * 5)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.eval(F, Mv, tr, c["bins"], c["q"], out=out, want_overlap=False, workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.timing(False)
    k_ms, k_n = ctx.timing_read(B.TIMER_HARD)
    best = int(np.argmax(out[:, 0].cpu().numpy()))
    vox = c["fixed"].size * n
    balg = algorithmic_bytes_per_voxel_xform(c["fixed"], c["moving"], c["transforms"], c["bins"])
    k_avg = k_ms / max(k_n, 1)
    return {"value": vox * reps / dt, "unit": "voxel-transform evals/s", "mi_evals_per_s": n * reps / dt,
            "ms_per_sweep": dt / reps * 1e3, "kernel_ms": k_avg,
            "kernel_hbm_frac": balg * vox / (k_avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "argmax_tx": float(c["transforms"][best][3]),
            "config": "64^3 u8 head phantom, moving translated by (3.5, -2, 1.25) voxels, 32 bins, "
                      "Shannon, 21 x-translations in [-10, 10]"}


def grad_leg(ctx, B, inputs, dev, args, cache: str) -> dict:
    """MI-grad evaluations per second: mi_grad (Parzen forward, MI, dMI/dp,
    backward) over the 128^3 f32 workload's 64 random affines, 64 bins,
    Shannon and Tsallis q = 1.5."""
    import torch
    g = inputs.parzen_gradient()
    F = B.Volume.from_numpy(g["fixed"], 0.0, 1.0, dev)
    M = B.Volume.from_numpy(g["moving"], 0.0, 1.0, dev)
    tr = torch.from_numpy(g["transforms"]).to(dev)
    n, bins, q = len(tr), g["bins"], g["q"]
    flags = B.BOUNDARY_CLAMP
    ws = torch.empty(ctx.workspace_size(F, M, n, bins, len(q), flags | B.HIST_PARZEN | B.GRADIENT),
                     dtype=torch.uint8, device=dev)
    log(f"gradient leg: {n} transforms x 128^3 f32, {bins} Parzen bins; tuning the Parzen sweeps")
    if not args.no_tune:
        ctx.tune(F, M, tr, bins, flags | B.HIST_PARZEN, workspace=ws)
    shape = tuned_shape(B, cache, "gemi-tune-parzen", fnx=g["fixed"].shape[2], bins=bins,
                        n_bucket=(n - 1).bit_length())
    for _ in range(2):
        ctx.grad(F, M, tr, bins, q, flags=flags, workspace=ws)
    torch.cuda.synchronize()
    for w in (B.TIMER_PARZEN_FWD, B.TIMER_PARZEN_BWD):
        ctx.timing_read(w)
    steps = max(3, args.steps // 2)
    ctx.timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.grad(F, M, tr, bins, q, flags=flags, workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.timing(False)
    fwd_ms, fwd_n = ctx.timing_read(B.TIMER_PARZEN_FWD)
    bwd_ms, bwd_n = ctx.timing_read(B.TIMER_PARZEN_BWD)
    fwd_k, bwd_k = fwd_ms / max(fwd_n, 1), bwd_ms / max(bwd_n, 1)
    # algorithmic bytes per voxel-transform of one sweep: the f32 fixed voxel
    # and the f32 moving voxels it covers (|det| of the linear part)
    dets = np.abs(np.linalg.det(g["transforms"].reshape(-1, 3, 4)[:, :, :3]))
    balg = 4.0 + 4.0 * float(dets.mean())
    vox = g["fixed"].size * n
    frac = lambda ms: balg * vox / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    return {"value": n * steps / dt, "unit": "MI-grad evals/s (forward + backward, 2 entropies)",
            "voxel_xf_per_s": g["fixed"].size * n * steps / dt, "ms_per_call": dt / steps * 1e3,
            "fwd_kernel_ms": fwd_k, "bwd_kernel_ms": bwd_k,
            "roofline": {"bound": "hbm", "algorithmic_bytes_per_voxel_xform_per_sweep": balg,
                         "fwd_frac": frac(fwd_k), "bwd_frac": frac(bwd_k),
                         "fwd_plus_bwd_frac": 2 * balg * vox / ((fwd_k + bwd_k) * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "launch": {"parzen_shape": shape, "shape_source": shape_source(args, shape)},
            "config": "128^3 f32 phantoms, 64 random affines, 64-bin cubic B-spline Parzen "
                      "histogram, Shannon + Tsallis q=1.5, clamp boundary"}


def register_leg(ctx, B, inputs, dev, args, cache: str, steps: int = 200) -> dict:
    """Gradient-ascent registration of the 512x512x300 i16 CT-like phantom to
    the 256^3 u16 MR-like one (2 mm spacing), 256 Parzen bins, from a known
    misregistration (rot_z 6 deg, t (8, -5, 4) mm, scale 1.04; the truth is
    the identity): one mi_grad (forward + backward, Shannon and Tsallis
    q = 1.3) and one Adam step per iteration, Shannon gradients for rotation,
    scale and shear, Tsallis gradients for translation."""
    import numpy as np
    import torch
    from paper_1909_10690_amd import transforms as T
    from paper_1909_10690_amd.register import affine_to_decomposed, register, volume_centre
    log("register leg: building the 512x512x300 / 256^3 CT-MR pair")
    c = inputs.ct_mr_pair()
    F = B.Volume.from_numpy(c["fixed"], *c["fixed_range"], dev, spacing=c["fixed_spacing"])
    M = B.Volume.from_numpy(c["moving"], *c["moving_range"], dev, spacing=c["moving_spacing"],
                            origin=c["moving_origin"])
    st = c["start"]
    p0 = T.params_from(T.affine_matrix(st["angles"], st["scale"]), st["t"])
    log("register leg: tuning the Parzen sweeps at the start transform")
    P0 = T.centred_matrix(p0[:9], p0[9:], volume_centre(F)).reshape(1, 12)
    if not args.no_tune:
        ctx.tune(F, M, torch.from_numpy(P0).to(dev), c["bins"], B.BOUNDARY_CLAMP | B.HIST_PARZEN)
    shape = tuned_shape(B, cache, "gemi-tune-parzen", fnx=c["fixed"].shape[2], bins=c["bins"], n_bucket=0)
    register(ctx, F, M, c["bins"], p0, steps=3, q_translation=c["q"][0], param="decomposed")
    torch.cuda.synchronize()
    log(f"register leg: {steps} iterations")
    t0 = time.perf_counter()
    s = register(ctx, F, M, c["bins"], p0, steps=steps, q_translation=c["q"][0], param="decomposed")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # kernel times of the same loop, timed apart (events around every
    # launch would add their own overhead to the iteration time above)
    ctx.timing_read(B.TIMER_PARZEN_FWD)
    ctx.timing_read(B.TIMER_PARZEN_BWD)
    ctx.timing(True)
    register(ctx, F, M, c["bins"], p0, steps=20, q_translation=c["q"][0], param="decomposed")
    torch.cuda.synchronize()
    ctx.timing(False)
    fwd_ms, fwd_n = ctx.timing_read(B.TIMER_PARZEN_FWD)
    bwd_ms, bwd_n = ctx.timing_read(B.TIMER_PARZEN_BWD)
    fwd_k, bwd_k = fwd_ms / max(fwd_n, 1), bwd_ms / max(bwd_n, 1)
    # algorithmic bytes per fixed voxel and sweep: the i16 fixed voxel and
    # the u16 moving voxels it covers (2 mm against 1 mm: 1/8 of a voxel)
    balg = 2.0 + 2.0 / 8.0
    nvox = c["fixed"].size
    frac = lambda ms: balg * nvox / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    p = s.affine()
    A, t = p[:9].reshape(3, 3), p[9:]
    R = T.rotation_matrix(np.degrees(affine_to_decomposed(p)[:3]))   # rotation factor of A
    cos = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    return {"value": steps / dt, "unit": "MI-grad evals/s (one transform, forward + backward, 2 entropies)",
            "ms_per_iteration": dt / steps * 1e3, "iterations": steps,
            "voxel_xf_per_s": c["fixed"].size * steps / dt,
            "start_error": {"rotation_deg": 6.0, "translation_mm": float(np.abs(st["t"]).max()),
                            "linear_max_abs": float(np.abs(p0[:9].reshape(3, 3) - np.eye(3)).max())},
            "final_error": {"rotation_deg": float(np.degrees(np.arccos(cos))),
                            "translation_mm": float(np.abs(t).max()),
                            "linear_max_abs": float(np.abs(A - np.eye(3)).max())},
            "mi_first": s.history[0][1], "mi_last": s.history[-1][1],
            "fwd_kernel_ms": fwd_k, "bwd_kernel_ms": bwd_k,
            "roofline": {"bound": "hbm", "algorithmic_bytes_per_voxel_per_sweep": balg,
                         "fwd_frac": frac(fwd_k), "bwd_frac": frac(bwd_k),
                         "fwd_plus_bwd_frac": 2 * balg * nvox / ((fwd_k + bwd_k) * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "launch": {"parzen_shape": shape, "shape_source": shape_source(args, shape)},
            "config": "fixed 512x512x300 i16 CT-like (1 mm), moving 256^3 u16 MR-like (2 mm), "
                      "256-bin cubic B-spline Parzen, Shannon + Tsallis q=1.3, clamp boundary, "
                      "Adam over angles / log-scales / shears / translation"}


def pairs_leg(ctx, B, inputs, dev, args, cache: str) -> dict:
    """256 uneven u8 pairs x 16 rigid transforms, 64 bins, one persistent
    launch: the launch shape tuned first (mi_tune_pairs), kernel time from
    eager calls, then the call replayed as a HIP graph with the pairs'
    preparation reused (MI_USE_GRAPH | MI_VOLUMES_UNCHANGED)."""
    import torch
    log("pairs leg: generating 256 uneven pairs")
    raw = inputs.uneven_pairs()
    pairs = [(B.Volume.from_numpy(p["fixed"], 0, 255, dev), B.Volume.from_numpy(p["moving"], 0, 255, dev),
              torch.from_numpy(p["transforms"]).to(dev)) for p in raw]
    vox = sum(p["fixed"].size for p in raw) * 16
    bins = 64
    ws = torch.empty(ctx.pairs_workspace_size(pairs, bins, 1), dtype=torch.uint8, device=dev)
    out = torch.empty((16 * len(pairs), 1), dtype=torch.float64, device=dev)
    if not args.no_tune:
        log("pairs leg: tuning the persistent launch")
        ctx.tune_pairs(pairs, bins, workspace=ws)
    shape = tuned_shape(B, cache, "gemi-tune-pairs", bins=bins)
    for _ in range(2):
        ctx.eval_pairs(pairs, bins, [1.0], workspace=ws, out=out)
    torch.cuda.synchronize()
    ref = out.clone()
    ctx.timing_read(B.TIMER_PAIRS)
    ctx.timing(True)
    steps = 5
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.eval_pairs(pairs, bins, [1.0], workspace=ws, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.timing(False)
    k_ms, k_n = ctx.timing_read(B.TIMER_PAIRS)
    gs = torch.cuda.Stream()
    gflags = B.USE_GRAPH | B.VOLUMES_UNCHANGED
    out.zero_()
    torch.cuda.synchronize()
    for _ in range(2):
        ctx.eval_pairs(pairs, bins, [1.0], flags=gflags, workspace=ws, out=out, stream=gs)
    gs.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.eval_pairs(pairs, bins, [1.0], flags=gflags, workspace=ws, out=out, stream=gs)
    gs.synchronize()
    gdt = time.perf_counter() - t0
    return {"value": vox * steps / gdt, "unit": "voxel-transform evals/s", "ms_per_call": gdt / steps * 1e3,
            "kernel_ms": k_ms / max(k_n, 1), "voxel_transforms": int(vox),
            "eager": {"value": vox * steps / dt, "ms_per_call": dt / steps * 1e3},
            "launch": {"pairs_shape": shape, "shape_source": shape_source(args, shape),
                       "graph": True, "volumes_unchanged": True, "mi_identical": bool(torch.equal(out, ref))},
            "config": "256 u8 pairs, edges from {64,96,128,160,192,256} per axis, 16 rigid transforms "
                      "each, 64 bins, Shannon"}


def maps_leg(ctx, B, inputs, dev, n: int = 51) -> dict:
    """Parameter-space maps of the same 256x256x180 u16 image: 51^3 grids
    of translations (+-25 mm), rotations (versors, the whole unit ball) and
    scales (+-25%), 128 bins, six entropies from each histogram, then the
    discrete gradient paths and capture range of every entropy's map."""
    import torch
    from paper_1909_10690_amd import maps
    log("maps leg: generating the 256x256x180 u16 same-image phantom")
    c = inputs.same_image()
    F = B.Volume.from_numpy(c["fixed"], *c["fixed_range"], dev)
    Mv = F  # the same image on both sides
    q, bins = tuple(c["q"]), c["bins"]
    shape_xyz = c["fixed"].shape[::-1]
    mats = {f: torch.from_numpy(maps.map_transforms(f, n, shape_xyz)).to(dev) for f in maps.FAMILIES}
    maps.mi_map(ctx, F, Mv, "translation", 3, 2.0, bins=bins, q=q)  # warm-up (workspace, kernels)
    torch.cuda.synchronize()
    out, total_s = {}, 0.0
    for fam in maps.FAMILIES:
        log(f"maps leg: {fam} {n}^3")
        t0 = time.perf_counter()
        m = maps.mi_map(ctx, F, Mv, fam, n, bins=bins, q=q, transforms=mats[fam])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = maps.map_paths(ctx, m, 1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        total_s += t2 - t0
        centre = ((n // 2) * n + n // 2) * n + n // 2
        caps = {}
        for qi, r in zip(q, res):
            ext, target, basin, radius = (int(x) for x in r["stats"].cpu().tolist())
            caps[f"q={qi:g}"] = {"extrema": ext, "centre_is_optimum": target == centre,
                                 "basin_fraction": basin / n ** 3, "capture_radius": radius}
        out[fam] = {"ms_map": (t1 - t0) * 1e3, "ms_paths": (t2 - t1) * 1e3,
                    "mi_evals_per_s": n ** 3 / (t1 - t0), "capture": caps}
    # Mattes-style maps (Discussion: random sampling and binned Parzen
    # histograms, whose effect the paper leaves open): cubic B-spline Parzen
    # bins, 64 of them, over a 10% random subset of the fixed voxels
    from paper_1909_10690_amd import binding as BB
    mattes, mattes_s = {}, 0.0
    for fam in maps.FAMILIES:
        log(f"maps leg: {fam} {n}^3, Parzen 64 bins, 10% of the voxels")
        t0 = time.perf_counter()
        m = maps.mi_map(ctx, F, Mv, fam, n, bins=64, q=q, flags=BB.HIST_PARZEN | BB.BOUNDARY_CLAMP,
                        transforms=mats[fam], sample=(0.1, 2019))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = maps.map_paths(ctx, m, 1)
        torch.cuda.synchronize()
        mattes_s += t1 - t0
        centre = ((n // 2) * n + n // 2) * n + n // 2
        caps = {}
        for qi, r in zip(q, res):
            ext, target, basin, radius = (int(x) for x in r["stats"].cpu().tolist())
            caps[f"q={qi:g}"] = {"extrema": ext, "centre_is_optimum": target == centre,
                                 "basin_fraction": basin / n ** 3, "capture_radius": radius}
        mattes[fam] = {"ms_map": (t1 - t0) * 1e3, "mi_evals_per_s": n ** 3 / (t1 - t0), "capture": caps}
    evals = 3 * n ** 3
    return {"value": evals / total_s, "unit": "MI evaluations/s (one transform, 6 entropies, incl. paths)",
            "voxel_xf_per_s": evals * c["fixed"].size / total_s, "families": out,
            "parzen64_sampled10": {"mi_evals_per_s": evals / mattes_s, "families": mattes,
                                   "config": "cubic B-spline Parzen, 64 bins, clamp boundary, 10% of the "
                                             "fixed voxels (SplitMix64 seed 2019), same grids and q"},
            "config": f"same 256x256x180 u16 image both sides, {n}^3 grids of translation (+-25 mm), "
                      f"rotation (versor, unit ball) and scale (+-25%), 128 bins, q = {list(q)}, "
                      "exclude boundary, ascent paths"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum wall time of the CPU-oracle sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle leg")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-shape tuners (shapes then come from the MI_TUNE_CACHE file, "
                         "if the caller names one, else the defaults); for profiled runs")
    ap.add_argument("--no-extras", action="store_true", help="skip the plain-path and gradient legs")
    ap.add_argument("--pairs", action="store_true",
                    help="time the 256 uneven pairs in one launch even with --no-extras")
    ap.add_argument("--register", action="store_true",
                    help="run the 200-iteration CT/MR registration (512x512x300 vs 256^3, 256 bins) "
                         "even with --no-extras")
    ap.add_argument("--maps", action="store_true",
                    help="map the metric over 51^3 translation, rotation and scale grids (with paths) "
                         "even with --no-extras")
    ap.add_argument("--no-maps", action="store_true", help="skip the parameter-space maps leg")
    ap.add_argument("--no-pairs", action="store_true", help="skip the uneven-pairs leg")
    ap.add_argument("--no-register", action="store_true", help="skip the registration leg")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run an elementwise copy of MIB MiB (read + write), the reference "
                         "kernel for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the library runs the "
              f"metric path on a single GPU and has no multi-GPU leg", file=sys.stderr)
        return 2

    import torch
    from paper_1909_10690_amd import binding as B
    from paper_1909_10690_amd import inputs

    log("building the multi-modal sweep inputs (256x256x180 u16, 1000 transforms)")
    c = inputs.multimodal_sweep()
    fixed, moving, mats = c["fixed"], c["moving"], c["transforms"]
    n, bins, q = len(mats), c["bins"], c["q"]
    # the tuners record their choices in MI_TUNE_CACHE; a private file unless
    # the caller names one, so that the line can say which shapes ran
    own_cache = "MI_TUNE_CACHE" not in os.environ
    if own_cache:
        fd, cache = tempfile.mkstemp(prefix="gemi-tune-", suffix=".txt")
        os.close(fd)
        os.environ["MI_TUNE_CACHE"] = cache
    cache = os.environ["MI_TUNE_CACHE"]
    ctx = B.Context(0)
    dev = "cuda:0"
    F = B.Volume.from_numpy(fixed, *c["fixed_range"], dev)
    Mv = B.Volume.from_numpy(moving, *c["moving_range"], dev)
    tr = torch.from_numpy(mats).to(dev)
    ws = torch.empty(ctx.workspace_size(F, Mv, n, bins, len(q)), dtype=torch.uint8, device=dev)
    out = torch.empty((n, len(q)), dtype=torch.float64, device=dev)

    def step():
        ctx.eval(F, Mv, tr, bins, q, out=out, want_overlap=False, workspace=ws)

    if not args.no_tune:
        log("tuning the hard sweep's launch shape for this problem class")
        ctx.tune(F, Mv, tr, bins, workspace=ws)
    hard_shape = tuned_shape(B, cache, "gemi-tune", fnx=fixed.shape[2], bins=bins, mnx=moving.shape[2],
                             n_bucket=(n - 1).bit_length())
    log(f"tuned shape: {hard_shape}")
    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing_read(B.TIMER_HARD)
    ctx.timing(True)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.timing(False)
    k_ms, k_n = ctx.timing_read(B.TIMER_HARD)
    r_ms, r_n = ctx.timing_read(B.TIMER_REDUCE)
    vox_xf = fixed.size * n
    value = vox_xf * args.steps / dt
    ms_step = dt / args.steps * 1e3
    k_avg_ms = k_ms / max(k_n, 1)
    balg = algorithmic_bytes_per_voxel_xform(fixed, moving, mats, bins)
    achieved = balg * vox_xf / (k_avg_ms * 1e-3) / 1e9
    kv = kernel_version()
    traffic = read_profile(kv, "hbm_bytes_per_launch")
    valu_per_vx = read_profile(kv, "valu_insts_per_voxel_xform")
    log(f"{value:.3e} voxel-xf/s, {ms_step:.2f} ms/step, hist kernel {k_avg_ms:.2f} ms, "
        f"reduce {r_ms / max(r_n, 1):.3f} ms")

    result = {
        "metric": METRIC, "value": value, "unit": "voxel-transform evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "multi-modal sweep: 256x256x180 u16 T1-like vs T2-like phantoms, "
                               "1000 affine transforms (10 tx x 10 rot_z x 10 scale), 128 bins, "
                               "Shannon + Tsallis q={0.5,0.8,1.2,1.5,2.0}",
                   "transforms": n, "bins": bins, "n_q": len(q), "fixed_voxels": int(fixed.size)},
        "mi_evals_per_s": n * args.steps / dt,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "hist_hard_kernel<uint16_t>", "kernel_ms": k_avg_ms,
                     "algorithmic_bytes_per_voxel_xform": balg},
    }

    # the same step replayed as a HIP graph (MI_USE_GRAPH) on a side stream;
    # graph replays carry no per-launch events, so this pass has wall time
    # only, and its MI must equal the eager step's bit for bit
    ref_out = out.clone()
    gs = torch.cuda.Stream()

    def gstep():
        ctx.eval(F, Mv, tr, bins, q, flags=B.USE_GRAPH, out=out, want_overlap=False, workspace=ws, stream=gs)

    log(f"graph replay: {args.steps} steps")
    out.zero_()
    torch.cuda.synchronize()
    for _ in range(max(2, args.warmup)):
        gstep()
    gs.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gstep()
    gs.synchronize()
    gdt = time.perf_counter() - t0
    result["launch"] = {
        "hist_shape": hard_shape, "shape_source": shape_source(args, hard_shape),
        "timed_region": "eager mi_eval calls on the default stream, HIP events around each kernel",
        "graph": {"ms_per_step": gdt / args.steps * 1e3, "value": vox_xf * args.steps / gdt,
                  "vs_eager": dt / gdt, "mi_identical": bool(torch.equal(out, ref_out))}}

    # LDS-atomic rate of the sweep (one 32-bit LDS add per counted voxel)
    # against the measured peak of conflict-free LDS adds on this device
    _, ov, _ = ctx.eval(F, Mv, tr, bins, q, workspace=ws)
    atomics = float(ov.sum().item())
    lds_peak = ctx.probe_lds_atomics()
    lds_rate = atomics / (k_avg_ms * 1e-3)
    result["lds_atomic"] = {"achieved": lds_rate, "peak": lds_peak, "unit": "lane-atomics/s",
                            "frac": lds_rate / lds_peak, "per_voxel_xform": atomics / vox_xf,
                            "peak_source": "mi_probe_lds_atomics (conflict-free ds_add_u32, measured)"}
    # bank conflicts of the same kernel build (committed SQ_LDS_BANK_CONFLICT
    # summary): stall cycles per LDS instruction and as a share of the LDS's
    # active cycles
    for key in ("lds_conflict_cycles_per_lds_inst", "lds_conflict_frac_of_active"):
        v = read_profile(kv, key)
        if v is not None:
            result["lds_atomic"][key] = v
    # VALU issue: wave64 VALU instructions per voxel-transform (committed
    # SQ_INSTS_VALU summary of this kernel build) x 64 lanes, against
    # 256 CUs x 64 lanes/clock x 2.4 GHz
    if valu_per_vx is not None:
        alu = valu_per_vx * vox_xf / (k_avg_ms * 1e-3)
        result["alu"] = {"achieved": alu / 1e12, "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s",
                         "frac": alu / 1e12 / VALU_PEAK_TOPS, "valu_per_voxel_xform": valu_per_vx}

    if args.calibrate_copy:
        nel = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        result["copy_calibration"] = {"bytes_read": 4 * nel, "bytes_written": 4 * nel,
                                      "launches": 3}

    if not args.no_extras:
        # one transform per launch: the same kernels, no batching
        sub = 100
        log(f"plain path: {sub} transforms, one mi_eval call each")
        ws1 = torch.empty(ctx.workspace_size(F, Mv, 1, bins, len(q)), dtype=torch.uint8, device=dev)
        out1 = torch.empty((1, len(q)), dtype=torch.float64, device=dev)
        trs = [tr[i:i + 1] for i in range(sub)]
        for i in range(3):
            ctx.eval(F, Mv, trs[i], bins, q, out=out1, want_overlap=False, workspace=ws1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(sub):
            ctx.eval(F, Mv, trs[i], bins, q, out=out1, want_overlap=False, workspace=ws1)
        torch.cuda.synchronize()
        plain = fixed.size * sub / (time.perf_counter() - t0)
        result["plain_one_transform_per_launch"] = {"value": plain, "unit": "voxel-transform evals/s",
                                                    "batched_speedup": value / plain}

    if not args.no_extras:
        result["mi_grad"] = grad_leg(ctx, B, inputs, dev, args, cache)
        result["plain_sweep"] = plain_sweep_leg(ctx, B, inputs, dev, args.steps)

    if (args.pairs or not args.no_extras) and not args.no_pairs:
        result["pairs"] = pairs_leg(ctx, B, inputs, dev, args, cache)
    if (args.maps or not args.no_extras) and not args.no_maps:
        result["maps"] = maps_leg(ctx, B, inputs, dev)
    if (args.register or not args.no_extras) and not args.no_register:
        result["register"] = register_leg(ctx, B, inputs, dev, args, cache)

    # the targets this measures against, stated with whether they are met
    targets = {"hbm_roofline_frac": {"target": 0.60, "achieved": result["roofline"]["frac"]}}
    if "plain_one_transform_per_launch" in result:
        targets["batched_vs_plain"] = {"target": 10.0,
                                       "achieved": result["plain_one_transform_per_launch"]["batched_speedup"]}
    if "mi_grad" in result:
        targets["gradient_path_hbm_roofline_frac"] = {
            "target": 0.60, "achieved": result["mi_grad"]["roofline"]["fwd_plus_bwd_frac"]}
    for v in targets.values():
        v["met"] = bool(v["achieved"] >= v["target"])
    result["targets"] = targets

    if not args.no_cpu:
        log(f"CPU oracle for at least {args.cpu_seconds} s")
        result["cpu_baseline"] = cpu_baseline(c, args.cpu_seconds)

    print(json.dumps(result), flush=True)
    ctx.close()
    if own_cache:
        os.remove(cache)
    return 0


if __name__ == "__main__":
    sys.exit(main())
