"""Throughput of the Voronoi-walk renderer on one MI355X.

Headline workload (the largest configuration that fits one GPU): 4M sites in
the shell structure (2.8M jittered on the unit sphere with density 50, 1.2M
uniform in [-2,2]^3 with density 0.01), Morton-ordered, 8x8 octahedral
texels stored in binary16, and 8 mixed views rendered in one launch each
way: 2 pinhole 1280x840, 2 equidistant 180 deg fisheye 1024x1024 (no rays
outside the image circle), 2 rolling shutter 960x540 (0.1 units along the
camera's +x over the frame), 2 thin lens 640x480 x 4 aperture samples.

One step = what a training step spends on rendering: gradient buffers
cleared, the scene records prepared, the forward launch (in-kernel ray
generation, start cells, walk, compositing) and the adjoint launch (replay
and gradient scatter, FP32 gradients).  Mrays/s = rays per step x steps /
timed seconds.  Scene construction (Delaunay adjacency), Morton reordering
and texel casts are one-time preprocessing outside the timed region, as in
the paper's viewer protocol (Sec. 6.1, App. B).

Prints one JSON line.  Also reported (outside `value`): the same workload
forward only; the 100k-site shell scene at 8 orbit poses (forward with f32,
f16 and bf16 texels, forward + backward, their error against the FP64
oracle on two 64x64 crops, the cell-skip sweep, half-precision edge vectors,
motion blur, the full appearance model, spherical harmonics); the 2M-site
ellipsoid scene forward + backward through the autograd Function; the
512-site scene; a plain device copy as the attainable HBM bandwidth; and the
FP64 oracle timed on the host cores.

    python bench.py [--steps K] [--warmup W]
    python bench.py --workload config5 --steps 1 --warmup 0 --profile
                                          (one workload, only its step's launches: profiling)
    python bench.py --copy-probe                              (1 GiB device copy only)
    python bench.py --summarise-counters OUT.json --kernel NAME --pmc DIR [DIR ...]
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# one wave64 VALU instruction per CU per clock (4 SIMD16 units, 4 cycles per
# wave instruction), 256 CUs at 2.4 GHz
VALU_PEAK_GINST = 256 * 2.4
N_POSES = 8
COUNTERS = {
    "bwd": os.path.join(ROOT, "profiles", "counters_views_bwd_shell4M_8views.json"),
    "fwd": os.path.join(ROOT, "profiles", "counters_views_fwd_shell4M_8views.json"),
}


# the sources the multi-view kernels are compiled from: committed counters
# stay valid while these are unchanged
KERNEL_SOURCES = ["include/voro.h"] + [
    f"paper_2608_17682_amd/csrc/{n}" for n in
    ("cameras.hip", "camera_impl.hpp", "host_common.hpp", "locate_impl.hpp", "voro_device.hpp",
     "walk_impl.hpp")]


def _code_only(text: str) -> str:
    """The source with its comments and blank lines removed (counters depend
    on the code, not on how it is commented).  String literals in these
    sources hold no comment markers."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def source_hash(root: str = None) -> str:
    """Hash of the code (comments stripped) of the sources the multi-view
    kernels are compiled from; the committed counter summaries carry it."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(root or ROOT, rel), "r", encoding="utf-8") as f:
            h.update(rel.encode())
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def fwd_step_bytes(stats, texel_bytes, stored=0):
    """Algorithmic bytes of a forward pass: per visited cell the cell record
    (xyz + sigma, 16 B), its adjacency bounds (8 B), per neighbour its id and
    position (4 + 12 B) and 4 RGBA texels; per ray 44 B of ray in / colour out;
    8 B per stored exit (`stored` of the steps)."""
    return (float(stats["steps"]) * (16 + 8 + 4 * texel_bytes) + 16.0 * stats["degree_sum"]
            + 44.0 * stats["rays"] + 8.0 * stored)


def bwd_step_bytes(stats, texel_bytes, stored=0):
    """Algorithmic bytes of an adjoint pass: the forward's reads (the replay),
    plus per visited cell the gradient read-modify-writes of its density (4 B),
    the two sites of its exit face (2 x 12 B) and the RGB of its 4 texels
    (4 x 12 B), plus per ray the saved colour and transmittance and the
    upstream gradient (32 B).  A step whose exit was stored reads those 8 B
    instead of its edge row (rows of the other steps taken at the mean degree)."""
    steps = float(stats["steps"])
    rows = 16.0 * stats["degree_sum"] * (1.0 - stored / max(1.0, steps))
    return (steps * (16 + 8 + 4 * texel_bytes) + rows + 8.0 * stored
            + steps * (4 + 24 + 48) + 32.0 * stats["rays"])


def stats_dict(t):
    from paper_2608_17682_amd import voro
    a = t.cpu().numpy()
    return {name: int(a[i]) for i, name in enumerate(voro.STAT_NAMES)}


# ----------------------------------------------------------- oracle legs
# Both run before this process touches the GPU: the oracle's pool forks.

def oracle_config5_sample(scene, workers, px_per_view=4):
    """FP64 oracle forward + adjoint on a few pixels of each of the 8 views."""
    from oracle import batch, cameras
    from paper_2608_17682_amd import synth
    cams = synth.config5_cameras(1.0)
    npx = [c.n_pixels for c in cams]
    g_all = synth.upstream(int(sum(npx)), 5, with_gT=False)[0]
    o_l, d_l, t_l, g_l = [], [], [], []
    for v, cam in enumerate(cams):
        o, d, tm, valid = cameras.camera_rays_of(cam)
        cand = np.nonzero(valid.reshape(cam.n_pixels, cam.spp).all(1))[0]
        for p in cand[synth.sample_pixels(len(cand), px_per_view, 90 + v)]:
            rs = slice(p * cam.spp, (p + 1) * cam.spp)
            o_l.append(o[rs])
            d_l.append(d[rs])
            t_l.append(tm[rs])
            g_l.append(np.repeat(g_all[sum(npx[:v]) + p][None], cam.spp, 0) / cam.spp)
    o, d, tm = (np.concatenate(x).astype(np.float32) for x in (o_l, d_l, t_l))
    g = np.concatenate(g_l)
    tex = scene.texels.astype(np.float16).astype(np.float32)   # binary16 storage
    sites = scene.sites.astype(np.float64)
    t0 = time.perf_counter()
    res = batch.evaluate(sites, scene.density, tex, o, d, tm, keep_records=np.ones(len(o), bool),
                         workers=workers, chunk=1)
    batch.sparse_gradients(sites, scene.density, tex, o, d, tm, res["records"], g)
    dt = time.perf_counter() - t0
    return {"rays": len(o), "seconds": dt, "mean_K": float(res["K"].mean()),
            "views": len(cams), "px_per_view": px_per_view}


def oracle_config2_crops(scene, cam, workers):
    """FP64 oracle on the two 64x64 crops (centre + seeded) of pose 0, f32 texels."""
    from oracle import batch, cameras, walk
    from paper_2608_17682_amd import synth
    pix = np.concatenate([synth.crop_pixels(cam, 64, 0, True), synth.crop_pixels(cam, 64, 2, False)])
    o, d, tm, _ = cameras.camera_rays_of(cam)
    o, d, tm = (x[pix].astype(np.float32) for x in (o, d, tm))
    sites = scene.sites.astype(np.float64)
    t0 = time.perf_counter()
    start = np.full(len(o), walk.nearest_site(sites, o[0])[0])
    res = batch.evaluate(sites, scene.density, scene.texels, o, d, tm, starts=start,
                         workers=workers)
    res["seconds"] = time.perf_counter() - t0
    res["pixels"] = pix
    return res


# -------------------------------------------------------------- GPU legs

def timed_fn(torch):
    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3
    return timed


def launch_ms(torch, fn, reps):
    """Mean duration of one launch, HIP events on the stream the library launches on."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def load_counters(direction):
    """Committed per-launch counters of the headline kernels, if the kernel
    sources have not changed since they were taken."""
    path = COUNTERS[direction]
    if not os.path.exists(path):
        return None
    with open(path) as f:
        c = json.load(f)
    if c.get("source_hash") != source_hash():
        return None
    return c


def roofline_of(counters, ms, algo_bytes, kernel):
    """Roofline entry of one kernel.  The binding roof is the most used of:
    HBM (calibrated FETCH_SIZE + WRITE_SIZE per launch over the live launch
    time, against 8 TB/s), VALU issue (wave instructions per launch over the
    chip's 614.4 G/s), the texture address / data units and the LDS (busy
    cycles over the kernel's cycles, per CU, from the profile run).  The byte model's
    bytes over the same live time are reported as `effective`, never as
    `frac`."""
    s = ms * 1e-3
    eff = algo_bytes / s / 1e9
    out = {"kernel": kernel, "launch_ms": round(ms, 4),
           "effective": {"algorithmic_bytes_per_launch": int(algo_bytes),
                         "gbs": round(eff, 1), "frac_of_hbm_peak": round(eff / HBM_PEAK_GBS, 4)}}
    if counters is None:
        out.update({"bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
                    "traffic": None,
                    "note": "no counters for the current kernel sources in profiles/"})
        return out
    hbm = counters["hbm_bytes_per_launch"]
    valu = counters["valu_insts_per_launch"]
    hbm_gbs = hbm / s / 1e9
    valu_g = valu / s / 1e9
    util = {"hbm": round(hbm_gbs / HBM_PEAK_GBS, 4),
            "valu_issue": round(valu_g / VALU_PEAK_GINST, 4)}
    busy = counters.get("unit_busy", {})
    util.update(busy)
    roof = max(util, key=util.get)
    if roof == "hbm":
        out.update({"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": util["hbm"]})
    elif roof == "valu_issue":
        out.update({"bound": "alu", "achieved": round(valu_g, 2), "peak": VALU_PEAK_GINST,
                    "unit": "G VALU wave-instructions/s", "frac": util["valu_issue"]})
    else:
        cyc = counters["cycles_per_launch"]
        out.update({"bound": roof, "achieved": round(busy[roof] * cyc / 1e6, 3),
                    "peak": round(cyc / 1e6, 3), "unit": "M busy cycles per CU per launch",
                    "frac": busy[roof]})
    out["traffic"] = int(hbm)
    out["utilisation"] = util
    out["l2_hit_rate"] = counters.get("l2_hit_rate")
    out["counters"] = os.path.relpath(counters["_path"], ROOT)
    return out


# Steps per ray whose exits the headline's forward stores for its adjoint:
# 7.7M rays x 256 x 8 B = 15.9 GB; the few rays that walk further (longest
# about 300 cells here) have their later exits searched again.
EXIT_STEPS = 256


def bench_config5(scene, dev, args, timed):
    """The headline: 4M sites, binary16 texels, 8 mixed views per launch, fwd + bwd
    (the forward stores each ray's first EXIT_STEPS exits for the adjoint)."""
    import torch
    from paper_2608_17682_amd import autotune, synth, voro
    cams = synth.config5_cameras(1.0)
    ds0 = voro.device_scene(scene, dev, tex_dtype="float16")
    ds, _, _ = voro.voro_morton_reorder(ds0)
    del ds0
    voro.voro_prepare(ds)
    ccams = [voro.camera_of(c) for c in cams]
    nr, npx = voro.voro_camera_counts(ccams)
    pf, pb = autotune.params_for(ds, cams, "fwd"), autotune.params_for(ds, cams, "bwd")
    rgb = torch.empty((npx, 3), device=dev)
    T = torch.empty(npx, device=dev)
    ray = torch.empty((nr, 4), device=dev)
    st = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    ks = torch.empty(nr, dtype=torch.int32, device=dev)
    trace = torch.empty((EXIT_STEPS, nr, 2), dtype=torch.int32, device=dev)
    voro.voro_render_views_fwd(ds, ccams, pf, rgb, T, ray, nsteps=ks, stats=st, trace=trace)
    stats = stats_dict(st)
    stored = int(torch.clamp(ks, max=EXIT_STEPS).sum())
    rays = stats["rays"]   # fisheye pixels outside the image circle emit no ray
    kv = ks[ks > 0].float()
    kq = torch.quantile(kv[torch.randperm(kv.numel(), device=dev)[:1 << 20]],
                        torch.tensor([0.5, 0.99], device=dev)).cpu().numpy()
    g = torch.from_numpy(synth.upstream(npx, 5, with_gT=False)[0]).to(dev)
    gs = torch.zeros((ds.n, 3), device=dev)
    gd = torch.zeros(ds.n, device=dev)
    gt = torch.zeros(tuple(ds.texels.shape), device=dev)

    def fwd(tr):
        voro.voro_prepare(ds)
        voro.voro_render_views_fwd(ds, ccams, pf, rgb, T, ray, trace=tr)

    def bwd():
        voro.voro_render_views_bwd(ds, ccams, rgb, T, ray, g, None, pb, gs, gd, gt, trace=trace)

    def step():
        gs.zero_()
        gd.zero_()
        gt.zero_()
        fwd(trace)
        bwd()

    secs = timed(step, args.steps, args.warmup)
    fwdt_ms = launch_ms(
        torch, lambda: voro.voro_render_views_fwd(ds, ccams, pf, rgb, T, ray, trace=trace), 3)
    bwd_ms = launch_ms(torch, bwd, 3)
    sf = fwd_ms = None
    if not args.profile:
        # the forward alone, as an inference pass renders (no stored exits);
        # left out of profiled runs so that every forward launch they see is
        # the step's
        sf = timed(lambda: fwd(None), args.steps, 1)
        fwd_ms = launch_ms(torch, lambda: voro.voro_render_views_fwd(ds, ccams, pf, rgb, T, ray),
                           3)
    del trace
    res = {"rays_per_step": rays, "secs": secs, "fwd_secs": sf, "stats": stats,
           "fwd_launch_ms": fwd_ms, "fwd_stored_launch_ms": fwdt_ms, "bwd_launch_ms": bwd_ms,
           "stored_exits": {"steps_per_ray": EXIT_STEPS, "stored": stored,
                            "searched_again": int(stats["steps"]) - stored,
                            "bytes": EXIT_STEPS * nr * 8},
           "cells_per_ray": {"mean": round(stats["steps"] / max(1, rays), 2),
                             "p50": float(kq[0]), "p99": float(kq[1]),
                             "max": int(ks.max())},
           "launch_fwd": dict(autotune.lookup(ds, cams, "fwd") or {}),
           "launch_bwd": dict(autotune.lookup(ds, cams, "bwd") or {})}
    del gs, gd, gt, ds
    torch.cuda.empty_cache()
    return res


def bench_config2(scene, cams, dev, args, timed, oracle2):
    """100k-site shell scene, 8 x 800x800 poses per step: the texel-precision
    comparison and the inference variants; forward + backward with each
    frame's exits stored for its adjoint."""
    import torch
    from paper_2608_17682_amd import autotune, synth, voro
    ds0 = voro.device_scene(scene, dev)
    ds, perm, inv = voro.voro_morton_reorder(ds0)
    del ds0
    voro.voro_prepare(ds)
    params = autotune.params_for(ds, cams, "fwd")
    params_bwd = autotune.params_for(ds, cams, "bwd")
    ccams = [voro.camera_of(c) for c in cams]
    rays_per_step = cams[0].n_rays * N_POSES
    npx = cams[0].n_pixels
    rgb = torch.empty((npx, 3), device=dev)
    T = torch.empty(npx, device=dev)
    out = {"workload": "shell100k: 100k sites (70% unit-sphere shell, sigma 50; 30% uniform "
                       "[-2,2]^3, sigma 0.01), 8x8 texels, 8 orbit poses of 800x800 per step"}

    def frame(i, p, dscene, out_rgb=rgb, out_T=T, stats=None, nsteps=None, trace=None):
        voro.voro_render_views_fwd(dscene, [ccams[i]], p, rgb=out_rgb, T=out_T, stats=stats,
                                   nsteps=nsteps, trace=trace)

    # forward + backward: each frame's forward stores its rays' first
    # EXIT_STEPS exits for that frame's adjoint (all poses have one size)
    trace = torch.empty((EXIT_STEPS, voro.voro_camera_counts([ccams[0]])[0], 2),
                        dtype=torch.int32, device=dev)

    def step(dscene, p):
        voro.voro_prepare(dscene)
        for i in range(N_POSES):
            frame(i, p, dscene)

    def mrays(s, steps):
        return round(rays_per_step * steps / s / 1e6, 2)

    st = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    for i in range(N_POSES):
        frame(i, params, ds, stats=st)
    stats = stats_dict(st)
    out["mean_cells_per_ray"] = round(stats["steps"] / max(1, stats["rays"]), 2)
    s = timed(lambda: step(ds, params), args.steps, args.warmup)
    out["fwd_f32_mrays_s"] = mrays(s, args.steps)
    ms = launch_ms(torch, lambda: frame(0, params, ds), 8)
    out["fwd_f32_frame_ms"] = round(ms, 4)
    out["fwd_f32_effective_gbs"] = round(fwd_step_bytes(stats, 16) / N_POSES / (ms * 1e-3) / 1e9, 1)
    dsh = {}
    for name in ("float16", "bfloat16"):
        dsh[name] = ds.with_arrays(texels=voro.voro_cast_texels(ds.texels, name))
        s = timed(lambda: step(dsh[name], params), args.steps, args.warmup)
        out[f"fwd_{name}_mrays_s"] = mrays(s, args.steps)
    g_rgb = torch.from_numpy(synth.upstream(npx, 2, with_gT=False)[0]).to(dev)
    kb = max(2, args.steps // 2)
    for name, dsc in (("f32", ds), ("float16", dsh["float16"])):
        gs = torch.zeros((ds.n, 3), device=dev)
        gd = torch.zeros(ds.n, device=dev)
        gt = torch.zeros(tuple(ds.texels.shape), device=dev)

        def fb():
            gs.zero_()
            gd.zero_()
            gt.zero_()
            voro.voro_prepare(dsc)
            for i in range(N_POSES):
                frame(i, params, dsc, trace=trace)
                voro.voro_render_views_bwd(dsc, [ccams[i]], rgb, T, None, g_rgb, None, params_bwd,
                                           gs, gd, gt, trace=trace)
        s = timed(fb, kb, 1)
        out[f"fwd_bwd_{name}_mrays_s"] = mrays(s, kb)
        del gs, gd, gt
    voro.voro_prepare(ds)

    # errors against the FP64 oracle on the two crops of pose 0 (f32 texels);
    # the GPU renders the same pixels through the benchmarked launch
    if oracle2 is not None:
        pix = oracle2["pixels"]
        sd = ~oracle2["stop_degenerate"]
        errs = {}

        def err_of(dscene, p):
            frame(0, p, dscene)
            e = np.abs(rgb.cpu().numpy()[pix] - oracle2["rgb"])[sd]
            return {"max": float(e.max()), "mean": float(e.mean())}
        errs["f32"] = err_of(ds, params)
        for name in ("float16", "bfloat16"):
            voro.voro_prepare(dsh[name])
            errs[name] = err_of(dsh[name], params)
        voro.voro_prepare(ds)
        p16 = voro.voro_params.from_buffer_copy(params)
        p16.edge_fp16 = 1
        p16.lanes_per_ray = 1
        errs["edge_fp16"] = err_of(ds, p16)
        out["rgb_error_vs_fp64_oracle_two_crops"] = dict(
            errs, rays=int(len(pix)), excluded_stop_degenerate=int((~sd).sum()),
            note="per channel |rgb - oracle rgb on the f32 texels|; the half-precision rows "
                 "carry the texel rounding (bound 2^-12 / 2^-9 x (1-T))")

    # cell-skip sweep (Sec. 5.6 / the supplementary threshold table)
    sweep = []
    ref_rgb = torch.empty((N_POSES, npx, 3), device=dev)
    for i in range(N_POSES):
        frame(i, params, ds, out_rgb=ref_rgb[i])
    for sw in (0.0, 1e-5, 1e-4, 3e-4, 1e-3, 3e-3, 1e-2):
        q = voro.voro_params.from_buffer_copy(params)
        q.skip_w = sw
        s = timed(lambda: step(ds, q), args.steps, args.warmup)
        err = 0.0
        for i in range(N_POSES):
            frame(i, q, ds)
            err = max(err, float((rgb - ref_rgb[i]).abs().max()))
        sweep.append({"skip_w": sw, "mrays_s": mrays(s, args.steps), "max_abs_rgb_change": err})
    out["skip_sweep"] = sweep
    del ref_rgb
    # half-precision edge vectors (Sec. 5.6 inference variant)
    p16 = voro.voro_params.from_buffer_copy(params)
    p16.edge_fp16 = 1
    p16.lanes_per_ray = 1
    s = timed(lambda: step(ds, p16), args.steps, args.warmup)
    same, dmax, dsum = 0.0, 0.0, 0.0
    ref = torch.empty((npx, 3), device=dev)
    for i in range(N_POSES):
        frame(i, params, ds, out_rgb=ref)
        frame(i, p16, ds)
        d = (rgb - ref).abs().max(1).values
        same += float((d == 0).float().mean()) / N_POSES
        dmax = max(dmax, float(d.max()))
        dsum += float(d.mean()) / N_POSES
    out["edge_fp16"] = {"fwd_mrays_s": mrays(s, args.steps),
                        "pixels_identical_to_exact": round(same, 6),
                        "max_abs_rgb_diff_vs_exact": dmax, "mean_abs_rgb_diff_vs_exact": dsum}
    del ref
    # motion blur (Sec. 6.5): 2 views of 960x540 pixels x 5 time samples
    mb = [voro.camera_of(c) for c in synth.motion_blur_cameras(1.0, spp=5)]
    mb_rays, mb_px = voro.voro_camera_counts(mb)
    mb_rgb = torch.empty((mb_px, 3), device=dev)
    mb_T = torch.empty(mb_px, device=dev)
    mb_ray = torch.empty((mb_rays, 4), device=dev)
    s = timed(lambda: voro.voro_render_views_fwd(ds, mb, params, mb_rgb, mb_T, mb_ray),
              args.steps, args.warmup)
    out["motion_blur_2x960x540x5_fwd_mrays_s"] = round(mb_rays * args.steps / s / 1e6, 2)
    del mb_rgb, mb_T, mb_ray
    # the paper's full appearance model (Sec. 5.1/5.2): surface + view maps
    full = torch.from_numpy(synth.full_texels(scene.n, scene.tex_res, seed=2)).to(dev)
    full = full[perm.long()].contiguous()
    dsf = ds.with_arrays(texels=full)
    voro.voro_prepare(dsf)

    def with_app(p, app):
        q = voro.voro_params.from_buffer_copy(p)
        q.appearance = app
        return q
    pf, pfb = with_app(params, 1), with_app(params_bwd, 1)
    fa = {}
    s = timed(lambda: step(dsf, pf), args.steps, args.warmup)
    fa["fwd_f32_mrays_s"] = mrays(s, args.steps)
    dsf16 = dsf.with_arrays(texels=voro.voro_cast_texels(full, "float16"))
    s = timed(lambda: step(dsf16, pf), args.steps, args.warmup)
    fa["fwd_float16_mrays_s"] = mrays(s, args.steps)
    del dsf16
    gs = torch.zeros((ds.n, 3), device=dev)
    gd = torch.zeros(ds.n, device=dev)
    gt = torch.zeros(tuple(full.shape), device=dev)

    def fbf():
        voro.voro_prepare(dsf)
        for i in range(N_POSES):
            frame(i, pf, dsf, trace=trace)
            voro.voro_render_views_bwd(dsf, [ccams[i]], rgb, T, None, g_rgb, None, pfb, gs, gd, gt,
                                       trace=trace)
    s = timed(fbf, kb, 1)
    fa["fwd_bwd_f32_mrays_s"] = mrays(s, kb)
    out["full_appearance"] = fa
    del gs, gd, gt, dsf, full
    # appearance comparison (Sec. 3.3 vs 5.1/5.2): values and bytes per visited cell
    ksh = torch.from_numpy(synth.sh_coeffs(scene.n, seed=2)).to(dev)[perm.long()].contiguous()
    psh = with_app(params, 2)
    cmp_ = {"single_map": {"values_per_cell": 12, "bytes_f32": 64, "bytes_f16": 32,
                           "fwd_f32_mrays_s": out["fwd_f32_mrays_s"],
                           "fwd_float16_mrays_s": out["fwd_float16_mrays_s"]},
            "surface_plus_view_maps": {"values_per_cell": 24, "bytes_f32": 128, "bytes_f16": 64,
                                       "fwd_f32_mrays_s": fa["fwd_f32_mrays_s"],
                                       "fwd_float16_mrays_s": fa["fwd_float16_mrays_s"]},
            "sh_degree3": {"values_per_cell": 48, "bytes_f32": 192, "bytes_f16": 96}}
    for name, kk in (("f32", ksh), ("float16", voro.voro_cast_texels(ksh, "float16"))):
        dss = ds.with_arrays(texels=kk)
        s = timed(lambda: step(dss, psh), args.steps, args.warmup)
        cmp_["sh_degree3"][f"fwd_{name}_mrays_s"] = mrays(s, args.steps)
    out["appearance_comparison"] = cmp_
    del ksh, ds, dsh
    torch.cuda.empty_cache()
    return out


def bench_config3(scene, dev, args, timed):
    """2M sites on 20 ellipsoid surfaces, one 1280x840 interior pinhole view;
    forward + backward through the autograd Functions (FP32), upstream dL/dRGB
    ~ N(0,1).  A step: gradients reset (as zero_grad(set_to_none=True) does),
    prepare, the forward launch (storing each ray's first EXIT_STEPS exits),
    dL/dsigma through sigma = exp(rho), the backward launch (reading them).
    Headline render_views (in-kernel ray generation, tuned
    launches); also render over explicit rays."""
    import torch
    from paper_2608_17682_amd import autotune, synth, voro
    from paper_2608_17682_amd.autograd import render, render_views
    cam = synth.config3_camera(scene)
    ds0 = voro.device_scene(scene, dev)
    ds, _, _ = voro.voro_morton_reorder(ds0)
    del ds0
    sites = ds.sites.clone().requires_grad_(True)
    rho = torch.log(ds.density.clamp_min(1e-30)).requires_grad_(True)
    tex = ds.texels.clone().requires_grad_(True)
    g = torch.from_numpy(synth.upstream(cam.n_rays, 3, with_gT=False)[0]).to(dev)
    ccam = [voro.camera_of(cam)]
    pf, pb = autotune.params_for(ds, [cam], "fwd"), autotune.params_for(ds, [cam], "bwd")

    def reset():
        sites.grad = None
        rho.grad = None
        tex.grad = None

    def step_views():
        reset()
        rgb, T = render_views(sites, torch.exp(rho), tex, ds.nbr_off, ds.nbr_idx, ccam, pf, pb,
                              stored_exits=EXIT_STEPS)
        (rgb * g).sum().backward()

    def step_explicit(dist=False):
        reset()
        O, D, TM = voro.voro_gen_rays(ccam, dev)
        S = voro.voro_locate_origins(ds, O[:1]).expand(O.shape[0]).contiguous()
        out = render(sites, torch.exp(rho), tex, ds.nbr_off, ds.nbr_idx, O, D, TM, S,
                     voro.default_params(img_w=cam.width), distortion=dist,
                     stored_exits=EXIT_STEPS)
        loss = (out[0] * g).sum()
        if dist:   # the training objective with the distortion regulariser (Sec. 5.3)
            loss = loss + 0.01 * out[2].sum()
        loss.backward()

    st = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    voro.voro_prepare(ds)
    tr = torch.empty((EXIT_STEPS, cam.n_rays, 2), dtype=torch.int32, device=dev)
    voro.voro_render_views_fwd(ds, ccam, pf, stats=st, trace=tr)   # as the step's forward
    del tr
    stats = stats_dict(st)
    steps = max(2, args.steps // 2)
    s = timed(step_views, steps, 1)

    def mr(x):
        return round(cam.n_rays * steps / x / 1e6, 2)
    res = {"workload": "ellipsoids2M: 1.8M sites on 20 ellipsoid surfaces (sigma 50) + 200k "
                       "uniform [-4,4]^3 (sigma 0.01), 8x8 f32 texels, 1280x840 interior "
                       "pinhole, tmax 14, fwd+bwd via torch.autograd.Function",
           "fwd_bwd_mrays_s": mr(s), "ms_per_step": round(s * 1e3 / steps, 3),
           "mean_cells_per_ray": round(stats["steps"] / max(1, stats["rays"]), 2)}
    if args.profile:   # profiled runs: only the render_views step's launches
        return res
    se = timed(step_explicit, steps, 1)
    sd = timed(lambda: step_explicit(True), steps, 1)
    fwd_s = timed(lambda: voro.voro_render_views_fwd(ds, ccam, pf), steps, 1)
    res.update({"fwd_bwd_explicit_rays_mrays_s": mr(se),
                "fwd_bwd_explicit_rays_with_distortion_mrays_s": mr(sd),
                "fwd_kernel_mrays_s": mr(fwd_s)})
    return res


def bench_config1(dev, args, timed):
    """512 uniform sites, 4x4 f32 texels, one 64x64 pinhole: ray generation,
    start cell, forward (and adjoint) on explicit rays."""
    import torch
    from paper_2608_17682_amd import synth, voro
    scene, cams = synth.config1()
    ds = voro.device_scene(scene, dev)
    ccam = [voro.camera_of(cams[0])]
    R = cams[0].n_rays
    g = torch.from_numpy(synth.upstream(R, 1)[0]).to(dev)
    gT = torch.from_numpy(synth.upstream(R, 1)[1]).to(dev)
    gs = torch.zeros((ds.n, 3), device=dev)
    gd = torch.zeros(ds.n, device=dev)
    gt = torch.zeros(tuple(ds.texels.shape), device=dev)

    def fwd():
        voro.voro_prepare(ds)
        O, D, TM = voro.voro_gen_rays(ccam, dev)
        S = voro.voro_locate_origins(ds, O[:1]).expand(R).contiguous()
        return O, D, TM, S, voro.voro_render_fwd(ds, O, D, TM, S)

    def fb():
        O, D, TM, S, (rgb, T) = fwd()
        voro.voro_render_bwd(ds, O, D, TM, S, rgb, T, g, gT, None, gs, gd, gt)
    steps = max(20, args.steps * 5)
    sf = timed(fwd, steps, 3)
    sb = timed(fb, steps, 3)
    return {"workload": "uniform512: 512 sites in [-1,1]^3, 4x4 f32 texels, one 64x64 pinhole",
            "fwd_mrays_s": round(R * steps / sf / 1e6, 3),
            "fwd_bwd_mrays_s": round(R * steps / sb / 1e6, 3),
            "fwd_ms_per_step": round(sf * 1e3 / steps, 4),
            "fwd_bwd_ms_per_step": round(sb * 1e3 / steps, 4),
            "note": "4096 rays: a few launches of a few microseconds each, launch-latency bound"}


def copy_bandwidth(dev):
    """A plain 1 GiB device-to-device copy: the attainable HBM bandwidth."""
    import torch
    n = 1 << 28
    a = torch.ones(n, device=dev)
    b = torch.empty(n, device=dev)
    ms = launch_ms(torch, lambda: b.copy_(a), 10)
    del a, b
    return {"bytes_per_copy": 8 * n, "ms": round(ms, 4), "gbs": round(8 * n / (ms * 1e-3) / 1e9, 1),
            "frac_of_hbm_peak": round(8 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


# -------------------------------------------------------- counter summary

def summarise_counters(out_path, kernel, dirs, copy_dirs):
    """Per-launch means of the rocprofv3 --pmc counters of one kernel (name
    substring) from counter-collection CSVs, HBM bytes calibrated against a
    plain copy's FETCH_SIZE / WRITE_SIZE; written as JSON with the source hash."""
    import csv
    import glob

    def read(dirs_, name_sub):
        vals = {}
        for d in dirs_:
            for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
                with open(path) as f:
                    for row in csv.DictReader(f):
                        if name_sub not in row["Kernel_Name"]:
                            continue
                        key = (row["Counter_Name"], row["Dispatch_Id"])
                        vals[key] = vals.get(key, 0.0) + float(row["Counter_Value"])
        per = {}
        for (cname, _), v in vals.items():
            per.setdefault(cname, []).append(v)
        return {k: (float(np.mean(v)), len(v)) for k, v in per.items()}

    k = read(dirs, kernel)
    c = read(copy_dirs, "copyBuffer") if copy_dirs else {}
    copy_bytes = 1 << 30
    fscale = copy_bytes / (c["FETCH_SIZE"][0] * 1024) if "FETCH_SIZE" in c else 1.0
    wscale = copy_bytes / (c["WRITE_SIZE"][0] * 1024) if "WRITE_SIZE" in c else 1.0
    out = {"kernel": kernel, "source_hash": source_hash(),
           "counters_per_launch": {n: v for n, (v, _) in sorted(k.items())},
           "launches": {n: cnt for n, (_, cnt) in sorted(k.items())},
           "fetch_scale": fscale, "write_scale": wscale}
    if "FETCH_SIZE" in k and "WRITE_SIZE" in k:
        out["hbm_bytes_per_launch"] = (k["FETCH_SIZE"][0] * fscale + k["WRITE_SIZE"][0] * wscale) * 1024
    if "SQ_INSTS_VALU" in k:
        out["valu_insts_per_launch"] = k["SQ_INSTS_VALU"][0]
    if "TCC_HIT_sum" in k and "TCC_MISS_sum" in k:
        h, m = k["TCC_HIT_sum"][0], k["TCC_MISS_sum"][0]
        out["l2_hit_rate"] = h / max(1.0, h + m)
    if "GRBM_GUI_ACTIVE" in k:
        cyc = k["GRBM_GUI_ACTIVE"][0] / 8.0      # summed over the 8 XCDs
        out["cycles_per_launch"] = cyc
        busy = {}
        for name, key in (("texture_addr", "TA_TA_BUSY_sum"), ("texture_data", "TD_TD_BUSY_sum"),
                          ("lds", "SQ_LDS_IDX_ACTIVE")):
            if key in k:
                busy[name] = round(k[key][0] / 256.0 / cyc, 4)
        if busy:
            out["unit_busy"] = busy
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1, sort_keys=True))


# ------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["all", "config5", "config2", "config3", "config1"],
                    default="all", help="one workload only (no oracle legs), e.g. for profiling")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="run only the timed step's launches (for rocprofv3)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--summarise-counters", metavar="OUT_JSON")
    ap.add_argument("--kernel", default="k_views_bwd")
    ap.add_argument("--pmc", nargs="*", default=[])
    ap.add_argument("--copy-pmc", nargs="*", default=[])
    args = ap.parse_args()

    if args.summarise_counters:
        summarise_counters(args.summarise_counters, args.kernel, args.pmc, args.copy_pmc)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(rays would shard by view or screen tile with a replicated scene)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2608_17682_amd import synth, voro

    if args.copy_probe:
        dev = torch.device("cuda:0")
        n = 1 << 28  # 1 GiB of float32
        a = torch.ones(n, device=dev)
        b = torch.empty(n, device=dev)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                          "launches": 5}))
        return

    w = args.workload
    want = {k: w in ("all", k) for k in ("config5", "config2", "config3", "config1")}
    # scenes first: the 2M/4M-site adjacencies are built by child processes (cached)
    scenes = {}
    for name in ("config5", "config3"):
        if want[name]:
            t0 = time.perf_counter()
            scenes[name] = synth.scene_cached(name)
            log(f"{name}: {scenes[name].n} sites ready in {time.perf_counter() - t0:.1f}s")
    if want["config2"]:
        t0 = time.perf_counter()
        scenes["config2"] = synth.config2()
        log(f"config2: scene built in {time.perf_counter() - t0:.1f}s")

    # oracle legs before this process touches the GPU (their pools fork)
    workers = min(16, os.cpu_count() or 1)
    cpu_baseline, oracle2 = None, None
    if w == "all" and not args.no_cpu_baseline:
        o5 = oracle_config5_sample(scenes["config5"], workers)
        log(f"oracle config5: {o5['rays']} rays fwd+bwd in {o5['seconds']:.1f}s")
        cpu_baseline = {"value": round(o5["rays"] / o5["seconds"] / 1e6, 9), "unit": "Mrays/s",
                        "cores": workers, "kind": "oracle", "cpu_model": cpu_model(),
                        "sample": f"{o5['rays']} rays of the headline workload ({o5['px_per_view']} "
                                  f"pixels of each of the 8 views, thin-lens pixels 4 rays), "
                                  f"forward + adjoint, FP64 brute force over all "
                                  f"{scenes['config5'].n} sites per step (mean K "
                                  f"{o5['mean_K']:.1f}), {workers} processes, "
                                  f"{o5['seconds']:.1f} s"}
        scene2, cams2 = scenes["config2"]
        oracle2 = oracle_config2_crops(scene2, cams2[0], workers)
        log(f"oracle config2 crops: {len(oracle2['pixels'])} rays in {oracle2['seconds']:.1f}s")

    dev = torch.device("cuda:0")
    timed = timed_fn(torch)
    extras = {}
    out = None
    if want["config5"]:
        r5 = bench_config5(scenes.pop("config5"), dev, args, timed)
        rays = r5["rays_per_step"]
        value = rays * args.steps / r5["secs"] / 1e6
        ms_per_step = r5["secs"] * 1e3 / args.steps
        log(f"config5 fwd+bwd: {ms_per_step:.3f} ms/step, {value:.1f} Mrays/s")
        st = r5["stats"]
        cb = load_counters("bwd")
        if cb:
            cb["_path"] = COUNTERS["bwd"]
        sx = r5["stored_exits"]
        roof = roofline_of(cb, r5["bwd_launch_ms"], bwd_step_bytes(st, 8, sx["stored"]),
                           "k_views_bwd (adjoint reading stored exits, 8 views, persistent "
                           "queue)")
        cf = load_counters("fwd")
        if cf:
            cf["_path"] = COUNTERS["fwd"]
        extras["config5_fwd_in_step"] = {
            "launch_ms": round(r5["fwd_stored_launch_ms"], 3),
            "roofline": roofline_of(cf, r5["fwd_stored_launch_ms"],
                                    fwd_step_bytes(st, 8, sx["stored"]),
                                    "k_views_fwd (storing exits, 8 views, persistent queue)")}
        extras["config5_stored_exits"] = sx
        if r5["fwd_secs"] is not None:
            extras["config5_fwd_only"] = {
                "mrays_s": round(rays * args.steps / r5["fwd_secs"] / 1e6, 2),
                "ms_per_step": round(r5["fwd_secs"] * 1e3 / args.steps, 3),
                "launch_ms": round(r5["fwd_launch_ms"], 3)}
        extras["config5_cells_per_ray"] = r5["cells_per_ray"]
        extras["config5_fp64_redecisions_per_step"] = st["fp64_redecide"]
        extras["config5_adjoint_share_of_step"] = round(r5["bwd_launch_ms"] / ms_per_step, 3)
        out = {
            "metric": "Mrays/s fwd and fwd+bwd at 1 MI355X (fp32 vs fp16 texels); % HBM peak",
            "value": round(value, 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "shell4M_8views: 4M sites (2.8M jittered unit-sphere shell, "
                                   "sigma 50; 1.2M uniform [-2,2]^3, sigma 0.01), 8x8 binary16 "
                                   "texels, FP32 compositing and gradients; 8 mixed views per "
                                   "launch (2 pinhole 1280x840, 2 equidistant fisheye 180deg "
                                   "1024x1024, 2 rolling shutter 960x540, 2 thin lens 640x480 x4 "
                                   "samples) on a radius-3 orbit, tmax 8; step = zero grads + "
                                   "prepare + forward launch (storing each ray's first "
                                   f"{EXIT_STEPS} exits) + adjoint launch (reading them)",
                       "rays_per_step": rays, "sites": 4_000_000, "texels": "f16",
                       "morton": True, "launch_fwd": r5["launch_fwd"],
                       "launch_bwd": r5["launch_bwd"]},
            "roofline": roof, "cpu_baseline": cpu_baseline}
    if want["config2"]:
        scene2, cams2 = scenes.pop("config2")
        extras["config2"] = bench_config2(scene2, cams2, dev, args, timed, oracle2)
        log(f"config2: {extras['config2']}")
    if want["config3"]:
        extras["config3"] = bench_config3(scenes.pop("config3"), dev, args, timed)
        log(f"config3: {extras['config3']}")
        torch.cuda.empty_cache()
    if want["config1"]:
        extras["config1"] = bench_config1(dev, args, timed)
        log(f"config1: {extras['config1']}")
    if w == "all":
        extras["hbm_copy"] = copy_bandwidth(dev)
        log(f"copy: {extras['hbm_copy']}")
    if oracle2 is not None:
        extras["oracle_config2_two_crops"] = {
            "rays": int(len(oracle2["pixels"])), "seconds": round(oracle2["seconds"], 2),
            "mrays_s": round(len(oracle2["pixels"]) / oracle2["seconds"] / 1e6, 9),
            "processes": workers, "degenerate_ray_frac": float(oracle2["degenerate"].mean())}
    if out is None:
        out = {"workload_only": w}
    out["extras"] = extras
    out["source_hash"] = source_hash()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
