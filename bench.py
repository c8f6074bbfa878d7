"""Throughput of the Voronoi-walk renderer on one MI355X.

Workload (default): the 100k-site shell scene (70% of the sites jittered on
the unit sphere with density 50, 30% uniform in [-2,2]^3 with density 0.01),
8x8 FP32 octahedral texels per cell, 800x800 pinhole views (60 deg FOV) at 8
poses evenly spaced on a radius-3 orbit, tmax 8, early stop at T < 1e-4.

One step = prepare the scene records once, then render the 8 poses as 8
frames; each frame is one voro_render_views_fwd call (camera-centre cell
search + in-kernel ray generation + walk + compositing).  Mrays/s = rays per
step * K / timed seconds.  Scene construction (Qhull adjacency), Morton
reordering and texel casts are one-time preprocessing outside the timed
region, as in the paper's viewer protocol (Sec. 6.1, App. B).

Prints one JSON line.  Also reported, outside `value`: FP16/BF16-texel
forward throughput and their error against the FP64 oracle on sampled rays,
forward+backward throughput, the dominant kernel's algorithmic bandwidth
against the HBM peak, and the FP64 oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_POSES = 8


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2608_17682_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def step_bytes(stats, tex_bytes, n_rays):
    """Algorithmic bytes of a forward pass: per visited cell the cell record
    (xyz + sigma, 16 B), its adjacency bounds (8 B), per neighbour its id and
    position (4 + 12 B), and 4 RGBA texels; per ray 44 B of ray in / colour out."""
    steps = float(stats["steps"])
    deg = float(stats["degree_sum"])
    return steps * (16 + 8 + 4 * tex_bytes) + 16.0 * deg + 44.0 * n_rays


def stats_dict(t):
    from paper_2608_17682_amd import voro
    a = t.cpu().numpy()
    return {name: int(a[i]) for i, name in enumerate(voro.STAT_NAMES)}


def oracle_sample(scene, cam, n_rays, workers, texels=None, seed=7):
    """FP64 oracle on n_rays rays of the 64x64 centre crop (and the GPU pixel ids)."""
    from oracle import cameras, render
    from paper_2608_17682_amd import synth
    o, d, tm, _ = cameras.camera_rays_of(cam)
    crop = synth.crop_pixels(cam, 64, 0, True)
    pick = crop[synth.sample_pixels(len(crop), n_rays, seed)]
    o32 = o[pick].astype(np.float32)
    d32 = d[pick].astype(np.float32)
    tm32 = tm[pick].astype(np.float32)
    tex = scene.texels if texels is None else texels
    t0 = time.perf_counter()
    rgb, T, recs = render.render_rays_parallel(scene.sites, scene.density, tex, o32, d32, tm32,
                                               workers=workers, chunk=max(1, n_rays // workers))
    dt = time.perf_counter() - t0
    from oracle.margins import degenerate
    degen = float(np.mean([degenerate(r) for r in recs]))
    return pick, rgb, T, dt, degen


def bench_config3(scene, dev, args, timed):
    """2M sites on 20 ellipsoid surfaces, one 1280x840 interior pinhole view;
    forward + backward through the autograd Functions (FP32), upstream dL/dRGB
    ~ N(0,1).  A step is what a training step spends on rendering: gradients
    reset (as zero_grad(set_to_none=True) does), prepare, the forward launch,
    dL/dsigma through sigma = exp(rho), and the backward launch.  Headline:
    render_views (in-kernel ray generation, tuned launches); also reported:
    render over explicit rays (ray generation + centre cell + both walks)."""
    import torch
    from paper_2608_17682_amd import autotune, synth, voro
    from paper_2608_17682_amd.autograd import render, render_views
    cam = synth.config3_camera(scene)
    ds0 = voro.device_scene(scene, dev)
    ds, perm, inv = voro.voro_morton_reorder(ds0)
    del ds0
    sites = ds.sites.clone().requires_grad_(True)
    rho = torch.log(ds.density.clamp_min(1e-30)).requires_grad_(True)
    tex = ds.texels.clone().requires_grad_(True)
    g = torch.from_numpy(synth.upstream(cam.n_rays, 3, with_gT=False)[0]).to(dev)
    ccam = [voro.camera_of(cam)]
    pf, pb = autotune.params_for("config3", "fwd"), autotune.params_for("config3", "bwd")

    def reset():
        sites.grad = None
        rho.grad = None
        tex.grad = None

    def step_views():
        reset()
        rgb, T = render_views(sites, torch.exp(rho), tex, ds.nbr_off, ds.nbr_idx, ccam, pf, pb)
        (rgb * g).sum().backward()

    def step_explicit():
        reset()
        O, D, TM = voro.voro_gen_rays(ccam, dev)
        S = voro.voro_locate_origins(ds, O[:1]).expand(O.shape[0]).contiguous()
        rgb, T = render(sites, torch.exp(rho), tex, ds.nbr_off, ds.nbr_idx, O, D, TM, S,
                        voro.default_params(img_w=cam.width))
        (rgb * g).sum().backward()

    def step_explicit_dist():
        # the training objective with the distortion regulariser (Sec. 5.3)
        reset()
        O, D, TM = voro.voro_gen_rays(ccam, dev)
        S = voro.voro_locate_origins(ds, O[:1]).expand(O.shape[0]).contiguous()
        rgb, T, ld = render(sites, torch.exp(rho), tex, ds.nbr_off, ds.nbr_idx, O, D, TM, S,
                            voro.default_params(img_w=cam.width), distortion=True)
        ((rgb * g).sum() + 0.01 * ld.sum()).backward()

    # instrumented forward for the step counts
    st = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    voro.voro_prepare(ds)
    voro.voro_render_views_fwd(ds, ccam, pf, stats=st)
    stats = stats_dict(st)
    steps = max(2, args.steps // 2)
    s = timed(step_views, steps, 1)
    se = timed(step_explicit, steps, 1)
    sd = timed(step_explicit_dist, steps, 1)
    fwd_s = timed(lambda: voro.voro_render_views_fwd(ds, ccam, pf), steps, 1)
    return {"workload": "ellipsoids2M: 1.8M sites on 20 ellipsoid surfaces (sigma 50) + 200k "
                        "uniform [-4,4]^3 (sigma 0.01), 8x8 f32 texels, 1280x840 interior "
                        "pinhole, tmax 14, fwd+bwd via torch.autograd.Function",
            "fwd_bwd_mrays_s": round(cam.n_rays * steps / s / 1e6, 2),
            "fwd_bwd_explicit_rays_mrays_s": round(cam.n_rays * steps / se / 1e6, 2),
            "fwd_bwd_explicit_rays_with_distortion_mrays_s": round(cam.n_rays * steps / sd / 1e6,
                                                                   2),
            "fwd_kernel_mrays_s": round(cam.n_rays * steps / fwd_s / 1e6, 2),
            "ms_per_step": round(s * 1e3 / steps, 3),
            "mean_cells_per_ray": round(stats["steps"] / max(1, stats["rays"]), 2)}


def bench_config5(scene, dev, args, timed):
    """4M sites (config-2 structure), binary16 texels, 8 views in one launch: 2 pinhole 1280x840, 2 fisheye 180 deg 1024x1024, 2 rolling shutter
    960x540, 2 thin lens 640x480 x 4 samples.  Forward, and forward + backward."""
    import torch
    from paper_2608_17682_amd import synth, voro
    cams = synth.config5_cameras(1.0)
    ds0 = voro.device_scene(scene, dev, tex_dtype="float16")
    ds, perm, inv = voro.voro_morton_reorder(ds0)
    del ds0
    voro.voro_prepare(ds)
    ccams = [voro.camera_of(c) for c in cams]
    nr, npx = voro.voro_camera_counts(ccams)
    rgb = torch.empty((npx, 3), device=dev)
    T = torch.empty(npx, device=dev)
    ray = torch.empty((nr, 4), device=dev)
    st = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    voro.voro_render_views_fwd(ds, ccams, None, rgb, T, ray, stats=st)
    stats = stats_dict(st)
    rays = stats["rays"]   # fisheye pixels outside the image circle emit no ray

    from paper_2608_17682_amd import autotune
    pf, pb = autotune.params_for("config5", "fwd"), autotune.params_for("config5", "bwd")

    def fwd():
        voro.voro_prepare(ds)
        voro.voro_render_views_fwd(ds, ccams, pf, rgb, T, ray)

    g = torch.from_numpy(synth.upstream(npx, 5, with_gT=False)[0]).to(dev)
    gs = torch.zeros((ds.n, 3), device=dev)
    gd = torch.zeros(ds.n, device=dev)
    gt = torch.zeros(tuple(ds.texels.shape), device=dev)

    def fwdbwd():
        fwd()
        voro.voro_render_views_bwd(ds, ccams, rgb, T, ray, g, None, pb, gs, gd, gt)

    steps = max(2, args.steps // 2)
    sf = timed(fwd, steps, 1)
    sb = timed(fwdbwd, steps, 1)
    return {"workload": "shell4M: 2.8M shell + 1.2M uniform sites, 8x8 f16 texels, 8 mixed views "
                        "(2 pinhole 1280x840, 2 fisheye 1024^2, 2 rolling shutter 960x540, "
                        "2 thin lens 640x480x4) in one launch",
            "rays": rays, "fwd_mrays_s": round(rays * steps / sf / 1e6, 2),
            "fwd_bwd_mrays_s": round(rays * steps / sb / 1e6, 2),
            "fwd_ms": round(sf * 1e3 / steps, 3), "fwd_bwd_ms": round(sb * 1e3 / steps, 3),
            "mean_cells_per_ray": round(stats["steps"] / max(1, rays), 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--lanes-per-ray", type=int, default=0)
    ap.add_argument("--tile", type=str, default="")
    ap.add_argument("--no-morton", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip half texels and fwd+bwd")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 2M-site (fwd+bwd) and 4M-site (8 views) workloads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-rays", type=int, default=1536)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()

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

    t0 = time.perf_counter()
    scene, cams = synth.config2()
    log(f"scene built in {time.perf_counter() - t0:.1f}s: N={scene.n} M={len(scene.nbr_idx)}")

    # The oracle leg runs first, in forked worker processes, before this
    # process touches the GPU.
    oracle_leg = None
    if not args.no_cpu_baseline:
        workers = min(16, os.cpu_count() or 1)
        oracle_leg = (workers,) + oracle_sample(scene, cams[0], args.oracle_rays, workers)
        log(f"oracle leg: {len(oracle_leg[1])} rays in {oracle_leg[4]:.1f}s on {workers} processes")

    # the 2M/4M-site scenes: adjacency built in a child process (cached)
    large = {}
    if not args.no_large and not args.no_extras:
        for name in ("config3", "config5"):
            t0 = time.perf_counter()
            try:
                large[name] = synth.scene_cached(name)
                log(f"{name}: {large[name].n} sites ready in {time.perf_counter() - t0:.1f}s")
            except Exception as e:  # a large workload must never cost the headline
                large[name] = e
                log(f"{name}: scene failed: {e!r}")

    dev = torch.device("cuda:0")
    ds0 = voro.device_scene(scene, dev)
    if args.no_morton:
        ds = ds0
    else:
        ds, perm, inv = voro.voro_morton_reorder(ds0)
    voro.voro_prepare(ds)
    from paper_2608_17682_amd import autotune
    params = autotune.params_for("shell100k", "fwd")
    params_bwd = autotune.params_for("shell100k", "bwd")
    if args.lanes_per_ray or args.tile:
        params = voro.default_params(lanes_per_ray=args.lanes_per_ray)
        if args.tile:
            tw, th = (int(x) for x in args.tile.split("x"))
            params.tile_w, params.tile_h = tw, th
        params_bwd = params
    ccams = [voro.camera_of(c) for c in cams]
    rays_per_frame = cams[0].n_rays
    rays_per_step = rays_per_frame * N_POSES
    npx = cams[0].n_pixels
    rgb = torch.empty((npx, 3), device=dev)
    T = torch.empty(npx, device=dev)

    def frame(i, p, dscene, out_rgb=rgb, out_T=T, stats=None, nsteps=None):
        voro.voro_render_views_fwd(dscene, [ccams[i]], p, rgb=out_rgb, T=out_T, stats=stats,
                                   nsteps=nsteps)

    def step(dscene, p):
        voro.voro_prepare(dscene)
        for i in range(N_POSES):
            frame(i, p, dscene)

    # instrumented pass (untimed): steps and degree sums for the byte model,
    # cells per ray over all poses
    st = torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev)
    ks = torch.empty((N_POSES, rays_per_frame), dtype=torch.int32, device=dev)
    for i in range(N_POSES):
        frame(i, params, ds, stats=st, nsteps=ks[i])
    torch.cuda.synchronize()
    stats = stats_dict(st)
    kq = torch.quantile(ks.flatten().float(), torch.tensor([0.5, 0.99], device=dev)).cpu().numpy()
    k_dist = {"mean": round(float(ks.float().mean()), 2), "p50": float(kq[0]),
              "p99": float(kq[1]), "max": int(ks.max())}
    log(f"stats per step: {stats}; cells per ray {k_dist}")

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

    # the timed region
    secs = timed(lambda: step(ds, params), args.steps, args.warmup)
    ms_per_step = secs * 1e3 / args.steps
    value = rays_per_step * args.steps / secs / 1e6
    log(f"fwd f32: {ms_per_step:.3f} ms/step, {value:.1f} Mrays/s")

    # dominant kernel: per-frame views launch timed with events on its stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(N_POSES * 3)]
    for k, (a, b) in enumerate(ev):
        a.record()
        frame(k % N_POSES, params, ds)
        b.record()
    torch.cuda.synchronize()
    frame_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    algo_bytes_frame = step_bytes(stats, 16, rays_per_step) / N_POSES
    achieved = algo_bytes_frame / (frame_ms * 1e-3) / 1e9
    traffic = None
    unit_busy = None
    tfile = os.path.join(ROOT, "profiles", "traffic_views_fwd_shell100k_800x800.json")
    if os.path.exists(tfile):
        with open(tfile) as f:
            tj = json.load(f)
        if tj.get("source_hash") == source_hash():
            traffic = tj.get("bytes_per_launch")
            unit_busy = tj.get("unit_busy")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_views_fwd", "launch_ms": round(frame_ms, 4),
                "algorithmic_bytes_per_launch": int(algo_bytes_frame),
                "mean_cells_per_ray": round(stats["steps"] / max(1, stats["rays"]), 2),
                "mean_degree": round(stats["degree_sum"] / max(1, stats["steps"]), 2)}
    if unit_busy:
        # the cache-resident walk beats the HBM roofline; what bounds it is
        # the issue rate and the texture path, from the committed counters
        roofline["unit_busy"] = {k: v for k, v in unit_busy.items() if k != "note"}

    extras = {"cells_per_ray": k_dist, "fp64_redecisions_per_step": stats["fp64_redecide"]}
    if not args.no_extras:
        # half-precision texels (Sec. 5.6), FP32 compositing
        for name in ("float16", "bfloat16"):
            th = voro.voro_cast_texels(ds.texels, name)
            dsh = ds.with_arrays(texels=th)
            voro.voro_prepare(dsh)
            s = timed(lambda: step(dsh, params), args.steps, args.warmup)
            extras[f"fwd_{name}_mrays_s"] = round(rays_per_step * args.steps / s / 1e6, 2)
        # forward + backward (replay adjoint) per frame, FP32 gradients
        g_rgb = torch.from_numpy(synth.upstream(npx, 2, with_gT=False)[0]).to(dev)
        gs = torch.zeros((ds.n, 3), device=dev)
        gd = torch.zeros(ds.n, device=dev)
        gt = torch.zeros(tuple(ds.texels.shape), device=dev)

        def fb():
            voro.voro_prepare(ds)
            for i in range(N_POSES):
                frame(i, params, ds)
                voro.voro_render_views_bwd(ds, [ccams[i]], rgb, T, None, g_rgb, None, params_bwd,
                                           gs, gd, gt)
        s = timed(fb, max(2, args.steps // 2), 1)
        extras["fwd_bwd_f32_mrays_s"] = round(rays_per_step * max(2, args.steps // 2) / s / 1e6, 2)
        # the same with binary16 texels (colour from f16, gradients in FP32)
        dsh = ds.with_arrays(texels=voro.voro_cast_texels(ds.texels, "float16"))

        def fb16():
            voro.voro_prepare(dsh)
            for i in range(N_POSES):
                frame(i, params, dsh)
                voro.voro_render_views_bwd(dsh, [ccams[i]], rgb, T, None, g_rgb, None, params_bwd,
                                           gs, gd, gt)
        s = timed(fb16, max(2, args.steps // 2), 1)
        extras["fwd_bwd_float16_mrays_s"] = round(
            rays_per_step * max(2, args.steps // 2) / s / 1e6, 2)
        del gs, gd, gt, dsh
        # cell-skip sweep (Sec. 5.6 / the supplementary threshold table): the
        # colour of a segment with weight below skip_w is not looked up
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
            sweep.append({"skip_w": sw, "mrays_s": round(rays_per_step * args.steps / s / 1e6, 2),
                          "max_abs_rgb_change": err})
        extras["skip_sweep"] = sweep
        del ref_rgb
        # half-precision edge vectors for ranking (Sec. 5.6 inference variant):
        # throughput and agreement with the exact walk over the 8 poses
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
        extras["edge_fp16"] = {"fwd_mrays_s": round(rays_per_step * args.steps / s / 1e6, 2),
                               "pixels_identical_to_exact": round(same, 6),
                               "max_abs_rgb_diff": dmax, "mean_abs_rgb_diff": dsum}
        del ref
        # motion blur (Sec. 6.5): 2 views of 960x540 pixels x 5 time samples
        # in one launch, pixel = mean of its samples
        mb = [voro.camera_of(c) for c in synth.motion_blur_cameras(1.0, spp=5)]
        mb_rays, mb_px = voro.voro_camera_counts(mb)
        mb_rgb = torch.empty((mb_px, 3), device=dev)
        mb_T = torch.empty(mb_px, device=dev)
        mb_ray = torch.empty((mb_rays, 4), device=dev)
        s = timed(lambda: voro.voro_render_views_fwd(ds, mb, params, mb_rgb, mb_T, mb_ray),
                  args.steps, args.warmup)
        extras["motion_blur_2x960x540x5_fwd_mrays_s"] = round(mb_rays * args.steps / s / 1e6, 2)
        del mb_rgb, mb_T, mb_ray
        # the paper's full appearance model (Sec. 5.1/5.2): surface + view maps
        # of seeded logits, same scene, walk and launches
        full = torch.from_numpy(synth.full_texels(scene.n, scene.tex_res, seed=2)).to(dev)
        if not args.no_morton:
            full = full[perm.long()].contiguous()
        dsf = ds.with_arrays(texels=full)
        voro.voro_prepare(dsf)

        def with_app(p):
            q = voro.voro_params.from_buffer_copy(p)
            q.appearance = 1
            return q
        pf, pfb = with_app(params), with_app(params_bwd)
        fa = {}
        s = timed(lambda: step(dsf, pf), args.steps, args.warmup)
        fa["fwd_f32_mrays_s"] = round(rays_per_step * args.steps / s / 1e6, 2)
        dsf16 = dsf.with_arrays(texels=voro.voro_cast_texels(full, "float16"))
        voro.voro_prepare(dsf16)
        s = timed(lambda: step(dsf16, pf), args.steps, args.warmup)
        fa["fwd_float16_mrays_s"] = round(rays_per_step * args.steps / s / 1e6, 2)
        del dsf16
        gs = torch.zeros((ds.n, 3), device=dev)
        gd = torch.zeros(ds.n, device=dev)
        gt = torch.zeros(tuple(full.shape), device=dev)

        def fbf():
            voro.voro_prepare(dsf)
            for i in range(N_POSES):
                frame(i, pf, dsf)
                voro.voro_render_views_bwd(dsf, [ccams[i]], rgb, T, None, g_rgb, None, pfb,
                                           gs, gd, gt)
        s = timed(fbf, max(2, args.steps // 2), 1)
        fa["fwd_bwd_f32_mrays_s"] = round(rays_per_step * max(2, args.steps // 2) / s / 1e6, 2)
        extras["full_appearance"] = fa
        del gs, gd, gt, dsf, full
        # appearance comparison (Sec. 3.3 vs 5.1/5.2): appearance values and
        # bytes loaded per visited cell, and forward throughput, same walk
        ksh = torch.from_numpy(synth.sh_coeffs(scene.n, seed=2)).to(dev)
        if not args.no_morton:
            ksh = ksh[perm.long()].contiguous()
        psh = with_app(params)
        psh.appearance = 2
        cmp_ = {"single_map": {"values_per_cell": 12, "bytes_f32": 64, "bytes_f16": 32,
                               "fwd_f32_mrays_s": round(value, 2),
                               "fwd_float16_mrays_s": extras.get("fwd_float16_mrays_s")},
                "surface_plus_view_maps": {"values_per_cell": 24, "bytes_f32": 128,
                                           "bytes_f16": 64,
                                           "fwd_f32_mrays_s": fa["fwd_f32_mrays_s"],
                                           "fwd_float16_mrays_s": fa["fwd_float16_mrays_s"]},
                "sh_degree3": {"values_per_cell": 48, "bytes_f32": 192, "bytes_f16": 96}}
        for name, kk in (("f32", ksh), ("float16", voro.voro_cast_texels(ksh, "float16"))):
            dss = ds.with_arrays(texels=kk)
            voro.voro_prepare(dss)
            s = timed(lambda: step(dss, psh), args.steps, args.warmup)
            cmp_["sh_degree3"][f"fwd_{name}_mrays_s"] = round(rays_per_step * args.steps / s / 1e6,
                                                              2)
        extras["appearance_comparison"] = cmp_
        voro.voro_prepare(ds)
        del ksh
        log(f"extras: {extras}")
        for name, fn in (("config3", bench_config3), ("config5", bench_config5)):
            if name not in large:
                continue
            try:
                if isinstance(large[name], Exception):
                    raise large[name]
                extras[name] = fn(large[name], dev, args, timed)
            except Exception as e:
                extras[name] = {"error": repr(e)}
            log(f"{name}: {extras[name]}")
            large[name] = None
            torch.cuda.empty_cache()

    cpu_baseline = None
    if oracle_leg is not None:
        workers, pick, rgb_o, T_o, dt, degen = oracle_leg
        extras["oracle_sample_degenerate_ray_frac"] = degen
        # GPU colours of the same rays (pose 0, un-reordered scene) for the error report
        rgb0 = torch.empty((npx, 3), device=dev)
        T0 = torch.empty(npx, device=dev)
        voro.voro_prepare(ds0)
        frame(0, params, ds0, rgb0, T0)
        rgb_h = {}
        for name in ("float16", "bfloat16"):
            th = voro.voro_cast_texels(ds0.texels, name)
            dsh = ds0.with_arrays(texels=th)
            voro.voro_prepare(dsh)
            r_ = torch.empty((npx, 3), device=dev)
            frame(0, params, dsh, r_, torch.empty(npx, device=dev))
            rgb_h[name] = r_.cpu().numpy()
        torch.cuda.synchronize()
        err32 = np.abs(rgb0.cpu().numpy()[pick] - rgb_o)
        extras["max_abs_err_f32_vs_oracle"] = float(err32.max())
        for name in ("float16", "bfloat16"):
            e = np.abs(rgb_h[name][pick] - rgb_o)
            extras[f"max_abs_err_{name}_vs_oracle"] = float(e.max())
            extras[f"mean_abs_err_{name}_vs_oracle"] = float(e.mean())
        cpu_baseline = {"value": round(len(pick) / dt / 1e6, 8), "unit": "Mrays/s",
                        "cores": workers, "kind": "oracle",
                        "sample": f"{len(pick)} rays of the 64x64 centre crop of pose 0, "
                                  f"FP64 brute-force walk over all {scene.n} sites, "
                                  f"{workers} processes, {dt:.1f} s"}
        log(f"cpu baseline: {cpu_baseline}")

    out = {
        "metric": "Mrays/s fwd and fwd+bwd at 1 MI355X (fp32 vs fp16 texels); % HBM peak",
        "value": round(value, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "shell100k: 100k sites (70% unit-sphere shell, sigma 50; 30% "
                               "uniform [-2,2]^3, sigma 0.01), 8x8 f32 texels, 800x800 pinhole "
                               "60deg, 8 orbit poses (r=3) per step, tmax 8, forward",
                   "rays_per_step": rays_per_step, "sites": scene.n,
                   "morton": not args.no_morton,
                   "launch_fwd": {"lanes_per_ray": params.lanes_per_ray or 1,
                                  "tile": f"{params.tile_w or 8}x{params.tile_h or 8}",
                                  "block": params.block or 256,
                                  "schedule": ["grid", "grid", "persistent"][params.schedule]},
                   "launch_source": "autotune table" if autotune.lookup("shell100k", "fwd")
                   and not (args.lanes_per_ray or args.tile) else "flags/defaults"},
        "roofline": roofline,
        "cpu_baseline": cpu_baseline,
        "extras": extras,
        "source_hash": source_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
