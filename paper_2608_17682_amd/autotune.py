"""Launch-shape autotuner for the walk kernels.

Picks, per workload class and direction (forward / adjoint), the number of
lanes that share a ray's neighbour tests (rays per wave = 64 / lanes), the
screen tile a wave walks, the workgroup size and the schedule (grid,
persistent queue or lane refill), by timing the multi-view launch with HIP
events on the caller's device.  The forward is timed as an inference pass
runs it; the adjoint reads the exits the forward stored (STORED_EXITS steps
per ray), as a training step does.

A workload class is keyed by what changes the best launch: the scene size
(rounded up to a power of two), the texture resolution, the texel storage
type and the set of camera models in the launch.  Results live in
``autotune_table.json`` next to this file.  ``lookup`` returns the tuned
fields for the exact class, or else for the tuned class with the same
texture, texel type, camera set and direction and the nearest scene size,
or else None (the library's defaults then apply).

    python -m paper_2608_17682_amd.autotune shell100k [config3] [config5]
"""
from __future__ import annotations

import json
import math
import os
import sys
import time
from typing import Dict, Iterable, List, Optional

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_table.json")
LAUNCH_FIELDS = ("lanes_per_ray", "tile_w", "tile_h", "block", "schedule")
MODEL_NAMES = {0: "pinhole", 1: "fisheye", 2: "rolling_shutter", 3: "thin_lens",
               4: "motion_blur"}
DTYPE_NAMES = {0: "f32", 1: "f16", 2: "bf16"}


def candidates() -> List[dict]:
    """Lanes per ray x wave tile (tile_w * tile_h * lanes = 64, aspect <= 8) x workgroup
    x schedule (1 = grid, 2 = persistent queue, 3 = lane refill with one lane per ray)."""
    out = []
    for lpr in (1, 2, 4, 8, 16):
        rays = 64 // lpr
        w = 1
        while w <= rays:
            h = rays // w
            if max(w, h) <= 8 * min(w, h):
                for block in (128, 256):
                    for schedule in ((1, 2, 3) if lpr == 1 else (1, 2)):
                        out.append({"lanes_per_ray": lpr, "tile_w": w, "tile_h": h,
                                    "block": block, "schedule": schedule})
            w *= 2
    return out


def size_bucket(n_sites: int) -> int:
    """Scene size rounded up to a power of two."""
    return 1 << max(0, int(math.ceil(math.log2(max(1, int(n_sites))))))


def workload_key(n_sites: int, tex_res: int, tex_dtype: int, models, direction: str) -> str:
    """Table key of a workload class, e.g. 'n4194304|r8|f16|fisheye+pinhole|bwd'."""
    mix = "+".join(sorted(MODEL_NAMES[int(m)] for m in set(int(m) for m in models)))
    return f"n{size_bucket(n_sites)}|r{int(tex_res)}|{DTYPE_NAMES[int(tex_dtype)]}|{mix}|{direction}"


def _models(cams) -> List[int]:
    return [int(c.model) for c in cams]


def key_of(ds, cams, direction: str) -> str:
    """Key of a prepared DeviceScene and its cameras."""
    return workload_key(ds.n, ds.tex_res, ds.tex_dtype, _models(cams), direction)


def _load() -> Dict[str, dict]:
    if os.path.exists(TABLE):
        with open(TABLE) as f:
            return json.load(f)
    return {}


def lookup_key(key: str, table: Optional[Dict[str, dict]] = None) -> Optional[dict]:
    """Tuned launch fields for a key: exact, else the nearest scene size with the
    same texture, texel type, camera set and direction, else None."""
    table = _load() if table is None else table
    e = table.get(key)
    if e is None:
        n, rest = key.split("|", 1)
        target = math.log2(int(n[1:]))
        near = [(abs(math.log2(int(k.split("|", 1)[0][1:])) - target), k)
                for k in table if k.split("|", 1)[1] == rest]
        if not near:
            return None
        e = table[min(near)[1]]
    return {k: e[k] for k in LAUNCH_FIELDS if k in e}


def lookup(ds, cams, direction: str) -> Optional[dict]:
    """Tuned launch fields for (scene, cameras, 'fwd' | 'bwd'), or None."""
    return lookup_key(key_of(ds, cams, direction))


def params_for(ds, cams, direction: str):
    """voro_params with the library defaults and the tuned launch shape (if any)."""
    from . import voro
    p = voro.default_params()
    t = lookup(ds, cams, direction)
    if t:
        for k, v in t.items():
            setattr(p, k, v)
    return p


def _time(fn, reps: int, warmup: int = 1) -> float:
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


# steps per ray of the stored exits the adjoint is timed with
STORED_EXITS = 256


def tune(ds, cams, reps: int = 3, cands: Iterable[dict] = None, log=print) -> Dict[str, dict]:
    """Time every candidate on the multi-view launch over `cams` (prepared
    DeviceScene `ds`); returns {'fwd': best, 'bwd': best} with times in ms."""
    import torch
    from . import synth, voro
    cands = list(cands or candidates())
    arr = [voro.camera_of(c) if not isinstance(c, voro.voro_camera) else c for c in cams]
    nr, npx = voro.voro_camera_counts(arr)
    dev = ds.sites.device
    rgb = torch.empty((npx, 3), device=dev)
    T = torch.empty(npx, device=dev)
    ray = torch.empty((nr, 4), device=dev)
    g = torch.from_numpy(synth.upstream(npx, 11, with_gT=False)[0]).to(dev)
    gs = torch.zeros((ds.n, 3), device=dev)
    gd = torch.zeros(ds.n, device=dev)
    gt = torch.zeros(tuple(ds.texels.shape), device=dev)
    base = voro.default_params()
    trace = torch.empty((STORED_EXITS, nr, 2), dtype=torch.int32, device=dev)
    voro.voro_render_views_fwd(ds, arr, base, rgb, T, ray, trace=trace)
    best = {}
    for direction in ("fwd", "bwd"):
        res = []
        for c in cands:
            if direction == "bwd" and c["schedule"] == 3:
                continue  # the adjoint has no refill kernel: it runs the persistent queue
            p = voro.default_params(**c)
            if direction == "fwd":
                fn = lambda: voro.voro_render_views_fwd(ds, arr, p, rgb, T, ray)  # noqa: E731
            else:
                fn = lambda: voro.voro_render_views_bwd(ds, arr, rgb, T, ray, g, None, p,  # noqa
                                                        gs, gd, gt, trace=trace)
            ms = _time(fn, reps)
            res.append((ms, c))
        res.sort(key=lambda x: x[0])
        ms, c = res[0]
        default_ms = next(m for m, cc in res if cc["lanes_per_ray"] == 1 and cc["tile_w"] == 8
                          and cc["block"] == 256 and cc["schedule"] == 1)
        best[direction] = dict(c, ms=round(ms, 4), default_ms=round(default_ms, 4),
                               rays=int(nr), candidates=len(res))
        if direction == "bwd":
            best[direction]["stored_exits"] = STORED_EXITS
        log(f"[autotune] {direction}: best {c} {ms:.3f} ms (default 1x8x8/256: {default_ms:.3f} ms)")
    return best


def _workload(name: str):
    """(DeviceScene, cameras) of a named benchmark workload, Morton-ordered."""
    import torch
    from . import synth, voro
    dev = torch.device("cuda:0")
    if name == "shell100k":
        scene, cams = synth.config2()
        cams = cams[:2]
        tex = None
    elif name == "config3":
        scene = synth.scene_cached("config3")
        cams = [synth.config3_camera(scene)]
        tex = None
    elif name == "config5":
        scene = synth.scene_cached("config5")
        cams = synth.config5_cameras(1.0)
        tex = "float16"
    else:
        raise ValueError(name)
    ds0 = voro.device_scene(scene, dev, tex_dtype=tex)
    ds, _, _ = voro.voro_morton_reorder(ds0)
    del ds0
    voro.voro_prepare(ds)
    return ds, cams


def main(argv):
    names = argv or ["shell100k"]
    # scenes first: big adjacencies are built by child processes
    from . import synth
    for n in names:
        if n in ("config3", "config5"):
            synth.scene_cached(n)
    table = _load()
    for n in names:
        t0 = time.perf_counter()
        ds, cams = _workload(n)
        best = tune(ds, cams, log=lambda m: print(f"{n}: {m}", flush=True))
        for direction, e in best.items():
            table[key_of(ds, cams, direction)] = dict(e, tuned_on=n)
        print(f"{n}: tuned in {time.perf_counter() - t0:.1f}s", flush=True)
        del ds
    out = os.environ.get("VORO_AUTOTUNE_OUT", TABLE)
    with open(out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(f"wrote {out}")


if __name__ == "__main__":
    main(sys.argv[1:])
