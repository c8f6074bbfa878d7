"""The allocation-free multi-view forward (its scratch in a static device array
of the library) against voro_render_views_fwd, through the C ABI: bit-identical
outputs on two calls in a row, the second with a smaller input, for the grid
and the persistent-queue schedules; more views than the scratch holds are
refused before anything is enqueued."""
import numpy as np
import pytest
import torch

from paper_2608_17682_amd import synth, voro

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def scene():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    voro.lib()
    dev = torch.device("cuda:0")
    sc = synth.scene_uniform(3000, 4, seed=12)
    ds = voro.device_scene(sc, dev)
    voro.voro_prepare(ds)
    return ds


def outputs(ds, cams):
    nr, npx = voro.voro_camera_counts(cams)
    dev = ds.sites.device
    return (torch.full((npx, 3), -1.0, device=dev), torch.full((npx,), -1.0, device=dev),
            torch.full((nr, 4), -1.0, device=dev), torch.full((nr,), -1, dtype=torch.int32,
                                                              device=dev),
            torch.zeros(voro.STAT_COUNT, dtype=torch.int64, device=dev))


@pytest.mark.parametrize("schedule", [voro.SCHEDULE_GRID, voro.SCHEDULE_PERSISTENT])
def test_noalloc_views_forward_equals_the_workspace_entry_point(scene, schedule):
    ds = scene
    p = voro.default_params(schedule=schedule)
    big = synth.config5_cameras(scale=0.08)            # 8 mixed views, thin lens 4 spp
    small = synth.config5_cameras(scale=0.03)[1:4]     # 3 smaller views
    for name, cams in (("8 views", big), ("3 smaller views", small)):
        announce(f"noalloc {name}, schedule {schedule}")
        want = outputs(ds, cams)
        voro.voro_render_views_fwd(ds, cams, p, want[0], want[1], want[2], want[3], want[4])
        got = outputs(ds, cams)
        voro.voro_render_views_fwd_noalloc(ds, cams, p, got[0], got[1], got[2], got[3], got[4])
        torch.cuda.synchronize()
        for a, b in zip(got, want):
            assert torch.equal(a, b), name
        assert int(got[4][voro.STAT_NAMES.index("rays")]) > 0


def test_noalloc_refuses_more_views_than_the_scratch_holds(scene):
    ds = scene
    cams = synth.config5_cameras(scale=0.02)
    cams = (cams * 3)[:voro.MAX_VIEWS + 1]
    rgb = torch.zeros((sum(c.n_pixels for c in cams), 3), device=ds.sites.device)
    T = torch.zeros(rgb.shape[0], device=ds.sites.device)
    ray = torch.zeros((sum(c.n_rays for c in cams), 4), device=ds.sites.device)
    with pytest.raises(voro.VoroError) as e:
        voro.voro_render_views_fwd_noalloc(ds, cams, voro.default_params(), rgb, T, ray)
    assert e.value.status == voro.VORO_EINVAL
    assert "maximum" in str(e.value)
