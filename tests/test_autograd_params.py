"""Host-side checks of the autograd wrappers (no device: every case raises
before anything reaches the library's compute entry points)."""
import numpy as np
import pytest
import torch

from paper_2608_17682_amd import synth, voro
from paper_2608_17682_amd.autograd import backward_params, render, render_views


def _args():
    sites = torch.zeros((4, 3), requires_grad=True)
    dens = torch.ones(4, requires_grad=True)
    tex = torch.zeros((4, 2, 2, 4), requires_grad=True)
    off = torch.zeros(5, dtype=torch.int32)
    idx = torch.zeros(0, dtype=torch.int32)
    cam = synth.Camera(synth.PINHOLE, 4, 4, synth.look_at((0, 0, -3), (0, 0, 0)),
                       np.radians(60.0), 6.0)
    return sites, dens, tex, off, idx, cam


def test_backward_params_take_the_forward_walk_and_the_own_launch_shape():
    pf = voro.default_params(tile_w=8, tile_h=8, block=128, schedule=1, t_stop=2e-4)
    pb = voro.default_params(tile_w=16, tile_h=4, block=256, schedule=2, t_stop=2e-4)
    q = backward_params(pf, pb)
    assert (q.tile_w, q.tile_h, q.block, q.schedule) == (16, 4, 256, 2)
    assert q.t_stop == pf.t_stop and q.max_steps == pf.max_steps
    q0 = backward_params(pf)
    assert bytes(q0) == bytes(pf)


@pytest.mark.parametrize("field,value", [("t_stop", 1e-3), ("max_steps", 7), ("tie_window", 0.0),
                                         ("appearance", 1), ("edge_fp16", 1), ("skip_w", 1e-3)])
def test_views_reject_a_backward_walk_other_than_the_forward(field, value):
    sites, dens, tex, off, idx, cam = _args()
    pb = voro.default_params()
    setattr(pb, field, value)
    with pytest.raises(ValueError, match=field):
        render_views(sites, dens, tex, off, idx, [cam], voro.default_params(), pb)


@pytest.mark.parametrize("field,value", [("edge_fp16", 1), ("skip_w", 1e-3)])
def test_gradients_refuse_forward_only_variants(field, value):
    sites, dens, tex, off, idx, cam = _args()
    p = voro.default_params()
    setattr(p, field, value)
    with pytest.raises(ValueError, match=field):
        render_views(sites, dens, tex, off, idx, [cam], p)
    o = torch.zeros((2, 3))
    d = torch.zeros((2, 3))
    tm = torch.ones(2)
    st = torch.zeros(2, dtype=torch.int32)
    with pytest.raises(ValueError, match=field):
        render(sites, dens, tex, off, idx, o, d, tm, st, p)


def test_stored_exits_must_not_be_negative():
    sites, dens, tex, off, idx, cam = _args()
    with pytest.raises(ValueError, match="stored_exits"):
        render_views(sites, dens, tex, off, idx, [cam], stored_exits=-1)
    o = torch.zeros((2, 3))
    d = torch.zeros((2, 3))
    tm = torch.ones(2)
    st = torch.zeros(2, dtype=torch.int32)
    with pytest.raises(ValueError, match="stored_exits"):
        render(sites, dens, tex, off, idx, o, d, tm, st, stored_exits=-1)
