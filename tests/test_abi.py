"""The C-ABI library loads, exports every entry point include/voro.h declares,
and validates arguments on the host (no device needed, no compute calls)."""
import ctypes
import os
import re

import pytest

from paper_2608_17682_amd import voro

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "voro.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(voro_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    return voro.lib()


def test_every_declared_symbol_is_exported(L):
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(voro.EXPORTS) == names


def test_struct_layouts_match_the_header(tmp_path):
    # compile a probe against include/voro.h and compare every field offset
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"voro_scene": voro.voro_scene, "voro_params": voro.voro_params,
               "voro_camera": voro.voro_camera}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "voro.h"', "int main(void){"]
    for sname, cls in structs.items():
        lines.append(f'printf("{sname} size %zu\\n", sizeof({sname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{sname} {fname} %zu\\n", offsetof({sname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for sname, cls in structs.items():
        assert got[(sname, "size")] == ctypes.sizeof(cls), sname
        for fname, _ in cls._fields_:
            assert got[(sname, fname)] == getattr(cls, fname).offset, (sname, fname)


def test_version_and_defaults(L):
    assert voro.version().startswith("voro ")
    p = voro.default_params()
    assert p.t_stop == pytest.approx(1e-4) and p.max_steps == 4096
    assert p.tie_window == pytest.approx(1e-6) and p.skip_w == 0.0
    assert L.voro_default_params(None) == voro.VORO_EINVAL


def fake_scene(n=10, m=40, res=4, dtype=0, addr=0x100000):
    s = voro.voro_scene()
    s.n_sites, s.tex_res, s.tex_dtype, s.tex_maps, s.n_edges = n, res, dtype, 0, m
    s.sites, s.density, s.nbr_off, s.nbr_idx, s.texels = addr, addr, addr, addr, addr
    return s


def test_workspace_size_host_only(L):
    s = fake_scene(100, 1500)
    n = ctypes.c_size_t()
    assert L.voro_workspace_size(ctypes.byref(s), ctypes.byref(n)) == 0
    assert n.value >= 100 * 32 + 1500 * 16 and n.value % 256 == 0


@pytest.mark.parametrize("field,value", [("n_sites", 0), ("tex_res", 1), ("tex_res", 17),
                                         ("tex_dtype", 7), ("n_edges", -1), ("tex_maps", 4)])
def test_bad_scene_is_einval(L, field, value):
    s = fake_scene()
    setattr(s, field, value)
    n = ctypes.c_size_t()
    assert L.voro_workspace_size(ctypes.byref(s), ctypes.byref(n)) == voro.VORO_EINVAL
    assert voro.last_error() != ""


def test_misaligned_texels_is_einval(L):
    s = fake_scene()
    s.texels = 0x100008  # f32 texels need 16-byte alignment
    n = ctypes.c_size_t()
    assert L.voro_workspace_size(ctypes.byref(s), ctypes.byref(n)) == voro.VORO_EINVAL


def test_render_validation_before_device(L):
    s = fake_scene()
    ws = 0x200000
    n = ctypes.c_size_t()
    L.voro_workspace_size(ctypes.byref(s), ctypes.byref(n))
    p = voro.default_params()
    A = 0x300000
    # workspace too small
    st = L.voro_render_fwd(ctypes.byref(s), ws, 16, A, A, A, A, 8, ctypes.byref(p), A, A, None,
                           None, None, None, 0, None, None)
    assert st == voro.VORO_EWORKSPACE
    # missing ray arrays
    st = L.voro_render_fwd(ctypes.byref(s), ws, n.value, None, A, A, A, 8, ctypes.byref(p), A, A,
                           None, None, None, None, 0, None, None)
    assert st == voro.VORO_EINVAL
    # bad params
    for field, value in [("max_steps", 0), ("lanes_per_ray", 3), ("block", 100),
                         ("t_stop", float("nan")), ("appearance", 1), ("appearance", 2),
                         ("appearance", 3)]:
        q = voro.default_params(**{field: value})
        st = L.voro_render_fwd(ctypes.byref(s), ws, n.value, A, A, A, A, 8, ctypes.byref(q), A, A,
                               None, None, None, None, 0, None, None)
        assert st in (voro.VORO_EINVAL, voro.VORO_EUNSUPPORTED), field
    q = voro.default_params(appearance=3)
    assert L.voro_render_fwd(ctypes.byref(s), ws, n.value, A, A, A, A, 8, ctypes.byref(q), A, A,
                             None, None, None, None, 0, None, None) == voro.VORO_EUNSUPPORTED
    # the spherical-harmonic comparison model is forward only and needs its
    # coefficient layout
    q = voro.default_params(appearance=2)
    assert L.voro_render_fwd(ctypes.byref(s), ws, n.value, A, A, A, A, 8, ctypes.byref(q), A, A,
                             None, None, None, None, 0, None, None) == voro.VORO_EINVAL
    assert "spherical-harmonic" in voro.last_error()
    assert L.voro_render_bwd(ctypes.byref(s), ws, n.value, A, A, A, A, 8, ctypes.byref(q), A, A, A,
                             None, None, None, None, 0, A, A, A, None, None) == voro.VORO_EUNSUPPORTED
    # the full appearance model needs two maps per cell, and the single-map
    # model one
    q = voro.default_params(appearance=1)
    assert L.voro_render_fwd(ctypes.byref(s), ws, n.value, A, A, A, A, 8, ctypes.byref(q), A, A,
                             None, None, None, None, 0, None, None) == voro.VORO_EINVAL
    assert "two texture maps" in voro.last_error()
    s2 = voro.voro_scene.from_buffer_copy(s)
    s2.tex_maps = 2
    n2 = ctypes.c_size_t()
    assert L.voro_workspace_size(ctypes.byref(s2), ctypes.byref(n2)) == 0
    assert L.voro_render_fwd(ctypes.byref(s2), ws, n2.value, A, A, A, A, 8, ctypes.byref(p), A, A,
                             None, None, None, None, 0, None, None) == voro.VORO_EINVAL
    assert "one texture map" in voro.last_error()
    q = voro.default_params(tile_w=8, tile_h=4)  # 8*4*1 != 64
    assert L.voro_render_fwd(ctypes.byref(s), ws, n.value, A, A, A, A, 8, ctypes.byref(q), A, A,
                             None, None, None, None, 0, None, None) == voro.VORO_EINVAL
    # backward refuses skip_w != 0
    q = voro.default_params(skip_w=1e-3)
    st = L.voro_render_bwd(ctypes.byref(s), ws, n.value, A, A, A, A, 8, ctypes.byref(q), A, A, A,
                           None, None, None, None, 0, A, A, A, None, None)
    assert st == voro.VORO_EINVAL and "skip_w" in voro.last_error()
    # the distortion loss's saved totals and its upstream gradient come together
    st = L.voro_render_bwd(ctypes.byref(s), ws, n.value, A, A, A, A, 8, ctypes.byref(p), A, A, A,
                           None, A, None, None, 0, A, A, A, None, None)
    assert st == voro.VORO_EINVAL and "g_dist" in voro.last_error()
    # R == 0 is a no-op even without a device
    assert L.voro_render_fwd(ctypes.byref(s), ws, n.value, None, None, None, None, 0,
                             ctypes.byref(p), None, None, None, None, None, None, 0, None, None) == 0


def test_valid_call_without_device_is_enodev(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    s = fake_scene()
    n = ctypes.c_size_t()
    L.voro_workspace_size(ctypes.byref(s), ctypes.byref(n))
    assert L.voro_prepare(ctypes.byref(s), 0x200000, n.value, None, None) == voro.VORO_ENODEV


def test_camera_validation(L):
    from paper_2608_17682_amd import synth
    cams = synth.config5_cameras(scale=0.05)
    nr, npx = voro.voro_camera_counts(cams)
    assert npx == sum(c.width * c.height for c in cams)
    assert nr == sum(c.width * c.height * c.spp for c in cams)
    bad = voro.camera_array(cams[:1])
    bad[0].spp = 4  # only thin lens takes several samples
    assert L.voro_camera_counts(bad, 1, None, None) == voro.VORO_EINVAL
    bad = voro.camera_array(cams[6:7])
    bad[0].spp = 3  # not a square
    assert L.voro_camera_counts(bad, 1, None, None) == voro.VORO_EINVAL
    assert L.voro_camera_counts(voro.camera_array(cams), 0, None, None) == voro.VORO_EINVAL
    many = voro.camera_array(cams + cams + cams[:1])
    assert L.voro_camera_counts(many, len(many), None, None) == voro.VORO_EINVAL


def test_views_trace_validation(L):
    # a stored-exit buffer needs a capacity of at least one step and 8-byte
    # alignment; both are checked before anything touches a device
    from paper_2608_17682_amd import synth
    arr = voro.camera_array(synth.config5_cameras(scale=0.05)[:1])
    s = fake_scene()
    p = voro.default_params()
    A = 0x10000
    args = (ctypes.byref(s), A, 1 << 20, arr, 1, ctypes.byref(p), A, A, None, None)
    assert L.voro_render_views_fwd(*args, A, 0, None, None) == voro.VORO_EINVAL
    assert "trace_cap" in voro.last_error()
    assert L.voro_render_views_fwd(*args, A + 4, 16, None, None) == voro.VORO_EINVAL
    assert "aligned" in voro.last_error()
    bargs = (ctypes.byref(s), A, 1 << 20, arr, 1, ctypes.byref(p), A, A, None)
    assert L.voro_render_views_bwd(*bargs, A, -3, A, None, A, A, A, None,
                                   None) == voro.VORO_EINVAL
    assert "trace_cap" in voro.last_error()
    import torch
    with pytest.raises(ValueError):
        voro._trace_args(torch.zeros((4, 7, 2), dtype=torch.int64), 7)
    with pytest.raises(ValueError):
        voro._trace_args(torch.zeros((4, 6, 2), dtype=torch.int32), 7)
    with pytest.raises(ValueError, match="device memory"):
        voro._trace_args(torch.zeros((4, 7, 2), dtype=torch.int32), 7)
    assert voro._trace_args(None, 7) == (None, 0)


def test_cast_and_reorder_validation(L):
    assert L.voro_cast_texels(0x1000, 0x2000, 16, 0, None) == voro.VORO_EINVAL
    assert L.voro_cast_texels(None, None, 0, 1, None) == 0
    n = ctypes.c_size_t()
    assert L.voro_reorder_scratch_size(1000, 15000, ctypes.byref(n)) == 0 and n.value > 12000
