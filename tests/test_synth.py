"""Input generation: determinism by seed and the parallel certified Delaunay
adjacency (must equal scipy's global Qhull exactly)."""
import numpy as np

from paper_2608_17682_amd import synth


def test_scenes_are_deterministic():
    a = synth.scene_uniform(300, 4, seed=3)
    b = synth.scene_uniform(300, 4, seed=3)
    for f in ("sites", "density", "texels", "nbr_off", "nbr_idx"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = synth.scene_uniform(300, 4, seed=4)
    assert not np.array_equal(a.sites, c.sites)


def test_parallel_adjacency_equals_qhull():
    s = synth.scene_shell(60_000, 2, seed=9, with_csr=False)
    off, idx = synth.delaunay_csr(s.sites)
    off2, idx2 = synth.delaunay_csr_parallel(s.sites, blocks_per_axis=3, workers=4)
    assert np.array_equal(off, off2) and np.array_equal(idx, idx2)


def test_parallel_adjacency_clustered():
    rng = np.random.default_rng(1)
    pts = np.concatenate([rng.normal(scale=0.05, size=(20_000, 3)) + c
                          for c in ([0, 0, 0], [1, 1, 0], [-1, 0.5, 1])]
                         + [rng.uniform(-2, 2, (10_000, 3))]).astype(np.float32)
    off, idx = synth.delaunay_csr(pts)
    off2, idx2 = synth.delaunay_csr_parallel(pts, blocks_per_axis=3, workers=4)
    assert np.array_equal(off, off2) and np.array_equal(idx, idx2)


def test_config_shapes():
    cams = synth.config5_cameras(scale=1.0)
    assert [c.model for c in cams] == [0, 0, 1, 1, 2, 2, 3, 3]
    assert sum(c.n_rays for c in cams) == 2 * 1280 * 840 + 2 * 1024 * 1024 + 2 * 960 * 540 + \
        2 * 640 * 480 * 4
    s, c = synth.config1()
    assert s.n == 512 and s.tex_res == 4 and c[0].width == 64
