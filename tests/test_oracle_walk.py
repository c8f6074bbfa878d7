"""Pins of the oracle's partition and walk (Sec. 3.1) against closed forms,
an independent O(N^2) interval method, and the Delaunay adjacency."""
import math

import numpy as np
import pytest

from oracle import walk, render
from paper_2608_17682_amd import synth


def test_two_site_bisector_at_midpoint():
    # p0 = (0,0,-1/2), p1 = (0,0,1/2), o = (0,0,-3), w = +z: the bisector is
    # the plane z = 0, crossed at t* = 3 exactly.
    sites = np.array([[0, 0, -0.5], [0, 0, 0.5]], np.float32)
    o = np.array([0.0, 0.0, -3.0])
    w = np.array([0.0, 0.0, 1.0])
    i0, gap = walk.nearest_site(sites, o)
    assert i0 == 0 and gap > 0
    t, j, _ = walk.exit_crossing(sites, 0, o, w)
    assert j == 1 and t == 3.0
    t2, j2, _ = walk.exit_crossing(sites, 1, o, w)
    assert j2 == -1 and math.isinf(t2)   # unbounded cell: no forward face


def test_single_site_one_segment():
    sites = np.array([[0.3, -0.2, 0.1]], np.float32)
    steps = list(walk.walk_stepwise(sites, [0, 0, -3], [0, 0, 1], 6.0))
    assert len(steps) == 1 and steps[0][0] == 0 and math.isinf(steps[0][1])
    cells, a, b = walk.cell_intervals(sites, [0, 0, -3], [0, 0, 1], 6.0)
    assert list(cells) == [0] and a[0] == 0.0 and b[0] == 6.0


def test_lattice_axis_ray_crosses_midplanes():
    # Integer lattice: a ray along +x at (y,z) = (0.1, 0.2) stays in the cells of
    # the sites (k,0,0) and crosses their bisectors at x = k + 1/2.
    sites = synth.lattice_sites(5, 1.0)
    o = np.array([-2.6, 0.1, 0.2])
    w = np.array([1.0, 0.0, 0.0])
    steps = list(walk.walk_stepwise(sites, o, w, 6.0))
    xs = [float(sites[s[0], 0]) for s in steps]
    assert xs == [-2.0, -1.0, 0.0, 1.0, 2.0]
    for s in steps:
        assert sites[s[0], 1] == 0.0 and sites[s[0], 2] == 0.0
    exits = [s[1] for s in steps[:-1]]
    np.testing.assert_allclose(exits, [1.1, 2.1, 3.1, 4.1], rtol=0, atol=1e-12)
    assert math.isinf(steps[-1][1])


def test_nearest_site_ties_to_smallest_index():
    sites = np.array([[1, 0, 0], [-1, 0, 0], [0, 5, 0]], np.float32)
    i, gap = walk.nearest_site(sites, [0, 0, 0])
    assert i == 0 and gap == 0.0
    sites2 = sites[[1, 0, 2]]
    i2, _ = walk.nearest_site(sites2, [0, 0, 0])
    assert i2 == 0


def test_nearest_site_on_lattice():
    sites = synth.lattice_sites(4, 0.5)
    rng = np.random.default_rng(0)
    for _ in range(20):
        x = rng.uniform(-0.7, 0.7, 3)
        i, _ = walk.nearest_site(sites, x)
        # nearest lattice point: round to the half-offset grid
        g = np.round((x + 0.75) / 0.5) * 0.5 - 0.75
        g = np.clip(g, -0.75, 0.75)
        np.testing.assert_allclose(sites[i], g, atol=1e-7)


@pytest.mark.parametrize("seed,n", [(0, 48), (1, 96), (2, 160)])
def test_interval_method_equals_stepwise(seed, n):
    rng = np.random.default_rng(seed)
    sites = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    for _ in range(12):
        o = rng.uniform(-1.5, 1.5, 3)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        tmax = 4.0
        cells, a, b = walk.cell_intervals(sites, o, w, tmax)
        steps = list(walk.walk_stepwise(sites, o, w, tmax))
        assert [s[0] for s in steps] == list(cells)
        ex = [min(s[1], tmax) for s in steps]
        np.testing.assert_allclose(ex, b, rtol=0, atol=1e-11)
        np.testing.assert_allclose(a[1:], b[:-1], rtol=0, atol=1e-11)
        assert a[0] == 0.0 and b[-1] == tmax


def test_no_repeats_and_lengths_sum_to_extent():
    scene = synth.scene_uniform(256, 4, seed=7)
    rng = np.random.default_rng(3)
    dens = np.full(scene.n, 1e-9, np.float32)
    for _ in range(10):
        o = rng.uniform(-1.2, 1.2, 3)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        rec = render.render_ray(scene.sites, dens, scene.texels, o, w, 5.0, t_stop=0.0)
        assert len(set(rec.cells)) == rec.K
        assert abs(sum(rec.delta) - 5.0) < 1e-12


def test_next_cell_in_delaunay_row():
    scene = synth.scene_uniform(512, 4, seed=1)
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(12):
        o = rng.uniform(-1.5, 1.5, 3)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        for i, ex, j, _ in walk.walk_stepwise(scene.sites, o, w, 6.0):
            if j >= 0 and ex < 6.0:
                assert walk.csr_contains(scene.nbr_off, scene.nbr_idx, i, j)
                checked += 1
    assert checked > 50


def test_csr_symmetric_no_self_loops():
    scene = synth.scene_uniform(300, 4, seed=5)
    off, idx = scene.nbr_off, scene.nbr_idx
    rows = np.repeat(np.arange(scene.n), np.diff(off))
    assert not np.any(rows == idx)
    fwd = set(zip(rows.tolist(), idx.tolist()))
    assert all((j, i) in fwd for i, j in fwd)


@pytest.mark.parametrize("kind", ["uniform", "shell", "lattice"])
def test_per_ray_bisectors_equal_exit_crossing(kind):
    # The per-ray form (dot products s = p.w, h = |p|^2/2 - p.o taken once)
    # must take every decision exit_crossing takes: the same next cell, the
    # same crossing to rounding, the same gap; on the integer lattice exact
    # ties must still go to the smaller index.
    rng = np.random.default_rng({"uniform": 0, "shell": 1, "lattice": 2}[kind])
    if kind == "uniform":
        sites = rng.uniform(-1, 1, (400, 3)).astype(np.float32)
    elif kind == "shell":
        v = rng.normal(size=(400, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        sites = (v + rng.normal(scale=0.01, size=v.shape)).astype(np.float32)
    else:
        sites = synth.lattice_sites(6, 1.0)
    checked = ties = 0
    for _ in range(8):
        if kind == "lattice":
            # axis-aligned rays through lattice planes: many exact ties
            o = np.round(rng.uniform(-3, 3, 3) * 2) / 2
            w = np.zeros(3)
            w[rng.integers(3)] = rng.choice([-1.0, 1.0])
        else:
            o = rng.uniform(-1.5, 1.5, 3)
            w = rng.normal(size=3)
            w /= np.linalg.norm(w)
        ray = walk.RayBisectors(sites, o, w)
        for i in range(0, len(sites), 7):
            t0, j0, g0 = walk.exit_crossing(sites, i, o, w)
            t1, j1, g1 = ray.exit(i)
            assert j1 == j0, (i, t0, t1)
            if j0 < 0:
                assert math.isinf(t1) and math.isinf(g1)
                continue
            # both forms round n.w differently by ~1e-16: at a grazing face
            # (small n.w) the crossing moves by |t| 1e-16 / |n.w|
            b = float((sites[j0].astype(np.float64) - sites[i]) @ w)
            tol = 1e-12 * max(1.0, abs(t0)) + 4e-16 * abs(t0) / abs(b)
            assert abs(t1 - t0) <= tol
            if math.isinf(g0):
                assert math.isinf(g1)
            else:
                assert abs(g1 - g0) <= 2 * tol + 1e-12 * abs(g0)
                ties += g0 == 0.0
            checked += 1
    assert checked > 100
    if kind == "lattice":
        assert ties > 10
