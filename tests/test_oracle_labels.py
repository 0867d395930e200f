"""Pins of the exact any-hit labels (visible = no triangle hit with 0 < t < t_max):
hand cases of the watertight test and BVH == brute force."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2306_07191_amd import synth as S

TRI = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)


def test_centroid_hit_and_misses():
    c = TRI.mean(axis=0).astype(np.float64)
    o = c + [0, 0, 2]
    assert O.ray_tri(o, [0, 0, -1], np.inf, TRI)          # through the centroid
    assert O.ray_tri(c - [0, 0, 2], [0, 0, 1], np.inf, TRI)  # from behind: double-sided
    assert not O.ray_tri(o, [0, 0, 1], np.inf, TRI)       # triangle behind the origin
    assert not O.ray_tri([2, 2, 2], [0, 0, -1], np.inf, TRI)  # outside the triangle
    assert not O.ray_tri(o, [1, 0, 0], np.inf, TRI)       # parallel to the plane


def test_tmax_is_strict():
    o = np.array([0.25, 0.25, 2.0])
    assert not O.ray_tri(o, [0, 0, -1], 2.0, TRI)  # hit exactly at t = t_max is not an occluder
    assert O.ray_tri(o, [0, 0, -1], 2.0 + 1e-12, TRI)
    assert not O.ray_tri(o, [0, 0, -1], 1.999, TRI)
    # a hit at t = 0 (origin on the surface) does not occlude
    assert not O.ray_tri([0.25, 0.25, 0.0], [0, 0, 1], np.inf, TRI)


def test_shared_edge_is_watertight():
    """Two triangles sharing the diagonal of a square: rays through the shared edge
    must hit at least one of them (no leak)."""
    a = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0]], np.float32)
    b = np.array([[0, 0, 0], [1, 1, 0], [0, 1, 0]], np.float32)
    g = np.random.default_rng(0)
    for s in g.uniform(0, 1, 200):
        p = np.array([s, s, 0.0])
        o = p + [0.3, -0.2, 1.5]
        d = p - o
        assert O.ray_tri(o, d, np.inf, a) or O.ray_tri(o, d, np.inf, b)
    # a shared vertex as well
    o = np.array([0.2, 0.7, -3.0])
    d = -o
    assert O.ray_tri(o, d, np.inf, a) or O.ray_tri(o, d, np.inf, b)


def test_bvh_equals_brute_force_random_meshes():
    g = np.random.default_rng(1)
    for trial in range(200):
        T = int(g.integers(1, 65))
        tris = S.random_triangles(T, g)
        if trial % 4 == 0:  # shared edges and vertices: a fan
            c = g.uniform(-1, 1, 3)
            ring = g.uniform(-1, 1, (T + 1, 3))
            tris = np.stack([np.broadcast_to(c, (T, 3)), ring[:-1], ring[1:]], axis=1).astype(np.float32)
        box = S.mesh_aabb(tris)
        rays, tmax = S.rays_sphere_to_box(300, box, g)
        tmax = np.where(g.uniform(size=300) < 0.3, g.uniform(0.5, 4.0, 300), tmax).astype(np.float32)
        vb = O.anyhit_brute(tris, rays, tmax, nthreads=1)
        vv = O.BVH(tris).anyhit(rays, tmax, nthreads=1)
        np.testing.assert_array_equal(vb, vv)


def test_bvh_equals_brute_force_tiny_workload():
    w = S.tiny_workload()
    vb = O.anyhit_brute(w["tris"], w["rays"], w["tmax"])
    vv = O.BVH(w["tris"]).anyhit(w["rays"], w["tmax"])
    np.testing.assert_array_equal(vb, vv)
    assert 0.0 < vb.mean() < 0.2  # the tiny mesh occludes most rays aimed into its box


def test_visible_when_no_triangles():
    w = S.tiny_workload(n_rays=50)
    empty = np.zeros((0, 3, 3), np.float32)
    assert (O.anyhit_brute(empty, w["rays"], w["tmax"]) == 1).all()
    assert (O.BVH(empty).anyhit(w["rays"], w["tmax"]) == 1).all()


# ---- closest hit (primary rays: the depth the network can encode, Sec. 7) ----

def test_closest_hit_hand_cases():
    near = np.array([[-1, -1, 1, 2, -1, 1, -1, 2, 1]], np.float32)   # plane z = 1
    far = np.array([[-1, -1, 3, 2, -1, 3, -1, 2, 3]], np.float32)    # plane z = 3
    tris = np.concatenate([far, near])
    rays = np.array([[0.2, 0.1, -2, 0, 0, 1],      # both planes: nearest at t = 3
                     [0.2, 0.1, -2, 0, 0, 2],      # t in units of d: 1.5
                     [0.2, 0.1, -2, 0, 0, 1],      # t_max = 3 exactly: the near hit is excluded (strict)
                     [0.2, 0.1, 2, 0, 0, 1],       # between the planes, looking up: t = 1
                     [0.2, 0.1, 2, 0, 0, -1],      # looking down: t = 1 (double-sided)
                     [5.0, 5.0, -2, 0, 0, 1]],     # misses both
                    np.float32)
    tmax = np.array([np.inf, np.inf, 3.0, np.inf, np.inf, np.inf], np.float32)
    t = O.closest_brute(tris, rays, tmax, nthreads=1)
    np.testing.assert_array_equal(t, [3.0, 1.5, np.inf, 1.0, 1.0, np.inf])
    np.testing.assert_array_equal(O.BVH(tris).closest(rays, tmax, nthreads=1), t)


def test_closest_bvh_equals_brute_force_and_agrees_with_any_hit():
    g = np.random.default_rng(7)
    for trial in range(100):
        T = int(g.integers(1, 200))
        tris = S.random_triangles(T, g)
        box = S.mesh_aabb(tris)
        rays, tmax = S.rays_sphere_to_box(300, box, g)
        tmax = np.where(g.uniform(size=300) < 0.3, g.uniform(0.5, 4.0, 300), tmax).astype(np.float32)
        tb = O.closest_brute(tris, rays, tmax, nthreads=1)
        np.testing.assert_array_equal(O.BVH(tris).closest(rays, tmax, nthreads=1), tb)
        # a closest hit exists iff the any-hit test reports an occluder, and it lies in (0, t_max)
        vis = O.anyhit_brute(tris, rays, tmax, nthreads=1)
        np.testing.assert_array_equal(np.isfinite(tb), vis == 0)
        hit = np.isfinite(tb)
        assert (tb[hit] > 0).all() and (tb[hit] < tmax[hit]).all()
        # and it is the smallest of the individual hit distances
        k = int(np.nonzero(hit)[0][0]) if hit.any() else None
        if k is not None:
            ts = [O.ray_tri_t(rays[k, :3].astype(np.float64), rays[k, 3:].astype(np.float64), float(tmax[k]), tr)
                  for tr in tris]
            assert tb[k] == min(x for x in ts if x is not None)


# ---- the watertight test in binary32 (the GPU caster's precision) ----

def test_binary32_test_hand_cases_and_watertightness():
    near = np.array([[-1, -1, 1, 2, -1, 1, -1, 2, 1]], np.float32)
    far = np.array([[-1, -1, 3, 2, -1, 3, -1, 2, 3]], np.float32)
    rays = np.array([[0.2, 0.1, -2, 0, 0, 1], [0.2, 0.1, -2, 0, 0, 1], [5.0, 5.0, -2, 0, 0, 1]], np.float32)
    vis, t = O.trace_brute32(np.concatenate([far, near]), rays, np.array([np.inf, 3.0, np.inf], np.float32), 1)
    np.testing.assert_array_equal(vis, [0, 1, 1])  # t_max = 3 exactly excludes the hit at 3 (strict)
    assert t[0] == np.float32(3.0) and np.isinf(t[1]) and np.isinf(t[2])
    # two triangles sharing an edge: rays through points of the edge never leak
    a = np.array([0, 0, 0, 1, 0, 0, 0, 1, 0], np.float32)
    b = np.array([1, 0, 0, 1, 1, 0, 0, 1, 0], np.float32)
    g = np.random.default_rng(2)
    s = g.uniform(0, 1, 2000)
    p = np.stack([s, 1 - s, np.zeros_like(s)], 1)
    o = p + g.normal(size=(2000, 3)) * [0.3, 0.3, 0.0] + [0, 0, 1.5]
    r = np.concatenate([o, p - o], 1).astype(np.float32)
    v, _ = O.trace_brute32(np.stack([a, b]), r, np.full(2000, np.inf, np.float32), 1)
    assert (v == 0).all()


def test_binary32_bvh_equals_brute_force_and_tracks_binary64():
    g = np.random.default_rng(12)
    agree = []
    for trial in range(60):
        T = int(g.integers(1, 300))
        tris = S.random_triangles(T, g)
        box = S.mesh_aabb(tris)
        rays, tmax = S.rays_sphere_to_box(400, box, g)
        tmax = np.where(g.uniform(size=400) < 0.3, g.uniform(0.5, 4.0, 400), tmax).astype(np.float32)
        vb, tb = O.trace_brute32(tris, rays, tmax, nthreads=1)
        vv, tv = O.BVH(tris).trace32(rays, tmax, nthreads=1)
        np.testing.assert_array_equal(vv, vb)
        np.testing.assert_array_equal(tv, tb)
        v64 = O.anyhit_brute(tris, rays, tmax, nthreads=1)
        agree.append((v64 == vb).mean())
        t64 = O.closest_brute(tris, rays, tmax, nthreads=1)
        both = np.isfinite(t64) & np.isfinite(tb)
        assert (np.abs(tb[both] - t64[both]) <= 1e-5 * t64[both]).mean() >= 0.999
    assert np.mean(agree) >= 0.999
