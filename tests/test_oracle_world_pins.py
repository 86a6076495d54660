"""Pins of the oracle's shared scenes (Sec. 3.4: KiloNeuS objects rendered with
classic primitives): primitive intersections in closed form, the reduction to
the single-object renderer, instance transforms, occlusion between objects,
continuation past an instance box, and path-tracing mixtures.  CPU only."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2206_10885_amd import synth

RNG = np.random.default_rng(2024)


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def test_sphere_hits_closed_form():
    for _ in range(200):
        c = RNG.uniform(-1, 1, 3)
        r = RNG.uniform(0.1, 0.8)
        d = _unit(RNG.standard_normal(3))
        dist = RNG.uniform(1.0, 3.0)
        o = c - (r + dist) * d      # on the line through the centre, outside
        ok, t, n = O.prim_hit(O.PRIM_SPHERE, [*c, r], o, d)
        assert ok and abs(t - dist) < 1e-12
        assert np.allclose(n, -d, atol=1e-12)         # facing the ray
        # from the centre: the exit at t = r, normal turned toward the ray
        ok, t, n = O.prim_hit(O.PRIM_SPHERE, [*c, r], c, d)
        assert ok and abs(t - r) < 1e-12 and np.allclose(n, -d, atol=1e-12)
        # a ray that passes at distance > r misses
        side = _unit(np.cross(d, RNG.standard_normal(3)))
        ok, _, _ = O.prim_hit(O.PRIM_SPHERE, [*c, r], o + 1.01 * r * side, d)
        assert not ok
    # t_min past both roots
    ok, _, _ = O.prim_hit(O.PRIM_SPHERE, [0, 0, 0, 1], [0, 0, 5], [0, 0, -1], t_min=6.5)
    assert not ok


def test_box_hits_closed_form():
    lo, hi = np.array([-0.5, -0.2, 0.1]), np.array([0.4, 0.7, 0.9])
    for axis in range(3):
        for sgn in (1.0, -1.0):
            d = np.zeros(3)
            d[axis] = sgn
            o = (lo + hi) / 2
            o[axis] = (lo[axis] - 2.0) if sgn > 0 else (hi[axis] + 2.0)
            ok, t, n = O.prim_hit(O.PRIM_BOX, [*lo, *hi], o, d)
            assert ok and abs(t - 2.0) < 1e-12
            want = np.zeros(3)
            want[axis] = -sgn
            assert np.array_equal(n, want)
            # from inside: the far face
            ok, t, n = O.prim_hit(O.PRIM_BOX, [*lo, *hi], (lo + hi) / 2, d)
            assert ok and abs(t - (hi[axis] - lo[axis]) / 2) < 1e-12 and np.array_equal(n, want)
    # parallel to a slab and outside it: no hit
    ok, _, _ = O.prim_hit(O.PRIM_BOX, [*lo, *hi], [0.0, 5.0, 0.5], [1.0, 0.0, 0.0])
    assert not ok


def test_triangle_hits_closed_form():
    A, B, C = np.array([0.1, -0.2, 0.3]), np.array([0.9, 0.0, 0.2]), np.array([0.2, 0.8, 0.5])
    nrm = _unit(np.cross(B - A, C - A))
    for _ in range(200):
        u, v = RNG.uniform(0, 1, 2)
        if u + v > 1:
            u, v = 1 - u, 1 - v
        x = A + u * (B - A) + v * (C - A)
        d = _unit(RNG.standard_normal(3))
        if abs(d @ nrm) < 0.1:
            continue
        dist = RNG.uniform(0.5, 2.0)
        ok, t, n = O.prim_hit(O.PRIM_TRIANGLE, [*A, *B, *C], x - dist * d, d)
        assert ok and abs(t - dist) < 1e-10
        assert np.allclose(n, -np.sign(d @ nrm) * nrm, atol=1e-12)
    # outside an edge (barycentric u + v > 1): no hit
    x = A + 0.7 * (B - A) + 0.6 * (C - A)
    ok, _, _ = O.prim_hit(O.PRIM_TRIANGLE, [*A, *B, *C], x + nrm, -nrm)
    assert not ok


@pytest.fixture(scope="module")
def c1():
    return synth.config_scene("c1"), synth.config_views("c1")[0]


def test_single_instance_world_is_the_single_object_renderer(c1):
    """A world with one instance at identity and no primitives renders
    exactly what the single-object renderer does (same operations)."""
    sc, view = c1
    os_ = O.OracleScene.from_scene(sc)
    w = O.OracleWorld([(os_, (0, 0, 0), 1.0)])
    a = w.render(view, 48, 40, 64, 1e-4)
    b = os_.render(view, 48, 40, 64, 1e-4)
    for k in ("rgb", "depth", "normal", "hit"):
        assert np.array_equal(a[k], b[k]), k
    assert set(np.unique(a["object"])) <= {-1, 0}
    env = synth.env_map(64, 32, seed=3)
    pa = w.path_trace(view, 24, 20, 64, 1e-4, spp=2, bounces=2, seed=11, env=env)
    pb = os_.path_trace(view, 24, 20, 64, 1e-4, spp=2, bounces=2, seed=11, env=env)
    for k in ("rgb", "depth", "normal", "hit"):
        assert np.array_equal(pa[k], pb[k]), k


def test_instance_transform_scales_depth(c1):
    """An instance scaled by s and translated by T, seen from the camera
    moved the same way, renders the same colours and normals at s times the
    depth (its MLPs see the same local points)."""
    sc, view = c1
    os_ = O.OracleScene.from_scene(sc)
    T, s = np.array([3.0, -1.5, 0.75]), 2.5
    w = O.OracleWorld([(os_, T, s)])
    v2 = synth.View(eye=tuple(T + s * np.asarray(view.eye)), look_at=tuple(T + s * np.asarray(view.look_at)),
                    up=view.up, tan_half_diag=1.0 / math.sqrt(2.5 ** 2 - 1))
    a = w.render(v2, 40, 40, 64, 1e-4)
    b = os_.render(view, 40, 40, 64, 1e-4)
    same = a["hit"] == b["hit"]
    assert same.mean() > 0.995            # rays within rounding of a grazing hit may flip
    both = same & (a["hit"] == 1)
    assert np.abs(a["depth"][both] - s * b["depth"][both]).max() < 1e-6
    assert np.abs(a["rgb"][both] - b["rgb"][both]).max() < 1e-6
    assert np.abs(a["normal"][both] - b["normal"][both]).max() < 1e-5


def test_primitive_occludes_and_is_occluded(c1):
    """A sphere primitive in front of the object covers it (depth and normal
    of the sphere in closed form, colour = its albedo); moved behind the
    object's surface, the object wins where both are hit."""
    sc, view = c1
    os_ = O.OracleScene.from_scene(sc)
    eye = np.asarray(view.eye)
    alb = (0.2, 0.6, 0.9)
    front = (O.PRIM_SPHERE, [0.0, 0.0, 1.2, 0.35], alb)
    w = O.OracleWorld([(os_, (0, 0, 0), 1.0)], [front])
    W = H = 40
    a = w.render(view, W, H, 64, 1e-4)
    alone = os_.render(view, W, H, 64, 1e-4)
    sph = 0
    for p in range(W * H):
        o, d = O.camera_ray(view, W, H, p // W, p % W)
        ok, t, n = O.prim_hit(O.PRIM_SPHERE, front[1], o, d)
        if ok:
            sph += 1
            assert a["object"][p] == -2 and abs(a["depth"][p] - t) < 1e-12
            assert np.allclose(a["rgb"][p], alb) and np.allclose(a["normal"][p], n)
        else:
            assert a["hit"][p] == alone["hit"][p] and abs(a["depth"][p] - alone["depth"][p]) < 1e-12
    assert sph > 50
    # inside the box, mostly behind the surface: the object wins exactly
    # where its march stops (hits) before the sphere, and keeps the depth it
    # has alone; elsewhere on the sphere, the sphere
    behind = (O.PRIM_SPHERE, [0.0, 0.0, -0.3, 0.45], alb)
    w2 = O.OracleWorld([(os_, (0, 0, 0), 1.0)], [behind])
    b = w2.render(view, W, H, 64, 1e-4)
    n_obj = n_prim = 0
    for p in range(W * H):
        o, d = O.camera_ray(view, W, H, p // W, p % W)
        ok, t, _ = O.prim_hit(O.PRIM_SPHERE, behind[1], o, d)
        tr = os_.trace(o, d, 64, 1e-4)
        if tr["status"] == O.HIT and (not ok or tr["t"] <= t):
            n_obj += 1
            assert b["object"][p] == 0 and abs(b["depth"][p] - alone["depth"][p]) < 1e-12
        elif ok:
            n_prim += 1
            assert b["object"][p] == -2 and abs(b["depth"][p] - t) < 1e-12
    assert n_obj > 500 and n_prim > 10, (n_obj, n_prim)


def test_ray_continues_past_a_missed_instance():
    """Two instances side by side along the view axis: rays that miss the
    near object's surface inside its box go on to the far one, which then
    renders as it would alone (depth offset by nothing: world distances)."""
    near = synth.sphere_scene(4, 32, 0.3, 0.0, seed=41)
    far = synth.sphere_scene(4, 32, 0.6, 0.0, seed=42)
    on, of = O.OracleScene.from_scene(near), O.OracleScene.from_scene(far)
    view = synth.View(eye=(0.0, 0.0, 6.0), tan_half_diag=0.18)
    w = O.OracleWorld([(on, (0.0, 0.0, 2.5), 1.0), (of, (0.0, 0.0, -1.0), 1.0)])
    W = H = 48
    a = w.render(view, W, H, 128, 1e-4)
    only_far = O.OracleWorld([(of, (0.0, 0.0, -1.0), 1.0)]).render(view, W, H, 128, 1e-4)
    only_near = O.OracleWorld([(on, (0.0, 0.0, 2.5), 1.0)]).render(view, W, H, 128, 1e-4)
    nh = only_near["hit"] == 1
    assert nh.sum() > 50 and (a["object"][nh] == 0).all()
    assert np.abs(a["depth"][nh] - only_near["depth"][nh]).max() < 1e-12
    rest = ~nh
    assert (a["hit"][rest] == only_far["hit"][rest]).all()
    fh = rest & (only_far["hit"] == 1)
    assert fh.sum() > 50 and (a["object"][fh] == 1).all()
    assert np.abs(a["depth"][fh] - only_far["depth"][fh]).max() < 1e-12


def test_path_trace_furnace_with_primitives():
    """Constant environment E and a convex sphere primitive of albedo a with
    one bounce: a scattered ray never meets the sphere again, so every sample
    contributes a E (hit) or E (miss), and each pixel is an exact mixture."""
    E, a = float(np.float32(0.8)), 0.35     # the map holds float32 texels
    env = np.full((16, 32, 3), E, np.float32)
    w = O.OracleWorld([], [(O.PRIM_SPHERE, [0.1, -0.05, 0.0, 0.7], (a, a, a))])
    view = synth.View(eye=(0.0, 0.0, 2.5))
    spp = 4
    r = w.path_trace(view, 32, 32, 64, 1e-4, spp=spp, bounces=1, seed=5, env=env)
    k = r["rgb"][:, 0] * spp / E              # = hits * a + misses, hits + misses = spp
    hits = (spp - k) / (1 - a)
    assert np.abs(hits - np.round(hits)).max() < 1e-9
    assert (np.round(hits) >= 0).all() and (np.round(hits) <= spp).all()
    assert (np.round(hits) == spp).sum() > 100 and (np.round(hits) == 0).sum() > 100


def test_interval_cut_inside_a_cell():
    """A sphere primitive just above a plane instance, inside one cell of
    it: rays that meet the sphere first show the sphere (the instance's
    march ends where the sphere cuts its interval, also inside a cell, so it
    does not go on to the plane below), the others the plane at its
    closed-form distance."""
    n = np.array([0.0, 1.0, 0.0])
    sc = synth.constant_color_plane_scene(2, 32, n, -0.3, [0.6, 0.35, 0.8], seed=3)
    sph = [0.5, -0.15, 0.5, 0.1]     # inside the cell [0, 1] x [-1, 0] x [0, 1]
    w = O.OracleWorld([(O.OracleScene.from_scene(sc), (0, 0, 0), 1.0)], [(O.PRIM_SPHERE, sph, (0.5, 0.5, 0.5))])
    view = synth.View(eye=(0.9, 1.6, 1.4), look_at=(0.5, -0.2, 0.5), tan_half_diag=0.25)
    W, H = 40, 30
    r = w.render(view, W, H, 128, 1e-4)
    n_s = n_p = 0
    for p in range(W * H):
        o, d = O.camera_ray(view, W, H, p // W, p % W)
        ok, ts, _ = O.prim_hit(O.PRIM_SPHERE, sph, o, d)
        tp = (-0.3 - o[1]) / d[1] if d[1] < 0 else np.inf
        xp = o + tp * d if np.isfinite(tp) else None
        in_box = xp is not None and abs(xp[0]) <= 1 and abs(xp[2]) <= 1
        if ok and (not in_box or ts < tp):
            n_s += 1
            assert r["object"][p] == -2 and abs(r["depth"][p] - ts) < 1e-12
        elif in_box and not (abs(abs(xp[0]) - 1) < 1e-3 or abs(abs(xp[2]) - 1) < 1e-3):
            n_p += 1
            assert r["object"][p] == 0 and abs(r["depth"][p] - tp) < 1e-4
    assert n_s > 50 and n_p > 50, (n_s, n_p)
