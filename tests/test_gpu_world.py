"""Shared scenes (Sec. 3.4: KiloNeuS objects rendered with classic
primitives) and progressive path tracing on the GPU, against the FP64 oracle
and against kn_render, through the C ABI (libkn.so via the ctypes binding)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2206_10885_amd import synth
from tests import parity as P

pytestmark = pytest.mark.gpu

PS, PB, PT_ = O.PRIM_SPHERE, O.PRIM_BOX, O.PRIM_TRIANGLE


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible: GPU tests need an MI355X")
    from paper_2206_10885_amd import kn
    c = kn.Context(0)
    yield c
    c.close()


def _np(out):
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


def _world_render(ctx, wid, view, W, H, S, precision="fp32", unclamped=False, **pt):
    from paper_2206_10885_amd import kn
    env = pt.pop("env", None)
    envt = None if env is None else torch.tensor(env, device="cuda")
    cam = kn.make_camera(view, W, H, S, 1e-4, precision, unclamped=unclamped, env=envt, **pt)
    out = ctx.alloc_frame(W, H, with_trace=True)
    out["stats"] = ctx.render_world_into(wid, cam, out)
    return _np(out)


def _objects(g, cell_ranges):
    """Object id per pixel from the trace records: instance k (its global
    cell range), primitive i as -(2 + i), nothing as -1."""
    tr = g["trace"].reshape(-1, 4)
    cell, status = tr[:, 2], tr[:, 3]
    obj = np.full(len(cell), -1, np.int64)
    for k, (lo, hi) in enumerate(cell_ranges):
        obj[(status == 1) & (cell >= lo) & (cell < hi)] = k
    prim = (status == 1) & (cell <= -2)
    obj[prim] = cell[prim]
    return obj


# two instances (scaled and translated), a ground box, a sphere that cuts
# into the second instance's box, and a triangle behind
INST_A = (synth.sphere_scene(8, 64, 0.6, 0.0, seed=41), (-0.9, 0.0, 0.0), 0.8)
INST_B = (synth.sphere_scene(4, 32, 0.5, 0.0, seed=42), (1.0, 0.1, -0.3), 0.7)
PRIMS = [(PB, [-4.0, -1.2, -4.0, 4.0, -0.9, 4.0], (0.7, 0.7, 0.6)),
         (PS, [0.9, 0.5, 0.6, 0.4], (0.9, 0.2, 0.2)),
         (PT_, [-2.0, -1.0, -2.0, 2.0, -1.0, -2.0, 0.0, 2.0, -2.5], (0.2, 0.5, 0.9))]
VIEW = synth.View(eye=(0.3, 1.2, 4.0), look_at=(0.0, 0.0, 0.0), tan_half_diag=0.7)


@pytest.fixture(scope="module")
def world(ctx):
    sids = [ctx.scene_create(sc, precisions=("bf16",)) for sc, _, _ in (INST_A, INST_B)]
    wid = ctx.world_create([(sids[0], INST_A[1], INST_A[2]), (sids[1], INST_B[1], INST_B[2])], PRIMS)
    ow = O.OracleWorld([(O.OracleScene.from_scene(INST_A[0]), INST_A[1], INST_A[2]),
                        (O.OracleScene.from_scene(INST_B[0]), INST_B[1], INST_B[2])], PRIMS)
    ranges = [(0, 8 ** 3), (8 ** 3, 8 ** 3 + 4 ** 3)]
    yield wid, ow, ranges
    ctx.world_destroy(wid)
    for s in sids:
        ctx.scene_destroy(s)


@pytest.mark.parametrize("precision,unclamped", [("fp32", False), ("bf16", False), ("fp32", True)])
def test_one_instance_world_equals_render(ctx, precision, unclamped):
    """A world holding one instance at identity and nothing else renders what
    kn_render renders for the scene: every output identical on hits (the
    world path hands the march the same local ray and interval), and the
    same misses."""
    sc = synth.config_scene("c1")
    view = synth.config_views("c1")[0]
    sid = ctx.scene_create(sc, precisions=("bf16",))
    wid = ctx.world_create([(sid, (0.0, 0.0, 0.0), 1.0)])
    W, H = 97, 61
    a = _world_render(ctx, wid, view, W, H, 64, precision, unclamped)
    b = _np(ctx.render(sid, view, W, H, 64, 1e-4, precision, with_trace=True, unclamped=unclamped))
    hit = b["hit"] == 1
    log(f"one-instance world {precision} unclamped={unclamped}: hits {int(hit.sum())}, "
        f"stats {a['stats']['rounds']} rounds / {a['stats']['evals']} evals vs {b['stats']['evals']}")
    assert np.array_equal(a["hit"], b["hit"])
    for k in ("rgb", "depth", "normal"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["steps"][hit], b["steps"][hit])
    assert np.array_equal(a["trace"][hit], b["trace"][hit])
    assert a["stats"]["evals"] == b["stats"]["evals"]
    ctx.world_destroy(wid)
    ctx.scene_destroy(sid)


def test_world_primary_matches_oracle(ctx, world):
    """Two instances and three primitives, 96x72 float32: the object hit at
    each pixel agrees with the oracle's; primitive hits equal its closed-form
    depth, normal and albedo; instance hits are within the single-scene
    tolerance (depth in world units: scale x 1e-4)."""
    wid, ow, ranges = world
    W, H = 96, 72
    g = _world_render(ctx, wid, VIEW, W, H, 128, "fp32")
    ref = ow.render(VIEW, W, H, 128, 1e-4)
    og = _objects(g, ranges)
    orf = ref["object"].astype(np.int64)
    agree = np.mean(og == orf)
    counts = {int(k): int(np.sum(orf == k)) for k in np.unique(orf)}
    log(f"world primary: object agreement {agree:.5f}, oracle objects {counts}")
    assert agree >= 0.995
    for k in (0, 1, -2, -3, -4):
        assert counts.get(k, 0) > 30, counts
    depth, normal, rgb = g["depth"].reshape(-1), g["normal"].reshape(-1, 3), g["rgb"].reshape(-1, 3)
    same = og == orf
    prim = same & (orf <= -2)
    assert np.abs(depth[prim] - ref["depth"][prim]).max() <= 1e-5 * max(1.0, ref["depth"][prim].max())
    an = P.angle_deg(normal[prim], ref["normal"][prim])
    log(f"primitive normals: {np.mean(an <= 0.01):.5f} within 0.01 deg, max {an.max():.4f} deg; per primitive max "
        + str({int(k): float(an[orf[prim] == k].max()) for k in (-2, -3, -4)}))
    pi = np.flatnonzero(prim)[np.argsort(-an)[:4]]
    for q in pi:
        log(f"  pixel {q}: object {orf[q]}, gpu n {normal[q].tolist()} d {depth[q]:.7f}; "
            f"oracle n {ref['normal'][q].round(7).tolist()} d {ref['depth'][q]:.7f}")
    assert an.max() <= 0.01
    assert np.abs(rgb[prim] - ref["rgb"][prim]).max() <= 1e-7
    scale = np.array([INST_A[2], INST_B[2]])
    inst = same & (orf >= 0)
    tol_d = P.TOL_DEPTH * scale[orf[inst]]
    bad = ((np.abs(depth[inst] - ref["depth"][inst]) > tol_d) |
           (P.angle_deg(normal[inst], ref["normal"][inst]) > P.TOL_NORMAL_DEG) |
           (np.abs(rgb[inst] - ref["rgb"][inst]).max(1) > P.TOL_RGB))
    log(f"instance hits {int(inst.sum())}, outside tolerance {int(bad.sum())}")
    assert bad.mean() <= 5e-3
    assert (g["hit"].reshape(-1) == (orf != -1)).mean() >= 0.995


def test_world_bf16_march(ctx, world):
    """The same world with a bf16 march (float32 refinement and shading):
    objects agree with the oracle on >= 99% of pixels and refined instance
    depths stay close."""
    wid, ow, ranges = world
    W, H = 96, 72
    g = _world_render(ctx, wid, VIEW, W, H, 128, "bf16")
    ref = ow.render(VIEW, W, H, 128, 1e-4)
    og = _objects(g, ranges)
    orf = ref["object"].astype(np.int64)
    agree = np.mean(og == orf)
    inst = (og == orf) & (orf >= 0)
    dd = np.abs(g["depth"].reshape(-1)[inst] - ref["depth"][inst])
    log(f"world bf16: object agreement {agree:.5f}, instance depth diff p50 {np.median(dd):.2e} "
        f"p99 {np.percentile(dd, 99):.2e}")
    assert agree >= 0.99
    assert np.median(dd) < 1e-4


def test_ray_continues_past_an_instance(ctx):
    """Rays that miss the near object inside its box go on to the far one
    behind it (the march's exit continues the ray past the box)."""
    near = synth.sphere_scene(4, 32, 0.3, 0.0, seed=41)
    far = synth.sphere_scene(4, 32, 0.6, 0.0, seed=42)
    sn, sf = ctx.scene_create(near), ctx.scene_create(far)
    wid = ctx.world_create([(sn, (0.0, 0.0, 2.5), 1.0), (sf, (0.0, 0.0, -1.0), 1.0)])
    view = synth.View(eye=(0.0, 0.0, 6.0), tan_half_diag=0.18)
    W = H = 48
    g = _world_render(ctx, wid, view, W, H, 128)
    ow = O.OracleWorld([(O.OracleScene.from_scene(near), (0.0, 0.0, 2.5), 1.0),
                        (O.OracleScene.from_scene(far), (0.0, 0.0, -1.0), 1.0)])
    ref = ow.render(view, W, H, 128, 1e-4)
    og = _objects(g, [(0, 64), (64, 128)])
    orf = ref["object"].astype(np.int64)
    log(f"continuation: agreement {np.mean(og == orf):.5f}, near {int(np.sum(og == 0))}, far {int(np.sum(og == 1))}")
    assert np.mean(og == orf) >= 0.998
    assert np.sum(og == 1) > 50 and np.sum(og == 0) > 50
    both = (og == orf) & (orf >= 0)
    assert np.abs(g["depth"].reshape(-1)[both] - ref["depth"][both]).max() < 1e-3
    ctx.world_destroy(wid)
    ctx.scene_destroy(sn)
    ctx.scene_destroy(sf)


def test_primitive_inside_an_instance_box_occludes(ctx):
    """A sphere primitive just above a plane instance, inside one cell of
    it: the march of a ray that meets the sphere first ends where the
    sphere cuts its interval, also inside the cell, so the sphere is what
    the pixel shows, as in the oracle (whose pin fixes this case)."""
    n = np.array([0.0, 1.0, 0.0])
    sc = synth.constant_color_plane_scene(2, 32, n, -0.3, [0.6, 0.35, 0.8], seed=3)
    sid = ctx.scene_create(sc)
    prims = [(PS, [0.5, -0.15, 0.5, 0.1], (0.5, 0.5, 0.5))]
    wid = ctx.world_create([(sid, (0.0, 0.0, 0.0), 1.0)], prims)
    view = synth.View(eye=(0.9, 1.6, 1.4), look_at=(0.5, -0.2, 0.5), tan_half_diag=0.25)
    W, H = 64, 48
    g = _world_render(ctx, wid, view, W, H, 128)
    ref = O.OracleWorld([(O.OracleScene.from_scene(sc), (0.0, 0.0, 0.0), 1.0)], prims).render(
        view, W, H, 128, 1e-4)
    og = _objects(g, [(0, 8)])
    orf = ref["object"].astype(np.int64)
    log(f"primitive inside a cell: agreement {np.mean(og == orf):.5f}, sphere pixels {int(np.sum(orf == -2))}, "
        f"plane pixels {int(np.sum(orf == 0))}")
    assert np.sum(orf == -2) > 100 and np.sum(orf == 0) > 1000
    assert np.mean(og == orf) >= 0.999
    ctx.world_destroy(wid)
    ctx.scene_destroy(sid)


def test_primitives_only_path_trace_matches_oracle(ctx):
    """A world of primitives under an environment map, 2 bounces: every path
    runs in k_world_step (intersections, scatter, environment); pixels equal
    the oracle's up to float32 rounding."""
    prims = [(PB, [-3.0, -1.0, -3.0, 3.0, -0.8, 3.0], (0.6, 0.6, 0.5)),
             (PS, [0.0, 0.0, 0.0, 0.6], (0.8, 0.3, 0.3)),
             (PT_, [-1.5, -0.8, -1.0, 1.5, -0.8, -1.0, 0.0, 1.5, -1.2], (0.3, 0.4, 0.9))]
    wid = ctx.world_create([], prims)
    env = synth.env_map(128, 64, seed=5005)
    view = synth.View(eye=(0.4, 0.9, 3.0), look_at=(0.0, 0.0, 0.0), tan_half_diag=0.6)
    W, H = 64, 48
    g = _world_render(ctx, wid, view, W, H, 64, spp=4, bounces=2, seed=91, env=env)
    ref = O.OracleWorld([], prims).path_trace(view, W, H, 64, 1e-4, 4, 2, 91, env)
    d = np.abs(g["rgb"].reshape(-1, 3) - ref["rgb"]).max(1)
    log(f"primitives path trace: rgb diff p50 {np.median(d):.2e} p99 {np.percentile(d, 99):.2e} max {d.max():.2e}")
    assert np.mean(g["hit"].reshape(-1) == ref["hit"]) >= 0.999
    assert np.percentile(d, 99) < 1e-3
    ctx.world_destroy(wid)


def test_world_path_trace_furnace(ctx):
    """Constant environment E, an instance of constant albedo and a sphere
    primitive inside its box, 3 bounces: each path's radiance is a product of
    albedos times E, so pixels equal the oracle's wherever the two take the
    same bounces (all but a few grazing paths)."""
    n = np.array([0.0, 1.0, 0.0])
    sc = synth.constant_color_plane_scene(2, 32, n, -0.3, [0.6, 0.35, 0.8], seed=3)
    sid = ctx.scene_create(sc)
    prims = [(PS, [0.1, 0.1, 0.0, 0.35], (0.5, 0.5, 0.5))]
    wid = ctx.world_create([(sid, (0.0, 0.0, 0.0), 1.0)], prims)
    E = np.array([1.5, 2.0, 0.7], np.float32)
    env = np.tile(E[None, None, :], (8, 16, 1))
    # seen from above: no camera ray enters the box below the plane, where the
    # hit is at the box face inside the solid and whether the scattered ray
    # starts inside or outside the box is a matter of rounding
    view = synth.View(eye=(0.3, 3.0, 0.9), look_at=(0.0, -0.3, 0.0), tan_half_diag=0.45)
    W, H = 48, 36
    spp, B = 3, 3
    g = _world_render(ctx, wid, view, W, H, 128, spp=spp, bounces=B, seed=5006, env=env)
    ow = O.OracleWorld([(O.OracleScene.from_scene(sc), (0.0, 0.0, 0.0), 1.0)], prims)
    ref = ow.path_trace(view, W, H, 128, 1e-4, spp, B, 5006, env)
    rgb = g["rgb"].reshape(-1, 3)
    # a sample is E x the albedos of the surfaces it met before escaping, or
    # 0 when it meets a surface after its last scatter; a pixel is the mean
    # of spp such samples
    a_plane = 1.0 / (1.0 + np.exp(-synth.unpack_col(sc.col[0])["bc2"].astype(np.float64)))
    albs = [a_plane, np.full(3, 0.5)]
    vals = [np.zeros(3)]
    prods = [np.ones(3)]
    for _ in range(B + 1):
        vals += [E * p for p in prods]
        prods = [p * a for p in prods for a in albs]
    vals = np.unique(np.round(np.array(vals), 12), axis=0)
    import itertools
    mixes = np.array([np.mean(c, axis=0) for c in itertools.combinations_with_replacement(vals, spp)])
    err = np.abs(rgb[:, None, :] - mixes[None]).max(-1).min(1) / E.max()
    same = np.abs(rgb - ref["rgb"]).max(1) < 1e-5
    bad = np.flatnonzero(~same)[:5]
    log(f"world furnace: max mixture error {err.max():.2e}; equal to oracle {same.mean():.4f}; "
        f"first differing pixels {bad.tolist()}: gpu {rgb[bad].round(4).tolist()} oracle {ref['rgb'][bad].round(4).tolist()}")
    assert err.max() < 1e-5
    assert same.mean() > 0.99
    ctx.world_destroy(wid)
    ctx.scene_destroy(sid)


def _accumulate(ctx, render, view, W, H, splits, **pt):
    """Renders the samples in calls of `splits` samples each into one
    accumulation buffer; returns rgb after the last call."""
    from paper_2206_10885_amd import kn
    env = torch.tensor(pt.pop("env"), device="cuda")
    out = ctx.alloc_frame(W, H)
    out["accum"] = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    off = 0
    for k in splits:
        cam = kn.make_camera(view, W, H, 128, 1e-4, "fp32", spp=k, env=env, sample_offset=off, **pt)
        render(cam, out)
        off += k
    torch.cuda.synchronize()
    return out["rgb"].clone()


@pytest.mark.parametrize("kind", ["scene", "world"])
def test_progressive_accumulation_equals_one_call(ctx, kind):
    """Path tracing 4 samples per pixel in one call, in 4 calls of 1 sample
    and in 2 calls of 2 (kn_frame.accum, kn_camera.sample_offset): the same
    rgb, bit for bit (each sample is keyed by its index; the running sum
    adds the samples in the same order)."""
    sc = synth.sphere_scene(8, 64, 0.6, 0.02, seed=5000)
    sid = ctx.scene_create(sc)
    env = synth.env_map(128, 64, seed=5005)
    view = synth.orbit_views(1, seed=5500)[0]
    W, H = 64, 48
    if kind == "scene":
        render = lambda cam, out: ctx.render_into(sid, cam, out)
        wid = None
    else:
        wid = ctx.world_create([(sid, (0.0, 0.0, 0.0), 1.0)],
                               [(PB, [-3.0, -1.4, -3.0, 3.0, -1.1, 3.0], (0.7, 0.6, 0.5))])
        render = lambda cam, out: ctx.render_world_into(wid, cam, out)
    pt = dict(bounces=2, seed=77, env=env)
    one = _accumulate(ctx, render, view, W, H, [4], **dict(pt))
    four = _accumulate(ctx, render, view, W, H, [1, 1, 1, 1], **dict(pt))
    two = _accumulate(ctx, render, view, W, H, [2, 2], **dict(pt))
    log(f"progressive {kind}: max |one - four| {float((one - four).abs().max()):.3e}, "
        f"max |one - two| {float((one - two).abs().max()):.3e}")
    assert torch.equal(one, four) and torch.equal(one, two)
    # and the one-call result is the plain kn_render / kn_render_world output
    from paper_2206_10885_amd import kn
    envt = torch.tensor(env, device="cuda")   # held while the call runs
    cam = kn.make_camera(view, W, H, 128, 1e-4, "fp32", spp=4, env=envt, bounces=2, seed=77)
    out = ctx.alloc_frame(W, H)
    render(cam, out)
    torch.cuda.synchronize()
    assert torch.equal(out["rgb"], one)
    if wid is not None:
        ctx.world_destroy(wid)
    ctx.scene_destroy(sid)


def test_one_scene_placed_twice(ctx):
    """Two instances of one resident scene (shared weights) at different
    scales and places, with a ground box: objects, depths (world units),
    normals and colours against the oracle."""
    sc = synth.sphere_scene(8, 64, 0.6, 0.0, seed=43)
    sid = ctx.scene_create(sc, precisions=("bf16",))
    inst = [((-1.1, 0.0, 0.0), 0.9), ((1.2, -0.2, -0.6), 0.6)]
    ground = [(PB, [-5.0, -1.4, -5.0, 5.0, -1.0, 5.0], (0.5, 0.6, 0.7))]
    wid = ctx.world_create([(sid, t, s) for t, s in inst], ground)
    os_ = O.OracleScene.from_scene(sc)
    ow = O.OracleWorld([(os_, t, s) for t, s in inst], ground)
    view = synth.View(eye=(0.2, 1.4, 4.2), look_at=(0.0, -0.2, 0.0), tan_half_diag=0.6)
    W, H = 96, 72
    for precision in ("fp32", "bf16"):
        g = _world_render(ctx, wid, view, W, H, 128, precision)
        ref = ow.render(view, W, H, 128, 1e-4)
        og = _objects(g, [(0, 512), (512, 1024)])
        orf = ref["object"].astype(np.int64)
        inst_px = (og == orf) & (orf >= 0)
        scale = np.array([s for _, s in inst])
        dd = np.abs(g["depth"].reshape(-1)[inst_px] - ref["depth"][inst_px]) / scale[orf[inst_px]]
        an = P.angle_deg(g["normal"].reshape(-1, 3)[inst_px], ref["normal"][inst_px])
        dc = np.abs(g["rgb"].reshape(-1, 3)[inst_px] - ref["rgb"][inst_px]).max(1)
        log(f"shared weights {precision}: agreement {np.mean(og == orf):.5f}, objects "
            f"{ {int(k): int(np.sum(orf == k)) for k in np.unique(orf)} }, local depth max {dd.max():.2e}, "
            f"normal max {an.max():.4f} deg, rgb max {dc.max():.2e}")
        assert np.sum(orf == 0) > 300 and np.sum(orf == 1) > 150
        if precision == "fp32":
            assert np.mean(og == orf) >= 0.999
            bad = (dd > P.TOL_DEPTH) | (an > P.TOL_NORMAL_DEG) | (dc > P.TOL_RGB)
            assert bad.mean() <= 1e-3, bad.sum()
        else:
            # a bf16 march may stop at another crossing where the surface is
            # grazed; as for the world's bf16 test: objects and refined depths
            assert np.mean(og == orf) >= 0.995
            assert np.median(dd) < 1e-5
    ctx.world_destroy(wid)
    ctx.scene_destroy(sid)


def test_world_path_trace_matches_oracle(ctx):
    """Path tracing a world of two scaled instances (smooth spheres) and a
    ground box under an environment map, 2 spp, 2 bounces: per pixel against
    the oracle (the same Philox samples; float32 against FP64 along paths
    that cross instances and primitives)."""
    a = synth.sphere_scene(8, 64, 0.6, 0.0, seed=44)
    b = synth.sphere_scene(4, 32, 0.5, 0.0, seed=45)
    sa, sb = ctx.scene_create(a), ctx.scene_create(b)
    inst = [(sa, a, (-0.9, 0.0, 0.0), 0.8), (sb, b, (1.0, 0.1, -0.3), 0.7)]
    ground = [(PB, [-4.0, -1.2, -4.0, 4.0, -0.9, 4.0], (0.7, 0.7, 0.6)),
              (PS, [0.1, 0.9, -1.2, 0.3], (0.9, 0.3, 0.2))]
    wid = ctx.world_create([(sid, t, s) for sid, _, t, s in inst], ground)
    ow = O.OracleWorld([(O.OracleScene.from_scene(sc), t, s) for _, sc, t, s in inst], ground)
    env = synth.env_map(128, 64, seed=5005)
    W, H = 64, 48
    g = _world_render(ctx, wid, VIEW, W, H, 128, spp=2, bounces=2, seed=123, env=env)
    ref = ow.path_trace(VIEW, W, H, 128, 1e-4, 2, 2, 123, env)
    d = np.abs(g["rgb"].reshape(-1, 3) - ref["rgb"]).max(1)
    log(f"world path trace: rgb diff p50 {np.median(d):.2e} p99 {np.percentile(d, 99):.2e} max {d.max():.2e}; "
        f"within 1e-4: {np.mean(d < 1e-4):.4f}; primary hits {int(g['hit'].sum())}")
    assert np.mean(g["hit"].reshape(-1) == ref["hit"]) >= 0.999
    assert np.mean(d < 1e-4) >= 0.98
    ctx.world_destroy(wid)
    ctx.scene_destroy(sa)
    ctx.scene_destroy(sb)


def test_empty_and_tiny_worlds(ctx):
    """An empty world renders background (primary) or the environment (path
    tracing); a 1x1 frame of a world renders its one pixel as the oracle."""
    from paper_2206_10885_amd import kn
    wid = ctx.world_create()
    view = synth.View(eye=(0.0, 0.0, 3.0))
    g = _world_render(ctx, wid, view, 17, 9, 64)
    assert not g["hit"].any() and not g["rgb"].any() and not g["depth"].any()
    env = synth.env_map(64, 32, seed=3)
    g = _world_render(ctx, wid, view, 17, 9, 64, spp=2, bounces=1, seed=4, env=env)
    ref = O.OracleWorld([]).path_trace(view, 17, 9, 64, 1e-4, 2, 1, 4, env)
    assert np.abs(g["rgb"].reshape(-1, 3) - ref["rgb"]).max() < 1e-5
    ctx.world_destroy(wid)
    wid = ctx.world_create([], [(PS, [0.0, 0.0, 0.0, 0.5], (0.3, 0.6, 0.9))])
    g = _world_render(ctx, wid, view, 1, 1, 64)
    assert g["hit"].reshape(-1)[0] == 1 and abs(float(g["depth"].reshape(-1)[0]) - 2.5) < 1e-6
    assert np.allclose(g["rgb"].reshape(-1), [0.3, 0.6, 0.9])
    ctx.world_destroy(wid)


def test_world_argument_errors(ctx):
    from paper_2206_10885_amd import kn
    a = ctx.scene_create(synth.sphere_scene(4, 32, 0.5, 0.0, seed=1), precisions=())
    b = ctx.scene_create(synth.sphere_scene(4, 64, 0.5, 0.0, seed=2), precisions=("bf16",))
    with pytest.raises(kn.KnError) as e:
        ctx.world_create([(a, (0, 0, 0), 1.0), (b, (1.5, 0, 0), 1.0)])      # overlapping boxes
    assert e.value.status == -1
    with pytest.raises(kn.KnError):
        ctx.world_create([], [(PS, [0, 0, 0, -1.0], (0.5, 0.5, 0.5))])     # radius < 0
    with pytest.raises(kn.KnError):
        ctx.world_create([], [(PS, [0, 0, 0, 1.0], (1.5, 0.5, 0.5))])      # albedo > 1
    wid = ctx.world_create([(a, (0, 0, 0), 1.0), (b, (3.0, 0, 0), 1.0)])
    with pytest.raises(kn.KnError) as e:
        ctx.scene_destroy(a)                                                 # placed in a world
    assert e.value.status == -4
    out = ctx.alloc_frame(8, 8)
    with pytest.raises(kn.KnError) as e:                                     # mixed widths, unclamped
        ctx.render_world_into(wid, kn.make_camera(synth.front_view(), 8, 8, 64, 1e-4, unclamped=True), out)
    assert e.value.status == -7
    with pytest.raises(kn.KnError) as e:                                     # no bf16 copy of scene a
        ctx.render_world_into(wid, kn.make_camera(synth.front_view(), 8, 8, 64, 1e-4, "bf16"), out)
    assert e.value.status == -1
    with pytest.raises(kn.KnError) as e:
        ctx.render_world_into(wid + 99, kn.make_camera(synth.front_view(), 8, 8, 64, 1e-4), out)
    assert e.value.status == -3
    out["accum"] = torch.empty((8, 8, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(kn.KnError) as e:                                     # accumulation needs bounces
        ctx.render_world_into(wid, kn.make_camera(synth.front_view(), 8, 8, 64, 1e-4), out)
    assert e.value.status == -7
    ctx.world_destroy(wid)
    ctx.scene_destroy(a)
    ctx.scene_destroy(b)
