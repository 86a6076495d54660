"""GPU parity of the HIP path against the FP64 oracle (runs on an MI355X).

All calls go through the C ABI (libkn.so via the ctypes binding)."""
import math
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2206_10885_amd import synth
from tests import parity as P

pytestmark = pytest.mark.gpu


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


def _query_points(scene, n, seed):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-1, 1, (n, 3))
    # a few points exactly on cell faces and box corners
    N = scene.N
    pts[:8] = -1 + 2.0 * rng.integers(0, N + 1, (8, 3)) / N
    return pts.astype(np.float32)


def _oracle_points(scene, pts):
    os_ = O.OracleScene.from_scene(scene)
    N = scene.N
    out = np.zeros((len(pts), 16))
    grad = np.zeros((len(pts), 3))
    centers = synth.cell_centers(N)
    for i, x in enumerate(pts.astype(np.float64)):
        idx = np.clip(np.floor((x + 1) * N / 2).astype(int), 0, N - 1)
        cell = idx[0] + N * (idx[1] + N * idx[2])
        xl = (x - centers[cell]) * N
        o, g = os_.sdf_eval(cell, xl, grad=True)
        out[i] = o
        grad[i] = g * N
    return out, grad


@pytest.mark.parametrize("N,H,n", [(4, 32, 1000), (16, 64, 3000), (3, 64, 777)])
def test_query_fp32_matches_oracle(ctx, N, H, n):
    """SDF value, world gradient and feature of the per-cell MLPs at random
    points (kn_query), float32 MFMA path against the FP64 oracle."""
    log(f"query fp32 N={N} H={H} n={n}")
    sc = synth.sphere_scene(N, H, 0.5, 0.02, seed=N * 10 + H)
    sid = ctx.scene_create(sc)
    pts = _query_points(sc, n, seed=N + H)
    res = ctx.query(sid, torch.tensor(pts, device="cuda"), "fp32", grad=True, feat=True)
    ref, rgrad = _oracle_points(sc, pts)
    d = res["d"].cpu().numpy()
    g = res["grad"].cpu().numpy()
    z = res["z"].cpu().numpy()
    ed = np.abs(d - ref[:, 0])
    eg = np.abs(g - rgrad) / (1.0 + np.abs(rgrad))
    ez = np.abs(z - ref[:, 1:])
    log(f"  max |dd| {ed.max():.2e}  max rel dgrad {eg.max():.2e}  max |dz| {ez.max():.2e}")
    # float32: ~40-70 products per sum of O(1) terms, encoding error ~1e-7
    assert ed.max() < 2e-5
    assert ez.max() < 2e-5
    # gradients: float32 position rounding (~1e-7) times the second
    # derivative of the highest encoding frequency (2^5 pi / h)
    assert eg.max() < 2e-4
    ctx.scene_destroy(sid)


def test_query_bf16_matches_emulation(ctx):
    """bfloat16 march MLP against its float32 CPU emulation (weights and each
    layer input rounded to bfloat16, float32 accumulation)."""
    from oracle import quant
    sc = synth.sphere_scene(16, 64, 0.6, 0.02, seed=7)
    sid = ctx.scene_create(sc, precisions=("bf16",))
    pts = _query_points(sc, 4000, seed=3)
    d = ctx.query(sid, torch.tensor(pts, device="cuda"), "bf16")["d"].cpu().numpy()
    ref = quant.sdf_bf16(sc, pts)
    err = np.abs(d - ref)
    log(f"bf16 query: median {np.median(err):.2e} p99.9 {np.percentile(err, 99.9):.2e} max {err.max():.2e}")
    # accumulation order differs, which can flip the rounding of a layer
    # input to bfloat16 (one ulp = 2^-8 relative) on rare points
    assert np.median(err) < 1e-5
    assert np.percentile(err, 99.9) < 2e-3
    assert err.max() < 2e-2
    ctx.scene_destroy(sid)


@pytest.mark.parametrize("H", [32, 64])
def test_query_fp8_matches_emulation(ctx, H):
    """fp8 e4m3 march MLP (per-(cell, layer) power-of-two scales) against its
    float32 CPU emulation."""
    from oracle import quant
    sc = synth.sphere_scene(8, H, 0.6, 0.02, seed=70 + H)
    sid = ctx.scene_create(sc, precisions=("fp8",))
    pts = _query_points(sc, 4000, seed=4)
    d = ctx.query(sid, torch.tensor(pts, device="cuda"), "fp8")["d"].cpu().numpy()
    ref = quant.sdf_fp8(sc, pts)
    err = np.abs(d - ref)
    full = quant.sdf_fp8(sc, pts, quantize=False)
    log(f"fp8 query H={H}: median {np.median(err):.2e} p99.9 {np.percentile(err, 99.9):.2e} "
        f"max {err.max():.2e}; fp8 vs fp32 median {np.median(np.abs(ref - full)):.2e}")
    # an e4m3 ulp is 2^-3 relative; float32 sums in another order flip a
    # rounding of a layer-2 input on a few points
    assert np.median(err) < 1e-5
    assert np.percentile(err, 99) < 1e-3
    ctx.scene_destroy(sid)


def _render(ctx, sid, view, W, H, S, eps=1e-4, precision="fp32"):
    return ctx.render(sid, view, W, H, S, eps, precision, with_trace=True)


def test_render_c1_full_frame(ctx):
    """C1 (4^3, H=32, 64x64, S=64) full frame against the oracle."""
    c = synth.CONFIGS["c1"]
    sc = synth.config_scene("c1")
    view = synth.config_views("c1")[0]
    sid = ctx.scene_create(sc)
    out = _render(ctx, sid, view, c["width"], c["height"], c["max_steps"], c["eps"])
    g = P.gpu_arrays(out)
    rep = P.compare(sc, view, c["width"], c["height"], c["max_steps"], c["eps"], g)
    log("C1", rep.as_dict(), out["stats"])
    assert rep.ok(), rep.as_dict()
    ctx.scene_destroy(sid)


@pytest.mark.parametrize("N", [1, 4])
def test_render_plane_closed_form(ctx, N):
    """Check (a) on the GPU: plane scene depth and normal in closed form."""
    n = np.array([0.3, 0.5, 0.81]); n /= np.linalg.norm(n)
    sc = synth.plane_scene(N, 32, n, 0.1, seed=4)
    view = synth.View(eye=tuple(2.5 * n + np.array([0.2, -0.1, 0.05])))
    W = H = 48
    sid = ctx.scene_create(sc)
    out = _render(ctx, sid, view, W, H, 256)
    gq = P.gpu_arrays(out)
    os_ = O.OracleScene.from_scene(sc)
    checked = 0
    for p in range(W * H):
        o, d = O.camera_ray(view, W, H, p // W, p % W)
        ok, tn, tf = os_.slab(o, d)
        if not ok:
            assert gq["hit"][p] == 0
            continue
        t0 = max(tn, 0.0)
        g0, c0 = synth.plane_affine_map(sc, 0)
        f0 = g0 @ (o + t0 * d) + c0
        gn = g0 / np.linalg.norm(g0)
        if abs(f0) < 1e-4 or abs(gn @ d) < 0.2:
            continue   # starts on the plane or grazes it: both outcomes defensible
        ts = -(g0 @ o + c0) / (g0 @ d)
        expect_hit = f0 < 0 or (gn @ d < 0 and ts <= tf)
        if expect_hit and f0 > 0 and min(abs(ts - tn), abs(ts - tf)) < 1e-3:
            continue   # plane meets the box boundary
        assert gq["hit"][p] == int(expect_hit), p
        if not expect_hit:
            continue
        cell = int(gq["cell"][p])
        g_, c_ = synth.plane_affine_map(sc, cell)
        want = t0 if f0 < 0 else -(g_ @ o + c_) / (g_ @ d)
        assert abs(gq["depth"][p] - want) < 1e-4, (p, gq["depth"][p], want)
        assert P.angle_deg(gq["normal"][p], g_ / np.linalg.norm(g_)) < 0.1
        checked += 1
    log(f"plane N={N}: {checked} pixels checked against the closed form")
    assert checked > 300
    ctx.scene_destroy(sid)


def test_render_lipschitz_safe_all_pixels(ctx):
    """A noise-free, Lipschitz-safe sphere scene: sphere tracing is well
    conditioned, so every pixel must meet the tolerance."""
    base = synth.sphere_scene(8, 32, 0.55, 0.0, seed=31)
    sc = synth.lipschitz_safe(base, 0.6)
    view = synth.View(eye=(0.8, 0.9, 2.2))
    W, H = 97, 61   # ragged: not multiples of the 64-wide wave or 16-ray tiles
    sid = ctx.scene_create(sc)
    out = _render(ctx, sid, view, W, H, 512)
    g = P.gpu_arrays(out)
    rep = P.compare(sc, view, W, H, 512, 1e-4, g)
    log("lipschitz-safe", rep.as_dict())
    assert rep.hit_agree >= P.TOL_HIT_MASK
    assert rep.stable_frac > 0.99
    assert rep.stable_bad == 0 and rep.replay_bad == 0 and rep.point_bad == 0
    ctx.scene_destroy(sid)


@pytest.mark.parametrize("cfg,views,samples", [("c2", 2, 3000), ("c3", 1, 6000)])
def test_render_full_size_sampled(ctx, cfg, views, samples):
    """C2 (16^3, H=32, 800x800) and C3 (16^3, H=64, 1920x1080) in float32 at
    full size, compared with the oracle on seeded pixel samples."""
    c = synth.CONFIGS[cfg]
    sc = synth.config_scene(cfg)
    sid = ctx.scene_create(sc)
    for vi, view in enumerate(synth.config_views(cfg)[:views]):
        out = _render(ctx, sid, view, c["width"], c["height"], c["max_steps"], c["eps"])
        pix = synth.sample_pixels(c["width"], c["height"], samples, seed=c["seed"] + vi)
        g = P.gpu_arrays(out, pix)
        rep = P.compare(sc, view, c["width"], c["height"], c["max_steps"], c["eps"], g, pixels=pix)
        log(cfg, vi, rep.as_dict(), out["stats"])
        assert rep.ok(), rep.as_dict()
    ctx.scene_destroy(sid)


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_render_lowp_vs_fp32_report(ctx, precision):
    """BF16 or FP8 march (refinement and shading on split-bf16 MFMA) against
    the FP32 path on the same inputs, and the FP64 oracle on sampled pixels:
    reported; the masks must largely agree."""
    sc = synth.sphere_scene(16, 64, 0.6, 0.02, seed=3000)
    sid = ctx.scene_create(sc, precisions=(precision,))
    view = synth.config_views("c3")[0]
    a = P.gpu_arrays(_render(ctx, sid, view, 480, 270, 128))
    out = _render(ctx, sid, view, 480, 270, 128, precision=precision)
    b = P.gpu_arrays(out)
    agree = float(np.mean(a["hit"] == b["hit"]))
    both = (a["hit"] == 1) & (b["hit"] == 1)
    dd = np.abs(a["depth"] - b["depth"])[both]
    an = P.angle_deg(a["normal"][both], b["normal"][both])
    dc = np.abs(a["rgb"] - b["rgb"]).max(axis=1)
    log(f"{precision} vs fp32: mask agreement {agree:.4f}, depth p50 {np.median(dd):.2e} "
        f"p99 {np.percentile(dd, 99):.2e} max {dd.max():.2e}; normal p50 {np.median(an):.2e} "
        f"p99 {np.percentile(an, 99):.2e} deg; rgb p50 {np.median(dc):.2e} p99 {np.percentile(dc, 99):.2e}")
    pix = synth.sample_pixels(480, 270, 1500, seed=9)
    rep = P.compare(sc, view, 480, 270, 128, 1e-4, P.gpu_arrays(out, pix), pixels=pix)
    log(f"{precision} vs FP64 oracle (1500 pixels):", rep.as_dict())
    assert agree > 0.95
    ctx.scene_destroy(sid)


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_split_bf16_shading_on_the_same_surface(ctx, precision):
    MIN_OK = {"bf16": 0.99, "fp8": 0.95}
    """Pools marching in bf16 or fp8 refine and shade on bf16 MFMA with split
    (hi + lo) operands.  On a smooth scene (no per-cell noise) the
    low-precision march ends next to the same crossing as the float32 one
    (depths within 1e-3), and two Newton steps take both to the same point, so
    what is left is the refinement and shading arithmetic: depth, normal and
    colour must agree with the float32 frame to the parity tolerances."""
    sc = synth.sphere_scene(16, 64, 0.6, 0.0, seed=3001)
    sid = ctx.scene_create(sc, precisions=(precision,))
    view = synth.config_views("c3")[1]
    a = P.gpu_arrays(_render(ctx, sid, view, 480, 270, 128))
    b = P.gpu_arrays(_render(ctx, sid, view, 480, 270, 128, precision=precision))
    both = (a["hit"] == 1) & (b["hit"] == 1)
    dd = np.abs(a["depth"] - b["depth"])
    same = both & (dd < 1e-3)
    an = P.angle_deg(a["normal"][same], b["normal"][same])
    dc = np.abs(a["rgb"] - b["rgb"]).max(axis=1)[same]
    log(f"{precision}: same-surface {same.sum()} of {both.sum()} common hits; depth p99 "
        f"{np.percentile(dd[same], 99):.2e} max {dd[same].max():.2e}; normal p99 {np.percentile(an, 99):.2e} "
        f"max {an.max():.2e} deg; rgb p99 {np.percentile(dc, 99):.2e} max {dc.max():.2e}")
    ok = (dd[same] <= P.TOL_DEPTH) & (an <= P.TOL_NORMAL_DEG) & (dc <= P.TOL_RGB)
    log(f"{precision}: {ok.mean():.5f} of the same-surface pixels within all three tolerances")
    assert same.sum() > 0.9 * both.sum()
    assert ok.mean() >= MIN_OK[precision]
    ctx.scene_destroy(sid)


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_counter_layouts_give_the_same_frame(precision):
    """Per-cell counters one per 128-byte line (grids up to 65536 cells) or
    packed (larger pools): the same frame, bit for bit."""
    from paper_2206_10885_amd import kn
    sc = synth.config_scene("c1")
    view = synth.config_views("c1")[0]
    outs = []
    for stride in ("32", "1"):
        os.environ["KN_COUNTER_STRIDE"] = stride
        try:
            with kn.Context(0) as c:
                sid = c.scene_create(sc, precisions=("bf16",))
                out = _render(c, sid, view, 320, 180, 96, precision=precision)
                torch.cuda.synchronize()
                outs.append({k: v.cpu().clone() for k, v in out.items() if torch.is_tensor(v)})
        finally:
            del os.environ["KN_COUNTER_STRIDE"]
    for k in ("rgb", "depth", "normal", "hit", "steps"):
        assert torch.equal(outs[0][k], outs[1][k]), k


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_march_tallies_count_every_evaluation(ctx, precision):
    """Every SDF evaluation of the march adds one to its ray's step count, so
    the evaluations tallied over the workgroups' lines equal the sum of the
    per-pixel step counts."""
    sc = synth.config_scene("c1")
    view = synth.config_views("c1")[0]
    sid = ctx.scene_create(sc, precisions=("bf16",))
    out = _render(ctx, sid, view, 320, 180, 96, precision=precision)
    torch.cuda.synchronize()
    st = out["stats"]
    assert st["evals"] == int(out["steps"].long().sum())
    assert 0 < st["march_chunks"] <= st["march_tiles"] <= st["evals"]


def test_render_deterministic(ctx):
    sc = synth.config_scene("c1")
    sid = ctx.scene_create(sc)
    view = synth.View(eye=(1.0, 0.5, 2.0))
    a = _render(ctx, sid, view, 130, 70, 64)
    b = _render(ctx, sid, view, 130, 70, 64)
    for k in ("rgb", "depth", "normal", "hit", "steps", "trace"):
        assert torch.equal(a[k], b[k]), k
    ctx.scene_destroy(sid)


@pytest.mark.parametrize("W,H", [(1, 1), (1, 37), (333, 1), (65, 65)])
def test_render_small_and_ragged_sizes(ctx, W, H):
    sc = synth.config_scene("c1")
    sid = ctx.scene_create(sc)
    view = synth.front_view()
    out = _render(ctx, sid, view, W, H, 64)
    g = P.gpu_arrays(out)
    ref = P.oracle_render(sc, view, W, H, 64, 1e-4)
    assert np.mean(ref["hit"] == g["hit"]) >= (1.0 if W * H < 1000 else P.TOL_HIT_MASK)
    ctx.scene_destroy(sid)


def test_render_degenerate_cases(ctx):
    """Camera inside the box, camera facing away (every ray misses the box),
    and a step budget of one evaluation."""
    sc = synth.config_scene("c1")
    sid = ctx.scene_create(sc)
    for view, S in [(synth.View(eye=(0.9, 0.9, 0.9), tan_half_diag=1.0), 64),
                    (synth.View(eye=(0.0, 0.0, 2.5), look_at=(0.0, 0.0, 5.0)), 64),
                    (synth.front_view(), 1)]:
        out = _render(ctx, sid, view, 40, 30, S)
        g = P.gpu_arrays(out)
        ref = P.oracle_render(sc, view, 40, 30, S, 1e-4)
        assert np.mean(ref["hit"] == g["hit"]) >= 0.99, view
        m = g["hit"] == 0
        assert (g["depth"][m] == 0).all() and (g["rgb"][m] == 0).all()
        np.testing.assert_array_equal(ref["status"] == 0, g["status"] == 0)
    ctx.scene_destroy(sid)


def test_errors_leave_outputs_untouched(ctx):
    from paper_2206_10885_amd import kn
    sc = synth.config_scene("c1")
    sid = ctx.scene_create(sc, precisions=())
    out = ctx.alloc_frame(8, 8)
    for v in out.values():
        v.fill_(7)
    bad = [kn.make_camera(synth.front_view(), 8, 8, 0, 1e-4),          # max_steps 0
           kn.make_camera(synth.front_view(), 8, 8, 64, -1.0),         # eps < 0
           kn.make_camera(synth.View(eye=(0, 0, 0)), 8, 8, 64, 1e-4),  # eye == look_at
           kn.make_camera(synth.front_view(), 8, 8, 64, 1e-4, "bf16")]  # no bf16 copy
    for cam in bad:
        with pytest.raises(kn.KnError) as e:
            ctx.render_into(sid, cam, out)
        assert e.value.status == -1
    with pytest.raises(kn.KnError) as e:
        ctx.render_into(sid + 999, kn.make_camera(synth.front_view(), 8, 8, 64, 1e-4), out)
    assert e.value.status == -3
    for v in out.values():
        assert (v == 7).all()
    ctx.scene_destroy(sid)
