"""Path tracing (Lambertian bounces, environment lighting) on the GPU
against the FP64 oracle, through the C ABI."""
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


def _pt(ctx, sid, view, W, H, S, spp, bounces, seed, env, precision="fp32"):
    from paper_2206_10885_amd import kn
    envt = None if env is None else torch.tensor(env, device="cuda")
    cam = kn.make_camera(view, W, H, S, 1e-4, precision, spp=spp, bounces=bounces, seed=seed, env=envt)
    out = ctx.alloc_frame(W, H, with_trace=True)
    out["stats"] = ctx.render_into(sid, cam, out)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


def test_furnace_plane(ctx):
    """Constant environment and albedo: every path is a E or E, whatever
    the random numbers (see the oracle pin); GPU pixels are such mixtures
    and equal the oracle's."""
    n = np.array([0.2, 1.0, 0.1])
    n /= np.linalg.norm(n)
    sc = synth.constant_color_plane_scene(2, 32, n, -0.1, [0.6, 0.35, 0.8], seed=3)
    a = 1.0 / (1.0 + np.exp(-synth.unpack_col(sc.col[0])["bc2"].astype(np.float64)))
    E = np.array([1.5, 2.0, 0.7], np.float32)
    env = np.tile(E[None, None, :], (8, 16, 1))
    sid = ctx.scene_create(sc)
    view = synth.View(eye=(0.4, 2.0, 1.5))
    W, H = 48, 36
    for spp, bounces in [(1, 1), (3, 3)]:
        g = _pt(ctx, sid, view, W, H, 128, spp, bounces, 5006, env)
        rgb = g["rgb"].reshape(-1, 3)
        mixes = np.stack([(k * a * E + (spp - k) * E) / spp for k in range(spp + 1)])
        err = np.abs(rgb[:, None, :] - mixes[None]).max(-1).min(1) / E.max()
        ref = O.OracleScene.from_scene(sc).path_trace(view, W, H, 128, 1e-4, spp, bounces, 5006, env)
        same = np.abs(rgb - ref["rgb"]).max(1) < 1e-5
        log(f"furnace spp={spp} bounces={bounces}: max mixture err {err.max():.2e}, "
            f"equal to oracle {same.mean():.4f}, hits {int(g['hit'].sum())}")
        assert err.max() < 1e-5
        assert same.mean() > 0.99
    ctx.scene_destroy(sid)


def test_plane_one_bounce_matches_oracle(ctx):
    """One scatter off a plane under a varying environment: each hit pixel is
    albedo x env(direction from Philox), so this checks the GPU generator,
    the cosine sampling, the basis and the environment lookup."""
    n = np.array([0.0, 1.0, 0.0])
    sc = synth.constant_color_plane_scene(1, 32, n, -0.2, [0.5, 0.25, 0.75], seed=4)
    env = synth.env_map(128, 64, seed=5005)
    sid = ctx.scene_create(sc)
    view = synth.View(eye=(0.3, 1.8, 1.9))
    W, H = 64, 48
    for spp in (1, 4):
        g = _pt(ctx, sid, view, W, H, 128, spp, 1, 77, env)
        ref = O.OracleScene.from_scene(sc).path_trace(view, W, H, 128, 1e-4, spp, 1, 77, env)
        d = np.abs(g["rgb"].reshape(-1, 3) - ref["rgb"]).max(1)
        log(f"plane one bounce spp={spp}: rgb diff p50 {np.median(d):.2e} p99.9 {np.percentile(d, 99.9):.2e} "
            f"max {d.max():.2e}")
        assert np.mean(g["hit"].reshape(-1) == ref["hit"]) > 0.999
        assert np.percentile(d, 99) < 1e-3
    ctx.scene_destroy(sid)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
def test_c5_like_scene_report(ctx, precision):
    """A small C5-like scene (noisy sphere, 3 bounces, environment): primary
    hits against the oracle; path radiance reported (parity unpinned at the
    image level: FP32/FP64 differences compound over bounces)."""
    sc = synth.sphere_scene(8, 64, 0.6, 0.02, seed=5000)
    env = synth.env_map(256, 128, seed=5005)
    sid = ctx.scene_create(sc, precisions=("bf16", "fp8"))
    view = synth.orbit_views(1, seed=5500)[0]
    W, H = 96, 72
    g = _pt(ctx, sid, view, W, H, 256, 2, 3, 5006, env, precision)
    pix = np.arange(W * H)
    ref = O.OracleScene.from_scene(sc).path_trace(view, W, H, 256, 1e-4, 2, 3, 5006, env)
    agree = np.mean(g["hit"].reshape(-1) == ref["hit"])
    d = np.abs(g["rgb"].reshape(-1, 3) - ref["rgb"]).max(1)
    st = g["stats"]
    log(f"c5-like {precision}: primary hit agreement {agree:.4f}; rgb diff p50 {np.median(d):.2e} "
        f"p90 {np.percentile(d, 90):.2e} p99 {np.percentile(d, 99):.2e}; rounds {st['rounds']} "
        f"evals {st['evals']} hits {st['hits']}")
    # low precision: reported; e4m3 keeps 3 mantissa bits, so on this noisy
    # scene a few percent of the primary rays stop at a different crossing
    assert agree > {"fp32": 0.99, "bf16": 0.95, "fp8": 0.9}[precision]
    assert np.median(d) < (1e-3 if precision == "fp32" else 5e-2)
    ctx.scene_destroy(sid)


def test_path_tracing_argument_errors(ctx):
    from paper_2206_10885_amd import kn
    sc = synth.sphere_scene(4, 32, 0.5, 0.01, seed=1)
    sid = ctx.scene_create(sc)
    v = synth.front_view()
    out = ctx.alloc_frame(8, 8)
    with pytest.raises(kn.KnError, match="E_UNSUPPORTED"):
        ctx.render_into(sid, kn.make_camera(v, 8, 8, 64, 1e-4, spp=4, bounces=0), out)
    with pytest.raises(kn.KnError, match="E_INVALID"):
        ctx.render_into(sid, kn.make_camera(v, 8, 8, 64, 1e-4, spp=1, bounces=99), out)
    with pytest.raises(kn.KnError, match="E_INVALID"):
        ctx.render_into(sid, kn.make_camera(v, 8, 8, 64, 1e-4, spp=0, bounces=1), out)
    ctx.scene_destroy(sid)
