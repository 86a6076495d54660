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


@pytest.fixture(scope="module")
def c5_scene(ctx):
    """The C5 scene (32^3 grid, H = 64) resident in every precision."""
    sc = synth.config_scene("c5")
    sid = ctx.scene_create(sc, precisions=("bf16", "fp8"))
    yield sc, sid
    ctx.scene_destroy(sid)


def _uniforms(seed, pixel, sample, k):
    """The path's two uniforms at event k: Philox-4x32-10 keyed by the seed
    with counter (pixel, sample, k, 0), top 24 bits of the first two words
    times 2^-24 (the oracle's generator)."""
    x = O.philox4x32_10([pixel, sample, k, 0], [seed & 0xFFFFFFFF, seed >> 32])
    return (int(x[0]) >> 8) * 2.0 ** -24, (int(x[1]) >> 8) * 2.0 ** -24


@pytest.mark.parametrize("precision", ["fp8", "bf16", "fp32"])
def test_c5_per_segment_against_oracle(ctx, c5_scene, precision):
    """C5 (32^3, H = 64, 1920x1080, 4 spp, 3 bounces, 512x256 environment),
    path traced on the GPU with per-segment records, compared with the FP64
    oracle segment by segment on the paths of 120 sampled pixels (480 paths),
    each segment from the GPU's own origin and direction (identical rays, so
    FP32/FP64 differences do not compound over bounces):
      - segment 0 is the oracle's camera ray through the Philox jitter;
        segment k >= 1 starts 1e-3 above the GPU's previous hit along its
        normal, in the oracle's cosine-weighted direction about that normal
        for the Philox uniforms of event k;
      - every GPU hit is replayed by the oracle from the GPU's march state:
        where the replay is well conditioned, depth (along the segment),
        normal and albedo match it (1e-4, 0.1 degree, 1e-3) on all but 0.1%;
      - the FP64 SDF where each hit's march stopped is below eps plus the
        precision's stated bound (float32: 1e-5);
      - the oracle's own trace of the segment agrees on hit / miss (reported;
        float32: >= 99% of the segments whose oracle trace is stable);
      - each pixel's colour equals the mean over its samples of the radiance
        the GPU's own segments define (throughput = product of albedos, an
        escaping segment adds throughput x env(dir)), to 1e-4 relative.
    Image-level agreement with the oracle's independent paths is parity
    unpinned (compounding differences)."""
    from paper_2206_10885_amd import kn
    sc, sid = c5_scene
    c = synth.CONFIGS["c5"]
    W, H, spp, B, S, eps = c["width"], c["height"], c["spp"], c["bounces"], c["max_steps"], c["eps"]
    seed = c["path_seed"]
    env = synth.env_map(512, 256, seed=c["env_seed"])
    envt = torch.tensor(env, device="cuda")
    view = synth.orbit_views(1, c["seed"] + 500)[0]
    cam = kn.make_camera(view, W, H, S, eps, precision, spp=spp, bounces=B, seed=seed, env=envt)
    out = ctx.alloc_frame(W, H)
    log(f"c5 segments {precision}: allocating {W * H * spp * (B + 1) * 80 / 1e9:.2f} GB of records")
    out["segments"] = torch.empty((W * H * spp * (B + 1), kn.SEGMENT_WORDS), dtype=torch.int32, device="cuda")
    st = ctx.render_into(sid, cam, out)
    torch.cuda.synchronize()
    pix = synth.sample_pixels(W, H, 120, seed=c["seed"] + 77)
    paths = (pix[:, None] * spp + np.arange(spp)[None, :]).ravel()
    rows = (paths[:, None] * (B + 1) + np.arange(B + 1)[None, :]).ravel()
    seg = kn.segment_fields(out["segments"][torch.tensor(rows, device="cuda")].view(len(paths), B + 1, -1))
    rgb = out["rgb"].cpu().numpy().reshape(-1, 3)[pix].astype(np.float64)
    del out
    os_ = O.OracleScene.from_scene(sc)
    pert = [O.OracleScene.from_scene(P.perturbed(sc, 1e-6, 700 + k)) for k in range(3)]
    rng = np.random.default_rng(9)
    half = 1.0 / sc.N
    centers = synth.cell_centers(sc.N)
    bound = {"fp32": 1e-5}.get(precision)
    if bound is None:
        from tests.test_gpu_parity import _fstop_bound
        bound, _ = _fstop_bound(sc, precision, n=3000)
    n_seg = n_hit = n_rep = rep_bad = chain_bad = fstop_bad = agree_n = agree_ok = 0
    worst = dict(depth=0.0, normal=0.0, albedo=0.0, origin=0.0, dir=0.0, rgb=0.0)
    Lpix = np.zeros((len(pix), 3))
    for q, pth in enumerate(paths):
        p, smp = divmod(int(pth), spp)
        T = np.ones(3)
        L = np.zeros(3)
        for k in range(B + 1):
            o, d = seg["origin"][q, k], seg["dir"][q, k]
            status = int(seg["status"][q, k])
            if k == 0:
                xi = _uniforms(seed, p, smp, 0) if spp > 1 else (0.5, 0.5)
                oo, od = O.camera_ray(view, W, H, p // W, p % W, *xi)
            else:
                prev = {f: seg[f][q, k - 1] for f in ("origin", "dir", "t", "normal")}
                u1, u2 = _uniforms(seed, p, smp, k)
                od = O.cosine_dir(prev["normal"], u1, u2)
                oo = prev["origin"] + prev["t"] * prev["dir"] + 1e-3 * prev["normal"]
            eo, ed = float(np.abs(o - oo).max()), float(P.angle_deg(d, od))
            worst["origin"], worst["dir"] = max(worst["origin"], eo), max(worst["dir"], ed)
            if eo > 1e-5 or ed > 1e-3:
                chain_bad += 1
            assert status in (0, 1, 2, 3), (q, k, status)
            n_seg += 1
            if status != 1:
                L += T * O.env_lookup(env, d)
                break
            n_hit += 1
            cell = int(seg["cell"][q, k])
            idx = (cell % sc.N, (cell // sc.N) % sc.N, cell // (sc.N * sc.N))
            cc = centers[cell]
            xs = o + seg["t_march"][q, k] * d
            if os_.sdf_eval(cell, (xs - cc) / half)[0] - eps > bound:
                fstop_bad += 1
            tr = P._trace_struct(idx, seg["t_march"][q, k], seg["t_entry"][q, k])
            sh = os_.shade(o, d, tr)
            stable = True
            for ps in pert:
                dj = d + 1e-7 * rng.standard_normal(3)
                dj /= np.linalg.norm(dj)
                s2 = ps.shade(o, dj, P._trace_struct(idx, seg["t_march"][q, k] * (1 + 1e-6 * rng.standard_normal()),
                                                     seg["t_entry"][q, k]))
                if (abs(s2["depth"] - sh["depth"]) > P.TOL_DEPTH / 2
                        or P.angle_deg(s2["normal"], sh["normal"]) > P.TOL_NORMAL_DEG / 2
                        or np.abs(s2["rgb"] - sh["rgb"]).max() > P.TOL_RGB / 2):
                    stable = False
                    break
            if stable:
                n_rep += 1
                e_d = abs(sh["depth"] - seg["t"][q, k])
                e_n = float(P.angle_deg(sh["normal"], seg["normal"][q, k]))
                e_c = float(np.abs(sh["rgb"] - seg["albedo"][q, k]).max())
                worst["depth"], worst["normal"] = max(worst["depth"], e_d), max(worst["normal"], e_n)
                worst["albedo"] = max(worst["albedo"], e_c)
                if e_d > P.TOL_DEPTH or e_n > P.TOL_NORMAL_DEG or e_c > P.TOL_RGB:
                    rep_bad += 1
            if k == B:
                break
            T = T * seg["albedo"][q, k]
        # the oracle's own trace of this path's first segment (hit / miss)
        r0 = os_.trace(seg["origin"][q, 0], seg["dir"][q, 0], S, eps)
        r1 = pert[0].trace(seg["origin"][q, 0], seg["dir"][q, 0], S, eps)
        if (r0["status"] == O.HIT) == (r1["status"] == O.HIT):
            agree_n += 1
            agree_ok += int((r0["status"] == O.HIT) == (seg["status"][q, 0] == 1))
        Lpix[q // spp] += L / spp
    erel = np.abs(Lpix - rgb).max(1) / (1.0 + np.abs(Lpix).max(1))
    worst["rgb"] = float(erel.max())
    agree = agree_ok / max(1, agree_n)
    log(f"c5 {precision}: {n_seg} segments ({n_hit} hits), chain errors {chain_bad}, replays {n_rep} "
        f"(bad {rep_bad}), stop over bound {fstop_bad}, primary hit agreement with the oracle {agree:.4f}; "
        f"worst {worst}; frame stats {st}")
    P.record(f"c5_segments_{precision}", dict(segments=n_seg, hits=n_hit, replays=n_rep, replay_bad=rep_bad,
                                              chain_bad=chain_bad, fstop_bad=fstop_bad, fstop_bound=bound,
                                              primary_hit_agreement=agree, worst=worst))
    assert n_hit > 300 and n_rep > 0.5 * n_hit
    assert chain_bad == 0
    assert rep_bad <= 1e-3 * n_rep
    assert fstop_bad == 0
    assert worst["rgb"] < 1e-4
    if precision == "fp32":
        assert agree >= 0.99
