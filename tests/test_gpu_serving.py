"""Serving loop (continuous batching) on the GPU, through the C ABI.

Requests of several resident scenes and resolutions share one ray pool; each
result must equal the same frame rendered alone (the per-ray arithmetic does
not depend on which other rays share a tile or a round, so equality is
exact), and sampled pixels must match the FP64 oracle."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2206_10885_amd import synth
from tests import parity as P

pytestmark = pytest.mark.gpu

FIELDS = ("rgb", "depth", "normal", "hit", "steps")


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _kn():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible: GPU tests need an MI355X")
    from paper_2206_10885_amd import kn
    return kn


def _scenes():
    return [synth.sphere_scene(4, 32, 0.5, 0.01, seed=11),
            synth.sphere_scene(6, 64, 0.55, 0.02, seed=12),
            synth.sphere_scene(16, 32, 0.6, 0.02, seed=13)]


def _requests(n, seed):
    rng = np.random.default_rng(seed)
    views = synth.orbit_views(n, seed=seed + 1)
    sizes = [(64, 64), (97, 61), (256, 256), (200, 120), (1, 1), (33, 300)]
    return [(int(rng.integers(0, 3)), views[i], *sizes[int(rng.integers(0, len(sizes)))]) for i in range(n)]


def _same(a, b):
    for f in FIELDS:
        x, y = a[f].cpu(), b[f].cpu()
        if not torch.equal(x, y):
            bad = (x != y).reshape(x.shape[0], x.shape[1], -1).any(-1)
            return f"{f} differs at {int(bad.sum())} pixels"
    return None


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_serving_mix_equals_alone(precision):
    kn = _kn()
    scenes = _scenes()
    with kn.Context(0) as ctx:
        sids = [ctx.scene_create(s, precisions=("bf16",)) for s in scenes]
        reqs = _requests(14, seed=5)
        alone = []
        for k, v, W, H in reqs:
            cam = kn.make_camera(v, W, H, 96, 1e-4, precision)
            out = ctx.alloc_frame(W, H)
            ctx.render_into(sids[k], cam, out)
            alone.append(out)
        torch.cuda.synchronize()
        log(f"{precision}: {len(reqs)} requests rendered alone")
        ctx.serve_start(max_inflight=8, precision=precision)
        mixed, ids = [], []
        for k, v, W, H in reqs:
            out = ctx.alloc_frame(W, H)
            for f in FIELDS:
                out[f].fill_(7)
            torch.cuda.synchronize()
            ids.append(ctx.serve_submit(sids[k], kn.make_camera(v, W, H, 96, 1e-4, precision), out))
            mixed.append(out)
        stats = [ctx.serve_poll(i, timeout_us=60_000_000) for i in ids]
        log(f"  served; latencies ms: {[round(s['wall_ms'], 2) for s in stats]}")
        for (k, v, W, H), a, m, st in zip(reqs, alone, mixed, stats):
            assert st["rays"] == W * H
            assert st["hits"] == int(a["hit"].sum().item())
            msg = _same(a, m)
            assert msg is None, f"scene {k} {W}x{H}: {msg}"
        # a second wave re-using the slots and pool ranges
        ids2 = [ctx.serve_submit(sids[k], kn.make_camera(v, W, H, 96, 1e-4, precision), m)
                for (k, v, W, H), m in zip(reqs[:5], mixed[:5])]
        for i in ids2:
            ctx.serve_poll(i, timeout_us=60_000_000)
        for a, m in zip(alone[:5], mixed[:5]):
            assert _same(a, m) is None
        ctx.serve_stop()


def test_serving_matches_oracle():
    kn = _kn()
    sc = synth.sphere_scene(4, 32, 0.5, 0.01, seed=1000)
    views = [synth.front_view()] + synth.orbit_views(2, seed=77)
    with kn.Context(0) as ctx:
        sid = ctx.scene_create(sc)
        ctx.serve_start(max_inflight=4, precision="fp32")
        outs, ids = [], []
        for v in views:
            out = ctx.alloc_frame(64, 64, with_trace=True)
            ids.append(ctx.serve_submit(sid, kn.make_camera(v, 64, 64, 64, 1e-4, "fp32"), out))
            outs.append(out)
        for i in ids:
            ctx.serve_poll(i, timeout_us=60_000_000)
        ctx.serve_stop()
    for v, out in zip(views, outs):
        rep = P.compare(sc, v, 64, 64, 64, 1e-4, P.gpu_arrays(out))
        log(rep.as_dict())
        assert rep.ok()


def test_serving_admission_by_budget():
    """A budget that leaves room for one large request at a time: the others
    wait in the queue and still come out equal to their alone renders."""
    kn = _kn()
    sc = synth.sphere_scene(4, 32, 0.5, 0.01, seed=21)
    W = H = 1024
    views = synth.orbit_views(4, seed=22)
    with kn.Context(0, hbm_budget_bytes=300 << 20) as ctx:
        sid = ctx.scene_create(sc)
        alone = []
        for v in views:
            out = ctx.alloc_frame(W, H)
            ctx.render_into(sid, kn.make_camera(v, W, H, 64, 1e-4, "bf16"), out)
            alone.append(out)
        torch.cuda.synchronize()
        ctx.serve_start(max_inflight=4, precision="bf16")
        outs = [ctx.alloc_frame(W, H) for _ in views]
        ids = [ctx.serve_submit(sid, kn.make_camera(v, W, H, 64, 1e-4, "bf16"), o)
               for v, o in zip(views, outs)]
        stats = [ctx.serve_poll(i, timeout_us=60_000_000) for i in ids]
        log("latencies", [round(s["wall_ms"], 2) for s in stats], "in pool",
            [round(s["gpu_ms"], 2) for s in stats])
        # later requests waited for pool space
        assert stats[-1]["wall_ms"] > stats[-1]["gpu_ms"]
        for a, o in zip(alone, outs):
            assert _same(a, o) is None
        big = ctx.alloc_frame(4096, 4096)
        with pytest.raises(kn.KnError, match="E_NOMEM"):
            ctx.serve_submit(sid, kn.make_camera(views[0], 4096, 4096, 64, 1e-4, "bf16"), big)
        ctx.serve_stop()


def test_serving_errors():
    kn = _kn()
    sc = synth.sphere_scene(4, 32, 0.5, 0.01, seed=31)
    v = synth.front_view()
    with kn.Context(0) as ctx:
        sid = ctx.scene_create(sc)
        out = ctx.alloc_frame(32, 32)
        cam = kn.make_camera(v, 32, 32, 64, 1e-4, "bf16")
        with pytest.raises(kn.KnError, match="E_SHUTDOWN"):
            ctx.serve_submit(sid, cam, out)
        with pytest.raises(kn.KnError, match="E_SHUTDOWN"):
            ctx.serve_poll(1, 0)
        with pytest.raises(kn.KnError, match="E_INVALID"):
            ctx.serve_start(max_inflight=0)
        ctx.serve_start(max_inflight=2, precision="bf16")
        with pytest.raises(kn.KnError, match="E_BUSY"):
            ctx.serve_start(max_inflight=2, precision="bf16")
        with pytest.raises(kn.KnError, match="E_INVALID"):
            ctx.serve_submit(sid, kn.make_camera(v, 32, 32, 64, 1e-4, "fp32"), out)
        with pytest.raises(kn.KnError, match="E_NOT_FOUND"):
            ctx.serve_submit(sid + 100, cam, out)
        with pytest.raises(kn.KnError, match="E_NOT_FOUND"):
            ctx.serve_poll(12345, 0)
        rid = ctx.serve_submit(sid, cam, out)
        st = ctx.serve_poll(rid, 0)
        if st is None:
            with pytest.raises(kn.KnError, match="E_BUSY"):
                ctx.scene_destroy(sid)
            st = ctx.serve_poll(rid, timeout_us=60_000_000)
        assert st["rays"] == 32 * 32
        with pytest.raises(kn.KnError, match="E_NOT_FOUND"):
            ctx.serve_poll(rid, 0)
        ctx.serve_stop()
        ctx.scene_destroy(sid)


def test_serving_c4_scenes_mix_equals_alone():
    """C4's eight resident scenes (grids 16^3, 16^3, 20^3, 24^3, 24^3, 28^3,
    32^3, 32^3; H = 32 for even k, 64 for odd k; r = 0.5 + 0.02 k; sigma
    0.02) in one serving pool, bf16, 256 steps: 24 requests at C4's
    resolutions {256^2, 512^2, 800^2, 1920x1080} submitted together, each
    equal bit for bit to the same frame rendered alone."""
    kn = _kn()
    Ns = [16, 16, 20, 24, 24, 28, 32, 32]
    scenes = [synth.sphere_scene(Ns[k], 32 if k % 2 == 0 else 64, 0.5 + 0.02 * k, 0.02, 4000 + k)
              for k in range(8)]
    sizes = [(256, 256), (512, 512), (800, 800), (1920, 1080)]
    rng = np.random.default_rng(44)
    with kn.Context(0) as ctx:
        sids = [ctx.scene_create(s, precisions=("bf16",)) for s in scenes]
        del scenes
        log("c4 scenes resident")
        reqs = []
        for i in range(24):
            k = i % 8
            v = synth.orbit_views(64, 4000 + k + 500)[int(rng.integers(0, 64))]
            reqs.append((k, v, *sizes[(i // 8 + i) % 4]))
        alone = []
        for k, v, W, H in reqs:
            out = ctx.alloc_frame(W, H)
            ctx.render_into(sids[k], kn.make_camera(v, W, H, 256, 1e-4, "bf16"), out)
            alone.append(out)
        torch.cuda.synchronize()
        log(f"c4: {len(reqs)} requests rendered alone")
        ctx.serve_start(max_inflight=32, precision="bf16")
        mixed, ids = [], []
        for k, v, W, H in reqs:
            out = ctx.alloc_frame(W, H)
            for f in FIELDS:
                out[f].fill_(7)
            torch.cuda.synchronize()
            ids.append(ctx.serve_submit(sids[k], kn.make_camera(v, W, H, 256, 1e-4, "bf16"), out))
            mixed.append(out)
        stats = [ctx.serve_poll(i, timeout_us=120_000_000) for i in ids]
        log(f"c4 served; latencies ms: {[round(s['wall_ms'], 1) for s in stats]}")
        for (k, v, W, H), a, m, st in zip(reqs, alone, mixed, stats):
            assert st["rays"] == W * H
            msg = _same(a, m)
            assert msg is None, f"scene {k} {W}x{H}: {msg}"
        ctx.serve_stop()
