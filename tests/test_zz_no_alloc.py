"""The allocation-free point query (kn_query_noalloc) against kn_query, through
the C ABI on the GPU: the same outputs bit for bit, on two calls in a row
(the second with fewer points, so it runs on what the first left in the
scratch array), for every precision; a call above the limit is refused and
changes no output."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2206_10885_amd import synth

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


def _points(n, N, seed):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-1, 1, (n, 3))
    pts[:16] = -1 + 2.0 * rng.integers(0, N + 1, (16, 3)) / N   # on cell faces and box corners
    return torch.tensor(pts.astype(np.float32), device="cuda")


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
def test_noalloc_query_equals_query(ctx, precision):
    from paper_2206_10885_amd import kn
    sc = synth.sphere_scene(16, 64, 0.6, 0.02, seed=5)
    sid = ctx.scene_create(sc, precisions=("bf16", "fp8"))
    for n, seed in ((200_000, 1), (1_537, 2)):
        log(f"no-alloc query {precision}: n={n}")
        pts = _points(n, sc.N, seed)
        ref = ctx.query(sid, pts, precision, grad=True, feat=True)
        got = ctx.query(sid, pts, precision, grad=True, feat=True, noalloc=True)
        torch.cuda.synchronize()
        for k in ("d", "grad", "z"):
            assert torch.equal(ref[k], got[k]), (precision, n, k)
    # above the limit: refused, outputs untouched
    n = (1 << 18) + 1
    pts = _points(n, sc.N, 3)
    out = dict(d=torch.full((n,), 7.0, device="cuda"))
    with pytest.raises(kn.KnError) as e:
        ctx.query(sid, pts, precision, noalloc=True, out=out)
    assert e.value.status == -1
    assert bool((out["d"] == 7.0).all())
    ctx.scene_destroy(sid)


def test_noalloc_query_small_grid_after_large(ctx):
    """A 4^3 scene after the 16^3 one: the counters of cells the small grid
    does not have are left from the earlier call and must not matter."""
    sc = synth.sphere_scene(4, 32, 0.5, 0.02, seed=6)
    sid = ctx.scene_create(sc, precisions=("bf16",))
    pts = _points(5_000, sc.N, 4)
    ref = ctx.query(sid, pts, "bf16")
    got = ctx.query(sid, pts, "bf16", noalloc=True)
    torch.cuda.synchronize()
    assert torch.equal(ref["d"], got["d"])
    ctx.scene_destroy(sid)
