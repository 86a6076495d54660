"""Early shading of large primary frames: once the rounds thin out, the
hits found so far are shaded on a second stream beside the remaining
rounds.  The frame must be the one-pass frame bit for bit (each hit is
refined and shaded on its own), whatever the fork point.

All calls go through the C ABI (libkn.so via the ctypes binding)."""
import os
import sys

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


def _render(ctx, sid, view, c, precision, frac, split=False):
    from paper_2206_10885_amd import kn
    old = os.environ.get("KN_EARLY_SHADE")
    os.environ["KN_EARLY_SHADE"] = frac
    try:
        cam = kn.make_camera(view, c["width"], c["height"], c["max_steps"], c["eps"], precision,
                             split_shading=split)
        out = ctx.alloc_frame(c["width"], c["height"], with_trace=True)
        out["stats"] = ctx.render_into(sid, cam, out)
        torch.cuda.synchronize()
    finally:
        if old is None:
            os.environ.pop("KN_EARLY_SHADE", None)
        else:
            os.environ["KN_EARLY_SHADE"] = old
    return out


@pytest.mark.parametrize("precision,split", [("bf16", False), ("fp32", False), ("bf16", True)])
def test_early_shading_equals_one_pass(ctx, precision, split):
    c = synth.CONFIGS["c3"]
    sc = synth.config_scene("c3")
    sid = ctx.scene_create(sc, precisions=("bf16",))
    for view in synth.config_views("c3")[:2]:
        ref = _render(ctx, sid, view, c, precision, "0", split)
        for frac in ("0.25", "0.6", "0.9"):
            out = _render(ctx, sid, view, c, precision, frac, split)
            log(f"{precision} split={split} early at {frac}: rounds {out['stats']['rounds']} vs "
                f"{ref['stats']['rounds']}, hits {out['stats']['hits']} vs {ref['stats']['hits']}, "
                f"gpu {out['stats']['gpu_ms']:.3f} vs {ref['stats']['gpu_ms']:.3f} ms")
            for k in ("rgb", "depth", "normal", "hit", "steps", "trace"):
                assert torch.equal(out[k], ref[k]), (frac, k)
            assert out["stats"]["hits"] == ref["stats"]["hits"]
            assert out["stats"]["evals"] == ref["stats"]["evals"]
    ctx.scene_destroy(sid)
