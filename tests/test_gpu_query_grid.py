"""GPU parity of the point-query workloads against the FP64 oracle: dense
lattice sampling (kn_grid_sample, the mesh-extraction input of Sec. 4.1) and
the finite-difference eikonal term (kn_eikonal_fd, Sec. 3.2 / 3.3).

All calls go through the C ABI (libkn.so via the ctypes binding)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2206_10885_amd import synth
from tests import parity as P

pytestmark = pytest.mark.gpu

# float32 MLP values: the tolerance of the float32 point query (~40-70
# products per sum of O(1) terms, encoding error ~1e-7)
TOL_D = 2e-5
# gradients (relative to 1 + |g|): float32 position rounding times the second
# derivative of the highest encoding frequency
TOL_G = 2e-4


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


def _lattice_cells(N, R, lin):
    """Cells and FP64 local coordinates of lattice points (flattened indices),
    written from the lattice definition: point i at -1 + 2 i / (R - 1) per
    axis, cell floor(i N / (R - 1)) clamped."""
    ijk = np.stack([lin % R, (lin // R) % R, lin // (R * R)], axis=1).astype(np.int64)
    idx = np.minimum(ijk * N // (R - 1), N - 1)
    x = -1.0 + 2.0 * ijk / (R - 1)
    c = -1.0 + (2.0 * idx + 1.0) / N
    cells = idx[:, 0] + N * (idx[:, 1] + N * idx[:, 2])
    return cells, (x - c) * N


@pytest.mark.parametrize("N,H,R", [(4, 32, 37), (3, 64, 20), (16, 64, 33), (4, 32, 2), (2, 64, 64)])
def test_grid_sample_fp32_every_point(ctx, N, H, R):
    """Every lattice point of small lattices (ragged cells, points on inner
    faces and the box faces, R = 2: the corners only) against the oracle:
    value and world gradient."""
    log(f"grid fp32 N={N} H={H} R={R}")
    sc = synth.sphere_scene(N, H, 0.5, 0.02, seed=100 + N * 10 + H)
    sid = ctx.scene_create(sc)
    res = ctx.grid_sample(sid, R, "fp32", grad=True)
    d = res["d"].cpu().numpy().reshape(-1).astype(np.float64)
    g = res["grad"].cpu().numpy().reshape(-1, 3).astype(np.float64)
    lin = np.arange(R ** 3, dtype=np.int64)
    ref = O.OracleScene.from_scene(sc).grid_sample(R, lin, grad=True)
    ed = np.abs(d - ref["d"])
    eg = np.abs(g - ref["grad"]) / (1.0 + np.abs(ref["grad"]))
    log(f"  max |dd| {ed.max():.2e}  max rel dgrad {eg.max():.2e}")
    assert ed.max() < TOL_D
    assert eg.max() < TOL_G
    # the value-only kernel (march block) gives the same values
    d2 = ctx.grid_sample(sid, R, "fp32")["d"].cpu().numpy().reshape(-1).astype(np.float64)
    assert np.abs(d2 - ref["d"]).max() < TOL_D
    ctx.scene_destroy(sid)


def _sample_lattice(R, n, seed):
    """Sampled flat indices: random points, the 8 corners, and points on the
    first and last lattice planes and on inner cell faces."""
    rng = np.random.default_rng(seed)
    ijk = rng.integers(0, R, (n, 3))
    ijk[:8] = np.array([[i, j, k] for i in (0, R - 1) for j in (0, R - 1) for k in (0, R - 1)])
    ijk[8:200, rng.integers(0, 3)] = R - 1
    ijk[200:400, 0] = 0
    return np.unique(ijk[:, 0] + R * (ijk[:, 1] + R * ijk[:, 2]))


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
def test_grid_sample_512_sampled(ctx, precision):
    """The mesh-extraction workload at full size: a 512^3 lattice over the
    16^3, H=64 scene (134 M points).  Every output is written (the buffer is
    filled with NaN first); sampled points match the oracle: float32 within
    the query tolerance, bf16 / fp8 within the worst-case rounding bound of
    their weights and layer inputs."""
    from oracle import quant
    R = 512
    sc = synth.config_scene("c3")
    sid = ctx.scene_create(sc, precisions=("bf16", "fp8"))
    out = dict(d=torch.full((R, R, R), float("nan"), device="cuda"))
    log(f"grid 512 {precision}")
    ctx.grid_sample(sid, R, precision, out=out)
    torch.cuda.synchronize()
    assert not bool(torch.isnan(out["d"]).any()), "lattice points left unwritten"
    lin = _sample_lattice(R, 4000, seed=11)
    d = out["d"].reshape(-1)[torch.tensor(lin, device="cuda")].cpu().numpy().astype(np.float64)
    if precision == "fp32":
        ref = O.OracleScene.from_scene(sc).grid_sample(R, lin)["d"]
        err = np.abs(d - ref)
        log(f"  fp32 max |dd| {err.max():.2e}")
        assert err.max() < TOL_D
    else:
        cells, xl = _lattice_cells(sc.N, R, lin)
        f = quant.sdf_fp64(sc, cells, xl)
        bound = quant.rounding_bound(sc, f, precision)
        err = np.abs(d - f["d"])
        log(f"  {precision} vs FP64: p50 {np.median(err):.2e} p99 {np.percentile(err, 99):.2e} "
            f"max {err.max():.2e}; worst error / bound {(err / bound).max():.4f}")
        P.record(f"grid512_{precision}", dict(kernel_vs_fp64=P.stats(err)))
        assert (err <= bound).all()
    ctx.scene_destroy(sid)


def _eik_points(N, n, delta, seed):
    """Uniform points in the box (the eikonal sampling of Sec. 3.2) with some
    placed within delta of a cell face, so that their stencils straddle a seam."""
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-1, 1, (n, 3))
    k = min(n // 4, 2000)
    ax = rng.integers(0, 3, k)
    face = -1 + 2.0 * rng.integers(1, N, k) / N
    pts[np.arange(k), ax] = face + rng.uniform(-0.9, 0.9, k) * delta
    return pts.astype(np.float32)


@pytest.mark.parametrize("n", [16384, 257, 1])
def test_eikonal_fd_fp32_matches_oracle(ctx, n):
    """kn_eikonal_fd on the 16^3, H=64 scene at the paper's M = 16384 points
    (and ragged counts), delta = 1e-3.

    1. Stencil values against the oracle's SDF at the same float32 stencil
       points (x +- delta formed in float32, as the kernel does).
    2. Gradient norms against the central differences of those oracle
       values: within sqrt(3) * 2 TOL_D / (2 delta) (each difference of two
       values within TOL_D), plus float32 rounding of the norm.
    3. Gradient norms and loss against the oracle's own eikonal term at the
       exact points, with the stencil-point rounding (|x| 2^-24 times the
       SDF's local slope) added to the bound; the loss within the bound's
       first-order effect on the mean of (g - 1)^2."""
    delta = np.float32(1e-3)
    sc = synth.config_scene("c3")
    sid = ctx.scene_create(sc)
    pts = _eik_points(sc.N, n, float(delta), seed=n)
    log(f"eikonal fp32 n={n}")
    res = ctx.eikonal_fd(sid, torch.tensor(pts, device="cuda"), float(delta), "fp32", stencil=True)
    torch.cuda.synchronize()
    gn = res["gnorm"].cpu().numpy().astype(np.float64)
    st = res["stencil"].cpu().numpy().astype(np.float64)
    loss = float(res["loss"].cpu().numpy()[0])
    os_ = O.OracleScene.from_scene(sc)
    sp = np.repeat(pts[:, None, :], 6, axis=1).copy()
    for a in range(3):
        sp[:, 2 * a, a] = pts[:, a] + delta
        sp[:, 2 * a + 1, a] = pts[:, a] - delta
    ref_st = os_.query(sp.reshape(-1, 3))["d"].reshape(n, 6)
    es = np.abs(st - ref_st)
    log(f"  stencil max |dd| {es.max():.2e}")
    assert es.max() < TOL_D
    g_ref = np.sqrt(sum(((ref_st[:, 2 * a] - ref_st[:, 2 * a + 1]) / (2.0 * float(delta))) ** 2
                        for a in range(3)))
    eg = np.abs(gn - g_ref)
    b1 = np.sqrt(3.0) * 2 * TOL_D / (2 * float(delta)) + 1e-6 * (1 + g_ref)
    log(f"  gnorm vs oracle stencil: max {eg.max():.2e} (bound {b1.max():.2e}); p50 {np.median(eg):.2e}")
    assert (eg <= b1).all()
    full = os_.eikonal_fd(pts.astype(np.float64), float(delta))
    # slope of d near each point, from the stencil itself (a local bound)
    slope = np.abs(ref_st[:, 0::2] - ref_st[:, 1::2]).max(axis=1) / (2 * float(delta)) + 1.0
    rnd = (np.abs(pts).max(axis=1) + float(delta)) * 2.0 ** -24 * slope
    b2 = b1 + np.sqrt(3.0) * 2 * rnd / (2 * float(delta))
    e2 = np.abs(gn - full["gnorm"])
    log(f"  gnorm vs oracle eikonal: max {e2.max():.2e} p50 {np.median(e2):.2e}; loss {loss:.6e} "
        f"vs {full['loss']:.6e}")
    assert (e2 <= b2).all()
    lb = np.mean(2 * np.abs(full["gnorm"] - 1) * b2 + b2 ** 2)
    assert abs(loss - full["loss"]) <= lb + 1e-12 * abs(full["loss"])
    if n == 16384:
        P.record("eikonal_fd_fp32", dict(gnorm_vs_oracle=P.stats(e2), loss=loss, oracle_loss=full["loss"]))
    # seams: some stencils straddle a cell face, and there the global SDF's
    # jump shows in the difference (the oracle sees the same cells)
    ctx.scene_destroy(sid)


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_eikonal_fd_lowp_is_the_point_query(ctx, precision):
    """In bf16 / fp8 the stencil values are the point query's values at the
    stencil points, bit for bit (the query itself is checked against the
    oracle's bounds elsewhere); gradient norms follow from them by the
    stated difference formula, and the loss is deterministic."""
    delta = np.float32(1e-3)
    sc = synth.config_scene("c3")
    sid = ctx.scene_create(sc, precisions=("bf16", "fp8"))
    n = 5000
    pts = _eik_points(sc.N, n, float(delta), seed=9)
    res = ctx.eikonal_fd(sid, torch.tensor(pts, device="cuda"), float(delta), precision, stencil=True)
    sp = np.repeat(pts[:, None, :], 6, axis=1).copy()
    for a in range(3):
        sp[:, 2 * a, a] = pts[:, a] + delta
        sp[:, 2 * a + 1, a] = pts[:, a] - delta
    q = ctx.query(sid, torch.tensor(sp.reshape(-1, 3), device="cuda"), precision)["d"].reshape(n, 6)
    torch.cuda.synchronize()
    assert torch.equal(q, res["stencil"])
    st = res["stencil"].cpu().numpy().astype(np.float64)
    g = np.sqrt(sum(((st[:, 2 * a] - st[:, 2 * a + 1]) / (2.0 * float(delta))) ** 2 for a in range(3)))
    gn = res["gnorm"].cpu().numpy().astype(np.float64)
    assert np.abs(gn - g).max() <= 1e-5 * (1 + g).max()
    res2 = ctx.eikonal_fd(sid, torch.tensor(pts, device="cuda"), float(delta), precision)
    assert torch.equal(res["loss"], res2["loss"]) and torch.equal(res["gnorm"], res2["gnorm"])
    ctx.scene_destroy(sid)


def test_grid_and_eikonal_argument_errors(ctx):
    from paper_2206_10885_amd import kn
    sc = synth.sphere_scene(4, 32, 0.5, 0.0, seed=3)
    sid = ctx.scene_create(sc)
    out = dict(d=torch.full((3, 3, 3), 7.0, device="cuda"), grad=torch.zeros((3, 3, 3, 3), device="cuda"))
    with pytest.raises(kn.KnError) as e:
        ctx.grid_sample(sid, 3, "fp8", out=out)     # no fp8 copy
    assert e.value.status == -1
    with pytest.raises(kn.KnError) as e:
        ctx.grid_sample(sid, 1, "fp32", out=out)
    assert e.value.status == -1
    assert bool((out["d"] == 7.0).all())
    with pytest.raises(kn.KnError) as e:
        ctx.eikonal_fd(sid, torch.zeros((4, 3), device="cuda"), 0.0)
    assert e.value.status == -1
    ctx.scene_destroy(sid)
