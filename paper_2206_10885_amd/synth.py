"""Seeded synthetic inputs for KiloNeuS rendering: scenes, camera views,
environment maps and serving request traces.

This module only *draws* inputs.  It holds none of the rendering arithmetic
(encoding, MLP evaluation, sphere tracing, shading); both the FP64 CPU oracle
and the HIP path receive the arrays made here and compute on them on their own.

Scene layout (the host-side parameter format of the C ABI, one block per cell,
cells ordered g = ix + N*(iy + N*iz), all float32):

  SDF block  (KiloSDF, eq. 3 of the paper, softplus MLP on gamma_6(x_local)):
      W1[H][39], b1[H], W2[H][H], b2[H], W3[16][H], b3[16]
      output row 0 is the SDF d, rows 1..15 the feature z (Sec. 3.1).
  Color block (KiloColor, eq. 4, ReLU MLP then sigmoid):
      Wc1[32][48], bc1[32], Wc2[3][32], bc2[3]
      input order [x_local(3), gamma_4(v)(27), n(3), z(15)].

The paper's trained per-cell weights (a DTU-trained model, Sec. 4) are not
available; the scenes here are seeded geometric initialisations toward a
sphere (Atzmon & Lipman's SAL initialisation, drawn once per scene in world
coordinates and folded exactly into every cell's local frame), plus seeded
per-cell Gaussian noise, which stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

POS_FREQS = 6          # L for the position encoding (Sec. 3.1)
DIR_FREQS = 4          # L for the view-direction encoding (Sec. 3.1)
FEAT_DIM = 15          # feature z; SDF MLP emits 1 + 15 outputs
COL_HIDDEN = 32        # KiloColor hidden width
SOFTPLUS_BETA = 100.0


def pe_dim(n: int, L: int) -> int:
    """Size of gamma_L on R^n: n + 2nL (Sec. 3.1, eq. 1-2)."""
    return n + 2 * n * L


SDF_IN = pe_dim(3, POS_FREQS)                          # 39
COL_IN = 3 + pe_dim(3, DIR_FREQS) + 3 + FEAT_DIM       # 48


def sdf_block_size(H: int) -> int:
    return SDF_IN * H + H + H * H + H + (1 + FEAT_DIM) * H + (1 + FEAT_DIM)


def col_block_size() -> int:
    return COL_IN * COL_HIDDEN + COL_HIDDEN + 3 * COL_HIDDEN + 3


def sdf_offsets(H: int) -> dict:
    """Offsets (in floats) of each tensor inside one SDF block."""
    o = {}
    p = 0
    for name, n in (("W1", SDF_IN * H), ("b1", H), ("W2", H * H), ("b2", H),
                    ("W3", (1 + FEAT_DIM) * H), ("b3", 1 + FEAT_DIM)):
        o[name] = (p, n)
        p += n
    return o


def col_offsets() -> dict:
    o = {}
    p = 0
    for name, n in (("Wc1", COL_IN * COL_HIDDEN), ("bc1", COL_HIDDEN),
                    ("Wc2", 3 * COL_HIDDEN), ("bc2", 3)):
        o[name] = (p, n)
        p += n
    return o


@dataclasses.dataclass
class Scene:
    N: int
    H: int
    sdf: np.ndarray            # float32 [N^3, sdf_block_size(H)]
    col: np.ndarray            # float32 [N^3, col_block_size()]
    bbox_min: tuple = (-1.0, -1.0, -1.0)
    bbox_max: tuple = (1.0, 1.0, 1.0)
    beta: float = SOFTPLUS_BETA
    name: str = ""

    @property
    def cells(self) -> int:
        return self.N ** 3


def unpack_sdf(block: np.ndarray, H: int) -> dict:
    o = sdf_offsets(H)
    shapes = {"W1": (H, SDF_IN), "b1": (H,), "W2": (H, H), "b2": (H,),
              "W3": (1 + FEAT_DIM, H), "b3": (1 + FEAT_DIM,)}
    return {k: block[p:p + n].reshape(shapes[k]) for k, (p, n) in o.items()}


def unpack_col(block: np.ndarray) -> dict:
    o = col_offsets()
    shapes = {"Wc1": (COL_HIDDEN, COL_IN), "bc1": (COL_HIDDEN,),
              "Wc2": (3, COL_HIDDEN), "bc2": (3,)}
    return {k: block[p:p + n].reshape(shapes[k]) for k, (p, n) in o.items()}


def pack_sdf(W1, b1, W2, b2, W3, b3) -> np.ndarray:
    return np.concatenate([np.asarray(a, np.float64).ravel()
                           for a in (W1, b1, W2, b2, W3, b3)]).astype(np.float32)


def pack_col(Wc1, bc1, Wc2, bc2) -> np.ndarray:
    return np.concatenate([np.asarray(a, np.float64).ravel()
                           for a in (Wc1, bc1, Wc2, bc2)]).astype(np.float32)


def cell_centers(N: int, bbox_min=(-1, -1, -1), bbox_max=(1, 1, 1)) -> np.ndarray:
    """Centers of the N^3 cells, ordered g = ix + N*(iy + N*iz) (float64)."""
    lo = np.asarray(bbox_min, np.float64)
    hi = np.asarray(bbox_max, np.float64)
    s = (hi - lo) / N
    i = np.arange(N, dtype=np.float64)
    iz, iy, ix = np.meshgrid(i, i, i, indexing="ij")
    c = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)
    return lo + (c + 0.5) * s


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def sphere_scene(N: int, H: int, radius: float, sigma: float, seed: int,
                 name: str = "") -> Scene:
    """Seeded geometric-initialisation scene toward a sphere of `radius`.

    One base network is drawn in world coordinates: hidden weights
    N(0, 2/fan_out), zero hidden biases, the encoding columns of the first
    layer zero, the SDF output row N(sqrt(pi)/sqrt(H), 1e-5^2) with bias
    -radius, feature rows N(0, 1/H) with zero bias.  It is folded exactly into
    every cell's local frame (x = c + h * x_local), then every weight and bias
    of every cell gets independent N(0, sigma^2) noise.  Color MLPs are
    He-normal with zero bias, drawn per cell.
    """
    rng = _rng(seed)
    n_cells = N ** 3
    # base network in world coordinates
    W1b = np.zeros((H, SDF_IN))
    W1b[:, 0:3] = rng.normal(0.0, math.sqrt(2.0 / H), size=(H, 3))
    b1b = np.zeros(H)
    W2b = rng.normal(0.0, math.sqrt(2.0 / H), size=(H, H))
    b2b = np.zeros(H)
    W3b = np.zeros((1 + FEAT_DIM, H))
    W3b[0] = rng.normal(math.sqrt(math.pi) / math.sqrt(H), 1e-5, size=H)
    W3b[1:] = rng.normal(0.0, math.sqrt(1.0 / H), size=(FEAT_DIM, H))
    b3b = np.zeros(1 + FEAT_DIM)
    b3b[0] = -radius

    P = sdf_block_size(H)
    o = sdf_offsets(H)
    centers = cell_centers(N)
    h = 1.0 / N                                   # half cell side in [-1,1]^3
    # float64 values rounded once to float32 (assignment into the float32
    # array); noise drawn in row chunks, the same stream as one draw
    sdf = np.empty((n_cells, P), np.float32)
    # per-cell fold: W1[:, 0:3] <- h * W1b[:, 0:3],  b1 <- b1b + W1b[:, 0:3] @ c
    W1c = W1b.copy()
    W1c[:, 0:3] *= h
    sdf[:, o["W1"][0]:o["W1"][0] + o["W1"][1]] = W1c.ravel()[None, :]
    sdf[:, o["b1"][0]:o["b1"][0] + H] = b1b[None, :] + centers @ W1b[:, 0:3].T
    sdf[:, o["W2"][0]:o["W2"][0] + H * H] = W2b.ravel()[None, :]
    sdf[:, o["b2"][0]:o["b2"][0] + H] = b2b[None, :]
    sdf[:, o["W3"][0]:o["W3"][0] + o["W3"][1]] = W3b.ravel()[None, :]
    sdf[:, o["b3"][0]:o["b3"][0] + 1 + FEAT_DIM] = b3b[None, :]
    if sigma > 0:
        rows = max(1, (1 << 22) // P)
        buf = np.empty((rows, P), np.float32)
        for r0 in range(0, n_cells, rows):
            r1 = min(n_cells, r0 + rows)
            nb = buf[:r1 - r0]
            rng.standard_normal(out=nb, dtype=np.float32)
            nb *= np.float32(sigma)
            sdf[r0:r1] += nb

    Pc = col_block_size()
    oc = col_offsets()
    col = np.zeros((n_cells, Pc), np.float32)
    w1 = col[:, oc["Wc1"][0]:oc["Wc1"][0] + COL_IN * COL_HIDDEN]
    w1[...] = rng.standard_normal((n_cells, COL_IN * COL_HIDDEN), dtype=np.float32)
    w1 *= np.float32(math.sqrt(2.0 / COL_IN))
    w2 = col[:, oc["Wc2"][0]:oc["Wc2"][0] + 3 * COL_HIDDEN]
    w2[...] = rng.standard_normal((n_cells, 3 * COL_HIDDEN), dtype=np.float32)
    w2 *= np.float32(math.sqrt(2.0 / COL_HIDDEN))
    return Scene(N=N, H=H, sdf=sdf, col=col, name=name or f"sphere N={N} H={H}")


def plane_scene(N: int, H: int, normal, offset: float, seed: int) -> Scene:
    """Scene whose SDF is the plane f(x) = n.x - offset (world units).

    First-layer rows are alpha_j * n with alpha_j ~ U(0.3, 0.5), encoding
    columns zero, b1 = 1.5; second-layer entries U(0, 2/H), b2 = 0.5.  Every
    pre-activation then exceeds 0.6 inside the box, where softplus with
    beta = 100 equals its argument to 1e-27 relative, so the network is
    affine.  The SDF row is a constant row scaled so the slope is the unit
    normal, and the bias sets the offset; magnitudes stay O(1) so single
    precision evaluates it to ~1e-6.  Folded into an N^3 grid with no noise.
    Color MLP in the positive ReLU regime (bc1 = 10, |Wc1| <= 0.05).
    The float32 rounding of the stored parameters moves the plane by ~1e-7;
    exact checks use the affine map of the stored parameters.
    """
    rng = _rng(seed)
    n = np.asarray(normal, np.float64)
    n = n / np.linalg.norm(n)
    alpha = rng.uniform(0.3, 0.5, size=H)
    W1b = np.zeros((H, SDF_IN))
    W1b[:, 0:3] = alpha[:, None] * n[None, :]
    b1b = np.full(H, 1.5)
    W2 = rng.uniform(0.0, 2.0 / H, size=(H, H))
    b2 = np.full(H, 0.5)
    W3 = np.zeros((1 + FEAT_DIM, H))
    W3[1:] = rng.normal(0.0, math.sqrt(1.0 / H), size=(FEAT_DIM, H))
    W3[0] = 1.0 / np.sum(W2 @ alpha)
    b3 = np.zeros(1 + FEAT_DIM)
    b3[0] = -offset - W3[0] @ (W2 @ b1b + b2)
    Wc1 = rng.uniform(-0.05, 0.05, size=(COL_HIDDEN, COL_IN))
    bc1 = np.full(COL_HIDDEN, 10.0)
    Wc2 = rng.normal(0.0, 0.05, size=(3, COL_HIDDEN))
    bc2 = rng.normal(0.0, 0.5, size=3)

    centers = cell_centers(N)
    h = 1.0 / N
    blocks = []
    for c in centers:
        W1 = W1b.copy()
        W1[:, 0:3] *= h
        b1 = b1b + W1b[:, 0:3] @ c
        blocks.append(pack_sdf(W1, b1, W2, b2, W3, b3))
    sdf = np.stack(blocks)
    col = np.tile(pack_col(Wc1, bc1, Wc2, bc2)[None, :], (N ** 3, 1))
    return Scene(N=N, H=H, sdf=sdf, col=col, name=f"plane N={N} H={H}")


def plane_affine_map(scene: Scene, cell: int):
    """(g, c0) with f(x) = g.x + c0 in world coordinates for one cell of a
    plane scene, computed in float64 from the stored float32 parameters
    (valid where every pre-activation is in softplus's linear regime)."""
    N = scene.N
    w = {k: v.astype(np.float64) for k, v in unpack_sdf(scene.sdf[cell], scene.H).items()}
    c = cell_centers(N)[cell]
    h = 1.0 / N
    row = w["W3"][0] @ w["W2"]                    # d f / d a1
    g = (row @ w["W1"][:, 0:3]) / h               # world gradient
    c0 = row @ (w["b1"] - w["W1"][:, 0:3] @ (c / h)) + w["W3"][0] @ w["b2"] + w["b3"][0]
    return g, c0


def constant_color_plane_scene(N: int, H: int, normal, offset: float,
                               albedo, seed: int) -> Scene:
    """Plane scene whose color MLP outputs a constant albedo: Wc = 0 and
    bc2 = logit(albedo), so sigmoid(bc2) = albedo."""
    sc = plane_scene(N, H, normal, offset, seed)
    a = np.asarray(albedo, np.float64)
    zero_w = np.zeros((COL_HIDDEN, COL_IN))
    blk = pack_col(zero_w, np.zeros(COL_HIDDEN), np.zeros((3, COL_HIDDEN)),
                   np.log(a / (1.0 - a)))
    sc.col = np.tile(blk[None, :], (N ** 3, 1))
    return sc


def lipschitz_safe(scene: Scene, factor: float) -> Scene:
    """Copy of `scene` with the SDF row (W3[0], b3[0]) scaled by `factor`."""
    o = sdf_offsets(scene.H)
    sdf = scene.sdf.copy()
    p = o["W3"][0]
    sdf[:, p:p + scene.H] *= np.float32(factor)
    sdf[:, o["b3"][0]] *= np.float32(factor)
    return Scene(N=scene.N, H=scene.H, sdf=sdf, col=scene.col.copy(),
                 name=scene.name + f" x{factor:g}")


# ----------------------------------------------------------------------------
# Cameras
# ----------------------------------------------------------------------------
ORBIT_DISTANCE = 2.5


def default_tan_half_diag(distance: float = ORBIT_DISTANCE) -> float:
    """Pinhole field of view whose half-diagonal angle is tangent to the
    bounding box's inscribed unit sphere: every primary ray then meets the box
    (the paper's performance setting has every ray intersect the bounding
    volume, Sec. 4.2)."""
    return 1.0 / math.sqrt(distance * distance - 1.0)


@dataclasses.dataclass
class View:
    eye: tuple
    look_at: tuple = (0.0, 0.0, 0.0)
    up: tuple = (0.0, 1.0, 0.0)
    tan_half_diag: float = 0.0   # 0 => 1/sqrt(|eye-look_at|^2 - 1)


def front_view(distance: float = ORBIT_DISTANCE) -> View:
    return View(eye=(0.0, 0.0, distance))


def orbit_views(count: int, seed: int, distance: float = ORBIT_DISTANCE) -> list:
    """`count` seeded orbit views: azimuth U[0, 2pi), elevation U[-45, 45]
    degrees, looking at the origin with +y up."""
    rng = _rng(seed)
    views = []
    for _ in range(count):
        az = rng.uniform(0.0, 2.0 * math.pi)
        el = rng.uniform(-math.pi / 4, math.pi / 4)
        eye = (distance * math.cos(el) * math.sin(az), distance * math.sin(el),
               distance * math.cos(el) * math.cos(az))
        views.append(View(eye=tuple(float(v) for v in eye)))
    return views


def sample_pixels(width: int, height: int, count: int, seed: int) -> np.ndarray:
    """Seeded sample of distinct pixel indices (row-major), sorted, int64."""
    rng = _rng(seed)
    n = width * height
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


# ----------------------------------------------------------------------------
# Configurations of the workloads (sizes only; seeds per scene)
# ----------------------------------------------------------------------------
CONFIGS = {
    # 4^3 grid, H=32, one 64x64 front view, 64 steps, eps 1e-4, FP32
    "c1": dict(N=4, H=32, radius=0.5, sigma=0.01, seed=1000, width=64, height=64,
               views=1, max_steps=64, eps=1e-4, precision="fp32"),
    # 16^3 grid, H=32, 8 orbit views of 800x800, 128 steps, FP32
    "c2": dict(N=16, H=32, radius=0.6, sigma=0.02, seed=2000, width=800, height=800,
               views=8, max_steps=128, eps=1e-4, precision="fp32"),
    # 16^3 grid, H=64, 8 orbit views of 1920x1080, 128 steps, BF16 vs FP32
    "c3": dict(N=16, H=64, radius=0.6, sigma=0.02, seed=3000, width=1920, height=1080,
               views=8, max_steps=128, eps=1e-4, precision="bf16"),
    # 32^3 grid, H=64, 1920x1080, 4 spp, 3 bounces, FP8 vs BF16
    "c5": dict(N=32, H=64, radius=0.6, sigma=0.02, seed=5000, width=1920, height=1080,
               views=1, max_steps=256, eps=1e-4, precision="fp8", spp=4, bounces=3,
               env_seed=5005, path_seed=5006),
}


def env_map(width: int = 512, height: int = 256, seed: int = 5005) -> np.ndarray:
    """Seeded procedural HDR environment, float32 [height][width][3] in the
    equirectangular layout of the renderer (row 0 looks up +y; column u
    looks along azimuth 2 pi (u - 1/2) from -z towards +x): a sky gradient
    from horizon to zenith, a darker ground, and three Gaussian lobes of
    random direction, width and intensity."""
    rng = np.random.default_rng(seed)
    v = (np.arange(height) + 0.5) / height
    u = (np.arange(width) + 0.5) / width
    th = np.pi * v[:, None]
    ph = 2.0 * np.pi * (u[None, :] - 0.5)
    d = np.stack([np.sin(th) * np.sin(ph), np.cos(th) * np.ones_like(ph), -np.sin(th) * np.cos(ph)], -1)
    up = np.clip(d[..., 1], 0.0, 1.0)[..., None]
    zenith = np.array([0.35, 0.55, 1.2])
    horizon = np.array([1.3, 1.15, 1.0])
    ground = np.array([0.25, 0.22, 0.2])
    img = np.where(d[..., 1:2] >= 0, horizon + (zenith - horizon) * np.sqrt(up), ground)
    for _ in range(3):
        c = rng.normal(size=3)
        c[1] = abs(c[1])
        c /= np.linalg.norm(c)
        k = rng.uniform(20.0, 200.0)
        inten = rng.uniform(2.0, 10.0) * rng.uniform(0.6, 1.0, 3)
        img = img + inten * np.exp(k * (d @ c - 1.0))[..., None]
    return img.astype(np.float32)


def config_scene(name: str) -> Scene:
    c = CONFIGS[name]
    return sphere_scene(c["N"], c["H"], c["radius"], c["sigma"], c["seed"],
                        name=f"{name}: N={c['N']} H={c['H']}")


def config_views(name: str) -> list:
    c = CONFIGS[name]
    if c["views"] == 1 and name == "c1":
        return [front_view()]
    return orbit_views(c["views"], c["seed"] + 500)
