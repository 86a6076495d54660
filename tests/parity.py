"""Comparison helpers shared by the GPU parity tests, smoke() and the bench.

Parity of a float32 render against the FP64 oracle, in four parts:
  1. hit masks agree on >= 99.9% of pixels, or -- when lower -- as often as
     the oracle agrees with itself when its inputs move by float32-sized
     amounts (weights x (1 + 1e-6 xi), eye + 1e-6 xi);
  2. on pixels whose oracle result is well conditioned (stays within half
     the tolerance under those perturbations), depth <= 1e-4, normal <= 0.1
     degree and RGB <= 1e-3;
  3. every GPU hit is valid at its own point: the FP64 SDF at the GPU's
     march stop is below eps, and where the FP64 normal there is well
     conditioned, the GPU normal and color equal the FP64 ones at that point;
  4. replay: the oracle refines and shades from the GPU's march state (cell,
     t_march, t_entry); where that replay is well conditioned, the GPU's
     depth, normal and color match it.
Parts 2-4 allow at most 0.1% of their cases outside the tolerance.  The
synthetic scenes' noisy SDFs are far from 1-Lipschitz (gradient norms of
10-50), so sphere tracing and Newton steps there can take different paths
under float32 rounding; such cases are counted and reported, not asserted.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from oracle import oracle as O
from paper_2206_10885_amd import synth

TOL_DEPTH = 1e-4      # scene units
TOL_NORMAL_DEG = 0.1
TOL_RGB = 1e-3
TOL_HIT_MASK = 0.999


def angle_deg(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Angle between vectors in degrees, in float64 from atan2(|a x b|, a.b),
    which stays accurate for small angles (arccos of a float32 cosine cannot
    resolve angles below about 0.02 degrees)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    cr = np.linalg.norm(np.cross(a, b), axis=-1)
    return np.degrees(np.arctan2(cr, np.sum(a * b, axis=-1)))


def perturbed(scene: synth.Scene, rel: float, seed: int) -> synth.Scene:
    rng = np.random.default_rng(seed)
    sdf = (scene.sdf.astype(np.float64) * (1.0 + rel * rng.standard_normal(scene.sdf.shape))).astype(np.float32)
    return synth.Scene(N=scene.N, H=scene.H, sdf=sdf, col=scene.col, name=scene.name + " perturbed")


def jittered(view: synth.View, amount: float, seed: int) -> synth.View:
    rng = np.random.default_rng(seed)
    e = np.asarray(view.eye, np.float64) + amount * rng.standard_normal(3)
    return synth.View(eye=tuple(e), look_at=view.look_at, up=view.up, tan_half_diag=view.tan_half_diag)


def oracle_render(scene, view, W, H, S, eps, pixels=None, unclamped: bool = False) -> dict:
    return O.OracleScene.from_scene(scene).render(view, W, H, S, eps, pixels=pixels, unclamped=unclamped)


def stable_mask(scene, view, W, H, S, eps, ref: dict, pixels=None, trials: int = 6, unclamped: bool = False):
    """Pixels whose oracle result stays within half the tolerance under
    float32-sized perturbations of the inputs (weights x (1 + 1e-6 xi), eye
    + 1e-6 xi), and the oracle's own worst hit-mask agreement across them."""
    ok = np.ones(len(ref["hit"]), bool)
    self_agree = 1.0
    for k in range(trials):
        r = oracle_render(perturbed(scene, 1e-6, 100 + k), jittered(view, 1e-6, 200 + k), W, H, S, eps,
                          pixels, unclamped)
        same_hit = r["hit"] == ref["hit"]
        self_agree = min(self_agree, float(np.mean(same_hit)))
        both = (r["hit"] == 1) & (ref["hit"] == 1)
        dd = np.abs(r["depth"] - ref["depth"])
        an = angle_deg(r["normal"], ref["normal"])
        dc = np.abs(r["rgb"] - ref["rgb"]).max(axis=1)
        ok &= same_hit
        ok &= ~both | ((dd <= TOL_DEPTH / 2) & (an <= TOL_NORMAL_DEG / 2))
        ok &= dc <= TOL_RGB / 2
    return ok, self_agree


@dataclasses.dataclass
class Report:
    n: int                      # pixels compared
    hit_agree: float            # fraction with equal hit flags
    oracle_self_agree: float    # oracle vs itself under float32-sized input perturbation
    stable_frac: float          # fraction well conditioned in the oracle
    stable_checked: int         # well-conditioned pixels with equal hit flags
    stable_bad: int             # ... of which outside the tolerance
    depth_max_stable: float
    normal_max_stable: float
    rgb_max_stable: float
    point_n: int                # GPU hits (well conditioned there) checked at their own point
    point_bad: int              # normal or color differs from FP64 at that point
    point_normal_max: float
    point_rgb_max: float
    fstop_max: float            # max over GPU hits of f_FP64(march stop) - eps
    replay_n: int               # GPU hits whose FP64 replay is well conditioned
    replay_bad: int
    replay_depth_max: float
    replay_normal_max: float
    replay_rgb_max: float
    all_depth_p99: float        # all pixels where both hit (reported only)
    all_normal_p99: float
    # every pixel where both hit (depth, normal in degrees) or whose masks
    # agree (rgb): p50 / p99 / max, reported
    err_all: dict = dataclasses.field(default_factory=dict)
    # per GPU hit: the march's stop point (world) and its cell, for checks of
    # low-precision marches in their own arithmetic
    stop_pts: np.ndarray = None
    stop_cells: np.ndarray = None
    fstop: np.ndarray = None    # f_FP64(stop) - eps per GPU hit

    def as_dict(self):
        skip = ("stop_pts", "stop_cells", "fstop")
        return {f.name: (round(getattr(self, f.name), 9) if isinstance(getattr(self, f.name), float)
                         else getattr(self, f.name)) for f in dataclasses.fields(self) if f.name not in skip}

    def ok(self, frac: float = 1e-3) -> bool:
        """The parity bar: hit masks agree on >= 99.9% of pixels (or as often as
        the oracle agrees with itself under float32-sized perturbations, if
        that is lower); on
        well-conditioned pixels and replays at most `frac` outside the
        tolerance; every GPU hit valid at its own point."""
        return (self.hit_agree >= min(TOL_HIT_MASK, self.oracle_self_agree)
                and self.stable_bad <= frac * max(1, self.stable_checked)
                and self.replay_bad <= frac * max(1, self.replay_n)
                and self.point_bad <= frac * max(1, self.point_n)
                and self.fstop_max < 1e-5)


def gpu_arrays(out: dict, pixels=None) -> dict:
    """Flattens a GPU frame (torch tensors) to numpy, optionally at pixels."""
    g = {k: v.detach().cpu().numpy() for k, v in out.items() if k != "stats"}
    res = dict(rgb=g["rgb"].reshape(-1, 3).astype(np.float64),
               depth=g["depth"].reshape(-1).astype(np.float64),
               normal=g["normal"].reshape(-1, 3).astype(np.float64),
               hit=g["hit"].reshape(-1),
               steps=g["steps"].reshape(-1).astype(np.int32))
    if "trace" in g:
        tr = g["trace"].reshape(-1, 4)
        res["t_march"] = tr[:, 0].copy().view(np.float32).astype(np.float64)
        res["t_entry"] = tr[:, 1].copy().view(np.float32).astype(np.float64)
        res["cell"] = tr[:, 2].astype(np.int64)
        res["status"] = tr[:, 3].astype(np.int32)
    if pixels is not None:
        res = {k: v[pixels] for k, v in res.items()}
    return res


def _trace_struct(cell_idx, t, t_entry):
    tr = O._Trace()
    tr.status = O.HIT
    tr.steps = 1
    tr.cell = (O.C.c_int32 * 3)(*cell_idx)
    tr.t = float(t)
    tr.t_entry = float(t_entry)
    tr.fmin = 0.0
    return dict(_raw=tr)


def compare(scene, view, W, H, S, eps, gpu: dict, pixels=None, unclamped: bool = False,
            trials: int = 6) -> Report:
    """Full comparison of a GPU frame (numpy dict from gpu_arrays, restricted
    to `pixels` if given) against the oracle (in the same step rule);
    `trials` perturbed oracle runs decide which pixels are well conditioned."""
    ref = oracle_render(scene, view, W, H, S, eps, pixels, unclamped)
    n = len(ref["hit"])
    hit_agree = float(np.mean(ref["hit"] == gpu["hit"]))
    stable, self_agree = stable_mask(scene, view, W, H, S, eps, ref, pixels, trials=trials, unclamped=unclamped)
    both = (ref["hit"] == 1) & (gpu["hit"] == 1)
    dd = np.abs(ref["depth"] - gpu["depth"])
    an = angle_deg(ref["normal"], gpu["normal"])
    dc = np.abs(ref["rgb"] - gpu["rgb"]).max(axis=1)
    chk = stable & (ref["hit"] == gpu["hit"])
    bad = chk & ((both & ((dd > TOL_DEPTH) | (an > TOL_NORMAL_DEG))) | (dc > TOL_RGB))
    bad |= stable & (ref["hit"] != gpu["hit"])
    sb = stable & both

    os_ = O.OracleScene.from_scene(scene)
    pert = [O.OracleScene.from_scene(perturbed(scene, 1e-6, 300 + k)) for k in range(6)]
    rng = np.random.default_rng(400)
    pix = np.arange(W * H) if pixels is None else np.asarray(pixels)
    N = scene.N
    centers = synth.cell_centers(N)
    half = 1.0 / N
    pb = rb = rn_ = pn_ = 0
    pn_max = pc_max = fstop = 0.0
    rd = rnm = rc = 0.0
    hits = np.nonzero(gpu["hit"] == 1)[0]
    stop_pts = np.zeros((len(hits), 3))
    stop_cells = np.zeros(len(hits), np.int64)
    fstops = np.zeros(len(hits))
    for hi_, q in enumerate(hits):
        p = int(pix[q])
        o, d = O.camera_ray(view, W, H, p // W, p % W)
        cell = int(gpu["cell"][q])
        idx = (cell % N, (cell // N) % N, cell // (N * N))
        c = centers[cell]
        # (1) validity at the GPU's own final point and march stop
        xg = o + gpu["depth"][q] * d
        y, gl = os_.sdf_eval(cell, (xg - c) / half, grad=True)
        nrm = gl / np.linalg.norm(gl)
        rgb = os_.color_eval(cell, (xg - c) / half, d, nrm, y[1:])
        # is the FP64 normal at this point well conditioned?
        point_stable = True
        for ps in pert:
            xj = xg + 1e-7 * rng.standard_normal(3)
            _, gj = ps.sdf_eval(cell, (xj - c) / half, grad=True)
            if angle_deg(gj, gl) > TOL_NORMAL_DEG / 2:
                point_stable = False
        if point_stable:
            pn_ += 1
            e_pn = float(angle_deg(nrm, gpu["normal"][q]))
            e_pc = float(np.abs(rgb - gpu["rgb"][q]).max())
            pn_max, pc_max = max(pn_max, e_pn), max(pc_max, e_pc)
            if e_pn > TOL_NORMAL_DEG or e_pc > TOL_RGB:
                pb += 1
        xs = o + gpu["t_march"][q] * d
        fstops[hi_] = os_.sdf_eval(cell, (xs - c) / half)[0] - eps
        fstop = max(fstop, fstops[hi_])
        stop_pts[hi_], stop_cells[hi_] = xs, cell
        # (2) FP64 replay of refinement and shading from the GPU's march state
        tr = _trace_struct(idx, gpu["t_march"][q], gpu["t_entry"][q])
        sh = os_.shade(o, d, tr)
        stable_r = True
        for k, ps in enumerate(pert):
            dj = d + 1e-7 * rng.standard_normal(3)
            dj /= np.linalg.norm(dj)
            trk = _trace_struct(idx, gpu["t_march"][q] * (1 + 1e-6 * rng.standard_normal()),
                                gpu["t_entry"][q])
            s2 = ps.shade(o, dj, trk)
            if (abs(s2["depth"] - sh["depth"]) > TOL_DEPTH / 2
                    or angle_deg(s2["normal"], sh["normal"]) > TOL_NORMAL_DEG / 2
                    or np.abs(s2["rgb"] - sh["rgb"]).max() > TOL_RGB / 2):
                stable_r = False
                break
        if not stable_r:
            continue
        rn_ += 1
        e_d = abs(sh["depth"] - gpu["depth"][q])
        e_n = float(angle_deg(sh["normal"], gpu["normal"][q]))
        e_c = float(np.abs(sh["rgb"] - gpu["rgb"][q]).max())
        rd, rnm, rc = max(rd, e_d), max(rnm, e_n), max(rc, e_c)
        if e_d > TOL_DEPTH or e_n > TOL_NORMAL_DEG or e_c > TOL_RGB:
            rb += 1
    return Report(
        n=n, hit_agree=hit_agree, oracle_self_agree=self_agree, stable_frac=float(stable.mean()), stable_checked=int(chk.sum()),
        stable_bad=int(bad.sum()),
        depth_max_stable=float(dd[sb].max()) if sb.any() else 0.0,
        normal_max_stable=float(an[sb].max()) if sb.any() else 0.0,
        rgb_max_stable=float(dc[chk].max()) if chk.any() else 0.0,
        point_n=pn_, point_bad=pb, point_normal_max=pn_max, point_rgb_max=pc_max,
        fstop_max=float(fstop),
        replay_n=rn_, replay_bad=rb, replay_depth_max=float(rd), replay_normal_max=rnm,
        replay_rgb_max=rc,
        all_depth_p99=float(np.percentile(dd[both], 99)) if both.any() else 0.0,
        all_normal_p99=float(np.percentile(an[both], 99)) if both.any() else 0.0,
        err_all=dict(depth=stats(dd[both]), normal_deg=stats(an[both]), rgb=stats(dc[ref["hit"] == gpu["hit"]])),
        stop_pts=stop_pts, stop_cells=stop_cells, fstop=fstops)


def stats(x) -> dict:
    """p50 / p99 / max of a sample (empty: zeros)."""
    x = np.asarray(x, np.float64).ravel()
    if x.size == 0:
        return dict(n=0, p50=0.0, p99=0.0, max=0.0)
    return dict(n=int(x.size), p50=float(np.median(x)), p99=float(np.percentile(x, 99)), max=float(x.max()))


def record(name: str, data: dict) -> None:
    """Appends one JSON line {name: data} to the file named by KN_REPORT (if
    set): the GPU tests' accuracy figures, kept beside the run's logs."""
    import json
    import os
    path = os.environ.get("KN_REPORT")
    if not path:
        return
    with open(path, "a") as fh:
        fh.write(json.dumps({"case": name, **data}) + "\n")
