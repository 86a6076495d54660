"""CPU emulations of the low-precision march MLP, and a rigorous per-point
bound on what the rounding can do to the SDF value (test infrastructure only).

The paper fixes no precision for the renderer (its kernels run in float32).
The low-precision variants are defined as readings of eq. 3 (Sec. 3.1):

  sdf_bf16 (the plain reading): every weight of the three layers (W1, W2 and
      the SDF row of W3) and every layer input (the encoding, a1, a2) rounded
      to bfloat16 (round to nearest even); products accumulated in float32;
      biases and softplus in float32.  This is written from the definition
      only, not from the GPU kernel's arithmetic.
  sdf_bf16_kernel_form: the same network in the algebra the bf16 march kernel
      evaluates: hidden layers written for u' = k u (k = beta / ln 2), so that
      2k softplus(u) = u' + |u'| + 2 log2(1 + 2^-|u'|); the rounded weights
      are k W1 and W2 / 2, the rounded layer inputs the encoding, 2k a1 and
      2k a2; the SDF row W3 / (2k) as a pair hi = bf16(w), lo = bf16(w - hi).
      Exact arithmetic gives eq. 3 again; the roundings differ from the plain
      reading's because k is not a power of two.
  sdf_fp8: W1 and W2 and their inputs (the encoding, a1) in OCP e4m3 with
      power-of-two per-(cell, layer) scales; a2 in bfloat16 and the SDF row
      as a hi + lo bfloat16 pair.

sdf_fp64 is eq. 3 in float64 (numpy), with its intermediate activations, and
rounding_bound() a first-order worst-case bound, per point, on
|d_lowp - d_fp64| for any evaluation that rounds weights with relative error
<= u_w, layer inputs with relative error <= u_in (plus an absolute term for
e4m3 subnormals), accumulates in float32 and evaluates the encoding and the
softplus in float32: each layer's error is the propagation of its input error
through |W| plus the new rounding terms, and softplus is 1-Lipschitz.  It
covers the plain reading and the kernel form alike, so the GPU kernels can be
checked against the FP64 oracle point by point with no statistics.

Pins (tests/test_quant_pins.py): the rounding functions against exact
e4m3 / bfloat16 values; with rounding switched off the emulations equal the
FP64 oracle to float32 precision; sdf_fp64 equals the C oracle; every
emulation stays inside rounding_bound() at every point, and the bound is
within a few orders of magnitude of the errors it covers.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def _bf16(x: torch.Tensor) -> torch.Tensor:
    return x.to(torch.bfloat16).to(torch.float32)


def _encode(xl: torch.Tensor, L: int) -> torch.Tensor:
    parts = [xl]
    for a in range(3):
        for k in range(L):
            w = (2.0 ** k) * math.pi * xl[:, a:a + 1].double()
            parts += [torch.sin(w).float(), torch.cos(w).float()]
    return torch.cat(parts, 1)


def _softplus(u: torch.Tensor, beta: float) -> torch.Tensor:
    return torch.clamp(u, min=0) + torch.log1p(torch.exp(-beta * u.abs())) / beta


E4M3_MAX = 448.0


def e4m3(x: torch.Tensor) -> torch.Tensor:
    """OCP fp8 e4m3fn rounding: saturate to [-448, 448], then nearest, ties
    to even (torch's float8_e4m3fn cast), back to float32."""
    return torch.clamp(x.float(), -E4M3_MAX, E4M3_MAX).to(torch.float8_e4m3fn).to(torch.float32)


def pow2_scale(bound: float) -> float:
    """Smallest power of two s with bound / s <= 448 (1 for bound <= 0)."""
    if not bound > 0 or not math.isfinite(bound):
        return 1.0
    e = math.ceil(math.log2(bound / E4M3_MAX))
    while bound / 2.0 ** (e - 1) <= E4M3_MAX:
        e -= 1
    while bound / 2.0 ** e > E4M3_MAX:
        e += 1
    return 2.0 ** e


def _softplus64(u: float, beta: float) -> float:
    return max(u, 0.0) + math.log1p(math.exp(-beta * abs(u))) / beta


def fp8_scales(W1: np.ndarray, b1: np.ndarray, W2: np.ndarray, beta: float):
    """Per-(cell, layer) power-of-two scales of the fp8 march MLP: weights by
    their largest magnitude; the layer-2 input by the bound
    softplus(sum_k |W1[j,k]| + b1[j]) on a1 for encodings with |e_k| <= 1
    (times 1.01 for points on the cell faces)."""
    W1 = np.asarray(W1, np.float64)
    s1 = pow2_scale(float(np.abs(W1).max()))
    s2 = pow2_scale(float(np.abs(np.asarray(W2, np.float64)).max()))
    bound = max(_softplus64(float(r) + float(b), beta) for r, b in zip(np.abs(W1).sum(1), b1))
    sa = pow2_scale(bound * 1.01)
    return s1, s2, sa


def _cell_blocks(scene, pts, cells=None):
    """Per cell: the mask of its points, their local coordinates (float32)
    and the cell's SDF weights.  Points belong to the cell containing them
    (clamped to the grid), or to the given cells."""
    N, H = scene.N, scene.H
    cell_np, xl_np = point_cells(N, pts, cells)
    cell = torch.tensor(cell_np)
    xl = torch.tensor(xl_np).float()
    din = 39
    for c in torch.unique(cell).tolist():
        m = cell == c
        blk = torch.tensor(scene.sdf[c])
        p = 0
        W1 = blk[p:p + din * H].view(H, din); p += din * H
        b1 = blk[p:p + H]; p += H
        W2 = blk[p:p + H * H].view(H, H); p += H * H
        b2 = blk[p:p + H]; p += H
        W3 = blk[p:p + 16 * H].view(16, H); p += 16 * H
        b3 = blk[p:p + 16]
        yield m, xl[m], (W1, b1, W2, b2, W3, b3)


def sdf_fp8(scene, pts: np.ndarray, quantize: bool = True, cells=None) -> np.ndarray:
    """SDF value of the cell containing each world point, fp8 e4m3 variant:
    the encoding (scale 1) and W1 / s1 rounded to e4m3; u1 = s1 (W1q eq) + b1;
    a1 = softplus(u1) scaled by 1 / sa and rounded; u2 = s2 sa (W2q a1q) + b2;
    a2 = softplus(u2) in bfloat16; the output row W3 as a hi + lo bfloat16
    pair.  quantize=False skips every rounding (float32 throughout)."""
    q = e4m3 if quantize else (lambda t: t.float())
    qb = _bf16 if quantize else (lambda t: t.float())
    out = torch.zeros(len(pts), dtype=torch.float32)
    for m, xl, (W1, b1, W2, b2, W3, b3) in _cell_blocks(scene, pts, cells):
        s1, s2, sa = fp8_scales(W1.numpy(), b1.numpy(), W2.numpy(), scene.beta)
        if not quantize:
            s1 = s2 = sa = 1.0
        e = q(_encode(xl, 6))
        u1 = (e @ q(W1 / s1).T) * s1 + b1
        a1 = _softplus(u1, scene.beta)
        u2 = (q(a1 / sa) @ q(W2 / s2).T) * (s2 * sa) + b2
        a2 = _softplus(u2, scene.beta)
        hi, lo = _split(W3[0], qb)
        out[m] = (qb(a2) @ hi + qb(a2) @ lo) + b3[0]
    return out.numpy()


def _split(w: torch.Tensor, qb) -> tuple:
    """A float32 row as hi = bf16(w) and lo = bf16(w - hi) (with qb the
    identity: w and 0)."""
    hi = qb(w.float())
    return hi, qb(w.float() - hi)


def _softplus_2k(up: torch.Tensor) -> torch.Tensor:
    """2k softplus(u) from u' = k u (k = beta / ln 2)."""
    return up + up.abs() + 2.0 * torch.log2(1.0 + torch.exp2(-up.abs()))


def sdf_bf16_kernel_form(scene, pts: np.ndarray, quantize: bool = True, cells=None) -> np.ndarray:
    """SDF value of the cell containing each world point (points clamped to
    the grid), bfloat16 variant in the bf16 march kernel's algebra (module
    docstring); quantize=False skips every rounding.  The scaled weights are
    formed in float64 and rounded to float32 first."""
    qb = _bf16 if quantize else (lambda t: t.float())
    k = scene.beta / math.log(2.0)
    out = torch.zeros(len(pts), dtype=torch.float32)
    for m, xl, (W1, b1, W2, b2, W3, b3) in _cell_blocks(scene, pts, cells):
        e = qb(_encode(xl, 6))
        a1 = _softplus_2k(e @ qb((k * W1.double()).float()).T + (k * b1.double()).float())
        a2 = _softplus_2k(qb(a1) @ qb(0.5 * W2).T + (k * b2.double()).float())
        hi, lo = _split((W3[0].double() * (0.5 / k)).float(), qb)
        out[m] = (qb(a2) @ hi + qb(a2) @ lo) + b3[0]
    return out.numpy()


def sdf_bf16(scene, pts: np.ndarray, quantize: bool = True, cells=None) -> np.ndarray:
    """SDF value of the cell containing each world point (points clamped to
    the grid), plain bfloat16 reading: bf16(W1), bf16(W2), bf16(W3[0]) and
    bf16 of the encoding, a1 and a2; float32 sums, biases and softplus."""
    qb = _bf16 if quantize else (lambda t: t.float())
    out = torch.zeros(len(pts), dtype=torch.float32)
    for m, xl, (W1, b1, W2, b2, W3, b3) in _cell_blocks(scene, pts, cells):
        e = qb(_encode(xl, 6))
        a1 = _softplus(e @ qb(W1).T + b1, scene.beta)
        a2 = _softplus(qb(a1) @ qb(W2).T + b2, scene.beta)
        out[m] = qb(a2) @ qb(W3[0]) + b3[0]
    return out.numpy()


# ---------------------------------------------------------------------------
# FP64 forward pass and the per-point rounding bound
# ---------------------------------------------------------------------------
def point_cells(N: int, pts: np.ndarray, cells=None):
    """Cell of each world point (the one containing it, clamped to the grid,
    box [-1,1]^3; or the given cells) and the cell-local coordinates
    x_l = (x - c) / h."""
    x = np.asarray(pts, np.float64)
    if cells is None:
        idx = np.clip(np.floor((x + 1.0) * N / 2.0).astype(np.int64), 0, N - 1)
        cell = idx[:, 0] + N * (idx[:, 1] + N * idx[:, 2])
    else:
        cell = np.asarray(cells, np.int64)
        idx = np.stack([cell % N, (cell // N) % N, cell // (N * N)], 1)
    centers = -1.0 + (idx + 0.5) * (2.0 / N)
    return cell, (x - centers) * N


def encode64(xl: np.ndarray, L: int = 6) -> np.ndarray:
    """gamma_L of each row (eq. 1-2): raw coordinates, then per axis
    sin(2^k pi x), cos(2^k pi x) for k = 0..L-1."""
    parts = [xl]
    for a in range(3):
        for k in range(L):
            w = (2.0 ** k) * math.pi * xl[:, a:a + 1]
            parts += [np.sin(w), np.cos(w)]
    return np.concatenate(parts, 1)


def softplus64(u: np.ndarray, beta: float) -> np.ndarray:
    return np.maximum(u, 0.0) + np.log1p(np.exp(-beta * np.abs(u))) / beta


def sdf_fp64(scene, cells: np.ndarray, xl: np.ndarray) -> dict:
    """Eq. 3 in float64 at local points xl of the given cells: the encoding
    e, pre-activations u1, u2, activations a1, a2 and d (row 0 of W3)."""
    H = scene.H
    cells = np.asarray(cells, np.int64)
    xl = np.asarray(xl, np.float64)
    n = len(cells)
    e = encode64(xl)
    out = dict(e=e, u1=np.zeros((n, H)), a1=np.zeros((n, H)), u2=np.zeros((n, H)), a2=np.zeros((n, H)),
               d=np.zeros(n), cells=cells)
    for c in np.unique(cells):
        m = cells == c
        w = _unpack64(scene, int(c))
        u1 = e[m] @ w["W1"].T + w["b1"]
        a1 = softplus64(u1, scene.beta)
        u2 = a1 @ w["W2"].T + w["b2"]
        a2 = softplus64(u2, scene.beta)
        out["u1"][m], out["a1"][m], out["u2"][m], out["a2"][m] = u1, a1, u2, a2
        out["d"][m] = a2 @ w["W3"][0] + w["b3"][0]
    return out


def _unpack64(scene, c: int) -> dict:
    H = scene.H
    blk = np.asarray(scene.sdf[c], np.float64)
    p = 0
    w = {}
    for name, shape in (("W1", (H, 39)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (16, H)),
                        ("b3", (16,))):
        n = int(np.prod(shape))
        w[name] = blk[p:p + n].reshape(shape)
        p += n
    return w


# unit roundoffs: bfloat16 (8 significant bits), e4m3 (4 significant bits),
# float32; e4m3 subnormals are multiples of 2^-9 (absolute error <= 2^-10
# times the scale)
U_BF16 = 2.0 ** -9
U_E4M3 = 2.0 ** -4
U_F32 = 2.0 ** -24
E4M3_SUB_HALF = 2.0 ** -10
ENC_ABS = 4e-6          # float32 encoding on the GPU's sin/cos units, absolute
SP_REL, SP_ABS = 4e-7, 1e-7   # float32 softplus: relative to |u|, absolute (in units of sp)


def rounding_bound(scene, f: dict, mode: str) -> np.ndarray:
    """First-order worst-case bound on |d_lowp - d| at each point of `f`
    (from sdf_fp64) for mode "bf16" (weights and layer inputs to bfloat16,
    the plain reading and the kernel form) or "fp8" (W1, W2 and their inputs
    to e4m3 with power-of-two scales, a2 and the SDF row to bfloat16).  Each
    layer: |du| <= sum_k |W| (dx_k + u_in (|x_k| + dx_k)) + u_w |W| (|x_k| +
    dx_k') + float32 accumulation; softplus is 1-Lipschitz plus its float32
    evaluation error."""
    cells = f["cells"]
    bound = np.zeros(len(cells))
    for c in np.unique(cells):
        m = cells == c
        w = _unpack64(scene, int(c))
        aW1, aW2, aw3 = np.abs(w["W1"]), np.abs(w["W2"]), np.abs(w["W3"][0])
        if mode == "bf16":
            uw1 = uw2 = U_BF16
            ui1 = ui2 = U_BF16
            ab1 = ab2 = 0.0
        elif mode == "fp8":
            s1, s2, sa = fp8_scales(w["W1"].astype(np.float32), w["b1"].astype(np.float32),
                                    w["W2"].astype(np.float32), scene.beta)
            uw1 = uw2 = U_E4M3
            ui1 = ui2 = U_E4M3
            ab1 = E4M3_SUB_HALF          # encoding scale 1
            ab2 = E4M3_SUB_HALF * sa     # a1 scale
            # weight subnormals: absolute 2^-10 s per weight
            aW1 = aW1 + E4M3_SUB_HALF * s1 / U_E4M3
            aW2 = aW2 + E4M3_SUB_HALF * s2 / U_E4M3
        else:
            raise ValueError(mode)
        e = np.abs(f["e"][m])
        de = ENC_ABS + ui1 * (e + ENC_ABS) + ab1
        x1 = e + de
        du1 = de @ np.abs(w["W1"]).T + uw1 * (x1 @ aW1.T) + 64 * U_F32 * (x1 @ aW1.T)
        a1 = np.abs(f["a1"][m])
        da1 = du1 + SP_REL * np.abs(f["u1"][m]) + SP_ABS
        dx2 = da1 + ui2 * (a1 + da1) + ab2
        x2 = a1 + dx2
        du2 = dx2 @ np.abs(w["W2"]).T + uw2 * (x2 @ aW2.T) + 64 * U_F32 * (x2 @ aW2.T)
        a2 = np.abs(f["a2"][m])
        da2 = du2 + SP_REL * np.abs(f["u2"][m]) + SP_ABS
        dx3 = da2 + U_BF16 * (a2 + da2)
        x3 = a2 + dx3
        bound[m] = dx3 @ aw3 + U_BF16 * (x3 @ aw3) + 64 * U_F32 * (x3 @ aw3 + abs(w["b3"][0]))
    return bound


# ---------------------------------------------------------------------------
# Kernel-form values with a per-point flip budget
# ---------------------------------------------------------------------------
def _bf16_np(x: np.ndarray) -> np.ndarray:
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(torch.bfloat16).to(torch.float32).numpy()


def _ulp_bf16(x: np.ndarray) -> np.ndarray:
    """Spacing of bfloat16 numbers at |x| (8 significant bits)."""
    a = np.maximum(np.abs(x).astype(np.float64), 2.0 ** -126)
    return np.exp2(np.floor(np.log2(a)) - 7.0)


def _near_midpoint(x: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """True where x lies within delta of a midpoint between two adjacent
    bfloat16 numbers (where a value moved by delta can round either way)."""
    u = _ulp_bf16(x)
    r = np.abs(x.astype(np.float64)) / u
    return np.abs(r - np.floor(r) - 0.5) * u <= delta


def kernel_form_with_flips(scene, pts: np.ndarray, enc_delta: float = 1e-6, cells=None):
    """The kernel-form bfloat16 value of each point (as sdf_bf16_kernel_form,
    in numpy float32), a flip budget and a float32 slack.

    A float32 sum taken in another order, or another float32 sine or
    exponential, moves a layer input by a few float32 ulps; where that input
    lies that close to a midpoint between two bfloat16 numbers it may round
    the other way (a flip: one bfloat16 ulp).  The inputs within reach of a
    midpoint are found per point (the encoding within enc_delta; a layer
    input within 64 float32 roundings of its pre-activation's sum of
    |terms|, plus the exponential and logarithm), and the budget is the sum
    of their flips' effects on d, propagated with |W| and the slope bound 2
    of 2k softplus in u':
      encoding e_j:   ulp(e_j) |k W1[:, j]| -> 2 |.| -> |W2 / 2| -> 2 |.| -> |w3|
      layer-2 input:  ulp(x_j) |W2[:, j] / 2| -> 2 |.| -> |w3|
      output input:   ulp(x_i) |w3_i|
    with w3 = W3[0] / (2k).  Without a flip the rounded inputs are equal and
    only the float32 output sum differs (the slack).  A GPU result may differ
    from the value by at most budget + slack."""
    k = scene.beta / math.log(2.0)
    cells, xl = point_cells(scene.N, pts, cells)
    val = np.zeros(len(cells))
    budget = np.zeros(len(cells))
    slack = np.zeros(len(cells))
    nflip = np.zeros(len(cells), np.int64)
    xl32 = xl.astype(np.float32)
    for c in np.unique(cells):
        m = cells == c
        w = _unpack64(scene, int(c))
        W1k = _bf16_np((k * w["W1"]).astype(np.float32)).astype(np.float64)
        W2h = _bf16_np((0.5 * w["W2"]).astype(np.float32)).astype(np.float64)
        w3 = (w["W3"][0] * (0.5 / k)).astype(np.float32).astype(np.float64)
        b1k = (k * w["b1"]).astype(np.float32).astype(np.float64)
        b2k = (k * w["b2"]).astype(np.float32).astype(np.float64)
        e32 = encode64(xl32[m].astype(np.float64)).astype(np.float32)
        e = _bf16_np(e32).astype(np.float64)
        u1 = (e @ W1k.T + b1k).astype(np.float32).astype(np.float64)
        x1f = u1 + np.abs(u1) + 2.0 * np.log2(1.0 + np.exp2(-np.abs(u1)))
        x1 = _bf16_np(x1f).astype(np.float64)
        u2 = (x1 @ W2h.T + b2k).astype(np.float32).astype(np.float64)
        x2f = u2 + np.abs(u2) + 2.0 * np.log2(1.0 + np.exp2(-np.abs(u2)))
        x2 = _bf16_np(x2f).astype(np.float64)
        val[m] = x2 @ w3 + float(w["b3"][0])
        aw3 = np.abs(w3)
        g2 = 2.0 * (np.abs(W2h).T @ aw3)              # d per unit of a layer-2 input
        g1 = 2.0 * (np.abs(W1k).T @ g2)               # d per unit of an encoding input
        # reach of float32 differences before each rounding
        d1 = 2.0 * (64 * U_F32 * (np.abs(e) @ np.abs(W1k).T + np.abs(b1k)) + 4e-7 * np.abs(u1)) + 1e-6
        d2 = 2.0 * (64 * U_F32 * (np.abs(x1) @ np.abs(W2h).T + np.abs(b2k)) + 4e-7 * np.abs(u2)) + 1e-6
        f0 = _near_midpoint(e32, np.full(e32.shape, enc_delta))
        f1 = _near_midpoint(x1f, d1)
        f2 = _near_midpoint(x2f, d2)
        budget[m] = (f0 * _ulp_bf16(e32)) @ g1 + (f1 * _ulp_bf16(x1f)) @ g2 + (f2 * _ulp_bf16(x2f)) @ aw3
        nflip[m] = f0.sum(1) + f1.sum(1) + f2.sum(1)
        slack[m] = 4e-6 * (np.abs(x2) @ aw3 + abs(float(w["b3"][0]))) + 1e-7
    return val, budget, slack, nflip
