"""CPU emulation of the low-precision march MLP (test infrastructure only).

The paper fixes no precision for the renderer; the bfloat16 variant used by
the march is defined here as: the SDF MLP of eq. 3 (Sec. 3.1) with its two
hidden layers written for u' = k u, k = beta / ln 2, which leaves eq. 3
unchanged in exact arithmetic since 2k softplus(u) = u' + |u'| +
2 log2(1 + 2^-|u'|); every weight (k W1, W2 / 2) and every layer input (the
encoding, 2k a1, 2k a2) rounded to bfloat16 (round to nearest even),
products accumulated in float32, biases and activations in float32; the
output row W3 / (2k) as a pair hi = bf16(w), lo = bf16(w - hi), whose two
products are added.  Plain torch CPU float32 ops, one cell
at a time.  The fp8 e4m3 variant (sdf_fp8) rounds the two hidden layers'
weights and inputs to e4m3 with power-of-two per-(cell, layer) scales.

Pins (tests/test_quant_pins.py): the rounding functions against exact
e4m3 / bfloat16 values; with rounding switched off the emulation equals the
FP64 oracle to float32 precision.  The GPU kernels are compared with it
statistically (float32 sums in a different order can flip a rounding).
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


def _cell_blocks(scene, pts):
    N, H = scene.N, scene.H
    x = torch.tensor(np.asarray(pts, np.float64))
    idx = torch.clamp(torch.floor((x + 1) * N / 2).long(), 0, N - 1)
    cell = idx[:, 0] + N * (idx[:, 1] + N * idx[:, 2])
    centers = -1 + (idx.double() + 0.5) * (2.0 / N)
    xl = ((x - centers) * N).float()
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


def sdf_fp8(scene, pts: np.ndarray, quantize: bool = True) -> np.ndarray:
    """SDF value of the cell containing each world point, fp8 e4m3 variant:
    the encoding (scale 1) and W1 / s1 rounded to e4m3; u1 = s1 (W1q eq) + b1;
    a1 = softplus(u1) scaled by 1 / sa and rounded; u2 = s2 sa (W2q a1q) + b2;
    a2 = softplus(u2) in bfloat16; the output row W3 as a hi + lo bfloat16
    pair.  quantize=False skips every rounding (float32 throughout)."""
    q = e4m3 if quantize else (lambda t: t.float())
    qb = _bf16 if quantize else (lambda t: t.float())
    out = torch.zeros(len(pts), dtype=torch.float32)
    for m, xl, (W1, b1, W2, b2, W3, b3) in _cell_blocks(scene, pts):
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


def sdf_bf16(scene, pts: np.ndarray, quantize: bool = True) -> np.ndarray:
    """SDF value of the cell containing each world point (points clamped to
    the grid), bfloat16 variant; quantize=False skips every rounding.  The
    scaled weights are formed in float64 and rounded to float32 first."""
    qb = _bf16 if quantize else (lambda t: t.float())
    k = scene.beta / math.log(2.0)
    out = torch.zeros(len(pts), dtype=torch.float32)
    for m, xl, (W1, b1, W2, b2, W3, b3) in _cell_blocks(scene, pts):
        e = qb(_encode(xl, 6))
        a1 = _softplus_2k(e @ qb((k * W1.double()).float()).T + (k * b1.double()).float())
        a2 = _softplus_2k(qb(a1) @ qb(0.5 * W2).T + (k * b2.double()).float())
        hi, lo = _split((W3[0].double() * (0.5 / k)).float(), qb)
        out[m] = (qb(a2) @ hi + qb(a2) @ lo) + b3[0]
    return out.numpy()
