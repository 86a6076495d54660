"""CPU emulation of the low-precision march MLP (test infrastructure only).

The paper fixes no precision for the renderer; the bfloat16 variant used by
the march is defined here as: the SDF MLP of eq. 3 (Sec. 3.1) with every
weight and every layer input rounded to bfloat16 (round to nearest even),
products accumulated in float32, biases and softplus in float32, the SDF
output row's weights also in bfloat16.  Plain torch CPU float32 ops, one cell
at a time.  Parity unpinned beyond its construction from those rounding
points: it is compared with the GPU kernel statistically (float32 sums in a
different order can flip a bfloat16 rounding).
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


def sdf_bf16(scene, pts: np.ndarray) -> np.ndarray:
    """SDF value of the cell containing each world point (points clamped to
    the grid), bfloat16 variant."""
    N, H = scene.N, scene.H
    x = torch.tensor(np.asarray(pts, np.float64))
    idx = torch.clamp(torch.floor((x + 1) * N / 2).long(), 0, N - 1)
    cell = idx[:, 0] + N * (idx[:, 1] + N * idx[:, 2])
    centers = -1 + (idx.double() + 0.5) * (2.0 / N)
    xl = ((x - centers) * N).float()
    out = torch.zeros(len(pts), dtype=torch.float32)
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
        e = _bf16(_encode(xl[m], 6))
        a1 = _softplus(e @ _bf16(W1).T + b1, scene.beta)
        a2 = _softplus(_bf16(a1) @ _bf16(W2).T + b2, scene.beta)
        out[m] = _bf16(a2) @ _bf16(W3[0]) + b3[0]
    return out.numpy()
