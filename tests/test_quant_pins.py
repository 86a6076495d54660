"""Pins of the low-precision rounding (CPU).

The packer's host rounding (kn_quant.h) and the emulation's rounding
(oracle/quant.py, torch casts) against exact values of the formats; the
emulation's MLP with rounding switched off against the FP64 oracle."""
import ctypes as C
import math
import os
import subprocess

import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import quant
from paper_2206_10885_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def qlib(tmp_path_factory):
    out = tmp_path_factory.mktemp("q") / "libquant_check.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", os.path.join(HERE, "quant_check.cpp"),
                    "-o", str(out)], check=True)
    L = C.CDLL(str(out))
    L.pow2_scale_of.restype = C.c_float
    L.pow2_scale_of.argtypes = [C.c_double]
    return L


# exact values of OCP e4m3fn (3 mantissa bits, exponent bias 7, max 448,
# subnormal step 2^-9), chosen to exercise ties to even and saturation
E4M3_CASES = [
    (448.0, 448.0), (460.0, 448.0), (1e6, 448.0), (-1e6, -448.0),
    (1.0625, 1.0),            # tie between 1 and 1.125 -> even mantissa
    (1.1875, 1.25),           # tie between 1.125 and 1.25 -> even
    (2.0 ** -6, 2.0 ** -6),   # smallest normal
    (2.0 ** -9, 2.0 ** -9),   # smallest subnormal
    (2.0 ** -10, 0.0),        # tie between 0 and 2^-9 -> even (0)
    (3 * 2.0 ** -10, 2.0 ** -8),  # tie between 1 and 2 subnormal steps -> 2
    (240.0, 240.0), (232.0, 224.0), (-3.0, -3.0), (0.3, 0.3125),
]


@pytest.mark.parametrize("x,want", E4M3_CASES)
def test_e4m3_rounding_exact_values(x, want, qlib):
    assert float(quant.e4m3(torch.tensor([x]))[0]) == want
    b = np.zeros(1, np.uint8)
    qlib.e4m3_many(np.array([x], np.float32).ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p), 1)
    v = np.zeros(1, np.float32)
    qlib.e4m3_decode(b.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p), 1)
    assert float(v[0]) == want


def test_e4m3_packer_matches_torch_cast(qlib):
    rng = np.random.default_rng(0)
    codes = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).float().numpy()
    codes = np.unique(codes[np.isfinite(codes)])
    mids = (codes[1:] + codes[:-1]) / 2
    x = np.concatenate([codes, mids, np.nextafter(mids.astype(np.float32), np.float32(np.inf)),
                        np.nextafter(mids.astype(np.float32), np.float32(-np.inf)),
                        rng.uniform(-500, 500, 100000), rng.normal(0, 1e-2, 100000)]).astype(np.float32)
    ours = np.zeros(len(x), np.uint8)
    qlib.e4m3_many(x.ctypes.data_as(C.c_void_p), ours.ctypes.data_as(C.c_void_p), len(x))
    ref = torch.tensor(np.clip(x, -448, 448)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref), np.nonzero(ours != ref)[0][:10]


def test_bf16_packer_matches_torch_cast(qlib):
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 1, 100000), rng.uniform(-1e4, 1e4, 10000),
                        1.0 + np.array([2.0 ** -8, 3 * 2.0 ** -8])]).astype(np.float32)
    ours = np.zeros(len(x), np.uint16)
    qlib.bf16_many(x.ctypes.data_as(C.c_void_p), ours.ctypes.data_as(C.c_void_p), len(x))
    ref = torch.tensor(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)
    # ties to even at 1 + half an ulp (ulp 2^-7) and 1 + 1.5 ulp
    assert float(quant._bf16(torch.tensor([1.0 + 2.0 ** -8]))[0]) == 1.0
    assert float(quant._bf16(torch.tensor([1.0 + 3 * 2.0 ** -8]))[0]) == 1.0 + 2.0 ** -6


def test_pow2_scale(qlib):
    rng = np.random.default_rng(2)
    for b in np.concatenate([[448.0, 449.0, 1.0, 224.0, 896.0], 10.0 ** rng.uniform(-6, 6, 500)]):
        s = quant.pow2_scale(float(b))
        assert s == qlib.pow2_scale_of(float(b))
        assert math.log2(s) == round(math.log2(s))
        assert b / s <= 448.0 < b / (s / 2)


@pytest.mark.parametrize("fn", ["sdf_bf16", "sdf_bf16_kernel_form", "sdf_fp8"])
def test_emulation_without_rounding_equals_oracle(fn):
    sc = synth.sphere_scene(4, 32, 0.5, 0.02, seed=9)
    rng = np.random.default_rng(3)
    pts = rng.uniform(-1, 1, (800, 3)).astype(np.float32)
    got = getattr(quant, fn)(sc, pts, quantize=False)
    os_ = O.OracleScene.from_scene(sc)
    N = sc.N
    centers = synth.cell_centers(N)
    ref = np.zeros(len(pts))
    for i, x in enumerate(pts.astype(np.float64)):
        idx = np.clip(np.floor((x + 1) * N / 2).astype(int), 0, N - 1)
        cell = idx[0] + N * (idx[1] + N * idx[2])
        ref[i] = os_.sdf_eval(cell, (x - centers[cell]) * N)[0]
    assert np.abs(got - ref).max() < 2e-5


def test_fp8_activation_bound_holds():
    """The layer-2 input scale never saturates: a1 / sa <= 448 on points of
    the cell (and on its faces)."""
    sc = synth.sphere_scene(3, 64, 0.5, 0.02, seed=4)
    rng = np.random.default_rng(5)
    H = sc.H
    for c in range(sc.N ** 3):
        blk = sc.sdf[c]
        W1 = blk[:39 * H].reshape(H, 39)
        b1 = blk[39 * H:40 * H]
        W2 = blk[40 * H:40 * H + H * H].reshape(H, H)
        s1, s2, sa = quant.fp8_scales(W1, b1, W2, sc.beta)
        xl = rng.uniform(-1, 1, (256, 3))
        xl[:16] = np.sign(xl[:16])
        e = np.array([O.encode(v, 6) for v in xl])
        a1 = np.maximum(e @ W1.T + b1, 0) + np.log1p(np.exp(-sc.beta * np.abs(e @ W1.T + b1))) / sc.beta
        assert a1.max() / sa <= 448.0
        assert np.abs(W1).max() / s1 <= 448.0 and np.abs(W2).max() / s2 <= 448.0


def test_fp64_forward_equals_c_oracle():
    """quant.sdf_fp64 (eq. 3 in numpy float64, with its activations) equals the
    C oracle's SDF value, and its activations are softplus of its
    pre-activations."""
    sc = synth.sphere_scene(4, 64, 0.5, 0.02, seed=21)
    rng = np.random.default_rng(8)
    pts = rng.uniform(-1, 1, (500, 3))
    cells, xl = quant.point_cells(sc.N, pts)
    f = quant.sdf_fp64(sc, cells, xl)
    os_ = O.OracleScene.from_scene(sc)
    ref = np.array([os_.sdf_eval(int(c), x)[0] for c, x in zip(cells, xl)])
    assert np.abs(ref - f["d"]).max() < 1e-12
    sp = np.vectorize(O.softplus)
    assert np.abs(f["a2"][:50] - sp(f["u2"][:50])).max() < 1e-14


@pytest.mark.parametrize("mode,fns", [("bf16", ("sdf_bf16", "sdf_bf16_kernel_form")), ("fp8", ("sdf_fp8",))])
def test_rounding_bound_covers_the_emulations(mode, fns):
    """Every emulation of a precision stays inside the worst-case per-point
    rounding bound at every point (H = 32 and 64, random points and points on
    cell faces).  The bound is loose by construction (sums of |terms|, no
    cancellation: typically 0.1-1% of it is used), so it catches gross errors
    (a wrong cell, layer or scale, a NaN); the sharp checks of the kernels are
    the flip budget and the comparison with the plain reading."""
    for H in (32, 64):
        sc = synth.sphere_scene(8, H, 0.6, 0.02, seed=40 + H)
        rng = np.random.default_rng(H)
        pts = rng.uniform(-1, 1, (3000, 3))
        pts[:64] = -1 + 2.0 * rng.integers(0, sc.N + 1, (64, 3)) / sc.N
        pts = pts.astype(np.float32)
        cells, xl = quant.point_cells(sc.N, pts)
        f = quant.sdf_fp64(sc, cells, xl)
        bound = quant.rounding_bound(sc, f, mode)
        for fn in fns:
            err = np.abs(getattr(quant, fn)(sc, pts).astype(np.float64) - f["d"])
            r = err / bound
            assert r.max() <= 1.0, (fn, H, r.max())
            assert np.median(r) > 1e-4, (fn, H, np.median(r))


def test_flip_budget_covers_a_reordered_evaluation():
    """kernel_form_with_flips (numpy float32) against sdf_bf16_kernel_form
    (torch float32, other summation order and exponentials): equal within
    float32 slack on almost every point, and within the per-point flip budget
    on every point.  A planted error, the SDF row without the low half of its
    hi + lo pair (the row itself rounded to bfloat16), breaks the budget at
    many points."""
    sc = synth.sphere_scene(16, 64, 0.6, 0.02, seed=7)
    rng = np.random.default_rng(3)
    pts = rng.uniform(-1, 1, (4000, 3)).astype(np.float32)
    val, budget, slack, nflip = quant.kernel_form_with_flips(sc, pts)
    ref = quant.sdf_bf16_kernel_form(sc, pts).astype(np.float64)
    diff = np.abs(val - ref)
    assert (diff <= budget + slack).all()
    assert np.mean(diff > slack) < 0.01
    # planted: W3[0] / (2k) replaced by its bfloat16 rounding, so the kernel
    # form's low half is (almost) zero
    k = sc.beta / math.log(2.0)
    bad = synth.Scene(N=sc.N, H=sc.H, sdf=sc.sdf.copy(), col=sc.col, beta=sc.beta)
    row0 = 39 * sc.H + sc.H + sc.H * sc.H + sc.H
    w = (bad.sdf[:, row0:row0 + sc.H].astype(np.float64) * (0.5 / k)).astype(np.float32)
    hi = torch.from_numpy(w).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    bad.sdf[:, row0:row0 + sc.H] = (hi * 2.0 * k).astype(np.float32)
    wrong = quant.sdf_bf16_kernel_form(bad, pts).astype(np.float64)
    assert np.mean(np.abs(wrong - val) > budget + slack) > 0.2
