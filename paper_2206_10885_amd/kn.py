"""Thin ctypes binding of the C ABI in include/kn.h.

Argument marshalling only: every step of rendering runs in the HIP library
libkn.so.  torch provides device memory (output tensors) and the stream.
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkn.so")

KN_OK, KN_PENDING = 0, 1
KN_FP32, KN_BF16, KN_FP8_E4M3 = 0, 1, 2
KN_ABI_VERSION = 3
KN_CAMERA_SPLIT_BF16_SHADING = 1
KN_CAMERA_UNCLAMPED_STEPS = 2
KN_PRIM_SPHERE, KN_PRIM_BOX, KN_PRIM_TRIANGLE = 1, 2, 3
_STATUS = {0: "KN_OK", 1: "KN_PENDING", -1: "KN_E_INVALID", -2: "KN_E_NOMEM", -3: "KN_E_NOT_FOUND",
           -4: "KN_E_BUSY", -5: "KN_E_DEVICE", -6: "KN_E_TIMEOUT", -7: "KN_E_UNSUPPORTED",
           -8: "KN_E_SHUTDOWN"}
PRECISIONS = {"fp32": KN_FP32, "bf16": KN_BF16, "fp8": KN_FP8_E4M3}


class KnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class SceneDesc(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("grid_n", C.c_uint32),
                ("bbox_min", C.c_float * 3), ("bbox_max", C.c_float * 3),
                ("pos_freqs", C.c_uint32), ("dir_freqs", C.c_uint32),
                ("sdf_hidden", C.c_uint32), ("sdf_layers", C.c_uint32), ("feat_dim", C.c_uint32),
                ("col_hidden", C.c_uint32), ("col_layers", C.c_uint32), ("col_in_has_x", C.c_uint32),
                ("softplus_beta", C.c_float),
                ("sdf_params", C.POINTER(C.c_float)), ("col_params", C.POINTER(C.c_float)),
                ("precisions", C.c_uint32)]


class Camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3),
                ("tan_half_diag", C.c_float), ("width", C.c_uint32), ("height", C.c_uint32),
                ("spp", C.c_uint32), ("bounces", C.c_uint32), ("max_steps", C.c_uint32),
                ("eps", C.c_float), ("precision", C.c_int), ("seed", C.c_uint64),
                ("env_rgb", C.c_void_p), ("env_w", C.c_uint32), ("env_h", C.c_uint32),
                ("flags", C.c_uint32), ("sample_offset", C.c_uint32)]


class Frame(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("normal", C.c_void_p),
                ("hit", C.c_void_p), ("steps", C.c_void_p), ("trace", C.c_void_p),
                ("segments", C.c_void_p), ("hip_stream", C.c_void_p), ("accum", C.c_void_p)]


class Primitive(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("p", C.c_float * 9), ("albedo", C.c_float * 3)]


class Instance(C.Structure):
    _fields_ = [("scene", C.c_uint32), ("translate", C.c_float * 3), ("scale", C.c_float)]


class WorldDesc(C.Structure):
    _fields_ = [("n_instances", C.c_uint32), ("instances", C.POINTER(Instance)),
                ("n_primitives", C.c_uint32), ("primitives", C.POINTER(Primitive))]


SEGMENT_WORDS = 20   # kn_segment_record: 80 bytes


def segment_fields(seg) -> dict:
    """Fields of kn_segment_record from a [..., 20] int32 tensor / array (as
    numpy): origin, dir, t_march, t_entry, t, normal, albedo, cell, status,
    steps."""
    a = seg.cpu().numpy() if hasattr(seg, "cpu") else np.asarray(seg)
    f = a.view(np.float32)
    return dict(origin=f[..., 0:3].astype(np.float64), dir=f[..., 3:6].astype(np.float64),
                t_march=f[..., 6].astype(np.float64), t_entry=f[..., 7].astype(np.float64),
                t=f[..., 8].astype(np.float64), normal=f[..., 9:12].astype(np.float64),
                albedo=f[..., 12:15].astype(np.float64), cell=a[..., 15].astype(np.int64),
                status=a[..., 16].astype(np.int64), steps=a[..., 17].astype(np.int64))


class Stats(C.Structure):
    _fields_ = [("gpu_ms", C.c_double), ("wall_ms", C.c_double), ("rays", C.c_uint64),
                ("evals", C.c_uint64), ("hits", C.c_uint64), ("rounds", C.c_uint64),
                ("kernel_times", C.c_uint32), ("march_launches", C.c_uint32),
                ("march_ms", C.c_double), ("shade_ms", C.c_double),
                ("march_tiles", C.c_uint64), ("march_chunks", C.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["kn_ctx_create", "kn_ctx_destroy", "kn_last_error", "kn_scene_create",
           "kn_scene_destroy", "kn_render", "kn_query", "kn_query_noalloc", "kn_grid_sample",
           "kn_eikonal_fd", "kn_world_create", "kn_world_destroy", "kn_render_world", "kn_serve_start",
           "kn_serve_submit", "kn_serve_poll", "kn_serve_stop"]

_lib = None


def lib():
    """Loads libkn.so (raises if it has not been built).

    torch is imported first: its wheel ships its own HIP runtime under another
    file name, and loading libkn.so first would map /opt/rocm's runtime as
    well, leaving two runtimes whose device pointers and streams are invalid
    in each other (kn_ctx_create refuses to run in such a process).  With
    torch loaded first, libkn.so binds to torch's runtime by its soname."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2206_10885_amd/build.py "
                              "(or __graft_entry__.build()) first")
        import torch  # noqa: F401  (one HIP runtime in the process: torch's)
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.kn_last_error.restype = C.c_char_p
        L.kn_ctx_create.argtypes = [C.c_int, C.c_uint64, C.POINTER(vp)]
        L.kn_ctx_destroy.argtypes = [vp]
        L.kn_scene_create.argtypes = [vp, C.POINTER(SceneDesc), C.POINTER(C.c_uint32)]
        L.kn_scene_destroy.argtypes = [vp, C.c_uint32]
        L.kn_render.argtypes = [vp, C.c_uint32, C.POINTER(Camera), C.POINTER(Frame), C.POINTER(Stats)]
        L.kn_query.argtypes = [vp, C.c_uint32, C.c_int, vp, C.c_uint64, vp, vp, vp, vp]
        L.kn_query_noalloc.argtypes = [vp, C.c_uint32, C.c_int, vp, C.c_uint64, vp, vp, vp, vp]
        L.kn_grid_sample.argtypes = [vp, C.c_uint32, C.c_int, C.c_uint32, vp, vp, vp]
        L.kn_eikonal_fd.argtypes = [vp, C.c_uint32, C.c_int, vp, C.c_uint64, C.c_float, vp, vp, vp, vp]
        L.kn_world_create.argtypes = [vp, C.POINTER(WorldDesc), C.POINTER(C.c_uint32)]
        L.kn_world_destroy.argtypes = [vp, C.c_uint32]
        L.kn_render_world.argtypes = [vp, C.c_uint32, C.POINTER(Camera), C.POINTER(Frame), C.POINTER(Stats)]
        L.kn_serve_start.argtypes = [vp, C.c_uint32, C.c_int]
        L.kn_serve_submit.argtypes = [vp, C.c_uint32, C.POINTER(Camera), C.POINTER(Frame),
                                      C.POINTER(C.c_uint64)]
        L.kn_serve_poll.argtypes = [vp, C.c_uint64, C.c_int64, C.POINTER(Stats)]
        L.kn_serve_stop.argtypes = [vp]
        for name in EXPORTS:
            if name != "kn_last_error":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(status: int) -> int:
    if status < 0:
        raise KnError(status, lib().kn_last_error().decode())
    return status


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def make_camera(view, width: int, height: int, max_steps: int, eps: float,
                precision: str = "fp32", spp: int = 1, bounces: int = 0, seed: int = 0,
                env=None, split_shading: bool = False, unclamped: bool = False,
                sample_offset: int = 0) -> Camera:
    """A kn_camera; split_shading selects the split-bfloat16 refinement and
    shading of bf16 / fp8 marches (float32 otherwise); unclamped selects
    Hart's unclamped steps across cells; sample_offset is the index of the
    call's first sample (progressive path tracing)."""
    env_ptr, ew, eh = None, 0, 0
    if env is not None:
        env_ptr, eh, ew = env.data_ptr(), env.shape[0], env.shape[1]
    return Camera((C.c_float * 3)(*view.eye), (C.c_float * 3)(*view.look_at),
                  (C.c_float * 3)(*view.up), float(view.tan_half_diag), width, height, spp,
                  bounces, max_steps, eps, PRECISIONS[precision], seed, env_ptr, ew, eh,
                  (KN_CAMERA_SPLIT_BF16_SHADING if split_shading else 0) |
                  (KN_CAMERA_UNCLAMPED_STEPS if unclamped else 0), sample_offset)


class Context:
    """A kn_ctx on one HIP device (torch device index)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.device = device
        h = C.c_void_p()
        check(lib().kn_ctx_create(device, hbm_budget_bytes, C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            check(lib().kn_ctx_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- scenes -------------------------------------------------------------
    def scene_create(self, scene, precisions=("bf16",)) -> int:
        sdf = np.ascontiguousarray(scene.sdf, np.float32)
        col = np.ascontiguousarray(scene.col, np.float32)
        bits = 0
        for p in precisions:
            bits |= 1 << PRECISIONS[p]
        d = SceneDesc(KN_ABI_VERSION, scene.N, (C.c_float * 3)(*scene.bbox_min),
                      (C.c_float * 3)(*scene.bbox_max), 6, 4, scene.H, 2, 15, 32, 1, 1,
                      float(scene.beta), sdf.ctypes.data_as(C.POINTER(C.c_float)),
                      col.ctypes.data_as(C.POINTER(C.c_float)), bits)
        sid = C.c_uint32()
        check(lib().kn_scene_create(self.h, C.byref(d), C.byref(sid)))
        return sid.value

    def scene_destroy(self, sid: int):
        check(lib().kn_scene_destroy(self.h, sid))

    # -- rendering ----------------------------------------------------------
    def alloc_frame(self, width: int, height: int, with_trace: bool = False) -> dict:
        import torch
        dev = torch.device("cuda", self.device)
        f = dict(rgb=torch.empty((height, width, 3), dtype=torch.float32, device=dev),
                 depth=torch.empty((height, width), dtype=torch.float32, device=dev),
                 normal=torch.empty((height, width, 3), dtype=torch.float32, device=dev),
                 hit=torch.empty((height, width), dtype=torch.uint8, device=dev),
                 steps=torch.empty((height, width), dtype=torch.int16, device=dev))
        if with_trace:
            f["trace"] = torch.empty((height, width, 4), dtype=torch.int32, device=dev)
        return f

    @staticmethod
    def _frame(out: dict, stream) -> Frame:
        return Frame(_ptr(out["rgb"]), _ptr(out.get("depth")), _ptr(out.get("normal")),
                     _ptr(out.get("hit")), _ptr(out.get("steps")), _ptr(out.get("trace")),
                     _ptr(out.get("segments")), None if stream is None else C.c_void_p(stream.cuda_stream),
                     _ptr(out.get("accum")))

    def render_into(self, sid: int, cam: Camera, out: dict, stream=None,
                    kernel_times: bool = False) -> dict:
        """kn_render into the tensors of `out` (rgb required; depth, normal,
        hit, steps, trace, segments and accum optional)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        fr = self._frame(out, stream)
        st = Stats()
        st.kernel_times = 1 if kernel_times else 0
        check(lib().kn_render(self.h, sid, C.byref(cam), C.byref(fr), C.byref(st)))
        return st.as_dict()

    def render(self, sid: int, view, width: int, height: int, max_steps: int, eps: float,
               precision: str = "fp32", with_trace: bool = False, split_shading: bool = False,
               unclamped: bool = False) -> dict:
        cam = make_camera(view, width, height, max_steps, eps, precision, split_shading=split_shading,
                          unclamped=unclamped)
        out = self.alloc_frame(width, height, with_trace)
        out["stats"] = self.render_into(sid, cam, out)
        return out

    # -- shared scenes -------------------------------------------------------
    def world_create(self, instances=(), primitives=()) -> int:
        """kn_world_create: instances = [(scene id, translate xyz, scale)],
        primitives = [(KN_PRIM_* kind, parameters (up to 9), albedo rgb)]."""
        ins = (Instance * max(1, len(instances)))()
        for k, (sid, T, s) in enumerate(instances):
            ins[k] = Instance(sid, (C.c_float * 3)(*T), float(s))
        prs = (Primitive * max(1, len(primitives)))()
        for k, (kind, p, alb) in enumerate(primitives):
            pp = list(p) + [0.0] * (9 - len(p))
            prs[k] = Primitive(kind, (C.c_float * 9)(*pp), (C.c_float * 3)(*alb))
        d = WorldDesc(len(instances), ins, len(primitives), prs)
        wid = C.c_uint32()
        check(lib().kn_world_create(self.h, C.byref(d), C.byref(wid)))
        return wid.value

    def world_destroy(self, wid: int):
        check(lib().kn_world_destroy(self.h, wid))

    def render_world_into(self, wid: int, cam: Camera, out: dict, stream=None,
                          kernel_times: bool = False) -> dict:
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        fr = self._frame(out, stream)
        st = Stats()
        st.kernel_times = 1 if kernel_times else 0
        check(lib().kn_render_world(self.h, wid, C.byref(cam), C.byref(fr), C.byref(st)))
        return st.as_dict()

    # -- serving ------------------------------------------------------------
    def serve_start(self, max_inflight: int = 16, precision: str = "bf16"):
        check(lib().kn_serve_start(self.h, max_inflight, PRECISIONS[precision]))

    def serve_submit(self, sid: int, cam: Camera, out: dict) -> int:
        """Queues a frame; `out` (from alloc_frame) must stay alive until
        serve_poll reports it finished."""
        fr = self._frame(out, None)
        rid = C.c_uint64()
        check(lib().kn_serve_submit(self.h, sid, C.byref(cam), C.byref(fr), C.byref(rid)))
        return rid.value

    def serve_poll(self, req: int, timeout_us: int = -1):
        """Stats of a finished request, or None while it is still pending."""
        st = Stats()
        r = check(lib().kn_serve_poll(self.h, req, timeout_us, C.byref(st)))
        return None if r == KN_PENDING else st.as_dict()

    def serve_stop(self):
        check(lib().kn_serve_stop(self.h))

    def query(self, sid: int, points, precision: str = "fp32", grad: bool = False,
              feat: bool = False, stream=None, noalloc: bool = False, out=None) -> dict:
        """kn_query (or kn_query_noalloc) on a [n, 3] float32 device tensor;
        `out` (a dict of d, grad, z tensors) receives the results if given."""
        import torch
        pts = points.contiguous()
        n = pts.shape[0]
        if out is not None:
            d, g, z = out.get("d"), out.get("grad"), out.get("z")
        else:
            d = torch.empty(n, dtype=torch.float32, device=pts.device)
            g = torch.empty((n, 3), dtype=torch.float32, device=pts.device) if grad else None
            z = torch.empty((n, 15), dtype=torch.float32, device=pts.device) if feat else None
        if stream is None:
            stream = torch.cuda.current_stream(pts.device)
        fn = lib().kn_query_noalloc if noalloc else lib().kn_query
        check(fn(self.h, sid, PRECISIONS[precision], _ptr(pts), n, _ptr(d), _ptr(g), _ptr(z),
                 C.c_void_p(stream.cuda_stream)))
        return dict(d=d, grad=g, z=z)

    def grid_sample(self, sid: int, R: int, precision: str = "fp32", grad: bool = False, stream=None,
                    out=None) -> dict:
        """kn_grid_sample: the SDF on the R^3 lattice spanning the box, as
        [R, R, R] tensors indexed [k, j, i] (z, y, x); `out` (d, grad) receives
        the results if given."""
        import torch
        dev = torch.device("cuda", self.device)
        if out is not None:
            d, g = out.get("d"), out.get("grad")
        else:
            d = torch.empty((R, R, R), dtype=torch.float32, device=dev)
            g = torch.empty((R, R, R, 3), dtype=torch.float32, device=dev) if grad else None
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        check(lib().kn_grid_sample(self.h, sid, PRECISIONS[precision], R, _ptr(d), _ptr(g),
                                   C.c_void_p(stream.cuda_stream)))
        return dict(d=d, grad=g)

    def eikonal_fd(self, sid: int, points, delta: float, precision: str = "fp32", stencil: bool = False,
                   stream=None) -> dict:
        """kn_eikonal_fd on a [n, 3] float32 device tensor: gradient norms,
        optionally the six stencil values per point, and the loss (a device
        float64 scalar)."""
        import torch
        pts = points.contiguous()
        n = pts.shape[0]
        gn = torch.empty(n, dtype=torch.float32, device=pts.device)
        st = torch.empty((n, 6), dtype=torch.float32, device=pts.device) if stencil else None
        loss = torch.empty(1, dtype=torch.float64, device=pts.device)
        if stream is None:
            stream = torch.cuda.current_stream(pts.device)
        check(lib().kn_eikonal_fd(self.h, sid, PRECISIONS[precision], _ptr(pts), n, float(delta), _ptr(gn),
                                  _ptr(st), _ptr(loss), C.c_void_p(stream.cuda_stream)))
        return dict(gnorm=gn, stencil=st, loss=loss)
