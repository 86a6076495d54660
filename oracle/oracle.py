"""ctypes front end of the FP64 CPU oracle (oracle/kno.c).

TEST INFRASTRUCTURE ONLY: the tests, the package's smoke check and the
benchmark's CPU-baseline leg use it; the product library never does.  It
imports nothing from the HIP package.  Scenes are passed as plain arrays in
the C ABI's host layout (one float32 block per cell).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkno.so")

BOX_MISS, HIT, EXIT_MISS, BUDGET_MISS = 0, 1, 2, 3


def build(verbose: bool = False) -> str:
    """Compile kno.c into libkno.so with gcc -O2 (no fast-math), OpenMP."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           os.path.join(HERE, "kno.c"), "-o", LIB_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB_PATH


class _Scene(C.Structure):
    _fields_ = [("N", C.c_int32), ("H", C.c_int32), ("pos_freqs", C.c_int32),
                ("dir_freqs", C.c_int32), ("beta", C.c_double),
                ("bmin", C.c_double * 3), ("bmax", C.c_double * 3),
                ("sdf", C.POINTER(C.c_float)), ("col", C.POINTER(C.c_float))]


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("look_at", C.c_double * 3), ("up", C.c_double * 3),
                ("tan_half_diag", C.c_double), ("width", C.c_int32), ("height", C.c_int32),
                ("max_steps", C.c_int32), ("eps", C.c_double), ("background", C.c_double * 3),
                ("step_mode", C.c_int32)]

STEP_CLAMPED, STEP_UNCLAMPED = 0, 1


class _Trace(C.Structure):
    _fields_ = [("status", C.c_int32), ("steps", C.c_int32), ("cell", C.c_int32 * 3),
                ("t", C.c_double), ("t_entry", C.c_double), ("fmin", C.c_double)]


class _Env(C.Structure):
    _fields_ = [("rgb", C.POINTER(C.c_float)), ("w", C.c_int32), ("h", C.c_int32)]


class _PT(C.Structure):
    _fields_ = [("spp", C.c_int32), ("bounces", C.c_int32), ("seed", C.c_uint64), ("env", _Env),
                ("jitter", C.c_int32)]


class _Prim(C.Structure):
    _fields_ = [("kind", C.c_int32), ("p", C.c_double * 9), ("albedo", C.c_double * 3)]


class _Instance(C.Structure):
    _fields_ = [("scene", C.POINTER(_Scene)), ("translate", C.c_double * 3), ("scale", C.c_double)]


class _World(C.Structure):
    _fields_ = [("n_inst", C.c_int32), ("inst", C.POINTER(_Instance)), ("n_prim", C.c_int32),
                ("prim", C.POINTER(_Prim))]


PRIM_SPHERE, PRIM_BOX, PRIM_TRIANGLE = 1, 2, 3


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or (
                os.path.getmtime(LIB_PATH) < os.path.getmtime(os.path.join(HERE, "kno.c"))):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.kno_sdf_params.restype = C.c_int
        L.kno_col_params.restype = C.c_int
        L.kno_encode.argtypes = [dp, C.c_int, C.c_int, dp]
        L.kno_softplus.argtypes = [C.c_double, C.c_double]
        L.kno_softplus.restype = C.c_double
        L.kno_sdf_eval.argtypes = [C.POINTER(_Scene), C.c_int, dp, dp, dp]
        L.kno_color_eval.argtypes = [C.POINTER(_Scene), C.c_int, dp, dp, dp, dp, dp]
        L.kno_camera_ray.argtypes = [C.POINTER(_Camera), C.c_int, C.c_int, C.c_double,
                                     C.c_double, dp, dp]
        L.kno_slab.argtypes = [C.POINTER(_Scene), dp, dp, dp, dp]
        L.kno_slab.restype = C.c_int
        L.kno_cells_along_ray.argtypes = [C.POINTER(_Scene), dp, dp, C.c_int,
                                          C.POINTER(C.c_int32), dp]
        L.kno_cells_along_ray.restype = C.c_int
        L.kno_trace.argtypes = [C.POINTER(_Scene), dp, dp, C.c_int, C.c_double,
                                C.POINTER(_Trace)]
        L.kno_trace_mode.argtypes = [C.POINTER(_Scene), dp, dp, C.c_int, C.c_double, C.c_int,
                                     C.POINTER(_Trace)]
        L.kno_shade.argtypes = [C.POINTER(_Scene), dp, dp, C.POINTER(_Trace), dp, dp, dp, dp]
        L.kno_render.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.c_void_p, C.c_int64,
                                 dp, dp, dp, C.POINTER(C.c_uint8), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32), dp, C.c_int]
        u32p = C.POINTER(C.c_uint32)
        L.kno_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.kno_onb.argtypes = [dp, dp, dp]
        L.kno_cosine_dir.argtypes = [dp, C.c_double, C.c_double, dp]
        L.kno_env_lookup.argtypes = [C.POINTER(_Env), dp, dp]
        L.kno_path_trace.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_PT), C.c_void_p,
                                     C.c_int64, dp, dp, dp, C.POINTER(C.c_uint8), C.c_int]
        L.kno_query.argtypes = [C.POINTER(_Scene), dp, C.c_int64, dp, dp, dp, C.c_int]
        L.kno_prim_hit.argtypes = [C.POINTER(_Prim), dp, dp, C.c_double, dp, dp]
        L.kno_prim_hit.restype = C.c_int
        L.kno_world_render.argtypes = [C.POINTER(_World), C.POINTER(_Camera), C.c_void_p, C.c_int64, dp, dp, dp,
                                       C.POINTER(C.c_uint8), C.POINTER(C.c_int32), C.c_int]
        L.kno_world_path_trace.argtypes = [C.POINTER(_World), C.POINTER(_Camera), C.POINTER(_PT), C.c_void_p,
                                           C.c_int64, dp, dp, dp, C.POINTER(C.c_uint8), C.c_int]
        L.kno_grid_sample.argtypes = [C.POINTER(_Scene), C.c_int, C.POINTER(C.c_int64), C.c_int64,
                                      dp, dp, dp, C.c_int]
        L.kno_eikonal_fd.argtypes = [C.POINTER(_Scene), dp, C.c_int64, C.c_double, dp, dp, dp, C.c_int]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _vec(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, np.float64))


class OracleScene:
    """Holds a scene's float32 arrays alive for the C side."""

    def __init__(self, sdf: np.ndarray, col: np.ndarray, N: int, H: int,
                 bbox_min=(-1, -1, -1), bbox_max=(1, 1, 1), beta: float = 100.0,
                 pos_freqs: int = 6, dir_freqs: int = 4):
        self.sdf = np.ascontiguousarray(sdf, np.float32)
        self.col = np.ascontiguousarray(col, np.float32)
        assert self.sdf.shape == (N ** 3, lib().kno_sdf_params(H))
        assert self.col.shape == (N ** 3, lib().kno_col_params())
        self.N, self.H = N, H
        self.c = _Scene(N, H, pos_freqs, dir_freqs, beta, (C.c_double * 3)(*bbox_min),
                        (C.c_double * 3)(*bbox_max),
                        self.sdf.ctypes.data_as(C.POINTER(C.c_float)),
                        self.col.ctypes.data_as(C.POINTER(C.c_float)))

    @classmethod
    def from_scene(cls, sc) -> "OracleScene":
        return cls(sc.sdf, sc.col, sc.N, sc.H, sc.bbox_min, sc.bbox_max, sc.beta)

    # -- primitives --------------------------------------------------------
    def sdf_eval(self, cell: int, xl, grad: bool = False):
        x = _vec(xl)
        out = np.zeros(16)
        g = np.zeros(3)
        lib().kno_sdf_eval(C.byref(self.c), int(cell), _dp(x), _dp(out), _dp(g) if grad else None)
        return (out, g) if grad else out

    def color_eval(self, cell: int, xl, v, n, z):
        rgb = np.zeros(3)
        a, b, c, d = _vec(xl), _vec(v), _vec(n), _vec(z)
        lib().kno_color_eval(C.byref(self.c), int(cell), _dp(a), _dp(b), _dp(c), _dp(d), _dp(rgb))
        return rgb

    def slab(self, o, d):
        tn, tf = C.c_double(), C.c_double()
        ok = lib().kno_slab(C.byref(self.c), _dp(_vec(o)), _dp(_vec(d)), C.byref(tn), C.byref(tf))
        return bool(ok), tn.value, tf.value

    def cells_along_ray(self, o, d, max_cells: int = 4096):
        cells = np.zeros(max_cells, np.int32)
        tin = np.zeros(max_cells)
        n = lib().kno_cells_along_ray(C.byref(self.c), _dp(_vec(o)), _dp(_vec(d)), max_cells,
                                      cells.ctypes.data_as(C.POINTER(C.c_int32)), _dp(tin))
        return cells[:n], tin[:n]

    def trace(self, o, d, max_steps: int, eps: float, unclamped: bool = False) -> dict:
        r = _Trace()
        lib().kno_trace_mode(C.byref(self.c), _dp(_vec(o)), _dp(_vec(d)), max_steps, eps,
                             STEP_UNCLAMPED if unclamped else STEP_CLAMPED, C.byref(r))
        return dict(status=r.status, steps=r.steps, cell=tuple(r.cell), t=r.t,
                    t_entry=r.t_entry, fmin=r.fmin, _raw=r)

    def shade(self, o, d, tr: dict) -> dict:
        depth = C.c_double()
        n, rgb, z = np.zeros(3), np.zeros(3), np.zeros(15)
        lib().kno_shade(C.byref(self.c), _dp(_vec(o)), _dp(_vec(d)), C.byref(tr["_raw"]),
                        C.byref(depth), _dp(n), _dp(rgb), _dp(z))
        return dict(depth=depth.value, normal=n, rgb=rgb, z=z)

    def render(self, view, width: int, height: int, max_steps: int, eps: float,
               pixels=None, background=(0.0, 0.0, 0.0), nthreads: int = 0, unclamped: bool = False) -> dict:
        cam = make_camera(view, width, height, max_steps, eps, background, unclamped)
        if pixels is None:
            npix = width * height
            pix_ptr = None
        else:
            pixels = np.ascontiguousarray(pixels, np.int64)
            npix = pixels.size
            pix_ptr = pixels.ctypes.data
        rgb = np.zeros((npix, 3))
        depth = np.zeros(npix)
        normal = np.zeros((npix, 3))
        hit = np.zeros(npix, np.uint8)
        steps = np.zeros(npix, np.int32)
        status = np.zeros(npix, np.int32)
        fmin = np.zeros(npix)
        lib().kno_render(C.byref(self.c), C.byref(cam), pix_ptr, npix, _dp(rgb), _dp(depth),
                         _dp(normal), hit.ctypes.data_as(C.POINTER(C.c_uint8)),
                         steps.ctypes.data_as(C.POINTER(C.c_int32)),
                         status.ctypes.data_as(C.POINTER(C.c_int32)), _dp(fmin), nthreads)
        return dict(rgb=rgb, depth=depth, normal=normal, hit=hit, steps=steps,
                    status=status, fmin=fmin)


    def query(self, pts, grad: bool = False, feat: bool = False, nthreads: int = 0) -> dict:
        """The global piecewise SDF at world points [n, 3]: d, and on request
        the world gradient of the containing cell's MLP and the feature."""
        p = np.ascontiguousarray(pts, np.float64).reshape(-1, 3)
        n = p.shape[0]
        d = np.zeros(n)
        g = np.zeros((n, 3)) if grad else None
        z = np.zeros((n, 15)) if feat else None
        lib().kno_query(C.byref(self.c), _dp(p), n, _dp(d), _dp(g) if grad else None,
                        _dp(z) if feat else None, nthreads)
        out = dict(d=d)
        if grad:
            out["grad"] = g
        if feat:
            out["z"] = z
        return out

    def grid_sample(self, R: int, lin, grad: bool = False, feat: bool = False, nthreads: int = 0) -> dict:
        """The SDF at lattice points (flattened indices i + R (j + R k)) of
        the R^3 lattice spanning the box, corners included."""
        lin = np.ascontiguousarray(lin, np.int64).ravel()
        n = lin.size
        d = np.zeros(n)
        g = np.zeros((n, 3)) if grad else None
        z = np.zeros((n, 15)) if feat else None
        lib().kno_grid_sample(C.byref(self.c), int(R), lin.ctypes.data_as(C.POINTER(C.c_int64)), n, _dp(d),
                              _dp(g) if grad else None, _dp(z) if feat else None, nthreads)
        out = dict(d=d)
        if grad:
            out["grad"] = g
        if feat:
            out["z"] = z
        return out

    def eikonal_fd(self, pts, delta: float, nthreads: int = 0) -> dict:
        """Central-difference gradient norms of the global SDF at points
        [n, 3], the six stencil values per point (+x, -x, +y, -y, +z, -z)
        and the mean squared eikonal residual."""
        p = np.ascontiguousarray(pts, np.float64).reshape(-1, 3)
        n = p.shape[0]
        gn = np.zeros(n)
        st = np.zeros((n, 6))
        loss = C.c_double()
        lib().kno_eikonal_fd(C.byref(self.c), _dp(p), n, float(delta), _dp(gn), _dp(st), C.byref(loss), nthreads)
        return dict(gnorm=gn, stencil=st, loss=loss.value)

    def path_trace(self, view, width: int, height: int, max_steps: int, eps: float, spp: int,
                   bounces: int, seed: int, env=None, pixels=None, nthreads: int = 0,
                   unclamped: bool = False, jitter: bool = False) -> dict:
        """Path-traced pixels (mean radiance over spp) plus the primary
        segment's depth, normal and hit of sample 0; jitter: jittered
        pixel samples at spp = 1 too."""
        cam = make_camera(view, width, height, max_steps, eps, unclamped=unclamped)
        envp = _make_env(env)
        pt = _PT(spp, bounces, seed, envp, 1 if jitter else 0)
        if pixels is None:
            npix, pix_ptr = width * height, None
        else:
            pixels = np.ascontiguousarray(pixels, np.int64)
            npix, pix_ptr = pixels.size, pixels.ctypes.data
        rgb = np.zeros((npix, 3))
        depth = np.zeros(npix)
        normal = np.zeros((npix, 3))
        hit = np.zeros(npix, np.uint8)
        lib().kno_path_trace(C.byref(self.c), C.byref(cam), C.byref(pt), pix_ptr, npix, _dp(rgb),
                             _dp(depth), _dp(normal), hit.ctypes.data_as(C.POINTER(C.c_uint8)), nthreads)
        return dict(rgb=rgb, depth=depth, normal=normal, hit=hit)


_env_keep = []


def _make_env(env) -> _Env:
    if env is None:
        return _Env(None, 0, 0)
    a = np.ascontiguousarray(env, np.float32)
    _env_keep.append(a)
    if len(_env_keep) > 8:
        del _env_keep[0]
    return _Env(a.ctypes.data_as(C.POINTER(C.c_float)), a.shape[1], a.shape[0])


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    u32p = C.POINTER(C.c_uint32)
    lib().kno_philox4x32_10(c.ctypes.data_as(u32p), k.ctypes.data_as(u32p), out.ctypes.data_as(u32p))
    return out


def onb(n):
    n = _vec(n)
    b1, b2 = np.zeros(3), np.zeros(3)
    lib().kno_onb(_dp(n), _dp(b1), _dp(b2))
    return b1, b2


def cosine_dir(n, u1: float, u2: float) -> np.ndarray:
    n = _vec(n)
    out = np.zeros(3)
    lib().kno_cosine_dir(_dp(n), u1, u2, _dp(out))
    return out


def env_lookup(env, d) -> np.ndarray:
    e = _make_env(env)
    d = _vec(d)
    out = np.zeros(3)
    lib().kno_env_lookup(C.byref(e), _dp(d), _dp(out))
    return out


def make_camera(view, width, height, max_steps, eps, background=(0.0, 0.0, 0.0),
                unclamped: bool = False) -> _Camera:
    return _Camera((C.c_double * 3)(*view.eye), (C.c_double * 3)(*view.look_at),
                   (C.c_double * 3)(*view.up), float(view.tan_half_diag), width, height,
                   max_steps, eps, (C.c_double * 3)(*background),
                   STEP_UNCLAMPED if unclamped else STEP_CLAMPED)


def encode(p, L: int) -> np.ndarray:
    x = _vec(p)
    out = np.zeros(x.size + 2 * x.size * L)
    lib().kno_encode(_dp(x), x.size, L, _dp(out))
    return out


def softplus(u: float, beta: float = 100.0) -> float:
    return lib().kno_softplus(float(u), float(beta))


def camera_ray(view, width, height, row, col, xi1=0.5, xi2=0.5):
    cam = make_camera(view, width, height, 1, 1e-4)
    o, d = np.zeros(3), np.zeros(3)
    lib().kno_camera_ray(C.byref(cam), row, col, xi1, xi2, _dp(o), _dp(d))
    return o, d


def prim_hit(kind: int, params, o, d, t_min: float = 0.0):
    """Closest hit of one primitive past t_min: (hit, t, facing normal)."""
    pr = _Prim(kind, (C.c_double * 9)(*(list(params) + [0.0] * (9 - len(params)))), (C.c_double * 3)(0, 0, 0))
    t = C.c_double()
    n = np.zeros(3)
    ok = lib().kno_prim_hit(C.byref(pr), _dp(_vec(o)), _dp(_vec(d)), float(t_min), C.byref(t), _dp(n))
    return bool(ok), t.value, n


class OracleWorld:
    """A shared scene: KiloNeuS instances (OracleScene, translation, uniform
    scale) and Lambertian primitives (kind, params, albedo)."""

    def __init__(self, instances=(), prims=()):
        self._scenes = [sc for sc, _, _ in instances]   # keep the scenes alive
        n_i, n_p = len(instances), len(prims)
        self._inst = (_Instance * max(1, n_i))()
        for k, (sc, t, s_) in enumerate(instances):
            self._inst[k] = _Instance(C.pointer(sc.c), (C.c_double * 3)(*t), float(s_))
        self._prim = (_Prim * max(1, n_p))()
        for k, (kind, params, alb) in enumerate(prims):
            ps = list(params) + [0.0] * (9 - len(params))
            self._prim[k] = _Prim(kind, (C.c_double * 9)(*ps), (C.c_double * 3)(*alb))
        self.w = _World(n_i, self._inst, n_p, self._prim)

    def render(self, view, width: int, height: int, max_steps: int, eps: float, pixels=None,
               background=(0.0, 0.0, 0.0), nthreads: int = 0, unclamped: bool = False) -> dict:
        cam = make_camera(view, width, height, max_steps, eps, background, unclamped)
        if pixels is None:
            npix, pix_ptr = width * height, None
        else:
            pixels = np.ascontiguousarray(pixels, np.int64)
            npix, pix_ptr = pixels.size, pixels.ctypes.data
        rgb, depth, normal = np.zeros((npix, 3)), np.zeros(npix), np.zeros((npix, 3))
        hit, obj = np.zeros(npix, np.uint8), np.zeros(npix, np.int32)
        lib().kno_world_render(C.byref(self.w), C.byref(cam), pix_ptr, npix, _dp(rgb), _dp(depth), _dp(normal),
                               hit.ctypes.data_as(C.POINTER(C.c_uint8)), obj.ctypes.data_as(C.POINTER(C.c_int32)),
                               nthreads)
        return dict(rgb=rgb, depth=depth, normal=normal, hit=hit, object=obj)

    def path_trace(self, view, width: int, height: int, max_steps: int, eps: float, spp: int, bounces: int,
                   seed: int, env=None, pixels=None, nthreads: int = 0, jitter: bool = False,
                   unclamped: bool = False) -> dict:
        cam = make_camera(view, width, height, max_steps, eps, unclamped=unclamped)
        pt = _PT(spp, bounces, seed, _make_env(env), 1 if jitter else 0)
        if pixels is None:
            npix, pix_ptr = width * height, None
        else:
            pixels = np.ascontiguousarray(pixels, np.int64)
            npix, pix_ptr = pixels.size, pixels.ctypes.data
        rgb, depth, normal, hit = np.zeros((npix, 3)), np.zeros(npix), np.zeros((npix, 3)), np.zeros(npix, np.uint8)
        lib().kno_world_path_trace(C.byref(self.w), C.byref(cam), C.byref(pt), pix_ptr, npix, _dp(rgb), _dp(depth),
                                   _dp(normal), hit.ctypes.data_as(C.POINTER(C.c_uint8)), nthreads)
        return dict(rgb=rgb, depth=depth, normal=normal, hit=hit)
