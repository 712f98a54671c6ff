"""ctypes binding of the FP64 oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU product path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

NCOUNT = 10
COUNTER_NAMES = ["closest_rays", "closest_nodes", "closest_tris", "shadow_rays", "shadow_nodes",
                 "shadow_tris", "hits", "nee_visible", "candidates", "primary_miss"]


class _Field(C.Structure):
    _fields_ = [("levels", C.c_int32), ("log2_table", C.c_int32), ("n_min", C.c_int32), ("n_max", C.c_int32),
                ("lo", C.c_float * 3), ("hi", C.c_float * 3), ("table", C.c_void_p), ("w1", C.c_void_p),
                ("b1", C.c_void_p), ("w2", C.c_void_p), ("b2", C.c_void_p)]


class _Scene(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("nv", C.c_int32), ("faces", C.c_void_p), ("nf", C.c_int32),
                ("uv", C.c_void_p), ("mat_mode", C.c_int32), ("vmat", C.c_void_p),
                ("albedo", C.c_void_p), ("rough", C.c_void_p), ("metal", C.c_void_p),
                ("tw", C.c_int32), ("th", C.c_int32), ("env", C.c_void_p), ("ew", C.c_int32),
                ("eh", C.c_int32), ("field", C.c_void_p)]


class _View(C.Structure):
    _fields_ = [("c2w", C.c_float * 16), ("fov_y_deg", C.c_float), ("w", C.c_int32), ("h", C.c_int32),
                ("spp", C.c_int32), ("sample_offset", C.c_uint32)]


class _Reuse(C.Structure):
    _fields_ = [("spatial", C.c_int32), ("radius", C.c_int32), ("temporal", C.c_int32), ("m_cap", C.c_int32),
                ("prev", C.c_void_p), ("out", C.c_void_p)]


class _Options(C.Structure):
    _fields_ = [("bounces", C.c_int32), ("ris_m", C.c_int32), ("ris_m_brdf", C.c_int32),
                ("rr_start", C.c_int32), ("seed", C.c_uint64), ("brdf", C.c_int32),
                ("background", C.c_int32), ("grad_mode", C.c_int32), ("reuse", C.c_void_p),
                ("jitter", C.c_double), ("jitter_seed", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from .build import build as _build
            _build()
        _lib = C.CDLL(LIB_PATH)
        d, i32, i64, p = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        _lib.orc_create.restype = p
        _lib.orc_create.argtypes = [C.POINTER(_Scene), i32]
        _lib.orc_destroy.argtypes = [p]
        _lib.orc_philox.argtypes = [p, p, p]
        _lib.orc_render.restype = i32
        _lib.orc_render.argtypes = [p, p, i32, C.POINTER(_Options), p, i64, p, p, p, i32]
        _lib.orc_grad.restype = i32
        _lib.orc_grad.argtypes = [p, p, i32, C.POINTER(_Options), p, i64, p, p, p, p, p, p, i32]
        _lib.orc_grad_field.restype = i32
        _lib.orc_grad_field.argtypes = [p, p, i32, C.POINTER(_Options), p, i64, p, p, p, p, p, p, p, i32]
        _lib.orc_field_eval.restype = i32
        _lib.orc_field_eval.argtypes = [C.POINTER(_Field), p, i64, p]
        _lib.orc_field_vjp.restype = i32
        _lib.orc_field_vjp.argtypes = [C.POINTER(_Field), p, p, i64, p, p, p, p, p]
        _lib.orc_field_levels.restype = i32
        _lib.orc_field_levels.argtypes = [C.POINTER(_Field), p]
        _lib.orc_reuse_offset.restype = i32
        _lib.orc_reuse_offset.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, i32, i32,
                                          C.POINTER(i32), C.POINTER(i32)]
        _lib.orc_frozen.restype = i32
        _lib.orc_frozen.argtypes = [p, p, p, i32, C.POINTER(_Options), p, p]
        _lib.orc_trace.restype = i32
        _lib.orc_trace.argtypes = [p, p, p, i64, i32, i32, p, p, p, p]
        _lib.orc_env_sample.restype = i32
        _lib.orc_env_sample.argtypes = [p, d, d, p, p, p]
        _lib.orc_env_pdf.restype = d
        _lib.orc_env_pdf.argtypes = [p, p]
        _lib.orc_env_lookup.restype = i32
        _lib.orc_env_lookup.argtypes = [p, p, p]
        _lib.orc_brdf_eval.argtypes = [p, p, p, p, i32, p]
        _lib.orc_brdf_pdf.restype = d
        _lib.orc_brdf_pdf.argtypes = [p, p, p, p, i32]
        _lib.orc_brdf_sample.restype = i32
        _lib.orc_brdf_sample.argtypes = [p, p, p, i32, p, p]
        _lib.orc_ggx_d.restype = d
        _lib.orc_ggx_d.argtypes = [d, d]
        _lib.orc_ggx_g1.restype = d
        _lib.orc_ggx_g1.argtypes = [d, d]
        _lib.orc_frame.argtypes = [p, p, p]
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def reuse_offset(seed: int, pixel: int, sample: int, view: int, j: int, radius: int):
    dx, dy = C.c_int32(), C.c_int32()
    if lib().orc_reuse_offset(seed, pixel, sample, view, j, radius, C.byref(dx), C.byref(dy)) != 0:
        raise ValueError("oracle.reuse_offset: invalid arguments")
    return dx.value, dy.value


def philox(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def views_struct(views) -> C.Array:
    arr = (_View * len(views))()
    for i, v in enumerate(views):
        arr[i].c2w[:] = [float(x) for x in np.asarray(v.c2w, np.float32).reshape(16)]
        arr[i].fov_y_deg = float(v.fov_y_deg)
        arr[i].w, arr[i].h, arr[i].spp = int(v.w), int(v.h), int(v.spp)
        arr[i].sample_offset = int(v.sample_offset)
    return arr


def reuse_struct(o, prev: Optional[np.ndarray] = None, out: Optional[np.ndarray] = None) -> Optional[_Reuse]:
    """Reservoir-reuse settings of options `o` (None when reuse is off)."""
    sp, tm = int(getattr(o, "reuse_spatial", 0)), int(getattr(o, "reuse_temporal", 0))
    if sp <= 0 and not tm:
        return None
    return _Reuse(sp, int(getattr(o, "reuse_radius", 16)), tm, int(getattr(o, "reuse_m_cap", 20)), _ptr(prev),
                  _ptr(out))


def options_struct(o, reuse: Optional[_Reuse] = None) -> _Options:
    """The C options; `jitter` / `jitter_seed` attributes of `o`, when
    present, switch on the conditioning hook (orc_options.jitter)."""
    return _Options(int(o.bounces), int(o.ris_m), int(o.ris_m_brdf), int(o.rr_start), int(o.seed),
                    int(o.brdf), int(o.background), int(o.grad_mode),
                    C.addressof(reuse) if reuse is not None else None,
                    float(getattr(o, "jitter", 0.0)), int(getattr(o, "jitter_seed", 0)) & (2 ** 64 - 1))


class FieldRef:
    """The material field alone (TEST INFRASTRUCTURE): FP64 evaluation and
    pull-back of the C oracle over float32 parameters."""

    def __init__(self, field):
        self.f = field
        self._keep = [np.ascontiguousarray(a, np.float32) for a in (field.table, field.w1, field.b1, field.w2,
                                                                      field.b2)]
        t, w1, b1, w2, b2 = self._keep
        L, T = t.shape[0], t.shape[1]
        assert T & (T - 1) == 0 and t.shape[2] == 2 and w1.shape == (32, 2 * L)
        self.s = _Field(L, T.bit_length() - 1, int(field.n_min), int(field.n_max),
                        (C.c_float * 3)(*[float(v) for v in field.lo]), (C.c_float * 3)(*[float(v) for v in field.hi]),
                        _ptr(t), _ptr(w1), _ptr(b1), _ptr(w2), _ptr(b2))

    def levels(self) -> np.ndarray:
        res = np.zeros(16, np.int64)
        n = lib().orc_field_levels(C.byref(self.s), _ptr(res))
        if n < 0:
            raise ValueError("oracle: invalid field")
        return res[:n]

    def eval(self, x) -> np.ndarray:
        x = _d(x).reshape(-1, 3)
        m = np.zeros((x.shape[0], 4))
        if lib().orc_field_eval(C.byref(self.s), _ptr(x), x.shape[0], _ptr(m)) != 0:
            raise ValueError("oracle: invalid field")
        return m

    def vjp(self, x, g) -> Dict[str, np.ndarray]:
        x = _d(x).reshape(-1, 3)
        g = _d(g).reshape(-1, 4)
        out = {k: np.zeros(a.shape) for k, a in zip(("table", "w1", "b1", "w2", "b2"), self._keep)}
        rc = lib().orc_field_vjp(C.byref(self.s), _ptr(x), _ptr(g), x.shape[0], _ptr(out["table"]),
                                 _ptr(out["w1"]), _ptr(out["b1"]), _ptr(out["w2"]), _ptr(out["b2"]))
        if rc != 0:
            raise ValueError("oracle: invalid field")
        return out


class Oracle:
    """FP64 reference renderer over one scene (mesh, materials, env)."""

    def __init__(self, scene, use_bvh: bool = True):
        self._keep = dict(pos=_f32(scene.pos), faces=np.ascontiguousarray(scene.faces, np.int32),
                          uv=_f32(scene.uv), vmat=_f32(scene.vmat), albedo=_f32(scene.albedo),
                          rough=_f32(scene.rough), metal=_f32(scene.metal), env=_f32(scene.env))
        k = self._keep
        tw = th = 0
        if scene.mat_mode == 1:
            th, tw = k["rough"].shape
        self.scene = scene
        self.field = FieldRef(scene.field) if scene.mat_mode == 2 else None
        s = _Scene(_ptr(k["pos"]), k["pos"].shape[0], _ptr(k["faces"]), k["faces"].shape[0], _ptr(k["uv"]),
                   int(scene.mat_mode), _ptr(k["vmat"]), _ptr(k["albedo"]), _ptr(k["rough"]),
                   _ptr(k["metal"]), tw, th, _ptr(k["env"]), k["env"].shape[1], k["env"].shape[0],
                   C.addressof(self.field.s) if self.field else None)
        self._h = lib().orc_create(C.byref(s), 1 if use_bvh else 0)
        if not self._h:
            raise ValueError("oracle: invalid scene")

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    # ---------------------------------------------------------------- render
    def render(self, views, opts, items: np.ndarray, nthreads: int = 0, counters: bool = False,
               prev: Optional[np.ndarray] = None, reservoirs: bool = False):
        """Per-item radiance and decision hashes.  With reservoir reuse in
        `opts`, prev [S, 8] is the previous frame's records by global sample
        index, and reservoirs=True also returns each item's final record."""
        items = np.ascontiguousarray(items, np.int32).reshape(-1, 3)
        n = items.shape[0]
        rgb = np.zeros((n, 3))
        hsh = np.zeros(n, np.uint32)
        cnt = np.zeros(NCOUNT, np.int64)
        nt = nthreads or os.cpu_count() or 1
        vs = views_struct(views)
        prev = None if prev is None else np.ascontiguousarray(prev, np.float32).reshape(-1, 8)
        res = np.zeros((n, 8)) if reservoirs else None
        ru = reuse_struct(opts, prev, res)
        op = options_struct(opts, ru)
        rc = lib().orc_render(self._h, C.addressof(vs), len(views), C.byref(op), _ptr(items), n,
                              _ptr(rgb), _ptr(hsh), _ptr(cnt), nt)
        if rc != 0:
            raise ValueError("oracle.render: invalid arguments")
        out = [rgb, hsh]
        if counters:
            out.append(dict(zip(COUNTER_NAMES, cnt.tolist())))
        if reservoirs:
            out.append(res)
        return tuple(out)

    def grad(self, views, opts, items: np.ndarray, dldc: np.ndarray, nthreads: int = 0,
             prev: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
        items = np.ascontiguousarray(items, np.int32).reshape(-1, 3)
        dldc = _d(dldc).reshape(-1, 3)
        assert dldc.shape[0] == items.shape[0]
        sc = self.scene
        g = {"env": np.zeros(sc.env.shape)}
        vs = views_struct(views)
        prev = None if prev is None else np.ascontiguousarray(prev, np.float32).reshape(-1, 8)
        ru = reuse_struct(opts, prev)
        op = options_struct(opts, ru)
        nt = nthreads or os.cpu_count() or 1
        if sc.mat_mode == 2:
            for k, a in zip(("table", "w1", "b1", "w2", "b2"), self.field._keep):
                g[k] = np.zeros(a.shape)
            rc = lib().orc_grad_field(self._h, C.addressof(vs), len(views), C.byref(op), _ptr(items),
                                      items.shape[0], _ptr(dldc), _ptr(g["table"]), _ptr(g["w1"]), _ptr(g["b1"]),
                                      _ptr(g["w2"]), _ptr(g["b2"]), _ptr(g["env"]), nt)
            if rc != 0:
                raise ValueError("oracle.grad: invalid arguments")
            return g
        if sc.mat_mode == 0:
            g["vmat"] = np.zeros(sc.vmat.shape)
        else:
            g["albedo"] = np.zeros(sc.albedo.shape)
            g["rough"] = np.zeros(sc.rough.shape)
            g["metal"] = np.zeros(sc.metal.shape)
        rc = lib().orc_grad(self._h, C.addressof(vs), len(views), C.byref(op), _ptr(items), items.shape[0],
                            _ptr(dldc), _ptr(g.get("vmat")), _ptr(g.get("albedo")), _ptr(g.get("rough")),
                            _ptr(g.get("metal")), _ptr(g["env"]), nt)
        if rc != 0:
            raise ValueError("oracle.grad: invalid arguments")
        return g

    def frozen(self, eval_oracle: "Oracle", views, opts, item, prev: Optional[np.ndarray] = None) -> np.ndarray:
        it = np.ascontiguousarray(item, np.int32).reshape(3)
        out = np.zeros(3)
        vs = views_struct(views)
        prev = None if prev is None else np.ascontiguousarray(prev, np.float32).reshape(-1, 8)
        ru = reuse_struct(opts, prev)
        op = options_struct(opts, ru)
        rc = lib().orc_frozen(self._h, eval_oracle._h, C.addressof(vs), len(views), C.byref(op), _ptr(it),
                              _ptr(out))
        if rc != 0:
            raise ValueError("oracle.frozen: invalid arguments")
        return out

    # ----------------------------------------------------------- test hooks
    def trace(self, o, d, any_hit: bool = False, brute: bool = False):
        o = _d(o).reshape(-1, 3)
        d = _d(d).reshape(-1, 3)
        n = o.shape[0]
        prim = np.zeros(n, np.int32)
        t, b1, b2 = np.zeros(n), np.zeros(n), np.zeros(n)
        lib().orc_trace(self._h, _ptr(o), _ptr(d), n, int(any_hit), int(brute), _ptr(prim), _ptr(t), _ptr(b1),
                        _ptr(b2))
        return prim, t, b1, b2

    def env_sample(self, u0: float, u1: float):
        dvec = np.zeros(3)
        pdf = np.zeros(1)
        tex = np.zeros(1, np.int32)
        ok = lib().orc_env_sample(self._h, float(u0), float(u1), _ptr(dvec), _ptr(pdf), _ptr(tex))
        return bool(ok), dvec, float(pdf[0]), int(tex[0])

    def env_pdf(self, d) -> float:
        return float(lib().orc_env_pdf(self._h, _ptr(_d(d))))

    def env_lookup(self, d):
        out = np.zeros(3)
        t = lib().orc_env_lookup(self._h, _ptr(_d(d)), _ptr(out))
        return int(t), out


def brdf_eval(n, wo, wi, m, brdf: int = 1) -> np.ndarray:
    f = np.zeros(3)
    lib().orc_brdf_eval(_ptr(_d(n)), _ptr(_d(wo)), _ptr(_d(wi)), _ptr(_d(m)), int(brdf), _ptr(f))
    return f


def brdf_pdf(n, wo, wi, m, brdf: int = 1) -> float:
    return float(lib().orc_brdf_pdf(_ptr(_d(n)), _ptr(_d(wo)), _ptr(_d(wi)), _ptr(_d(m)), int(brdf)))


def brdf_sample(n, wo, m, u, brdf: int = 1):
    wi = np.zeros(3)
    lobe = lib().orc_brdf_sample(_ptr(_d(n)), _ptr(_d(wo)), _ptr(_d(m)), int(brdf), _ptr(_d(u)), _ptr(wi))
    return int(lobe), wi


def ggx_d(alpha: float, cos_h: float) -> float:
    return float(lib().orc_ggx_d(float(alpha), float(cos_h)))


def ggx_g1(alpha: float, cos_w: float) -> float:
    return float(lib().orc_ggx_g1(float(alpha), float(cos_w)))


def frame(n):
    t, b = np.zeros(3), np.zeros(3)
    lib().orc_frame(_ptr(_d(n)), _ptr(t), _ptr(b))
    return t, b
