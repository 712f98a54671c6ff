"""Python binding of libmirres (include/mirres.h): argument marshalling only.

Every step of the rendering path runs in the HIP library.  PyTorch provides
device memory and the current stream.  If the library is missing the import
of this module fails: there is no CPU fallback.

    bvh   = build_bvh(pos, faces)                       # pos [nv,3], faces [nf,3] on cuda
    scene = GpuScene(pos, faces, env, vmat=...)         # or uv/albedo/rough/metal
    img   = render(scene, views, RenderOptions(...))    # [sum W*H, 3]
    img   = render_autograd(scene, views, opts)         # differentiable w.r.t. materials and env
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Dict, List, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# MIRRES_LIB selects another build of the same library (e.g. a variant for an A/B timing run)
LIB_PATH = os.environ.get("MIRRES_LIB") or os.path.join(_HERE, "libmirres.so")

MRS_OK, MRS_EINVAL, MRS_ENOMEM, MRS_EHIP, MRS_EOVERFLOW, MRS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
MAT_VERTEX, MAT_TEXTURE, MAT_FIELD = 0, 1, 2
FIELD_KEYS = ("table", "w1", "b1", "w2", "b2")
TAPE_AUTO, TAPE_ON, TAPE_OFF = 0, 1, 2


class MirresError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mirres error {code}: {msg}")
        self.code = code


class _Field(C.Structure):
    _fields_ = [("levels", C.c_int32), ("log2_table", C.c_int32), ("n_min", C.c_int32), ("n_max", C.c_int32),
                ("lo", C.c_float * 3), ("hi", C.c_float * 3), ("table", C.c_void_p), ("w1", C.c_void_p),
                ("b1", C.c_void_p), ("w2", C.c_void_p), ("b2", C.c_void_p)]


class _FieldGrads(C.Structure):
    _fields_ = [("table", C.c_void_p), ("w1", C.c_void_p), ("b1", C.c_void_p), ("w2", C.c_void_p),
                ("b2", C.c_void_p)]


class _Scene(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("nv", C.c_int32), ("faces", C.c_void_p), ("nf", C.c_int32),
                ("uv", C.c_void_p), ("bvh", C.c_void_p), ("mat_mode", C.c_int32), ("vmat", C.c_void_p),
                ("albedo", C.c_void_p), ("rough", C.c_void_p), ("metal", C.c_void_p), ("tw", C.c_int32),
                ("th", C.c_int32), ("env", C.c_void_p), ("ew", C.c_int32), ("eh", C.c_int32), ("field", _Field)]


class _View(C.Structure):
    _fields_ = [("c2w", C.c_float * 16), ("fov_y_deg", C.c_float), ("w", C.c_int32), ("h", C.c_int32),
                ("spp", C.c_int32), ("sample_offset", C.c_uint32), ("pixel_offset", C.c_int64)]


class _Options(C.Structure):
    _fields_ = [("bounces", C.c_int32), ("ris_m", C.c_int32), ("ris_m_brdf", C.c_int32), ("rr_start", C.c_int32),
                ("seed", C.c_uint64), ("brdf", C.c_int32), ("background", C.c_int32), ("grad_mode", C.c_int32),
                ("tape_mode", C.c_int32), ("tape_budget", C.c_int64), ("pool", C.c_int32), ("block", C.c_int32),
                ("debug_sample_rgb", C.c_void_p), ("debug_hash", C.c_void_p), ("reuse_spatial", C.c_int32),
                ("reuse_radius", C.c_int32), ("reuse_temporal", C.c_int32), ("reuse_m_cap", C.c_int32),
                ("reservoir_prev", C.c_void_p), ("reservoir_out", C.c_void_p), ("deterministic", C.c_int32)]


class _Grads(C.Structure):
    _fields_ = [("vmat", C.c_void_p), ("albedo", C.c_void_p), ("rough", C.c_void_p), ("metal", C.c_void_p),
                ("env", C.c_void_p), ("field", _FieldGrads)]


def _grads_struct(grads: Dict[str, Optional[torch.Tensor]]) -> _Grads:
    fg = _FieldGrads(*[_ptr(grads.get(k)) for k in FIELD_KEYS])
    return _Grads(_ptr(grads.get("vmat")), _ptr(grads.get("albedo")), _ptr(grads.get("rough")),
                  _ptr(grads.get("metal")), _ptr(grads.get("env")), fg)


# BVH builders (MRS_BVH_*).  Scenes built here default to PLOC: on the
# 300k-triangle workload it needs 15 % fewer box tests per shadow ray than the
# LBVH (the C entry point mrs_build_bvh keeps the paper's LBVH).
BVH_LBVH, BVH_PLOC = 0, 1
DEFAULT_BUILDER = int(os.environ.get("MIRRES_BVH_BUILDER", BVH_PLOC))

# the C-ABI symbols declared in include/mirres.h
EXPORTS = ["mrs_build_bvh", "mrs_build_bvh_with", "mrs_bvh_refit", "mrs_bvh_destroy", "mrs_bvh_info", "mrs_trace", "mrs_render", "mrs_render_backward",
           "mrs_plan_create", "mrs_plan_forward", "mrs_plan_backward", "mrs_plan_info", "mrs_plan_destroy",
           "mrs_tape_bytes", "mrs_tape_destroy", "mrs_gbuffer", "mrs_denoise_work_bytes", "mrs_denoise",
           "mrs_denoise_backward", "mrs_denoise_noalloc", "mrs_field_eval", "mrs_field_backward", "mrs_profile_begin", "mrs_profile_end",
           "mrs_sort_pairs_tmp_bytes", "mrs_sort_pairs_u32", "mrs_release_workspace", "mrs_last_error"]


class _KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("ms", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2406_16360_amd/csrc/build.py "
                          "(there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    p, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.mrs_build_bvh.restype = i32
    lib.mrs_build_bvh.argtypes = [p, i32, p, i32, p, C.POINTER(p)]
    lib.mrs_build_bvh_with.restype = i32
    lib.mrs_build_bvh_with.argtypes = [p, i32, p, i32, i32, p, C.POINTER(p)]
    lib.mrs_bvh_refit.restype = i32
    lib.mrs_bvh_refit.argtypes = [p, p, i32, p]
    lib.mrs_gbuffer.restype = i32
    lib.mrs_gbuffer.argtypes = [p, p, i32, p, p, p]
    lib.mrs_denoise_work_bytes.restype = i64
    lib.mrs_denoise_work_bytes.argtypes = [p, i32, p]
    lib.mrs_denoise.restype = i32
    lib.mrs_denoise.argtypes = [p, i32, p, p, p, p, p, p, p]
    lib.mrs_denoise_backward.restype = i32
    lib.mrs_denoise_backward.argtypes = [p, i32, p, p, p, p, p, p, p]
    lib.mrs_denoise_noalloc.restype = i32
    lib.mrs_denoise_noalloc.argtypes = [p, i32, p, p, p, p, p, p]
    lib.mrs_field_eval.restype = i32
    lib.mrs_field_eval.argtypes = [C.POINTER(_Field), p, i64, p, p]
    lib.mrs_field_backward.restype = i32
    lib.mrs_field_backward.argtypes = [C.POINTER(_Field), p, p, i64, C.POINTER(_FieldGrads), p]
    lib.mrs_bvh_destroy.argtypes = [p]
    lib.mrs_bvh_info.restype = i32
    lib.mrs_bvh_info.argtypes = [p, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    lib.mrs_trace.restype = i32
    lib.mrs_trace.argtypes = [p, p, p, i64, i32, p, p]
    lib.mrs_render.restype = i32
    lib.mrs_render.argtypes = [C.POINTER(_Scene), p, i32, C.POINTER(_Options), p, C.POINTER(p), p]
    lib.mrs_render_backward.restype = i32
    lib.mrs_render_backward.argtypes = [C.POINTER(_Scene), p, i32, C.POINTER(_Options), p, C.POINTER(_Grads), p, p]
    lib.mrs_tape_bytes.restype = i64
    lib.mrs_tape_bytes.argtypes = [p, i32, C.POINTER(_Options)]
    lib.mrs_tape_destroy.argtypes = [p]
    lib.mrs_release_workspace.argtypes = []
    lib.mrs_profile_begin.restype = i32
    lib.mrs_profile_begin.argtypes = []
    lib.mrs_profile_end.restype = i32
    lib.mrs_profile_end.argtypes = [p, i32, C.POINTER(i32)]
    lib.mrs_plan_create.restype = i32
    lib.mrs_plan_create.argtypes = [C.POINTER(_Scene), p, i32, C.POINTER(_Options), p, p, C.POINTER(_Grads), i32,
                                    C.POINTER(p)]
    lib.mrs_plan_forward.restype = i32
    lib.mrs_plan_forward.argtypes = [p, p]
    lib.mrs_plan_backward.restype = i32
    lib.mrs_plan_backward.argtypes = [p, p]
    lib.mrs_plan_info.restype = i32
    lib.mrs_plan_info.argtypes = [p, C.POINTER(i64), C.POINTER(i32), C.POINTER(i32)]
    lib.mrs_plan_destroy.argtypes = [p]
    lib.mrs_sort_pairs_tmp_bytes.restype = C.c_size_t
    lib.mrs_sort_pairs_tmp_bytes.argtypes = [i64]
    lib.mrs_sort_pairs_u32.restype = i32
    lib.mrs_sort_pairs_u32.argtypes = [p, p, p, p, i64, p, C.c_size_t, p]
    lib.mrs_last_error.restype = C.c_char_p
    return lib


_lib = _load()


def lib():
    return _lib


def _check(code: int):
    if code != MRS_OK:
        raise MirresError(code, (_lib.mrs_last_error() or b"").decode())


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev(t: Optional[torch.Tensor], dtype=torch.float32) -> Optional[torch.Tensor]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("mirres: tensors must be on the GPU")
    return t.detach().to(dtype).contiguous()


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _need(t: Optional[torch.Tensor], name: str, shape, dtype=torch.float32) -> None:
    """Caller-supplied buffers the kernels write or read by element count:
    contiguous GPU tensors of exactly this dtype and shape (None passes)."""
    if t is None:
        return
    shape = tuple(int(x) for x in shape)
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous() \
            or tuple(t.shape) != shape:
        got = (f"{'cuda' if t.is_cuda else 'cpu'} {t.dtype} {tuple(t.shape)} "
               f"{'contiguous' if t.is_contiguous() else 'strided'}") if isinstance(t, torch.Tensor) else type(t)
        raise ValueError(f"mirres: {name} must be a contiguous {dtype} GPU tensor of shape {shape}, got {got}")


def _overlap(a: Optional[torch.Tensor], b: Optional[torch.Tensor]) -> bool:
    if a is None or b is None:
        return False
    a0, b0 = a.data_ptr(), b.data_ptr()
    return a0 < b0 + b.numel() * b.element_size() and b0 < a0 + a.numel() * a.element_size()


@dataclasses.dataclass
class RenderOptions:
    bounces: int = 3
    ris_m: int = 32
    ris_m_brdf: int = 16
    rr_start: int = -1
    seed: int = 1
    brdf: int = 1
    background: int = 0
    grad_mode: int = 0
    tape_mode: int = TAPE_AUTO
    tape_budget: int = 0
    pool: int = 0
    block: int = 0
    reuse_spatial: int = 0
    reuse_radius: int = 16
    reuse_temporal: int = 0
    reuse_m_cap: int = 20
    deterministic: int = 0

    @classmethod
    def from_any(cls, o) -> "RenderOptions":
        if isinstance(o, cls):
            return o
        names = [f.name for f in dataclasses.fields(cls)]
        return cls(**{n: getattr(o, n) for n in names if hasattr(o, n)})

    def struct(self, debug_rgb=None, debug_hash=None, reservoir_prev=None, reservoir_out=None) -> _Options:
        return _Options(self.bounces, self.ris_m, self.ris_m_brdf, self.rr_start, self.seed & (2 ** 64 - 1), self.brdf,
                        self.background, self.grad_mode, self.tape_mode, self.tape_budget, self.pool, self.block,
                        _ptr(debug_rgb), _ptr(debug_hash), self.reuse_spatial, self.reuse_radius,
                        self.reuse_temporal, self.reuse_m_cap, _ptr(reservoir_prev), _ptr(reservoir_out),
                        self.deterministic)


class Bvh:
    """BVH over a triangle mesh (library-owned), built on the GPU over the
    Morton order of the triangles: builder BVH_LBVH (the paper's linear BVH)
    or BVH_PLOC (locally-ordered clustering, fewer node visits per ray)."""

    def __init__(self, pos: torch.Tensor, faces: torch.Tensor, stream=None, builder: Optional[int] = None):
        pos = _dev(pos)
        faces = _dev(faces, torch.int32)
        h = C.c_void_p()
        b = DEFAULT_BUILDER if builder is None else builder
        _check(_lib.mrs_build_bvh_with(pos.data_ptr(), pos.shape[0], faces.data_ptr(), faces.shape[0], b,
                                       _stream(stream), C.byref(h)))
        self._h = h
        self.nf = int(faces.shape[0])

    @property
    def handle(self):
        return self._h

    def refit(self, pos: torch.Tensor, stream=None) -> None:
        """Moves the triangles to new positions of the same vertices and
        recomputes every box over the unchanged tree."""
        pos = _dev(pos)
        _check(_lib.mrs_bvh_refit(self._h, pos.data_ptr(), pos.shape[0], _stream(stream)))

    def info(self) -> Tuple[int, int, int]:
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib.mrs_bvh_info(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def trace(self, orig: torch.Tensor, dirs: torch.Tensor, any_hit: bool = False, stream=None) -> torch.Tensor:
        o = _dev(orig)
        d = _dev(dirs)
        out = torch.empty((o.shape[0], 4), dtype=torch.float32, device=o.device)
        _check(_lib.mrs_trace(self._h, o.data_ptr(), d.data_ptr(), o.shape[0], int(any_hit), out.data_ptr(),
                              _stream(stream)))
        return out

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mrs_bvh_destroy(self._h)
            self._h = None


def build_bvh(pos: torch.Tensor, faces: torch.Tensor, stream=None, builder: Optional[int] = None) -> Bvh:
    return Bvh(pos, faces, stream, builder=builder)


class Tape:
    """Per-vertex path records kept by render() for render_backward()."""

    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mrs_tape_destroy(self._h)
            self._h = None


class Field:
    """Material field F_m (hash-grid encoding + 2-layer MLP, include/mirres.h
    mrs_field) as GPU float32 tensors: table [L, T, 2], w1 [32, 2L], b1 [32],
    w2 [4, 32], b2 [4], over the box [lo, hi]."""

    def __init__(self, table, w1, b1, w2, b2, lo, hi, n_min: int = 16, n_max: int = 2048, device="cuda"):
        dev = torch.device(device)
        t = lambda x: torch.as_tensor(x).to(device=dev, dtype=torch.float32).contiguous()
        self.table, self.w1, self.b1, self.w2, self.b2 = t(table), t(w1), t(b1), t(w2), t(b2)
        self.lo = [float(v) for v in torch.as_tensor(lo).reshape(3).tolist()]
        self.hi = [float(v) for v in torch.as_tensor(hi).reshape(3).tolist()]
        self.n_min, self.n_max = int(n_min), int(n_max)
        T = int(self.table.shape[1])
        if T & (T - 1) or self.table.dim() != 3 or self.table.shape[2] != 2:
            raise ValueError("field table must be [L, 2^k, 2]")

    @classmethod
    def from_synth(cls, f, device="cuda") -> "Field":
        return cls(f.table, f.w1, f.b1, f.w2, f.b2, f.lo, f.hi, f.n_min, f.n_max, device=device)

    def with_params(self, **kw) -> "Field":
        f = object.__new__(Field)
        f.__dict__.update(self.__dict__)
        for k, v in kw.items():
            if v is not None:
                setattr(f, k, _dev(v))
        return f

    def zeros_like_params(self) -> Dict[str, torch.Tensor]:
        return {k: torch.zeros_like(getattr(self, k)) for k in FIELD_KEYS}

    def struct(self) -> _Field:
        L, T = int(self.table.shape[0]), int(self.table.shape[1])
        return _Field(L, T.bit_length() - 1, self.n_min, self.n_max, (C.c_float * 3)(*self.lo),
                      (C.c_float * 3)(*self.hi), _ptr(self.table), _ptr(self.w1), _ptr(self.b1), _ptr(self.w2),
                      _ptr(self.b2))

    def eval(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        """m [n, 4] = (albedo rgb, roughness) at the points x [n, 3]."""
        x = _dev(x).reshape(-1, 3)
        m = torch.empty((x.shape[0], 4), dtype=torch.float32, device=x.device)
        fs = self.struct()
        _check(_lib.mrs_field_eval(C.byref(fs), x.data_ptr(), x.shape[0], m.data_ptr(), _stream(stream)))
        return m

    def backward(self, x: torch.Tensor, grad_m: torch.Tensor, grads: Optional[Dict[str, torch.Tensor]] = None,
                 stream=None) -> Dict[str, torch.Tensor]:
        """Accumulates the pull-back of grad_m [n, 4] into `grads` (zeros if None)."""
        x = _dev(x).reshape(-1, 3)
        gm = _dev(grad_m).reshape(-1, 4)
        if grads is None:
            grads = self.zeros_like_params()
        fs = self.struct()
        fg = _FieldGrads(*[_ptr(grads.get(k)) for k in FIELD_KEYS])
        _check(_lib.mrs_field_backward(C.byref(fs), x.data_ptr(), gm.data_ptr(), x.shape[0], C.byref(fg),
                                       _stream(stream)))
        return grads


class GpuScene:
    """Mesh, materials and environment map as GPU float32 tensors."""

    def __init__(self, pos, faces, env, vmat=None, uv=None, albedo=None, rough=None, metal=None,
                 bvh: Optional[Bvh] = None, device="cuda", builder: Optional[int] = None,
                 field: Optional[Field] = None):
        dev = torch.device(device)

        def t(x, dt=torch.float32):
            if x is None:
                return None
            return torch.as_tensor(x).to(device=dev, dtype=dt).contiguous()

        self.pos = t(pos)
        self.faces = t(faces, torch.int32)
        self.env = t(env)
        self.vmat = t(vmat)
        self.uv = t(uv)
        self.albedo = t(albedo)
        self.rough = t(rough)
        self.metal = t(metal)
        self.field = field
        self.mat_mode = MAT_FIELD if field is not None else (MAT_VERTEX if self.vmat is not None else MAT_TEXTURE)
        self.bvh = bvh if bvh is not None else Bvh(self.pos, self.faces, builder=builder)

    @classmethod
    def from_synth(cls, sc, device="cuda", builder: Optional[int] = None) -> "GpuScene":
        field = Field.from_synth(sc.field, device=device) if sc.mat_mode == MAT_FIELD else None
        return cls(sc.pos, sc.faces, sc.env, vmat=sc.vmat if sc.mat_mode == 0 else None, uv=sc.uv,
                   albedo=sc.albedo, rough=sc.rough, metal=sc.metal, device=device, builder=builder, field=field)

    def with_params(self, vmat=None, albedo=None, rough=None, metal=None, env=None) -> "GpuScene":
        s = object.__new__(GpuScene)
        s.__dict__.update(self.__dict__)
        for k, v in dict(vmat=vmat, albedo=albedo, rough=rough, metal=metal, env=env).items():
            if v is not None:
                setattr(s, k, _dev(v))
        return s

    def struct(self) -> _Scene:
        tw = th = 0
        if self.mat_mode == MAT_TEXTURE:
            th, tw = self.rough.shape
        return _Scene(_ptr(self.pos), self.pos.shape[0], _ptr(self.faces), self.faces.shape[0], _ptr(self.uv),
                      self.bvh.handle, self.mat_mode, _ptr(self.vmat), _ptr(self.albedo), _ptr(self.rough),
                      _ptr(self.metal), tw, th, _ptr(self.env), self.env.shape[1], self.env.shape[0],
                      self.field.struct() if self.field is not None else _Field())

    def param_shapes(self) -> Dict[str, Tuple[int, ...]]:
        """Shapes of the parameter groups a gradient dict may hold."""
        sh = {"env": tuple(self.env.shape)}
        if self.mat_mode == MAT_VERTEX:
            sh["vmat"] = tuple(self.vmat.shape)
        elif self.mat_mode == MAT_FIELD:
            sh.update({k: tuple(getattr(self.field, k).shape) for k in FIELD_KEYS})
        else:
            sh.update(albedo=tuple(self.albedo.shape), rough=tuple(self.rough.shape), metal=tuple(self.metal.shape))
        return sh

    def check_grads(self, grads: Dict[str, Optional[torch.Tensor]]) -> None:
        """Every gradient buffer matches its parameter group (the adjoint
        adds into each element); unknown keys are an error."""
        sh = self.param_shapes()
        for k, t in grads.items():
            if t is None:
                continue
            if k not in sh:
                raise ValueError(f"mirres: no parameter group {k!r} in this scene (groups: {sorted(sh)})")
            _need(t, f"grads[{k!r}]", sh[k])

    def zero_grads(self) -> Dict[str, torch.Tensor]:
        """Zeroed gradient buffers for every parameter of the scene."""
        g = {"env": torch.zeros_like(self.env)}
        if self.mat_mode == MAT_VERTEX:
            g["vmat"] = torch.zeros_like(self.vmat)
        elif self.mat_mode == MAT_FIELD:
            g.update(self.field.zeros_like_params())
        else:
            g.update(albedo=torch.zeros_like(self.albedo), rough=torch.zeros_like(self.rough),
                     metal=torch.zeros_like(self.metal))
        return g


def views_struct(views: Sequence) -> Tuple[C.Array, int, List[int]]:
    """Packs views (objects with c2w, fov_y_deg, w, h, spp, sample_offset)
    back to back; returns the struct array, total pixels and per-view offsets."""
    arr = (_View * len(views))()
    off, offsets = 0, []
    for i, v in enumerate(views):
        c2w = torch.as_tensor(v.c2w, dtype=torch.float32).reshape(16).tolist()
        arr[i].c2w[:] = c2w
        arr[i].fov_y_deg = float(v.fov_y_deg)
        arr[i].w, arr[i].h, arr[i].spp = int(v.w), int(v.h), int(v.spp)
        arr[i].sample_offset = int(getattr(v, "sample_offset", 0))
        arr[i].pixel_offset = off
        offsets.append(off)
        off += int(v.w) * int(v.h)
    return arr, off, offsets


def total_samples(views: Sequence) -> int:
    return int(sum(int(v.w) * int(v.h) * int(v.spp) for v in views))


def render(scene: GpuScene, views: Sequence, opts, keep_tape: bool = False, debug: bool = False,
           out: Optional[torch.Tensor] = None, stream=None, reservoir_prev: Optional[torch.Tensor] = None,
           reservoir_out: Optional[torch.Tensor] = None):
    """Renders packed images [sum W*H, 3].  With keep_tape returns (image,
    tape or None); with debug also per-sample radiance and decision hashes.
    With reservoir reuse in opts, reservoir_prev / reservoir_out [S, 8] are
    the previous and this frame's final primary-vertex reservoirs."""
    o = RenderOptions.from_any(opts)
    vs, npix, _ = views_struct(views)
    dev = scene.pos.device
    S = total_samples(views)
    _need(out, "out", (npix, 3))
    _need(reservoir_prev, "reservoir_prev", (S, 8))
    _need(reservoir_out, "reservoir_out", (S, 8))
    if _overlap(reservoir_prev, reservoir_out):
        raise ValueError("mirres: reservoir_out must not share memory with reservoir_prev")
    img = out if out is not None else torch.empty((npix, 3), dtype=torch.float32, device=dev)
    dbg_rgb = dbg_hash = None
    if debug:
        dbg_rgb = torch.empty((S, 3), dtype=torch.float32, device=dev)
        dbg_hash = torch.empty((S,), dtype=torch.int32, device=dev)
    op = o.struct(dbg_rgb, dbg_hash, reservoir_prev, reservoir_out)
    sc = scene.struct()
    th = C.c_void_p()
    _check(_lib.mrs_render(C.byref(sc), C.addressof(vs), len(views), C.byref(op), img.data_ptr(),
                           C.byref(th) if keep_tape else None, _stream(stream)))
    tape = Tape(th) if (keep_tape and th.value) else None
    res = [img]
    if keep_tape:
        res.append(tape)
    if debug:
        res += [dbg_rgb, dbg_hash]
    return res[0] if len(res) == 1 else tuple(res)


def render_backward(scene: GpuScene, views: Sequence, opts, grad_image: torch.Tensor, tape: Optional[Tape] = None,
                    grads: Optional[Dict[str, torch.Tensor]] = None, stream=None,
                    reservoir_prev: Optional[torch.Tensor] = None) -> Dict[str, torch.Tensor]:
    """Accumulates d(sum grad_image . image)/d(materials, env) into `grads`
    (allocated zero if None) and returns it.  With reservoir reuse and no
    tape, reservoir_prev must be the one the forward call used."""
    o = RenderOptions.from_any(opts)
    vs, npix, _ = views_struct(views)
    gi = _dev(grad_image)
    if gi.numel() != 3 * npix:
        raise ValueError(f"mirres: grad_image must hold {npix} x 3 values, got {tuple(grad_image.shape)}")
    gi = gi.reshape(npix, 3)
    _need(reservoir_prev, "reservoir_prev", (total_samples(views), 8))
    if grads is None:
        grads = scene.zero_grads()
    scene.check_grads(grads)
    g = _grads_struct(grads)
    op = o.struct(reservoir_prev=reservoir_prev)
    sc = scene.struct()
    _check(_lib.mrs_render_backward(C.byref(sc), C.addressof(vs), len(views), C.byref(op), gi.data_ptr(),
                                    C.byref(g), tape.handle if tape is not None else None, _stream(stream)))
    return grads


def tape_bytes(views: Sequence, opts) -> int:
    vs, _, _ = views_struct(views)
    op = RenderOptions.from_any(opts).struct()
    return int(_lib.mrs_tape_bytes(C.addressof(vs), len(views), C.byref(op)))


class Plan:
    """A planned render (+ adjoint) over fixed views and bound tensors.

    All views share one persistent path pool; with use_graph each pass is
    captured once into a hipGraph and replayed.  The scene tensors, the image,
    the grad image and the gradient buffers are bound at creation: update
    their contents in place between passes (never rebind them)."""

    def __init__(self, scene: GpuScene, views: Sequence, opts, with_grad: bool = False, use_graph: bool = True,
                 debug: bool = False, reservoir_prev: Optional[torch.Tensor] = None,
                 reservoir_out: Optional[torch.Tensor] = None):
        self.scene, self.views = scene, list(views)
        self.opts = RenderOptions.from_any(opts)
        vs, npix, self.offsets = views_struct(self.views)
        dev = scene.pos.device
        self.image = torch.zeros((npix, 3), dtype=torch.float32, device=dev)
        self.dbg_rgb = self.dbg_hash = None
        if debug:
            S = total_samples(self.views)
            self.dbg_rgb = torch.zeros((S, 3), dtype=torch.float32, device=dev)
            self.dbg_hash = torch.zeros((S,), dtype=torch.int32, device=dev)
        self.grad_image = None
        self.grads: Dict[str, torch.Tensor] = {}
        g = None
        if with_grad:
            self.grad_image = torch.zeros_like(self.image)
            self.grads = scene.zero_grads()
            g = _grads_struct(self.grads)
        S = total_samples(self.views)
        _need(reservoir_prev, "reservoir_prev", (S, 8))
        _need(reservoir_out, "reservoir_out", (S, 8))
        if _overlap(reservoir_prev, reservoir_out):
            raise ValueError("mirres: reservoir_out must not share memory with reservoir_prev")
        self.reservoir_prev, self.reservoir_out = reservoir_prev, reservoir_out   # bound: keep them alive
        op = self.opts.struct(self.dbg_rgb, self.dbg_hash, reservoir_prev, reservoir_out)
        sc = scene.struct()
        h = C.c_void_p()
        _check(_lib.mrs_plan_create(C.byref(sc), C.addressof(vs), len(self.views), C.byref(op),
                                    self.image.data_ptr(), _ptr(self.grad_image), C.byref(g) if g else None,
                                    int(use_graph), C.byref(h)))
        self._h = h

    def forward(self, stream=None) -> torch.Tensor:
        _check(_lib.mrs_plan_forward(self._h, _stream(stream)))
        return self.image

    def backward(self, stream=None) -> Dict[str, torch.Tensor]:
        """Accumulates d(sum grad_image . image) into self.grads (zero them
        first for a fresh gradient)."""
        _check(_lib.mrs_plan_backward(self._h, _stream(stream)))
        return self.grads

    def zero_grad(self):
        for t in self.grads.values():
            t.zero_()

    def info(self) -> Tuple[int, bool, bool]:
        s, t, g = C.c_int64(), C.c_int32(), C.c_int32()
        _check(_lib.mrs_plan_info(self._h, C.byref(s), C.byref(t), C.byref(g)))
        return s.value, bool(t.value), bool(g.value)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mrs_plan_destroy(self._h)
            self._h = None


def profile_begin():
    """Start timing every kernel launch with HIP events on its stream."""
    _check(_lib.mrs_profile_begin())


def profile_end() -> Dict[str, Tuple[int, float]]:
    """Stop timing; returns {kernel: (launches, device milliseconds)}."""
    buf = (_KernelTime * 32)()
    n = C.c_int32()
    _check(_lib.mrs_profile_end(C.addressof(buf), 32, C.byref(n)))
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].ms)) for i in range(n.value)}


def release_workspace():
    _lib.mrs_release_workspace()


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, scene, views, opts, vmat, albedo, rough, metal, env):
        sc = scene.with_params(vmat=vmat, albedo=albedo, rough=rough, metal=metal, env=env)
        img, tape = render(sc, views, opts, keep_tape=True)
        ctx.scene, ctx.views, ctx.opts, ctx.tape = sc, views, opts, tape
        return img

    @staticmethod
    def backward(ctx, gimg):
        sc = ctx.scene
        need = ctx.needs_input_grad
        grads = {}
        if sc.mat_mode == MAT_VERTEX:
            grads["vmat"] = torch.zeros_like(sc.vmat) if need[3] else None
        else:
            grads["albedo"] = torch.zeros_like(sc.albedo) if need[4] else None
            grads["rough"] = torch.zeros_like(sc.rough) if need[5] else None
            grads["metal"] = torch.zeros_like(sc.metal) if need[6] else None
        grads["env"] = torch.zeros_like(sc.env) if need[7] else None
        render_backward(sc, ctx.views, ctx.opts, gimg, tape=ctx.tape, grads=grads)
        ctx.tape = None
        return (None, None, None, grads.get("vmat"), grads.get("albedo"), grads.get("rough"), grads.get("metal"),
                grads.get("env"))


def render_autograd(scene: GpuScene, views: Sequence, opts, vmat=None, albedo=None, rough=None, metal=None,
                    env=None) -> torch.Tensor:
    """Differentiable render: gradients flow to whichever of vmat / albedo /
    rough / metal / env are passed as tensors requiring grad (defaults: the
    scene's own tensors, without grad)."""
    vmat = scene.vmat if vmat is None else vmat
    albedo = scene.albedo if albedo is None else albedo
    rough = scene.rough if rough is None else rough
    metal = scene.metal if metal is None else metal
    env = scene.env if env is None else env
    return _RenderFn.apply(scene, list(views), opts, vmat, albedo, rough, metal, env)


class _FieldRenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, scene, views, opts, table, w1, b1, w2, b2, env):
        f = scene.field.with_params(table=table, w1=w1, b1=b1, w2=w2, b2=b2)
        sc = object.__new__(GpuScene)
        sc.__dict__.update(scene.__dict__)
        sc.field = f
        sc.env = _dev(env)
        img, tape = render(sc, views, opts, keep_tape=True)
        ctx.scene, ctx.views, ctx.opts, ctx.tape = sc, views, opts, tape
        return img

    @staticmethod
    def backward(ctx, gimg):
        sc = ctx.scene
        need = ctx.needs_input_grad
        grads = {k: torch.zeros_like(getattr(sc.field, k)) if need[3 + i] else None
                 for i, k in enumerate(FIELD_KEYS)}
        grads["env"] = torch.zeros_like(sc.env) if need[8] else None
        render_backward(sc, ctx.views, ctx.opts, gimg, tape=ctx.tape, grads=grads)
        ctx.tape = None
        return (None, None, None) + tuple(grads[k] for k in FIELD_KEYS) + (grads["env"],)


def render_field_autograd(scene: GpuScene, views: Sequence, opts, table=None, w1=None, b1=None, w2=None, b2=None,
                          env=None) -> torch.Tensor:
    """Differentiable render of a field-material scene: gradients flow to
    whichever of the field's table / w1 / b1 / w2 / b2 and env are passed as
    tensors requiring grad (defaults: the scene's own tensors)."""
    if scene.mat_mode != MAT_FIELD:
        raise ValueError("render_field_autograd needs a scene with a material field")
    f = scene.field
    args = [f.table if table is None else table, f.w1 if w1 is None else w1, f.b1 if b1 is None else b1,
            f.w2 if w2 is None else w2, f.b2 if b2 is None else b2, scene.env if env is None else env]
    return _FieldRenderFn.apply(scene, list(views), opts, *args)


# ------------------------------------------------------------------ denoiser
class _DenoiseParams(C.Structure):
    _fields_ = [("levels", C.c_int32), ("sigma_rt", C.c_float), ("sigma_n", C.c_float), ("sigma_x", C.c_float)]


def gbuffer(scene: GpuScene, views: Sequence, stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Position and normal of the closest hit through every pixel centre,
    packed like render()'s image (zeros where the ray misses)."""
    vs, npix, _ = views_struct(views)
    dev = scene.pos.device
    pos = torch.empty((npix, 3), dtype=torch.float32, device=dev)
    nrm = torch.empty((npix, 3), dtype=torch.float32, device=dev)
    sc = scene.struct()
    _check(_lib.mrs_gbuffer(C.byref(sc), C.addressof(vs), len(views), pos.data_ptr(), nrm.data_ptr(),
                            _stream(stream)))
    return pos, nrm


class Denoiser:
    """Edge-avoiding a-trous wavelet denoiser over packed images of `views`
    with a fixed G-buffer.  forward() keeps the per-level state in a device
    workspace that backward() reads."""

    def __init__(self, views: Sequence, normal: torch.Tensor, position: torch.Tensor, levels: int = 3,
                 sigma_rt: float = 1.0, sigma_n: float = 0.5, sigma_x: float = 0.5):
        self.vs, self.npix, _ = views_struct(views)
        self.nviews = len(views)
        self.params = _DenoiseParams(levels, sigma_rt, sigma_n, sigma_x)
        self.normal = _dev(normal)
        self.position = _dev(position)
        nbytes = _lib.mrs_denoise_work_bytes(C.addressof(self.vs), self.nviews, C.byref(self.params))
        if nbytes < 0:
            raise MirresError(-1, "invalid denoiser views or parameters")
        self.work = torch.empty(((nbytes + 3) // 4,), dtype=torch.float32, device=self.normal.device)
        self.generation = 0       # forwards run so far: the workspace holds the last one's state

    def forward(self, color: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        c = _dev(color)
        if c.numel() != 3 * self.npix:
            raise ValueError(f"mirres: color must hold {self.npix} x 3 values, got {tuple(color.shape)}")
        _need(out, "out", tuple(c.shape))
        res = out if out is not None else torch.empty_like(c)
        _check(_lib.mrs_denoise(C.addressof(self.vs), self.nviews, C.byref(self.params), c.data_ptr(),
                                self.normal.data_ptr(), self.position.data_ptr(), res.data_ptr(),
                                self.work.data_ptr(), _stream(stream)))
        self.generation += 1
        return res

    def backward(self, grad_out: torch.Tensor, stream=None) -> torch.Tensor:
        g = _dev(grad_out)
        gi = torch.empty_like(g)
        _check(_lib.mrs_denoise_backward(C.addressof(self.vs), self.nviews, C.byref(self.params),
                                         self.normal.data_ptr(), self.position.data_ptr(), self.work.data_ptr(),
                                         g.data_ptr(), gi.data_ptr(), _stream(stream)))
        return gi


def denoise_noalloc(views: Sequence, color: torch.Tensor, normal: torch.Tensor, position: torch.Tensor,
                    out: torch.Tensor, levels: int = 3, sigma_rt: float = 1.0, sigma_n: float = 0.5,
                    sigma_x: float = 0.5, stream=None) -> torch.Tensor:
    """The denoiser's forward into the caller's `out` without any device
    allocation: the library's static scratch holds the intermediate levels
    (mrs_denoise_noalloc).  No state is kept for a backward."""
    vs, npix, _ = views_struct(views)
    params = _DenoiseParams(levels, sigma_rt, sigma_n, sigma_x)
    bufs = {"color": color, "normal": normal, "position": position, "out": out}
    for k, t in bufs.items():
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == 3 * npix):
            raise ValueError(f"denoise_noalloc: {k} must be a contiguous float32 GPU tensor of {npix} x 3")
    _check(_lib.mrs_denoise_noalloc(C.addressof(vs), len(views), C.byref(params), color.data_ptr(),
                                    normal.data_ptr(), position.data_ptr(), out.data_ptr(), _stream(stream)))
    return out


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor):
    """Stable sort of (key, value) pairs by key (uint32 bits in int32 GPU
    tensors of one length): returns the sorted keys and values (new tensors)."""
    n = keys.numel()
    for t, name in ((keys, "keys"), (vals, "vals")):
        if not (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous() and t.numel() == n):
            raise ValueError(f"mirres: {name} must be a contiguous int32 GPU tensor of {n} entries")
    ko, vo = torch.empty_like(keys), torch.empty_like(vals)
    tmp = torch.empty(max(int(_lib.mrs_sort_pairs_tmp_bytes(n)), 16), dtype=torch.uint8, device=keys.device)
    _check(_lib.mrs_sort_pairs_u32(keys.data_ptr(), ko.data_ptr(), vals.data_ptr(), vo.data_ptr(), n, tmp.data_ptr(),
                                   tmp.numel(), _stream()))
    return ko, vo


class _DenoiseFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, color, den):
        ctx.den = den
        out = den.forward(color)
        ctx.generation = den.generation
        return out

    @staticmethod
    def backward(ctx, g):
        if ctx.den.generation != ctx.generation:
            raise RuntimeError("mirres: this Denoiser ran another forward after the one being differentiated; "
                               "its workspace no longer holds that call's levels (use one Denoiser per "
                               "denoised image in a graph)")
        return ctx.den.backward(g.contiguous()), None


def denoise_autograd(color: torch.Tensor, den: "Denoiser") -> torch.Tensor:
    """Differentiable denoise(color).  The backward reads the Denoiser's
    workspace, which holds the latest forward only: a second forward on the
    same Denoiser before this call's backward makes that backward raise."""
    return _DenoiseFn.apply(color, den)
