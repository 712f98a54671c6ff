"""Seeded synthetic inputs shaped like the paper's workloads.

The paper evaluates on object-centric multi-view captures under HDR
environment lighting (Sec. 5.1, TensoIR synthetic and OWL datasets) with a
256x512 environment map (Sec. 3, "Intrinsic decomposition") and three
bounces (Sec. 4.2).  Those datasets are not available here; this module
builds stand-ins of the same shape: a displaced sphere with concave
cavities on a ground plane or box, smooth-noise material textures, a
log-normal HDR environment with bright lobes, and pinhole cameras around
the object.

This module holds input generation only.  It contains none of the
renderer's arithmetic (no sampling, shading, intersection or gradients),
so both the FP64 oracle and the GPU path may consume what it produces.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
MAT_VERTEX = 0
MAT_TEXTURE = 1
MAT_FIELD = 2


@dataclasses.dataclass
class Field:
    """Parameters of a material field: a multi-resolution hash grid
    (levels x 2^log2_table entries of 2 features) and a 2-layer MLP
    (2L -> 32 -> 4), over the box [lo, hi]."""
    table: np.ndarray                  # float32 [L, T, 2]
    w1: np.ndarray                     # float32 [32, 2L]
    b1: np.ndarray                     # float32 [32]
    w2: np.ndarray                     # float32 [4, 32]
    b2: np.ndarray                     # float32 [4]
    lo: np.ndarray                     # float32 [3]
    hi: np.ndarray                     # float32 [3]
    n_min: int = 16
    n_max: int = 2048

    @property
    def levels(self) -> int:
        return int(self.table.shape[0])

    @property
    def log2_table(self) -> int:
        return int(self.table.shape[1]).bit_length() - 1


@dataclasses.dataclass
class Scene:
    pos: np.ndarray                    # float32 [nv, 3]
    faces: np.ndarray                  # int32 [nf, 3]
    env: np.ndarray                    # float32 [eh, ew, 3], row 0 = +y pole
    mat_mode: int = MAT_VERTEX
    vmat: Optional[np.ndarray] = None  # float32 [nv, 5] (albedo rgb, roughness, metallic)
    uv: Optional[np.ndarray] = None    # float32 [nv, 2]
    albedo: Optional[np.ndarray] = None  # float32 [th, tw, 3]
    rough: Optional[np.ndarray] = None   # float32 [th, tw]
    metal: Optional[np.ndarray] = None   # float32 [th, tw]
    field: Optional[Field] = None        # MAT_FIELD

    @property
    def nv(self) -> int:
        return int(self.pos.shape[0])

    @property
    def nf(self) -> int:
        return int(self.faces.shape[0])


@dataclasses.dataclass
class View:
    c2w: np.ndarray            # float32 [4, 4], camera looks down -z, +y up
    fov_y_deg: float
    w: int
    h: int
    spp: int
    sample_offset: int = 0


@dataclasses.dataclass
class Options:
    bounces: int = 3
    ris_m: int = 32
    ris_m_brdf: int = 16
    rr_start: int = -1
    seed: int = 1
    brdf: int = 1          # 0 Lambert, 1 Lambert + GGX
    background: int = 0    # 0 env, 1 black
    grad_mode: int = 0     # 0 full path, 1 primary vertex only
    reuse_spatial: int = 0   # reservoir reuse at primary vertices: neighbours merged (0 = none)
    reuse_radius: int = 16   # neighbour window half-size in pixels
    reuse_temporal: int = 0  # 1: merge the previous frame's reservoir first
    reuse_m_cap: int = 20    # temporal confidence cap, in multiples of ris_m


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    views: List[View]
    opts: Options

    @property
    def samples(self) -> int:
        return int(sum(v.w * v.h * v.spp for v in self.views))

    @property
    def pixels(self) -> int:
        return int(sum(v.w * v.h for v in self.views))


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
def icosphere(subdiv: int, radius: float = 1.0):
    """Loop-free icosphere by midpoint subdivision of an icosahedron."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
         (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        cache = {}
        new_faces = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    pos = np.array(verts, dtype=np.float64) * radius
    return pos.astype(np.float32), np.array(faces, dtype=np.int32)


def _perlin_perm(rng: np.random.Generator) -> np.ndarray:
    p = np.arange(256, dtype=np.int64)
    rng.shuffle(p)
    return np.concatenate([p, p])


def _perlin3(p: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """Improved gradient noise (Perlin, SIGGRAPH 2002) at points p [N, 3]."""
    fl = np.floor(p)
    f = p - fl
    i = fl.astype(np.int64) & 255
    fade = f * f * f * (f * (f * 6.0 - 15.0) + 10.0)

    def grad(h, x, y, z):
        h = h & 15
        u = np.where(h < 8, x, y)
        v = np.where(h < 4, y, np.where((h == 12) | (h == 14), x, z))
        return np.where(h & 1, -u, u) + np.where(h & 2, -v, v)

    X, Y, Z = i[:, 0], i[:, 1], i[:, 2]
    x, y, z = f[:, 0], f[:, 1], f[:, 2]
    A = perm[X] + Y
    AA = perm[A] + Z
    AB = perm[A + 1] + Z
    B = perm[X + 1] + Y
    BA = perm[B] + Z
    BB = perm[B + 1] + Z

    def lerp(t, a, b):
        return a + t * (b - a)

    u, v, w = fade[:, 0], fade[:, 1], fade[:, 2]
    return lerp(w,
                lerp(v, lerp(u, grad(perm[AA], x, y, z), grad(perm[BA], x - 1, y, z)),
                     lerp(u, grad(perm[AB], x, y - 1, z), grad(perm[BB], x - 1, y - 1, z))),
                lerp(v, lerp(u, grad(perm[AA + 1], x, y, z - 1), grad(perm[BA + 1], x - 1, y, z - 1)),
                     lerp(u, grad(perm[AB + 1], x, y - 1, z - 1), grad(perm[BB + 1], x - 1, y - 1, z - 1))))


def fbm3(p: np.ndarray, rng: np.random.Generator, octaves: int = 4, freq: float = 2.0) -> np.ndarray:
    perm = _perlin_perm(rng)
    out = np.zeros(p.shape[0])
    amp = 1.0
    for o in range(octaves):
        out += amp * _perlin3(p * (freq * 2.0 ** o) + 17.0 * o, perm)
        amp *= 0.5
    return out


def displaced_latlong_sphere(rows: int, cols: int, amp: float, rng: np.random.Generator):
    """Lat-long sphere (`rows` latitude bands, `cols` longitudes) with triangle
    fans at the poles (no degenerate triangles), a duplicated seam column so
    uv runs 0..1, and radial displacement r = 1 + amp * fBm(x)."""
    ring_theta = np.pi * np.arange(1, rows) / rows                  # rows - 1 rings
    phi = 2.0 * np.pi * np.arange(cols + 1) / cols                  # seam duplicated
    th, ph = np.meshgrid(ring_theta, phi, indexing="ij")
    dirs = np.stack([np.sin(th) * np.sin(ph), np.cos(th), -np.sin(th) * np.cos(ph)], -1).reshape(-1, 3)
    uv_ring = np.stack([(ph / (2 * np.pi)), th / np.pi], -1).reshape(-1, 2)
    # one pole vertex per fan triangle so each gets its own u
    pole_u = (np.arange(cols) + 0.5) / cols
    north = np.tile(np.array([[0.0, 1.0, 0.0]]), (cols, 1))
    south = np.tile(np.array([[0.0, -1.0, 0.0]]), (cols, 1))
    dirs_all = np.concatenate([north, dirs, south], 0)
    uv_all = np.concatenate([np.stack([pole_u, np.zeros(cols)], -1), uv_ring,
                             np.stack([pole_u, np.ones(cols)], -1)], 0)
    disp = fbm3(dirs_all, rng)
    pos = dirs_all * (1.0 + amp * disp)[:, None]
    nring = cols + 1
    base = cols

    def rv(r, c):  # vertex index of ring r (0..rows-2), column c (0..cols)
        return base + r * nring + c

    faces = []
    c = np.arange(cols)
    # north fan
    faces.append(np.stack([c, rv(0, c), rv(0, c + 1)], -1))
    for r in range(rows - 2):
        a, b = rv(r, c), rv(r, c + 1)
        a2, b2 = rv(r + 1, c), rv(r + 1, c + 1)
        faces.append(np.stack([a, a2, b2], -1))
        faces.append(np.stack([a, b2, b], -1))
    s0 = base + (rows - 1) * nring
    faces.append(np.stack([s0 + c, rv(rows - 2, c + 1), rv(rows - 2, c)], -1))
    faces = np.concatenate(faces, 0).astype(np.int32)
    return pos.astype(np.float32), faces, uv_all.astype(np.float32)


def ground_plane(y: float, half: float):
    pos = np.array([[-half, y, -half], [half, y, -half], [half, y, half], [-half, y, half]], np.float32)
    faces = np.array([[0, 2, 1], [0, 3, 2]], np.int32)
    uv = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32)
    return pos, faces, uv


def ground_box(y0: float, y1: float, half: float):
    """Axis-aligned slab [-half, half] x [y0, y1] x [-half, half], 12 triangles."""
    xs = (-half, half)
    pos, uv = [], []
    for yy in (y0, y1):
        for zz in xs:
            for xx in xs:
                pos.append((xx, yy, zz))
                uv.append(((xx + half) / (2 * half), (zz + half) / (2 * half)))
    pos = np.array(pos, np.float32)
    # corners: index = 4*top + 2*(z>0) + (x>0)
    quads = [(4, 6, 7, 5), (0, 1, 3, 2), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    faces = []
    for a, b, c, d in quads:
        faces += [(a, b, c), (a, c, d)]
    return pos, np.array(faces, np.int32), np.array(uv, np.float32)


def merge(parts):
    pos, faces, uv = [], [], []
    off = 0
    for p, f, u in parts:
        pos.append(p)
        faces.append(f + off)
        uv.append(u)
        off += p.shape[0]
    return (np.concatenate(pos).astype(np.float32), np.concatenate(faces).astype(np.int32),
            np.concatenate(uv).astype(np.float32))


# --------------------------------------------------------------------------
# textures and environment
# --------------------------------------------------------------------------
def _periodic_cubic_matrix(n_out: int, n_in: int) -> np.ndarray:
    """[n_out, n_in] periodic Catmull-Rom interpolation weights."""
    x = (np.arange(n_out) + 0.5) * n_in / n_out - 0.5
    i = np.floor(x).astype(np.int64)
    t = x - i
    w = [(-0.5 * t ** 3 + t ** 2 - 0.5 * t), (1.5 * t ** 3 - 2.5 * t ** 2 + 1.0),
         (-1.5 * t ** 3 + 2.0 * t ** 2 + 0.5 * t), (0.5 * t ** 3 - 0.5 * t ** 2)]
    A = np.zeros((n_out, n_in))
    rows = np.arange(n_out)
    for k in range(4):
        np.add.at(A, (rows, (i - 1 + k) % n_in), w[k])
    return A


def smooth_noise2(res: int, rng: np.random.Generator, base: int = 8, octaves: int = 4) -> np.ndarray:
    """Tileable fBm of cubic-interpolated random grids, roughly N(0, 1)."""
    out = np.zeros((res, res))
    amp, tot = 1.0, 0.0
    for o in range(octaves):
        g = min(base * 2 ** o, res)
        G = rng.standard_normal((g, g))
        A = _periodic_cubic_matrix(res, g)
        out += amp * (A @ G @ A.T)
        tot += amp * amp
        amp *= 0.5
    return out / math.sqrt(tot)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def noise_textures(res: int, rng: np.random.Generator):
    albedo = np.stack([0.05 + 0.9 * _sigmoid(1.5 * smooth_noise2(res, rng)) for _ in range(3)], -1)
    rough = 0.1 + 0.8 * _sigmoid(1.5 * smooth_noise2(res, rng))
    m = np.clip((smooth_noise2(res, rng) - 0.3) / 0.6, 0.0, 1.0)
    metal = m * m * (3.0 - 2.0 * m)
    return albedo.astype(np.float32), rough.astype(np.float32), metal.astype(np.float32)


def _texel_dirs(eh: int, ew: int) -> np.ndarray:
    v = (np.arange(eh) + 0.5) / eh
    u = (np.arange(ew) + 0.5) / ew
    th, ph = np.meshgrid(np.pi * v, 2 * np.pi * (u - 0.5), indexing="ij")
    return np.stack([np.sin(th) * np.sin(ph), np.cos(th), -np.sin(th) * np.cos(ph)], -1)


def _upper_dir(rng: np.random.Generator, elev_lo_deg=15.0, elev_hi_deg=75.0) -> np.ndarray:
    el = np.deg2rad(rng.uniform(elev_lo_deg, elev_hi_deg))
    az = rng.uniform(0, 2 * np.pi)
    return np.array([np.cos(el) * np.sin(az), np.sin(el), -np.cos(el) * np.cos(az)])


def hdr_env(eh: int, ew: int, rng: np.random.Generator, lobes) -> np.ndarray:
    """Log-normal(0, 1) texels plus Gaussian lobes (strength, sigma_deg)."""
    env = np.exp(rng.standard_normal((eh, ew, 3)))
    dirs = _texel_dirs(eh, ew)
    for strength, sigma_deg in lobes:
        c = _upper_dir(rng)
        gam = np.arccos(np.clip(dirs @ c, -1.0, 1.0))
        sig = np.deg2rad(sigma_deg)
        env += strength * np.exp(-gam ** 2 / (2 * sig ** 2))[..., None]
    return env.astype(np.float32)


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)) -> np.ndarray:
    eye = np.asarray(eye, np.float64)
    z = eye - np.asarray(target, np.float64)
    z /= np.linalg.norm(z)
    x = np.cross(np.asarray(up, np.float64), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    m = np.eye(4)
    m[:3, 0], m[:3, 1], m[:3, 2], m[:3, 3] = x, y, z, eye
    return m.astype(np.float32)


def orbit(radius, elev_deg, az_rad, target=(0.0, 0.0, 0.0)) -> np.ndarray:
    el = np.deg2rad(elev_deg)
    eye = radius * np.array([np.cos(el) * np.sin(az_rad), np.sin(el), np.cos(el) * np.cos(az_rad)])
    return look_at(eye + np.asarray(target), target)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def _displaced_scene(rows, cols, tex_res, env_hw, rng):
    sph = displaced_latlong_sphere(rows, cols, 0.2, rng)
    box = ground_box(-1.45, -1.25, 4.0)
    pos, faces, uv = merge([sph, box])
    albedo, rough, metal = noise_textures(tex_res, rng)
    env = hdr_env(env_hw[0], env_hw[1], rng,
                  [(rng.uniform(50, 100), 5.0) for _ in range(3)])
    return Scene(pos=pos, faces=faces, env=env, mat_mode=MAT_TEXTURE, uv=uv,
                 albedo=albedo, rough=rough, metal=metal)


def config1(seed_base: int = 1000) -> Workload:
    """Tiny: icosphere (subdiv 3) over a 2-triangle plane, per-vertex
    materials, 32x16 env with a sun lobe, one 64x64 view; B=2, spp=4, M=8."""
    rng = np.random.default_rng(seed_base + 1)
    sp, sf = icosphere(3, 1.0)
    gp, gf, _ = ground_plane(-1.05, 4.0)
    pos, faces, _ = merge([(sp, sf, np.zeros((sp.shape[0], 2), np.float32)),
                           (gp, gf, np.zeros((4, 2), np.float32))])
    nv = pos.shape[0]
    vmat = np.concatenate([rng.uniform(0.1, 0.9, (nv, 3)), rng.uniform(0.1, 0.9, (nv, 1)),
                           (rng.uniform(0, 1, (nv, 1)) < 0.2).astype(np.float64)], 1).astype(np.float32)
    env = hdr_env(16, 32, rng, [(100.0, 8.0)])
    scene = Scene(pos=pos, faces=faces, env=env, mat_mode=MAT_VERTEX, vmat=vmat)
    c2w = orbit(3.0, rng.uniform(10, 60), rng.uniform(0, 2 * np.pi))
    views = [View(c2w=c2w, fov_y_deg=40.0, w=64, h=64, spp=4)]
    return Workload("c1_tiny_icosphere_64x64", scene, views,
                    Options(bounces=2, ris_m=8, ris_m_brdf=4, rr_start=-1, seed=1))


def config2(seed_base: int = 1000, res: int = 512) -> Workload:
    """~100k-triangle displaced sphere on a ground box, 1024^2 textures,
    256x128 env with 3 lobes, one 512x512 view; B=3, spp=1, M=32, RR from 2."""
    rng = np.random.default_rng(seed_base + 2)
    scene = _displaced_scene(158, 316, 1024, (128, 256), rng)
    c2w = orbit(3.0, rng.uniform(15, 35), rng.uniform(0, 2 * np.pi))
    views = [View(c2w=c2w, fov_y_deg=40.0, w=res, h=res, spp=1)]
    return Workload("c2_100k_tris_512x512", scene, views,
                    Options(bounces=3, ris_m=32, ris_m_brdf=16, rr_start=2, seed=2))


def config3(seed_base: int = 1000, n_views: int = 8, res: int = 800, spp: int = 4,
            tex_res: int = 2048) -> Workload:
    """~300k-triangle displaced sphere, 2048^2 textures, 512x256 env, 8 views
    of 800x800 on a ring; B=3, spp=4, M=32 (the differentiation workload)."""
    rng = np.random.default_rng(seed_base + 3)
    scene = _displaced_scene(274, 548, tex_res, (256, 512), rng)
    views = []
    for i in range(n_views):
        az = 2 * np.pi * i / n_views + rng.uniform(-0.1, 0.1)
        views.append(View(c2w=orbit(3.0, 20.0 + rng.uniform(-5, 5), az), fov_y_deg=40.0,
                          w=res, h=res, spp=spp))
    return Workload(f"c3_300k_tris_{n_views}x{res}x{res}_spp{spp}", scene, views,
                    Options(bounces=3, ris_m=32, ris_m_brdf=16, rr_start=-1, seed=3))


def config4(seed_base: int = 1000, n_views: int = 64, scene: Optional[Scene] = None) -> Workload:
    """64 views of uneven square size in 256..1024 and spp in 1..16 over the
    config-3 mesh and env; B=3, M=16 (the batching workload)."""
    rng = np.random.default_rng(seed_base + 4)
    if scene is None:
        scene = _displaced_scene(274, 548, 2048, (256, 512), np.random.default_rng(seed_base + 3))
    views = []
    for i in range(n_views):
        s = int(rng.integers(256, 1025))
        spp = int(rng.integers(1, 17))
        c2w = orbit(3.0, rng.uniform(5, 60), rng.uniform(0, 2 * np.pi))
        views.append(View(c2w=c2w, fov_y_deg=40.0, w=s, h=s, spp=spp))
    return Workload(f"c4_batched_{n_views}views", scene, views,
                    Options(bounces=3, ris_m=16, ris_m_brdf=8, rr_start=-1, seed=4))


def fibonacci_upper(n: int) -> np.ndarray:
    i = np.arange(n) + 0.5
    y = 0.15 + 0.8 * i / n                      # elevation band above the ground
    r = np.sqrt(1 - y * y)
    phi = np.pi * (1 + 5 ** 0.5) * i
    return np.stack([r * np.sin(phi), y, r * np.cos(phi)], -1)


def config5(seed_base: int = 1000, n_views: int = 100, res: int = 800, rows: int = 500, cols: int = 1000,
            tex_res: int = 4096, env_hw=(512, 1024)) -> Workload:
    """1M-triangle mesh, 4096^2 textures, 1024x512 env, 100 views of 800x800
    on a Fibonacci hemisphere; B=5, spp=2, M=32 (the inverse-rendering loop)."""
    rng = np.random.default_rng(seed_base + 5)
    scene = _displaced_scene(rows, cols, tex_res, env_hw, rng)
    views = [View(c2w=look_at(3.0 * d), fov_y_deg=40.0, w=res, h=res, spp=2) for d in fibonacci_upper(n_views)]
    return Workload(f"c5_inverse_{n_views}x{res}x{res}", scene, views,
                    Options(bounces=5, ris_m=32, ris_m_brdf=16, rr_start=-1, seed=5))


def furnace_scene(env_value: float = 1.5, subdiv: int = 2, env_hw=(8, 16)) -> Scene:
    """Convex albedo-1 Lambertian icosphere under a constant environment."""
    pos, faces = icosphere(subdiv, 1.0)
    vmat = np.tile(np.array([[1.0, 1.0, 1.0, 0.5, 0.0]], np.float32), (pos.shape[0], 1))
    env = np.full((env_hw[0], env_hw[1], 3), env_value, np.float32)
    return Scene(pos=pos, faces=faces, env=env, mat_mode=MAT_VERTEX, vmat=vmat)


def plane_scene(albedo=(0.3, 0.5, 0.7), env_value: float = 2.0, env_hw=(8, 16)) -> Scene:
    """A single large square (unoccluded) under a constant environment."""
    pos, faces, _ = ground_plane(0.0, 50.0)
    vmat = np.tile(np.array([[albedo[0], albedo[1], albedo[2], 0.5, 0.0]], np.float32), (4, 1))
    env = np.full((env_hw[0], env_hw[1], 3), env_value, np.float32)
    return Scene(pos=pos, faces=faces, env=env, mat_mode=MAT_VERTEX, vmat=vmat)


def random_field(lo, hi, rng: np.random.Generator, levels: int = 16, log2_table: int = 19, n_min: int = 16,
                 n_max: int = 2048, table_scale: float = 0.5, decay: float = 0.0) -> Field:
    """Seeded field parameters: table entries uniform in +-table_scale
    (n_min / N_l)^decay at level l of resolution N_l (decay 1 keeps each
    level's slope per unit length alike, the fine levels carrying less
    amplitude, as in a trained field), layers with fan-in scaled normal
    weights, output biases around a mid-grey albedo and mid roughness."""
    T = 1 << log2_table
    table = rng.uniform(-table_scale, table_scale, (levels, T, 2))
    if decay:
        g = np.log(n_max / n_min) / max(levels - 1, 1)
        res = np.floor(n_min * np.exp(np.arange(levels) * g) + 1e-6)
        table *= ((n_min / res) ** decay)[:, None, None]
    w1 = rng.normal(0.0, 1.0 / np.sqrt(2 * levels), (32, 2 * levels)) * 2.0
    b1 = rng.normal(0.0, 0.1, 32)
    w2 = rng.normal(0.0, 1.0 / np.sqrt(32), (4, 32)) * 2.0
    b2 = np.array([0.0, -0.2, 0.2, 0.0]) + rng.normal(0.0, 0.1, 4)
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    return Field(table=f32(table), w1=f32(w1), b1=f32(b1), w2=f32(w2), b2=f32(b2), lo=f32(lo), hi=f32(hi),
                 n_min=n_min, n_max=n_max)


def with_field(scene: Scene, rng: np.random.Generator, margin: float = 0.05, decay: float = 1.0, **kw) -> Scene:
    """The same mesh and environment with a material field over the mesh's
    bounding box (enlarged by `margin` of its extent) instead of its
    per-vertex or texture materials; table amplitude falls as 1 / N_l
    (decay 1) by default."""
    lo, hi = scene.pos.min(0), scene.pos.max(0)
    ext = np.maximum(hi - lo, 1e-3)
    f = random_field(lo - margin * ext, hi + margin * ext, rng, decay=decay, **kw)
    return Scene(pos=scene.pos, faces=scene.faces, env=scene.env, mat_mode=MAT_FIELD, field=f)


def sample_items(workload: Workload, n: int, seed: int) -> np.ndarray:
    """Seeded subset of (view, pixel, sample) triples, uniform over samples."""
    rng = np.random.default_rng(seed)
    sizes = np.array([v.w * v.h * v.spp for v in workload.views], np.int64)
    cum = np.concatenate([[0], np.cumsum(sizes)])
    g = np.sort(rng.choice(int(cum[-1]), size=min(n, int(cum[-1])), replace=False))
    vi = np.searchsorted(cum, g, side="right") - 1
    local = g - cum[vi]
    spp = np.array([workload.views[i].spp for i in vi])
    return np.stack([vi, local // spp, local % spp], -1).astype(np.int32)


def sample_pixels(workload: Workload, n: int, seed: int) -> np.ndarray:
    """Seeded subset of (view, pixel) pairs, uniform over pixels, sorted."""
    rng = np.random.default_rng(seed)
    sizes = np.array([v.w * v.h for v in workload.views], np.int64)
    cum = np.concatenate([[0], np.cumsum(sizes)])
    g = np.sort(rng.choice(int(cum[-1]), size=min(n, int(cum[-1])), replace=False))
    vi = np.searchsorted(cum, g, side="right") - 1
    return np.stack([vi, g - cum[vi]], -1).astype(np.int32)


def pixel_items(workload: Workload, pixels: np.ndarray) -> np.ndarray:
    """Every sample of the given (view, pixel) pairs, pixel after pixel."""
    pixels = np.asarray(pixels, np.int32).reshape(-1, 2)
    spp = np.array([workload.views[v].spp for v in pixels[:, 0]], np.int64)
    rep = np.repeat(np.arange(len(pixels)), spp)
    first = np.concatenate([[0], np.cumsum(spp)[:-1]])
    s = np.arange(int(spp.sum())) - np.repeat(first, spp)
    return np.stack([pixels[rep, 0], pixels[rep, 1], s], -1).astype(np.int32)


def all_items(workload: Workload) -> np.ndarray:
    out = []
    for vi, v in enumerate(workload.views):
        p = np.repeat(np.arange(v.w * v.h), v.spp)
        s = np.tile(np.arange(v.spp), v.w * v.h)
        out.append(np.stack([np.full_like(p, vi), p, s], -1))
    return np.concatenate(out).astype(np.int32)
