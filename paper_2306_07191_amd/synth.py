"""Seeded synthetic inputs for the neural visibility workloads.

This module only draws inputs: meshes, shadow rays, MLP weights at their
Xavier initialisation and object assignments.  It holds none of the method's
arithmetic (no clipping, encoding or network evaluation), so that both the
HIP path and the CPU oracle can consume the same inputs without sharing code.

The paper evaluates on its own rendered scenes (Stanford models, Centaur,
Amazon Bistro; Sec. 6), which are not available here.  Every workload below is
a synthetic stand-in with the shape the paper's pipeline produces: shadow rays
from shading points towards a light (Sec. 4, Sec. 6 "Lights"), one query per
(ray, object AABB) pair (Sec. 4.1), per-object grids and Xavier-initialised
weights (Sec. 5 "Initialization").

Random streams: ``numpy.random.Generator(PCG64(SeedSequence([cfg, stream, ...])))``
with streams 0 mesh, 1 rays, 3 MLP, 4 object assignment, 5 training batch,
6 light samples, 7 calibration.  Grid latents are not drawn here: they come
from a counter-based generator (Philox4x64-10) that the library and the oracle
each implement from its published definition, because a 2 GB-per-object table
is too large to pass in from the host.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class ModelShape:
    """Grid and MLP sizes of one NIF model.

    levels/res_min/res_max/feats describe the multi-resolution grids (one set
    each for entry point, exit point and direction); hidden/width the MLP.
    grid_dtype is "f32" or "f16" (the paper stores latents in half, Sec. 5
    "Memory Footprint")."""

    levels: int
    res_min: int
    res_max: int
    feats: int
    hidden: int
    width: int
    grid_dtype: str

    @property
    def din(self) -> int:
        return 3 * self.levels * self.feats

    @property
    def mlp_params(self) -> int:
        """Weights of din->width, (hidden-1) x width->width, width->1; no biases."""
        return self.width * self.din + (self.hidden - 1) * self.width * self.width + self.width


TINY = ModelShape(levels=4, res_min=4, res_max=32, feats=2, hidden=3, width=64, grid_dtype="f32")
FRAME = ModelShape(levels=8, res_min=16, res_max=512, feats=2, hidden=4, width=64, grid_dtype="f16")

# configuration ids used as the first SeedSequence word
CFG_TINY, CFG_FRAME, CFG_TRAIN, CFG_MULTI, CFG_SCENE = 1, 2, 3, 4, 5

GRID_INIT_AMP = 1.0e-4  # latents ~ U(-1e-4, 1e-4), Sec. 5 "Initialization"


def rng(*words: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(words))))


# --------------------------------------------------------------------------
# Meshes
# --------------------------------------------------------------------------


def random_triangles(n: int, gen: np.random.Generator) -> np.ndarray:
    """n triangles with every vertex uniform in [-1, 1]^3; float32 [n, 3, 3]."""
    return gen.uniform(-1.0, 1.0, size=(n, 3, 3)).astype(np.float32)


def _value_noise(p: np.ndarray, gen: np.random.Generator) -> np.ndarray:
    """Seeded lattice value noise in [-1, 1]: lattice values from a 256-entry
    permutation hash, blended with the smoothstep 3t^2 - 2t^3 trilinearly."""
    perm = gen.permutation(256).astype(np.int64)
    vals = gen.uniform(-1.0, 1.0, size=256)
    fl = np.floor(p)
    i = fl.astype(np.int64)
    t = p - fl
    s = t * t * (3.0 - 2.0 * t)

    def lattice(ix, iy, iz):
        h = perm[(perm[(perm[ix & 255] + iy) & 255] + iz) & 255]
        return vals[h]

    out = np.zeros(p.shape[0])
    for bz in (0, 1):
        wz = s[:, 2] if bz else 1.0 - s[:, 2]
        for by in (0, 1):
            wy = s[:, 1] if by else 1.0 - s[:, 1]
            for bx in (0, 1):
                wx = s[:, 0] if bx else 1.0 - s[:, 0]
                out += wx * wy * wz * lattice(i[:, 0] + bx, i[:, 1] + by, i[:, 2] + bz)
    return out


def displaced_uv_sphere(n_lon: int, n_rings: int, center, radius: float, amp: float,
                        gen: np.random.Generator) -> np.ndarray:
    """UV sphere with n_lon longitudes and n_rings latitude rings between the
    poles, radius scaled by 1 + amp * noise(4 n).  Triangle count is
    2*n_lon (pole fans) + 2*n_lon*(n_rings-1) (quad bands).  float32 [T, 3, 3]."""
    theta = math.pi * np.arange(1, n_rings + 1) / (n_rings + 1)
    phi = 2.0 * math.pi * np.arange(n_lon) / n_lon
    st, ct = np.sin(theta)[:, None], np.cos(theta)[:, None]
    nrm = np.stack([st * np.cos(phi)[None, :], np.broadcast_to(ct, (n_rings, n_lon)),
                    st * np.sin(phi)[None, :]], axis=-1).reshape(-1, 3)
    nrm = np.concatenate([np.array([[0.0, 1.0, 0.0]]), nrm, np.array([[0.0, -1.0, 0.0]])])
    r = radius * (1.0 + amp * _value_noise(4.0 * nrm, gen))
    verts = np.asarray(center, dtype=np.float64)[None, :] + r[:, None] * nrm
    top, bot = 0, 1 + n_rings * n_lon
    j = np.arange(n_lon)
    jn = (j + 1) % n_lon
    ring = lambda k, jj: 1 + k * n_lon + jj  # noqa: E731
    tris = [np.stack([np.full(n_lon, top), ring(0, j), ring(0, jn)], axis=1)]
    for k in range(n_rings - 1):
        a, b, c, d = ring(k, j), ring(k, jn), ring(k + 1, j), ring(k + 1, jn)
        tris.append(np.stack([a, c, b], axis=1))
        tris.append(np.stack([b, c, d], axis=1))
    tris.append(np.stack([np.full(n_lon, bot), ring(n_rings - 1, jn), ring(n_rings - 1, j)], axis=1))
    idx = np.concatenate(tris)
    return verts[idx].astype(np.float32)


def uv_sphere_dims(target_tris: int) -> tuple[int, int]:
    """(n_lon, n_rings) with n_lon = 2 n_rings whose triangle count is closest to target."""
    best = None
    k0 = max(2, int(math.sqrt(target_tris / 4.0)))
    for k in range(max(2, k0 - 2), k0 + 3):
        t = 2 * (2 * k) + 2 * (2 * k) * (k - 1)
        if best is None or abs(t - target_tris) < abs(best[2] - target_tris):
            best = (2 * k, k, t)
    return best[0], best[1]


def mesh_aabb(tris: np.ndarray) -> np.ndarray:
    """float32 [6] = lo xyz, hi xyz of the vertices, widened symmetrically so
    that every axis spans at least 1e-6 of the largest one."""
    v = tris.reshape(-1, 3)
    lo = v.min(axis=0).astype(np.float64)
    hi = v.max(axis=0).astype(np.float64)
    ext = hi - lo
    need = 1e-6 * ext.max()
    pad = np.where(ext < need, 0.5 * (need - ext), 0.0)
    return np.concatenate([lo - pad, hi + pad]).astype(np.float32)


# --------------------------------------------------------------------------
# Rays
# --------------------------------------------------------------------------


def _normalize32(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.float32)
    n = np.sqrt((v.astype(np.float64) ** 2).sum(axis=1)).astype(np.float32)
    return (v / n[:, None]).astype(np.float32)


def rays_sphere_to_box(n: int, aabb: np.ndarray, gen: np.random.Generator,
                       radius: float = 3.0, center=None):
    """Origins uniform on a sphere (radius 3 about the box centre unless given),
    aimed at uniform points inside the box; t_max = +inf.
    Returns rays float32 [n, 6] (ox oy oz dx dy dz, d unit) and t_max float32 [n]."""
    lo, hi = aabb[:3].astype(np.float64), aabb[3:].astype(np.float64)
    c = np.zeros(3) if center is None else np.asarray(center, dtype=np.float64)
    g = gen.standard_normal(size=(n, 3))
    o = c[None, :] + radius * g / np.linalg.norm(g, axis=1, keepdims=True)
    tgt = lo[None, :] + gen.uniform(size=(n, 3)) * (hi - lo)[None, :]
    o32 = o.astype(np.float32)
    d = _normalize32(tgt.astype(np.float32) - o32)
    rays = np.concatenate([o32, d], axis=1).astype(np.float32)
    return rays, np.full(n, np.inf, dtype=np.float32)


# The single-object frame scene: a displaced sphere above a 4 x 4 ground quad,
# lit by a 0.5 x 0.5 area light at height 5.
FRAME_CENTER = (0.0, 2.0, 0.0)
FRAME_QUAD_HALF = 2.0
FRAME_LIGHT_Y = 5.0
FRAME_LIGHT_HALF = 0.25


def rays_ground_to_light(n: int, gen: np.random.Generator, quad_half=FRAME_QUAD_HALF,
                         light_y=FRAME_LIGHT_Y, light_half=FRAME_LIGHT_HALF, light_center=(0.0, 0.0)):
    """Shadow rays from uniform points of the ground quad (y = 0) to uniform
    points of the area light; d unit (float32) and t_max = distance to the
    light sample."""
    o = np.zeros((n, 3))
    o[:, 0] = gen.uniform(-quad_half, quad_half, n)
    o[:, 2] = gen.uniform(-quad_half, quad_half, n)
    lp = np.zeros((n, 3))
    lp[:, 0] = light_center[0] + gen.uniform(-light_half, light_half, n)
    lp[:, 1] = light_y
    lp[:, 2] = light_center[1] + gen.uniform(-light_half, light_half, n)
    o32 = o.astype(np.float32)
    v = lp.astype(np.float32) - o32
    d = _normalize32(v)
    tmax = np.sqrt((v.astype(np.float64) ** 2).sum(axis=1)).astype(np.float32)
    return np.concatenate([o32, d], axis=1).astype(np.float32), tmax


def frame_emitter(cells: int = 12, half: float = 1.5, height: float = FRAME_LIGHT_Y, sigma: float = 1.5):
    """An emitter above the frame scene for the sampling comparison: a
    2 half x 2 half square at `height` split into cells x cells squares of
    two triangles each, facing down, with log-normal radiance exp(sigma N(0,1))
    per square (seeded), so that the flux is concentrated on a few squares.
    Returns (triangles [2 cells^2, 9] float32, radiance [2 cells^2] float32)."""
    g = rng(CFG_TRAIN, 6, 1)
    e = np.linspace(-half, half, cells + 1)
    tris, rad = [], []
    for i in range(cells):
        for j in range(cells):
            x0, x1, z0, z1 = e[i], e[i + 1], e[j], e[j + 1]
            L = float(np.exp(sigma * g.normal()))
            tris.append([x0, height, z0, x1, height, z0, x1, height, z1])
            tris.append([x0, height, z0, x1, height, z1, x0, height, z1])
            rad += [L, L]
    return np.asarray(tris, np.float32), np.asarray(rad, np.float32)


def ground_points(n: int, gen: np.random.Generator, quad_half=FRAME_QUAD_HALF) -> np.ndarray:
    """Uniform points of the ground quad (y = 0), float32 [n, 3]."""
    p = np.zeros((n, 3), np.float32)
    p[:, 0] = gen.uniform(-quad_half, quad_half, n)
    p[:, 2] = gen.uniform(-quad_half, quad_half, n)
    return p


# --------------------------------------------------------------------------
# MLP weights
# --------------------------------------------------------------------------


def xavier_mlp(shape: ModelShape, gen: np.random.Generator) -> np.ndarray:
    """Flat float32 weights [W1 (width x din), W2..WH (width x width), w_out (width)],
    each matrix row-major [out][in], drawn U(+-sqrt(6/(fan_in+fan_out))) (Glorot
    uniform; Sec. 5 "Initialization").  No biases."""
    mats = [(shape.width, shape.din)] + [(shape.width, shape.width)] * (shape.hidden - 1) + [(1, shape.width)]
    parts = []
    for out_f, in_f in mats:
        lim = math.sqrt(6.0 / (in_f + out_f))
        parts.append(gen.uniform(-lim, lim, size=out_f * in_f))
    return np.concatenate(parts).astype(np.float32)


# The paper's own networks (Sec. 5 "Architecture", Table 1): (out, in) of each
# weight matrix, hidden layers then the output row.
PAPER_LAYERS = {0: [(64, 6), (64, 64), (1, 64)], 1: [(48, 13), (48, 48), (48, 48), (1, 48)]}


def xavier_layers(shapes, gen: np.random.Generator) -> np.ndarray:
    """Flat float32 Glorot-uniform weights of row-major [out][in] matrices."""
    parts = []
    for out_f, in_f in shapes:
        lim = math.sqrt(6.0 / (in_f + out_f))
        parts.append(gen.uniform(-lim, lim, size=out_f * in_f))
    return np.concatenate(parts).astype(np.float32)


def rays_inside_box(n: int, aabb: np.ndarray, gen: np.random.Generator):
    """Origins uniform strictly inside the box (5 %..95 % of each extent), unit
    directions uniform on the sphere, t_max = +inf: rays of the inner network
    (secondary rays that start on a surface inside the AABB)."""
    lo, hi = aabb[:3].astype(np.float64), aabb[3:].astype(np.float64)
    o = lo[None, :] + gen.uniform(0.05, 0.95, size=(n, 3)) * (hi - lo)[None, :]
    d = _normalize32(gen.standard_normal(size=(n, 3)).astype(np.float32))
    rays = np.concatenate([o.astype(np.float32), d], axis=1).astype(np.float32)
    return rays, np.full(n, np.inf, dtype=np.float32)


def rays_surface_to_light(n: int, tris: np.ndarray, gen: np.random.Generator, light_y=FRAME_LIGHT_Y,
                          light_half=FRAME_LIGHT_HALF, offset: float = 0.0):
    """Shadow rays of the inner network: origins at uniform barycentric points of
    uniformly chosen triangles (on the object, so inside its AABB), aimed at
    uniform points of the frame's area light; t_max = the distance.  offset > 0
    moves each origin that far towards the light (and shortens t_max), so that
    exact labels do not count the surface the ray starts on."""
    t = tris[gen.integers(0, tris.shape[0], n)].astype(np.float64).reshape(n, 3, 3)
    a, b = gen.uniform(size=n), gen.uniform(size=n)
    flip = a + b > 1.0
    a, b = np.where(flip, 1.0 - a, a), np.where(flip, 1.0 - b, b)
    o = t[:, 0] + a[:, None] * (t[:, 1] - t[:, 0]) + b[:, None] * (t[:, 2] - t[:, 0])
    lp = np.empty((n, 3))
    lp[:, 0] = gen.uniform(-light_half, light_half, n)
    lp[:, 1] = light_y
    lp[:, 2] = gen.uniform(-light_half, light_half, n)
    if offset > 0.0:
        u = lp - o
        o = o + offset * u / np.linalg.norm(u, axis=1, keepdims=True)
    o32 = o.astype(np.float32)
    v = lp.astype(np.float32) - o32
    d = _normalize32(v)
    tmax = np.sqrt((v.astype(np.float64) ** 2).sum(axis=1)).astype(np.float32)
    return np.concatenate([o32, d], axis=1).astype(np.float32), tmax


def scaled_mlp(shape: ModelShape, gen: np.random.Generator, gain: float) -> np.ndarray:
    """Xavier weights multiplied by gain: a wider logit range for parity cases."""
    return (xavier_mlp(shape, gen).astype(np.float64) * gain).astype(np.float32)


# --------------------------------------------------------------------------
# Workload bundles
# --------------------------------------------------------------------------


def tiny_workload(n_rays: int = 16384, n_tris: int = 2048):
    """One object of random triangles in [-1,1]^3 seen from a radius-3 sphere."""
    tris = random_triangles(n_tris, rng(CFG_TINY, 0))
    box = mesh_aabb(tris)
    rays, tmax = rays_sphere_to_box(n_rays, box, rng(CFG_TINY, 1))
    w = xavier_mlp(TINY, rng(CFG_TINY, 3))
    return dict(shape=TINY, tris=tris, aabb=box[None, :], rays=rays, tmax=tmax,
                ids=np.zeros(n_rays, np.int32), mlps=w[None, :], mlp_index=np.zeros(1, np.int32))


def frame_mesh(n_lon: int = 1000, n_rings: int = 500) -> np.ndarray:
    """1,000,000-triangle displaced sphere (amplitude 0.2) centred at (0, 2, 0)."""
    return displaced_uv_sphere(n_lon, n_rings, FRAME_CENTER, 1.0, 0.2, rng(CFG_FRAME, 0))


def frame_workload(n_rays: int = 1920 * 1080, with_mesh: bool = True, ray_stream: int = 1, cfg: int = CFG_FRAME):
    tris = frame_mesh() if with_mesh else None
    box = mesh_aabb(tris) if with_mesh else frame_aabb()
    rays, tmax = rays_ground_to_light(n_rays, rng(cfg, ray_stream))
    w = xavier_mlp(FRAME, rng(CFG_FRAME, 3))
    return dict(shape=FRAME, tris=tris, aabb=box[None, :], rays=rays, tmax=tmax,
                ids=np.zeros(n_rays, np.int32), mlps=w[None, :], mlp_index=np.zeros(1, np.int32))


_FRAME_AABB = None


def frame_aabb() -> np.ndarray:
    global _FRAME_AABB
    if _FRAME_AABB is None:
        _FRAME_AABB = mesh_aabb(frame_mesh())
    return _FRAME_AABB


def train_batch(step: int, n: int = 262144):
    """Fresh shadow rays of the frame scene for training step `step`."""
    return rays_ground_to_light(n, rng(CFG_TRAIN, 5, step))


def zipf_ids(n: int, k: int, s: float, gen: np.random.Generator) -> np.ndarray:
    """i.i.d. object ids with P(j) proportional to (j+1)^-s, j = 0..k-1."""
    p = (np.arange(1, k + 1, dtype=np.float64)) ** (-s)
    p /= p.sum()
    return gen.choice(k, size=n, p=p).astype(np.int32)


def multi_workload(n_objects: int = 32, n_rays: int = 4194304, zipf_s: float = 1.1,
                   tri_lo: float = 1e3, tri_hi: float = 2e6, with_mesh: bool = False):
    """Objects with log-uniform triangle counts, rays assigned by Zipf, each ray
    following the radius-3 sphere recipe relative to its object's box; the
    array is shuffled (unsorted arrival)."""
    g = rng(CFG_MULTI, 0)
    tri_counts = np.round(np.exp(g.uniform(math.log(tri_lo), math.log(tri_hi), n_objects))).astype(np.int64)
    centers = g.uniform(-20.0, 20.0, size=(n_objects, 3))
    meshes, boxes = [], []
    for k in range(n_objects):
        n_lon, n_rings = uv_sphere_dims(int(tri_counts[k]))
        if with_mesh:
            m = displaced_uv_sphere(n_lon, n_rings, centers[k], 1.0, 0.2, rng(CFG_MULTI, 0, k))
            meshes.append(m)
            boxes.append(mesh_aabb(m))
        else:
            boxes.append(np.concatenate([centers[k] - 1.2, centers[k] + 1.2]).astype(np.float32))
    boxes = np.stack(boxes)
    ids = zipf_ids(n_rays, n_objects, zipf_s, rng(CFG_MULTI, 4))
    rays = np.empty((n_rays, 6), np.float32)
    tmax = np.empty(n_rays, np.float32)
    gr = rng(CFG_MULTI, 1)
    for k in range(n_objects):
        sel = np.nonzero(ids == k)[0]
        if sel.size == 0:
            continue
        box = boxes[k]
        ctr = 0.5 * (box[:3].astype(np.float64) + box[3:])
        half = 0.5 * float((box[3:].astype(np.float64) - box[:3]).max())
        r, t = rays_sphere_to_box(sel.size, box, gr, radius=3.0 * half, center=ctr)
        rays[sel] = r
        tmax[sel] = t
    mlps = np.stack([xavier_mlp(FRAME, rng(CFG_MULTI, 3, k)) for k in range(n_objects)])
    return dict(shape=FRAME, tris=meshes if with_mesh else None, tri_counts=tri_counts, aabb=boxes,
                rays=rays, tmax=tmax, ids=ids, mlps=mlps, mlp_index=np.arange(n_objects, dtype=np.int32))


def multi_train_batch(box, obj: int, step: int, n: int = 262144):
    """Fresh training rays of one object of the multi-object workload: the same
    radius-3 sphere recipe relative to its box."""
    box = np.asarray(box, np.float32)
    ctr = 0.5 * (box[:3].astype(np.float64) + box[3:])
    half = 0.5 * float((box[3:].astype(np.float64) - box[:3]).max())
    return rays_sphere_to_box(n, box, rng(CFG_MULTI, 5, obj, step), radius=3.0 * half, center=ctr)


# --------------------------------------------------------------------------
# Large scene: 64 displaced spheres on a ground plane, 30M triangles in all,
# a 1920 x 1080 grid of ground points, 4 light samples per pixel.
# --------------------------------------------------------------------------
SCENE_OBJECTS = 64
SCENE_TRIANGLES = 30_000_000
SCENE_X, SCENE_Z = 24.0, 13.5          # ground half extents
SCENE_LIGHT_Y, SCENE_LIGHT_HALF = 30.0, 2.0
SCENE_W, SCENE_H, SCENE_SPP = 1920, 1080, 4


def scene_layout():
    """Triangle targets, (n_lon, n_rings), radii and centres of the 64 objects:
    counts log-uniform in [1e3, 2e6] rescaled to sum to 30M, radii U(0.5, 1.5),
    centres uniform on the ground, sunk to y = 0.9 r."""
    g = rng(CFG_SCENE, 0)
    t = np.exp(g.uniform(math.log(1e3), math.log(2e6), SCENE_OBJECTS))
    t *= SCENE_TRIANGLES / t.sum()
    dims = [uv_sphere_dims(int(round(x))) for x in t]
    radii = g.uniform(0.5, 1.5, SCENE_OBJECTS)
    centers = np.stack([g.uniform(-SCENE_X, SCENE_X, SCENE_OBJECTS), 0.9 * radii,
                        g.uniform(-SCENE_Z, SCENE_Z, SCENE_OBJECTS)], axis=1)
    counts = np.array([2 * a + 2 * a * (b - 1) for a, b in dims], np.int64)
    return dict(dims=dims, radii=radii, centers=centers, tri_counts=counts)


def scene_meshes():
    """The 64 meshes (float32 [T_k, 3, 3] each), displacement amplitude 0.2."""
    lay = scene_layout()
    return [displaced_uv_sphere(a, b, lay["centers"][k], float(lay["radii"][k]), 0.2, rng(CFG_SCENE, 0, k))
            for k, (a, b) in enumerate(lay["dims"])]


def scene_rays(light_seed: int = 0):
    """Shadow rays of the frame: pixel (i, j) -> ground point (x, 0, z) at the
    pixel centre, 4 light samples per pixel stratified 2 x 2 on the 4 x 4 light
    at height 30 and jittered; d unit (float32), t_max = distance to the
    sample.  Order: row j, column i, sample.  Returns rays [N, 6], t_max [N]."""
    i = (np.arange(SCENE_W) + 0.5) / SCENE_W
    j = (np.arange(SCENE_H) + 0.5) / SCENE_H
    gx = -SCENE_X + 2 * SCENE_X * i
    gz = -SCENE_Z + 2 * SCENE_Z * j
    n_pix = SCENE_W * SCENE_H
    o = np.zeros((n_pix, SCENE_SPP, 3))
    o[:, :, 0] = np.tile(gx, SCENE_H)[:, None]
    o[:, :, 2] = np.repeat(gz, SCENE_W)[:, None]
    g = rng(CFG_SCENE, 6, light_seed)
    jit = g.uniform(size=(n_pix, SCENE_SPP, 2))
    sx = np.array([0, 1, 0, 1])[None, :]
    sz = np.array([0, 0, 1, 1])[None, :]
    lx = -SCENE_LIGHT_HALF + SCENE_LIGHT_HALF * (sx + jit[:, :, 0])
    lz = -SCENE_LIGHT_HALF + SCENE_LIGHT_HALF * (sz + jit[:, :, 1])
    light = np.stack([lx, np.full_like(lx, SCENE_LIGHT_Y), lz], axis=-1)
    o32 = o.reshape(-1, 3).astype(np.float32)
    v = light.reshape(-1, 3).astype(np.float32) - o32
    d = _normalize32(v)
    tmax = np.sqrt((v.astype(np.float64) ** 2).sum(axis=1)).astype(np.float32)
    return np.concatenate([o32, d], axis=1).astype(np.float32), tmax


def scene_workload(light_seed: int = 0, with_mesh: bool = True):
    meshes = scene_meshes() if with_mesh else None
    lay = scene_layout()
    if with_mesh:
        boxes = np.stack([mesh_aabb(m) for m in meshes])
    else:  # the undisplaced bounds widened by the displacement amplitude
        r = (1.2 * lay["radii"])[:, None]
        boxes = np.concatenate([lay["centers"] - r, lay["centers"] + r], axis=1).astype(np.float32)
    rays, tmax = scene_rays(light_seed)
    mlps = np.stack([xavier_mlp(FRAME, rng(CFG_SCENE, 3, k)) for k in range(SCENE_OBJECTS)])
    return dict(shape=FRAME, tris=meshes, tri_counts=lay["tri_counts"], aabb=boxes, rays=rays, tmax=tmax,
                mlps=mlps, mlp_index=np.arange(SCENE_OBJECTS, dtype=np.int32))
