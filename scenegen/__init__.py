"""Seeded synthetic inputs for the polarized path tracer.

This module only *generates input data*: triangle meshes, analytic spheres, material
records, rectangular area lights, parameter tensors and camera views, serialised into
the binary scene blob that both the HIP library and the CPU oracle parse with their own
code.  It contains none of the rendering or differentiation arithmetic.

The workloads stand in for the paper's scenes, which are not available (Sec. 5 uses
Mitsuba scenes such as the Cornell box or the Modern Hall): every configuration below is
a seeded, synthetic scene of the stated size, structure and material mix.
"""
from __future__ import annotations

import struct
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------- constants
MAGIC = 0x31545050  # 'PPT1'
VERSION = 2

MAT_LAMBERT = 0        # depolarizing diffuse reflector (Sec. 4.1: only M00 is non-zero)
MAT_DIELECTRIC = 1     # smooth dielectric interface, polarized Fresnel R/T (delta lobes)
MAT_GGX_DIELECTRIC = 2 # reflection-only microfacet pBRDF, real IOR
MAT_GGX_CONDUCTOR = 3  # reflection-only microfacet pBRDF, complex IOR n + i k
MAT_SHEET = 4          # ideal linear polarizer sheet (delta transmission)
MAT_EMITTER = 5        # black, one-sided emitter (the geometry of an area light)
MAT_BLEND = 6          # stochastic 50/50-style blend of a Lambertian and a GGX dielectric lobe

SENSOR_NONE = 0        # output the full Stokes vector in the sensor frame
SENSOR_POLARIZER = 1   # ideal linear polarizer at angle theta (a parameter)
SENSOR_ANALYZER4 = 2   # four analyzers: 0, 45, 90 degree polarizers and QWP(0) + 45 degree polarizer
SENSOR_LIGHTSTAGE4 = 3 # four analyzers: 0, 45, 90 degree polarizers and QWP(0) + -45 degree polarizer

FLAG_NO_NEE = 1

VIEW_DTYPE = np.dtype([
    ("world", "<i4"), ("width", "<i4"), ("height", "<i4"), ("spp", "<i4"),
    ("crop_x0", "<i4"), ("crop_y0", "<i4"), ("crop_w", "<i4"), ("crop_h", "<i4"),
    ("origin", "<f4", 3), ("target", "<f4", 3), ("up", "<f4", 3), ("fov_y_deg", "<f4"),
    ("sensor", "<i4"), ("theta_slot", "<i4"), ("theta_off", "<i4"), ("view_id", "<u4"),
])
assert VIEW_DTYPE.itemsize == 88

MAT_DTYPE = np.dtype([
    ("type", "<u4"),
    ("albedo_slot", "<i4"), ("albedo_off", "<u4"), ("albedo_tw", "<u4"), ("albedo_th", "<u4"),
    ("alpha_slot", "<i4"), ("alpha_off", "<u4"), ("alpha_tw", "<u4"), ("alpha_th", "<u4"),
    ("eta_slot", "<i4"), ("eta_off", "<u4"),
    ("kappa_slot", "<i4"), ("kappa_off", "<u4"),
    ("emit_slot", "<i4"), ("emit_off", "<u4"),
    ("axis", "<f4", 3), ("blend", "<f4"),
    ("emit_circ", "<f4"),
    ("spec_slot", "<i4"), ("spec_off", "<u4"), ("spec_tw", "<u4"), ("spec_th", "<u4"),
    ("normal_slot", "<i4"), ("normal_off", "<u4"), ("normal_tw", "<u4"), ("normal_th", "<u4"),
    ("reserved", "<u4", 4),
])
assert MAT_DTYPE.itemsize == 128

LIGHT_DTYPE = np.dtype([
    ("p0", "<f4", 3), ("eu", "<f4", 3), ("ev", "<f4", 3),
    ("le_slot", "<i4"), ("le_off", "<u4"), ("circ", "<f4"),
])
assert LIGHT_DTYPE.itemsize == 48


def analyzer_count(sensor: int) -> int:
    return 4 if sensor in (SENSOR_ANALYZER4, SENSOR_LIGHTSTAGE4) else 1


# ----------------------------------------------------------------------------- containers
@dataclass
class World:
    tri_v: list = field(default_factory=list)    # arrays (n, 3, 3) float32
    tri_uv: list = field(default_factory=list)   # arrays (n, 3, 2) float32
    tri_mat: list = field(default_factory=list)  # arrays (n,) uint32
    spheres: list = field(default_factory=list)  # (cx, cy, cz, r, mat)
    materials: list = field(default_factory=list)
    lights: list = field(default_factory=list)

    def add_material(self, **kw) -> int:
        rec = np.zeros((), MAT_DTYPE)
        for k in ("albedo_slot", "alpha_slot", "eta_slot", "kappa_slot", "emit_slot", "spec_slot", "normal_slot"):
            rec[k] = -1
        rec["blend"] = 0.5
        for k, v in kw.items():
            rec[k] = v
        self.materials.append(rec)
        return len(self.materials) - 1

    def add_tris(self, v, uv, mat):
        v = np.asarray(v, np.float32).reshape(-1, 3, 3)
        uv = np.zeros((v.shape[0], 3, 2), np.float32) if uv is None else np.asarray(uv, np.float32).reshape(-1, 3, 2)
        m = np.broadcast_to(np.asarray(mat, np.uint32), (v.shape[0],)).copy()
        self.tri_v.append(v)
        self.tri_uv.append(uv)
        self.tri_mat.append(m)

    def add_quad(self, p0, eu, ev, mat, uv_rect=(0.0, 0.0, 1.0, 1.0)):
        """Two triangles p0, p0+eu, p0+eu+ev / p0, p0+eu+ev, p0+ev; normal along eu x ev."""
        p0, eu, ev = (np.asarray(a, np.float64) for a in (p0, eu, ev))
        a, b, c, d = p0, p0 + eu, p0 + eu + ev, p0 + ev
        u0, v0, u1, v1 = uv_rect
        ta, tb, tc, td = (u0, v0), (u1, v0), (u1, v1), (u0, v1)
        self.add_tris([[a, b, c], [a, c, d]], [[ta, tb, tc], [ta, tc, td]], mat)

    def add_sphere(self, c, r, mat):
        self.spheres.append((float(c[0]), float(c[1]), float(c[2]), float(r), int(mat)))

    def add_light(self, p0, eu, ev, le_slot, le_off=0, circ=0.0):
        """Rectangular one-sided area light; adds its emitter geometry and its NEE record.
        circ is the degree of circular polarization of the emission, Le (1, 0, 0, circ)."""
        m = self.add_material(type=MAT_EMITTER, emit_slot=le_slot, emit_off=le_off, emit_circ=circ)
        self.add_quad(p0, eu, ev, m)
        rec = np.zeros((), LIGHT_DTYPE)
        rec["p0"], rec["eu"], rec["ev"] = p0, eu, ev
        rec["le_slot"], rec["le_off"], rec["circ"] = le_slot, le_off, circ
        self.lights.append(rec)

    def n_tris(self):
        return int(sum(a.shape[0] for a in self.tri_v))


class Scene:
    """Parameter slots plus one or more worlds (independent geometry/material sets)."""

    def __init__(self):
        self.slot_names: list[str] = []
        self.slot_values: list[np.ndarray] = []
        self.worlds: list[World] = []

    def add_slot(self, name, values) -> int:
        assert name not in self.slot_names, name
        self.slot_names.append(name)
        self.slot_values.append(np.ascontiguousarray(np.asarray(values, np.float32).reshape(-1)))
        return len(self.slot_names) - 1

    def slot(self, name) -> int:
        return self.slot_names.index(name)

    def add_world(self) -> World:
        self.worlds.append(World())
        return self.worlds[-1]

    def params(self):
        """Fresh float32 copies of the initial parameter values, one array per slot."""
        return [v.copy() for v in self.slot_values]

    def to_blob(self) -> bytes:
        out = [struct.pack("<4I", MAGIC, VERSION, len(self.slot_values), len(self.worlds))]
        out.append(np.asarray([v.size for v in self.slot_values], "<u4").tobytes())
        for w in self.worlds:
            tv = np.concatenate(w.tri_v) if w.tri_v else np.zeros((0, 3, 3), np.float32)
            tuv = np.concatenate(w.tri_uv) if w.tri_uv else np.zeros((0, 3, 2), np.float32)
            tm = np.concatenate(w.tri_mat) if w.tri_mat else np.zeros((0,), np.uint32)
            sph = np.asarray([s[:4] for s in w.spheres], "<f4").reshape(-1, 4)
            sm = np.asarray([s[4] for s in w.spheres], "<u4").reshape(-1)
            mats = np.asarray(w.materials, MAT_DTYPE).reshape(-1)
            lights = np.asarray(w.lights, LIGHT_DTYPE).reshape(-1)
            out.append(struct.pack("<4I", tv.shape[0], sph.shape[0], mats.shape[0], lights.shape[0]))
            out += [tv.astype("<f4").tobytes(), tuv.astype("<f4").tobytes(), tm.astype("<u4").tobytes(),
                    sph.tobytes(), sm.tobytes(), mats.tobytes(), lights.tobytes()]
        return b"".join(out)


@dataclass
class Workload:
    name: str
    scene: Scene
    views: np.ndarray
    max_depth: int
    seed: int
    flags: int = 0
    grad_slots: tuple = ()
    meta: dict = field(default_factory=dict)

    def n_paths(self):
        v = self.views
        return int(np.sum(v["crop_w"].astype(np.int64) * v["crop_h"] * v["spp"]))

    def image_numel(self):
        return image_numel(self.views)


def image_numel(views) -> int:
    a = np.where(np.isin(views["sensor"], (SENSOR_ANALYZER4, SENSOR_LIGHTSTAGE4)), 4, 1)
    return int(np.sum(a * views["crop_w"].astype(np.int64) * views["crop_h"] * 12))


def view_offsets(views) -> np.ndarray:
    """Float offset of each view's block in the concatenated [V][A][h][w][3][4] output."""
    a = np.where(np.isin(views["sensor"], (SENSOR_ANALYZER4, SENSOR_LIGHTSTAGE4)), 4, 1)
    sizes = a * views["crop_w"].astype(np.int64) * views["crop_h"] * 12
    return np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)


def make_view(world=0, width=32, height=32, spp=4, origin=(0, 1, 6), target=(0, -0.5, 0), up=(0, 1, 0),
              fov=40.0, sensor=SENSOR_POLARIZER, theta_slot=-1, theta_off=0, view_id=0, crop=None):
    v = np.zeros((), VIEW_DTYPE)
    v["world"], v["width"], v["height"], v["spp"] = world, width, height, spp
    cx0, cy0, cw, ch = crop if crop is not None else (0, 0, width, height)
    v["crop_x0"], v["crop_y0"], v["crop_w"], v["crop_h"] = cx0, cy0, cw, ch
    v["origin"], v["target"], v["up"], v["fov_y_deg"] = origin, target, up, fov
    v["sensor"], v["theta_slot"], v["theta_off"], v["view_id"] = sensor, theta_slot, theta_off, view_id
    return v


def crop_views(views, cx0, cy0, cw, ch):
    """Same views restricted to one pixel window (the per-pixel RNG keeps crops exact)."""
    v = views.copy()
    v["crop_x0"], v["crop_y0"] = cx0, cy0
    v["crop_w"] = np.minimum(cw, v["width"] - cx0)
    v["crop_h"] = np.minimum(ch, v["height"] - cy0)
    return v


# ----------------------------------------------------------------------------- geometry helpers
def icosphere(subdiv: int):
    """Unit icosphere as (n, 3, 3) triangles with outward winding."""
    t = (1.0 + 5 ** 0.5) / 2
    verts = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t], [0, -1, -t],
                      [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], np.float64)
    faces = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4],
                      [11, 10, 2], [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8],
                      [3, 8, 9], [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]])
    tris = verts[faces]
    tris /= np.linalg.norm(tris, axis=-1, keepdims=True)
    for _ in range(subdiv):
        a, b, c = tris[:, 0], tris[:, 1], tris[:, 2]
        ab, bc, ca = (a + b), (b + c), (c + a)
        ab /= np.linalg.norm(ab, axis=-1, keepdims=True)
        bc /= np.linalg.norm(bc, axis=-1, keepdims=True)
        ca /= np.linalg.norm(ca, axis=-1, keepdims=True)
        tris = np.concatenate([np.stack([a, ab, ca], 1), np.stack([b, bc, ab], 1),
                               np.stack([c, ca, bc], 1), np.stack([ab, bc, ca], 1)])
    n = np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])
    flip = np.einsum("ij,ij->i", n, tris.mean(1)) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    return tris


def sphere_uv(p):
    """Equirectangular uv of unit-sphere points (input data for texture lookups)."""
    u = 0.5 + np.arctan2(p[..., 2], p[..., 0]) / (2 * np.pi)
    v = np.arccos(np.clip(p[..., 1], -1, 1)) / np.pi
    return np.stack([u, v], -1)


def random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def smooth_noise(rng, h, w, ch, coarse=8, lo=0.2, hi=0.8):
    """Seeded smooth texture in [lo, hi]: bilinear upsampling of a coarse uniform grid."""
    g = rng.uniform(0, 1, size=(coarse + 1, coarse + 1, ch))
    ys = np.linspace(0, coarse, h, endpoint=False) + coarse / (2 * h)
    xs = np.linspace(0, coarse, w, endpoint=False) + coarse / (2 * w)
    y0 = np.floor(ys).astype(int); x0 = np.floor(xs).astype(int)
    fy = (ys - y0)[:, None, None]; fx = (xs - x0)[None, :, None]
    y1 = np.minimum(y0 + 1, coarse); x1 = np.minimum(x0 + 1, coarse)
    t = (g[y0][:, x0] * (1 - fy) * (1 - fx) + g[y0][:, x1] * (1 - fy) * fx
         + g[y1][:, x0] * fy * (1 - fx) + g[y1][:, x1] * fy * fx)
    t = (t - t.min()) / max(t.max() - t.min(), 1e-12)
    return (lo + (hi - lo) * t).astype(np.float32)


def perlin2d(rng, n, cells):
    """Gradient (Perlin 2002 'improved' fade) noise on an n x n lattice with `cells` gradient cells."""
    ang = rng.uniform(0, 2 * np.pi, size=(cells + 1, cells + 1))
    gx, gy = np.cos(ang), np.sin(ang)
    xs = np.linspace(0, cells, n, endpoint=False)
    x0 = np.floor(xs).astype(int); fx = xs - x0
    X0, Y0 = np.meshgrid(x0, x0, indexing="xy")
    FX, FY = np.meshgrid(fx, fx, indexing="xy")

    def dot(ix, iy, dx, dy):
        return gx[iy, ix] * dx + gy[iy, ix] * dy

    fade = lambda t: t * t * t * (t * (t * 6 - 15) + 10)
    n00 = dot(X0, Y0, FX, FY); n10 = dot(X0 + 1, Y0, FX - 1, FY)
    n01 = dot(X0, Y0 + 1, FX, FY - 1); n11 = dot(X0 + 1, Y0 + 1, FX - 1, FY - 1)
    u, v = fade(FX), fade(FY)
    return (n00 * (1 - u) + n10 * u) * (1 - v) + (n01 * (1 - u) + n11 * u) * v


# ----------------------------------------------------------------------------- workloads
def _ground(world, y, half, mat, uv=True):
    # normal +y: eu x ev must point up -> eu = +z, ev = +x
    world.add_quad((-half, y, -half), (0, 0, 2 * half), (2 * half, 0, 0), mat,
                   uv_rect=(0.0, 0.0, 1.0, 1.0) if uv else (0, 0, 0, 0))


def config1(seed: int = 1, theta_deg: float = 30.0) -> Workload:
    """Tiny scene: ground plane, 3 analytic spheres, one 2x2 area light, polarizer camera.

    32x32, 4 spp, max depth 3; sphere 0 and the plane share one Lambertian RGB albedo,
    spheres 1-2 are a smooth dielectric with IOR 1.5.
    """
    rng = np.random.default_rng(seed)
    sc = Scene()
    s_theta = sc.add_slot("theta", [np.deg2rad(theta_deg)])
    s_alb = sc.add_slot("albedo", rng.uniform(0.2, 0.8, 3))
    s_ior = sc.add_slot("ior", [1.5])
    s_le = sc.add_slot("light_Le", [10.0, 10.0, 10.0])
    w = sc.add_world()
    m_lam = w.add_material(type=MAT_LAMBERT, albedo_slot=s_alb)
    m_die = w.add_material(type=MAT_DIELECTRIC, eta_slot=s_ior)
    _ground(w, -1.5, 10.0, m_lam)
    cs, rs = [], []
    while len(cs) < 3:  # non-overlapping spheres (rejection sampling)
        c = rng.uniform(-1, 1, 3); r = rng.uniform(0.2, 0.5)
        if all(np.linalg.norm(c - c2) > r + r2 + 1e-3 for c2, r2 in zip(cs, rs)):
            cs.append(c); rs.append(r)
    for i, (c, r) in enumerate(zip(cs, rs)):
        w.add_sphere(c, r, m_lam if i == 0 else m_die)
    w.add_light((-1, 3, -1), (2, 0, 0), (0, 0, 2), s_le)
    views = np.asarray([make_view(0, 32, 32, 4, (0, 1, 6), (0, -0.5, 0), (0, 1, 0), 40.0,
                                  SENSOR_POLARIZER, s_theta, 0, 0)], VIEW_DTYPE)
    return Workload("c1_tiny", sc, views, max_depth=3, seed=seed,
                    grad_slots=("theta", "albedo", "ior"), meta={"target_theta_deg": 45.0, "target_seed": seed + 1000})


def _icosphere_objects(rng, world, n_obj, materials, base):
    for k in range(n_obj):
        R = random_rotation(rng)
        S = np.diag(rng.uniform(0.3, 0.7, 3))
        t = np.array([rng.uniform(-3, 3), rng.uniform(-0.5, 1.0), rng.uniform(-3, 3)])
        A = R @ S
        tv = base @ A.T + t
        world.add_tris(tv, sphere_uv(base), materials[k])


def _c2_materials(rng, sc, w, n_obj, s_tex, tex_w, tex_h):
    """Object k gets material type k mod 3: GGX dielectric, GGX conductor, textured Lambertian."""
    kinds = [k % 3 for k in range(n_obj)]
    n_ggx = sum(1 for k in kinds if k in (0, 1))
    n_die = sum(1 for k in kinds if k == 0)
    n_con = sum(1 for k in kinds if k == 1)
    s_rough = sc.add_slot("roughness", np.zeros(n_ggx))
    s_ior = sc.add_slot("ior", np.zeros(max(n_die, 1)))
    s_n = sc.add_slot("cond_n", np.zeros(max(n_con, 1)))
    s_k = sc.add_slot("cond_k", np.zeros(max(n_con, 1)))
    mats, ig, idie, icon = [], 0, 0, 0
    for k in kinds:
        if k == 0:
            sc.slot_values[s_rough][ig] = rng.uniform(0.05, 0.5)
            sc.slot_values[s_ior][idie] = rng.uniform(1.3, 1.7)
            mats.append(w.add_material(type=MAT_GGX_DIELECTRIC, alpha_slot=s_rough, alpha_off=ig,
                                       eta_slot=s_ior, eta_off=idie))
            ig += 1; idie += 1
        elif k == 1:
            sc.slot_values[s_n][icon] = rng.uniform(0.2, 1.5)
            sc.slot_values[s_k][icon] = rng.uniform(2.0, 5.0)
            sc.slot_values[s_rough][ig] = rng.uniform(0.05, 0.5)
            mats.append(w.add_material(type=MAT_GGX_CONDUCTOR, alpha_slot=s_rough, alpha_off=ig,
                                       eta_slot=s_n, eta_off=icon, kappa_slot=s_k, kappa_off=icon))
            ig += 1; icon += 1
        else:
            mats.append(w.add_material(type=MAT_LAMBERT, albedo_slot=s_tex, albedo_tw=tex_w, albedo_th=tex_h))
    return mats


RING_R, RING_H = 8.0, 3.0


def ring_pose(k):
    a = np.deg2rad(90.0 * k)
    return (RING_R * np.sin(a), RING_H, RING_R * np.cos(a))


def scene2(seed: int = 2):
    """16 random icospheres (subdivision 3) + textured ground + one 3x3 light (~20.5k tris)."""
    rng = np.random.default_rng(seed)
    sc = Scene()
    s_theta = sc.add_slot("theta", [rng.uniform(0, np.pi)])
    s_tex = sc.add_slot("albedo_tex", smooth_noise(rng, 64, 64, 3))
    w = sc.add_world()
    mats = _c2_materials(rng, sc, w, 16, s_tex, 64, 64)
    s_le = sc.add_slot("light_Le", [10.0, 10.0, 10.0])
    m_ground = w.add_material(type=MAT_LAMBERT, albedo_slot=s_tex, albedo_tw=64, albedo_th=64)
    _ground(w, -1.5, 6.0, m_ground)
    _icosphere_objects(rng, w, 16, mats, icosphere(3))
    w.add_light((-1.5, 5, -1.5), (3, 0, 0), (0, 0, 3), s_le)
    return sc, s_theta


def config2(seed: int = 2) -> Workload:
    """Single view at scale: 256x256, 64 spp, depth 8, polarizer camera at theta ~ U[0, pi)."""
    sc, s_theta = scene2(seed)
    views = np.asarray([make_view(0, 256, 256, 64, ring_pose(0), (0, 0, 0), (0, 1, 0), 45.0,
                                  SENSOR_POLARIZER, s_theta, 0, 0)], VIEW_DTYPE)
    return Workload("c2_single_view", sc, views, max_depth=8, seed=seed,
                    grad_slots=("albedo_tex", "roughness", "theta"), meta={"delta_seed": 2002})


def config3(seed: int = 2, res: int = 128, spp: int = 32, n_angles: int = 32, n_poses: int = 4) -> Workload:
    """Batched: the config-2 scene, 4 ring poses x 32 polarizer angles k*pi/32 = 128 views."""
    sc, _ = scene2(seed)
    s_thetas = sc.add_slot("theta_views", [k * np.pi / n_angles for k in range(n_angles)])
    views = []
    for p in range(n_poses):
        for k in range(n_angles):
            vid = p * n_angles + k
            views.append(make_view(0, res, res, spp, ring_pose(p), (0, 0, 0), (0, 1, 0), 45.0,
                                   SENSOR_POLARIZER, s_thetas, k, vid))
    views = np.asarray(views, VIEW_DTYPE)
    return Workload("c3_batched", sc, views, max_depth=6, seed=seed,
                    grad_slots=("albedo_tex", "roughness", "theta_views"), meta={"delta_seed": 3003})


def scene4(seed: int = 4, tex: int = 256, truth: bool = False):
    """32 icospheres + ground with a Lambertian/GGX blend (256^2 albedo and roughness maps), 2 lights."""
    rng = np.random.default_rng(seed)
    sc = Scene()
    s_theta = sc.add_slot("theta_views", [k * np.pi / 8 for k in range(8)])
    alb_true = smooth_noise(rng, tex, tex, 3, coarse=16)
    rough_true = smooth_noise(rng, tex, tex, 1, coarse=16, lo=0.05, hi=0.6)
    le_true = np.array([8.0, 7.5, 7.0, 6.0, 6.5, 7.0], np.float32)
    le_init = le_true * rng.uniform(0.5, 1.5, 6).astype(np.float32)
    s_alb = sc.add_slot("albedo_tex", alb_true if truth else np.full(tex * tex * 3, 0.5))
    s_rgh = sc.add_slot("roughness_tex", rough_true if truth else np.full(tex * tex, 0.3))
    s_ior = sc.add_slot("ground_ior", [1.5])
    w = sc.add_world()
    s_obj_tex = sc.add_slot("object_tex", smooth_noise(rng, 64, 64, 3))
    mats = _c2_materials(rng, sc, w, 32, s_obj_tex, 64, 64)
    s_le = sc.add_slot("light_Le", le_true if truth else le_init)
    m_ground = w.add_material(type=MAT_BLEND, albedo_slot=s_alb, albedo_tw=tex, albedo_th=tex,
                              alpha_slot=s_rgh, alpha_tw=tex, alpha_th=tex, eta_slot=s_ior, blend=0.5)
    _ground(w, -1.5, 6.0, m_ground)
    _icosphere_objects(rng, w, 32, mats, icosphere(3))
    w.add_light((-3.5, 5, -1), (2, 0, 0), (0, 0, 2), s_le, 0)
    w.add_light((1.5, 4.5, 0.5), (2, 0, 0), (0, 0, 2), s_le, 3)
    return sc


def config4(seed: int = 4, res: int = 512, spp: int = 16, truth: bool = False) -> Workload:
    """Optimisation: 8 views at theta_k = k*pi/8 from one pose, 512^2, 16 spp, depth 6."""
    sc = scene4(seed, truth=truth)
    s_theta = sc.slot("theta_views")
    views = np.asarray([make_view(0, res, res, spp, (0.0, 6.0, 7.0), (0, -1, 0), (0, 1, 0), 50.0,
                                  SENSOR_POLARIZER, s_theta, k, k) for k in range(8)], VIEW_DTYPE)
    return Workload("c4_optimisation", sc, views, max_depth=6, seed=seed,
                    grad_slots=("albedo_tex", "roughness_tex", "light_Le"))


def scene5(seed: int, max_objects: int = 64):
    """Terrain from a 1000x1000 Perlin height lattice, meshed to a seeded triangle budget in
    [1e5, 1e6] (log-uniform), plus up to 64 random icospheres; four analyzers on the camera."""
    rng = np.random.default_rng(seed)
    sc = Scene()
    budget = float(np.exp(rng.uniform(np.log(1e5), np.log(1e6))))
    n_obj = int(rng.integers(8, max_objects + 1))
    obj_tris = n_obj * 320  # icosphere subdivision 2
    g = max(int(np.sqrt(max(budget - obj_tris, 2e4) / 2)), 16)
    h = perlin2d(rng, 1000, 12) * 1.2 + perlin2d(rng, 1000, 48) * 0.25
    s_tex = sc.add_slot("albedo_tex", smooth_noise(rng, 128, 128, 3))
    w = sc.add_world()
    mats = _c2_materials(rng, sc, w, n_obj, s_tex, 128, 128)
    s_le = sc.add_slot("light_Le", [12.0, 12.0, 12.0])
    m_ground = w.add_material(type=MAT_LAMBERT, albedo_slot=s_tex, albedo_tw=128, albedo_th=128)
    # sample the lattice at a G x G grid of vertices spanning [-8, 8]^2
    idx = np.linspace(0, 999, g + 1)
    ii = np.round(idx).astype(int)
    H = h[np.ix_(ii, ii)] - 1.5
    xs = np.linspace(-8, 8, g + 1)
    X, Z = np.meshgrid(xs, xs, indexing="xy")
    P = np.stack([X, H, Z], -1)
    UV = np.stack([(X + 8) / 16, (Z + 8) / 16], -1)
    a, b, c, d = P[:-1, :-1], P[:-1, 1:], P[1:, 1:], P[1:, :-1]
    ta, tb, tc, td = UV[:-1, :-1], UV[:-1, 1:], UV[1:, 1:], UV[1:, :-1]
    # normal up: winding (a, d, c), (a, c, b)
    t1 = np.stack([a, d, c], 2).reshape(-1, 3, 3); t2 = np.stack([a, c, b], 2).reshape(-1, 3, 3)
    u1 = np.stack([ta, td, tc], 2).reshape(-1, 3, 2); u2 = np.stack([ta, tc, tb], 2).reshape(-1, 3, 2)
    w.add_tris(np.concatenate([t1, t2]), np.concatenate([u1, u2]), m_ground)
    base = icosphere(2)
    for k in range(n_obj):
        R = random_rotation(rng)
        S = np.diag(rng.uniform(0.2, 0.6, 3))
        x, z = rng.uniform(-6, 6, 2)
        y = h[int((z + 8) / 16 * 999), int((x + 8) / 16 * 999)] - 1.5 + rng.uniform(0.3, 1.0)
        w.add_tris(base @ (R @ S).T + np.array([x, y, z]), sphere_uv(base), mats[k])
    w.add_light((-2, 7, -2), (4, 0, 0), (0, 0, 4), s_le)
    return sc


def config5(seeds=range(50, 58), crop=None):
    """Eight uneven scenes (resolutions 256..1024, 64..256 spp, depth 12) in one scene object.

    Each seed becomes one world of a multi-world scene; every world has its own parameter slots
    (prefixed with the world index) so gradients of all material parameters stay separate.
    """
    seeds = list(seeds)
    rng = np.random.default_rng(5000 + seeds[0])
    res_choices = [256, 384, 512, 640, 768, 896, 1024, 512][: len(seeds)]
    spp_choices = [64, 96, 128, 160, 192, 224, 256, 64][: len(seeds)]
    rng.shuffle(res_choices); rng.shuffle(spp_choices)
    merged = Scene()
    views = []
    for wi, s in enumerate(seeds):
        sc = scene5(s)
        remap = {}
        for name, val in zip(sc.slot_names, sc.slot_values):
            remap[sc.slot(name)] = merged.add_slot(f"w{wi}_{name}", val)
        w = sc.worlds[0]
        for rec in w.materials:
            for k in ("albedo_slot", "alpha_slot", "eta_slot", "kappa_slot", "emit_slot", "spec_slot", "normal_slot"):
                if rec[k] >= 0:
                    rec[k] = remap[int(rec[k])]
        for rec in w.lights:
            rec["le_slot"] = remap[int(rec["le_slot"])]
        merged.worlds.append(w)
        r = res_choices[wi]
        views.append(make_view(wi, r, r, spp_choices[wi], (0.0, 5.0, 10.0), (0, -1, 0), (0, 1, 0), 50.0,
                               SENSOR_ANALYZER4, -1, 0, wi))
    views = np.asarray(views, VIEW_DTYPE)
    if crop is not None:
        cw, ch = crop
        views = crop_views(views, 0, 0, cw, ch)
        views["crop_x0"] = (views["width"] - cw) // 2
        views["crop_y0"] = (views["height"] - ch) // 2
    grad = tuple(n for n in merged.slot_names)
    return Workload("c5_uneven", merged, views, max_depth=12, seed=50, grad_slots=grad)


def polarizer_stack(n_sheets: int = 85, width: int = 1280, height: int = 720, spp: int = 1, step_deg: float = 1.0,
                    max_depth: int = 128) -> Workload:
    """Deep-path benchmark scene: a Lambertian floor (RGB albedo parameter) and back wall under an
    area light, seen through a stack of linear polarizer sheets whose axes turn by step_deg from
    one sheet to the next, so that a camera path crosses n_sheets delta vertices before its first
    diffuse vertex.  1280x720 at 1 spp by default."""
    sc = Scene()
    s_alb = sc.add_slot("floor_albedo", [0.6, 0.5, 0.4])
    s_wall = sc.add_slot("wall_albedo", [0.7, 0.7, 0.7])
    s_le = sc.add_slot("light_Le", [20.0, 20.0, 20.0])
    w = sc.add_world()
    m_floor = w.add_material(type=MAT_LAMBERT, albedo_slot=s_alb)
    m_wall = w.add_material(type=MAT_LAMBERT, albedo_slot=s_wall)
    _ground(w, 0.0, 12.0, m_floor, uv=False)
    w.add_quad((-12, 0, -3), (24, 0, 0), (0, 12, 0), m_wall)  # back wall facing +z
    w.add_light((-1.5, 6.0, -1.5), (3.0, 0, 0), (0, 0, 3.0), s_le)  # facing -y (eu x ev = -y)
    for i in range(n_sheets):
        z = 6.0 - 4.0 * i / max(n_sheets - 1, 1)
        a = np.deg2rad(step_deg * i)
        m = w.add_material(type=MAT_SHEET, axis=(np.cos(a), np.sin(a), 0.0))
        w.add_quad((-3.0, -1.0, z), (6.0, 0, 0), (0, 6.0, 0), m)
    views = np.asarray([make_view(0, width, height, spp, (0.0, 2.0, 9.0), (0.0, 1.5, 0.0), (0, 1, 0), 45.0,
                                  SENSOR_NONE)], VIEW_DTYPE)
    return Workload("polarizer_stack", sc, views, max_depth=max_depth, seed=7,
                    grad_slots=("floor_albedo",))


def glossy_scene(seed: int = 3, width: int = 24, height: int = 16, spp: int = 4, max_depth: int = 8) -> Workload:
    """Microfacet-only scene (GGX conductors and a GGX dielectric, no depolarizing or polarizer
    surfaces) under one area light: every block of path vertices has an invertible Mueller
    throughput away from Brewster-like reflections.  Full Stokes camera."""
    rng = np.random.default_rng(seed)
    sc = Scene()
    s_rgh = sc.add_slot("roughness", [0.3, 0.2, 0.25])
    s_eta = sc.add_slot("eta", [0.8, 1.5])
    s_kap = sc.add_slot("kappa", [3.5])
    s_le = sc.add_slot("light_Le", [10.0, 10.0, 10.0])
    w = sc.add_world()
    m_gc = w.add_material(type=MAT_GGX_CONDUCTOR, alpha_slot=s_rgh, alpha_off=0, eta_slot=s_eta, eta_off=0,
                          kappa_slot=s_kap)
    m_gd = w.add_material(type=MAT_GGX_DIELECTRIC, alpha_slot=s_rgh, alpha_off=1, eta_slot=s_eta, eta_off=1)
    m_gc2 = w.add_material(type=MAT_GGX_CONDUCTOR, alpha_slot=s_rgh, alpha_off=2, eta_slot=s_eta, eta_off=0,
                           kappa_slot=s_kap)
    _ground(w, -1.0, 8.0, m_gc)
    for k in range(5):
        c = np.array([rng.uniform(-2, 2), rng.uniform(-0.3, 0.8), rng.uniform(-2, 1)])
        w.add_tris(0.6 * icosphere(2) + c, None, (m_gd, m_gc2)[k % 2])
    w.add_quad((-4, -1, -3), (8, 0, 0), (0, 6, 0), m_gc2)
    w.add_light((-1.5, 3.5, -1.5), (3, 0, 0), (0, 0, 3), s_le)
    views = np.asarray([make_view(0, width, height, spp, (0, 1.5, 6), (0, 0, 0), (0, 1, 0), 50.0, SENSOR_NONE)],
                       VIEW_DTYPE)
    return Workload("glossy", sc, views, max_depth=max_depth, seed=5, grad_slots=("roughness", "eta", "kappa"))


# ----------------------------------------------------------------------------- light stage
def normal_map(rng, h, w, amp, coarse=8):
    """Tangent-space normal map input (t, b, n) = (gx, gy, 1) with smooth seeded slopes in
    [-amp, amp]; the renderer normalises it."""
    g = smooth_noise(rng, h, w, 2, coarse=coarse, lo=-amp, hi=amp)
    return np.concatenate([g, np.ones((h, w, 1), np.float32)], -1).astype(np.float32)


def _facing_rect(center, size):
    """(p0, eu, ev) of a size x size rectangle centred at `center` emitting toward the origin."""
    c = np.asarray(center, np.float64)
    n = -c / np.linalg.norm(c)
    a = np.cross(np.array([0.0, 1.0, 0.0]), n)
    a = a / np.linalg.norm(a)
    b = np.cross(n, a)
    eu, ev = a * size, b * size
    if np.dot(np.cross(eu, ev), n) < 0:
        eu, ev = ev, eu
    return c - 0.5 * (eu + ev), eu, ev


def scene_lightstage(seed: int = 6, tex: int = 64):
    """Virtual light stage (the paper's multi-view capture with right-circular illumination,
    synthetic): a normal-mapped central object on a normal-mapped ground, a smooth dielectric and
    a conductor with normal maps, ringed by eight right-circularly polarized area lights."""
    rng = np.random.default_rng(seed)
    sc = Scene()
    w = sc.add_world()
    s_ior = sc.add_slot("ior", [1.5])
    # ground: Lambertian/GGX blend with albedo, roughness, specular and normal maps
    s_galb = sc.add_slot("ground_albedo", smooth_noise(rng, tex, tex, 3))
    s_grgh = sc.add_slot("ground_roughness", smooth_noise(rng, tex, tex, 1, lo=0.1, hi=0.5))
    s_gspc = sc.add_slot("ground_specular", smooth_noise(rng, tex, tex, 1, lo=0.5, hi=1.0))
    s_gnrm = sc.add_slot("ground_normal", normal_map(rng, tex, tex, 0.3))
    m_ground = w.add_material(type=MAT_BLEND, albedo_slot=s_galb, albedo_tw=tex, albedo_th=tex,
                              alpha_slot=s_grgh, alpha_tw=tex, alpha_th=tex, eta_slot=s_ior, blend=0.5,
                              spec_slot=s_gspc, spec_tw=tex, spec_th=tex,
                              normal_slot=s_gnrm, normal_tw=tex, normal_th=tex)
    _ground(w, -1.0, 5.0, m_ground)
    # central object (a stand-in for the captured bust): icosphere with all four maps
    s_oalb = sc.add_slot("object_albedo", smooth_noise(rng, tex, tex, 3, coarse=6))
    s_orgh = sc.add_slot("object_roughness", smooth_noise(rng, tex, tex, 1, coarse=6, lo=0.1, hi=0.6))
    s_ospc = sc.add_slot("object_specular", smooth_noise(rng, tex, tex, 1, coarse=6, lo=0.4, hi=1.0))
    s_onrm = sc.add_slot("object_normal", normal_map(rng, tex, tex, 0.4, coarse=12))
    m_obj = w.add_material(type=MAT_BLEND, albedo_slot=s_oalb, albedo_tw=tex, albedo_th=tex,
                           alpha_slot=s_orgh, alpha_tw=tex, alpha_th=tex, eta_slot=s_ior, blend=0.4,
                           spec_slot=s_ospc, spec_tw=tex, spec_th=tex,
                           normal_slot=s_onrm, normal_tw=tex, normal_th=tex)
    base = icosphere(4)
    w.add_tris(base * 0.9 + np.array([0.0, -0.1, 0.0]), sphere_uv(base), m_obj)
    # smooth dielectric with a normal map: its s/p frames move with the shading normal
    small = icosphere(3)
    s_gnm = sc.add_slot("glass_normal", normal_map(rng, 32, 32, 0.2))
    m_glass = w.add_material(type=MAT_DIELECTRIC, eta_slot=s_ior, normal_slot=s_gnm, normal_tw=32, normal_th=32)
    w.add_tris(small * 0.5 + np.array([1.7, -0.5, 0.6]), sphere_uv(small), m_glass)
    # GGX conductor with a constant specular scale and a normal map
    s_meta = sc.add_slot("metal_eta", [0.6])
    s_mkap = sc.add_slot("metal_kappa", [3.0])
    s_mrgh = sc.add_slot("metal_roughness", [0.25])
    s_mspc = sc.add_slot("metal_specular", [0.8])
    s_mnrm = sc.add_slot("metal_normal", normal_map(rng, 32, 32, 0.3))
    m_metal = w.add_material(type=MAT_GGX_CONDUCTOR, alpha_slot=s_mrgh, eta_slot=s_meta, kappa_slot=s_mkap,
                             spec_slot=s_mspc, normal_slot=s_mnrm, normal_tw=32, normal_th=32)
    w.add_tris(small * 0.5 + np.array([-1.7, -0.5, 0.4]), sphere_uv(small), m_metal)
    # eight right-circular lights on a ring above the object, facing its centre
    s_le = sc.add_slot("light_Le", [3.0, 3.0, 3.0])
    for k in range(8):
        a = 2 * np.pi * (k + 0.5) / 8
        p0, eu, ev = _facing_rect((4.0 * np.cos(a), 3.5, 4.0 * np.sin(a)), 1.6)
        w.add_light(p0, eu, ev, s_le, 0, circ=1.0)
    return sc


def lightstage(seed: int = 6, res: int = 256, spp: int = 16, n_views: int = 8, max_depth: int = 6) -> Workload:
    """Multi-view light-stage capture: n_views cameras on a ring, each with the four analyzer
    states 0, 45, 90 degrees and left-circular; gradients of the normal, specular and roughness
    maps (the parameters of the paper's light-stage gradient study)."""
    sc = scene_lightstage(seed)
    views = []
    for k in range(n_views):
        a = 2 * np.pi * k / n_views
        views.append(make_view(0, res, res, spp, (5.5 * np.cos(a), 1.2, 5.5 * np.sin(a)), (0.0, -0.3, 0.0),
                               (0, 1, 0), 40.0, SENSOR_LIGHTSTAGE4, -1, 0, k))
    return Workload("lightstage", sc, np.asarray(views, VIEW_DTYPE), max_depth=max_depth, seed=seed,
                    grad_slots=("ground_normal", "ground_specular", "ground_roughness", "object_normal",
                                "object_specular", "object_roughness", "glass_normal", "metal_normal",
                                "metal_specular"))


def tilted_plane_scene(phi=0.0, theta_light=0.5, material=MAT_LAMBERT, spec=None, normal_map_on=True):
    """A plane y = 0 (tangent +x along u) whose constant normal map tilts the shading normal by
    phi toward +x, lit by a tiny light at angle theta_light from the geometric normal in the
    xy-plane; the camera looks straight down at the origin through a very narrow field."""
    sc = Scene()
    s_alb = sc.add_slot("albedo", [0.6, 0.5, 0.4])
    s_rgh = sc.add_slot("roughness", [0.3])
    s_ior = sc.add_slot("ior", [1.5])
    s_nrm = sc.add_slot("normal", [np.sin(phi), 0.0, np.cos(phi)])
    s_spc = sc.add_slot("specular", [1.0 if spec is None else spec])
    s_le = sc.add_slot("light_Le", [5.0, 5.0, 5.0])
    w = sc.add_world()
    kw = dict(type=material, albedo_slot=s_alb, alpha_slot=s_rgh, eta_slot=s_ior)
    if normal_map_on:
        kw.update(normal_slot=s_nrm)
    if spec is not None:
        kw.update(spec_slot=s_spc)
    m = w.add_material(**kw)
    # eu = +x (u), ev = -z: normal eu x ev = +y, tangent +x, bitangent +y x +x = -z
    w.add_quad((-50.0, 0.0, 50.0), (100.0, 0.0, 0.0), (0.0, 0.0, -100.0), m)
    d = 20.0
    c = np.array([d * np.sin(theta_light), d * np.cos(theta_light), 0.0])
    p0, eu, ev = _facing_rect(c, 1e-3)
    w.add_light(p0, eu, ev, s_le)
    return sc


# ----------------------------------------------------------------------------- closed-form test scenes
def emitter_wall_scene(le=10.0, sheets=(), z_light=-5.0, size=50.0, circ=0.0):
    """Camera at the origin looking down -z at a huge one-sided emitter (Stokes Le (1, 0, 0,
    circ)); optional polarizer sheets (axis angles in radians, measured from +x toward +y)
    stacked in between."""
    sc = Scene()
    s_theta = sc.add_slot("theta", [0.0])
    s_le = sc.add_slot("light_Le", [le, le, le])
    w = sc.add_world()
    h = size / 2
    # emitter facing +z: eu x ev = +z -> eu = +x, ev = +y
    w.add_light((-h, -h, z_light), (size, 0, 0), (0, size, 0), s_le, circ=circ)
    n = len(sheets)
    for i, a in enumerate(sheets):
        z = -1.0 - (i + 1) * (abs(z_light) - 2.0) / (n + 1)
        m = w.add_material(type=MAT_SHEET, axis=(np.cos(a), np.sin(a), 0.0))
        w.add_quad((-h, -h, z), (size, 0, 0), (0, size, 0), m)
    return sc, s_theta


def furnace_scene(rho=0.6, le=1.0):
    """Camera inside a closed sphere whose inside is Lambertian (albedo rho) and emits le."""
    sc = Scene()
    s_theta = sc.add_slot("theta", [0.0])
    s_alb = sc.add_slot("albedo", [rho, rho, rho])
    s_le = sc.add_slot("emission", [le, le, le])
    w = sc.add_world()
    m = w.add_material(type=MAT_LAMBERT, albedo_slot=s_alb, emit_slot=s_le)
    w.add_sphere((0.0, 0.0, 0.0), -3.0, m)  # negative radius: normals point inward
    return sc, s_theta
