"""Seeded synthetic inputs for the sonar and underwater-camera paths.

This module holds input generation only: it never computes a return's
intensity, bin, speckle or fan value, nor any part of the camera model.  Both
the FP64 oracle and the GPU library consume what it produces.

Returns are generated the way the paper's point-cloud annotator would deliver
them (Sec. III-A.2): points in the sensor frame (x forward, y left, z up) with
surface normals and material ids.  Positions are placed through the inverse
of the polar grid: a range cell and an azimuth cell are drawn uniformly and
the point is put at a uniform fraction inside each, keeping a margin of
``EDGE_MARGIN`` cells from every cell edge, so that after rounding to float32
every hit still sits at least 1e-3 cells from an edge (bin indices are then
unique in any precision that resolves 1e-3 of a cell).  Uniform cells with
uniform in-cell fractions give the uniform range and azimuth laws of the
workloads, minus the excluded bands.

All randomness comes from numpy's ``Generator(Philox(key))`` through
``random()`` doubles only, with every law built by inversion, so the inputs
do not depend on numpy's distribution code.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

SPECKLE_OFF, SPECKLE_PAPER, SPECKLE_GAMMA = 0, 1, 2

BASE_SEED = 250301074
EDGE_MARGIN = 1.5e-3          # cells kept clear of every bin edge before float32 rounding
ELEV_MARGIN = 1e-4            # radians kept clear of the elevation cone edge
DEG = math.pi / 180.0


def _f32(v) -> float:
    return float(np.float32(v))


@dataclass
class SonarSpec:
    """Geometry, physical parameters and RNG key of one sonar frame.

    Floating values are float32-representable, since the GPU receives them as
    float32; the oracle promotes the same values to float64.
    """
    r_min: float
    r_max: float
    n_range: int
    n_azimuth: int
    fov_az: float = _f32(130 * DEG)
    fov_el: float = _f32(20 * DEG)
    fan_h: int = 0
    fan_w: int = 0
    kappa: float = 2.0
    alpha: float = _f32(0.1)
    gain: float = 1.0
    sigma_phi: float = 0.25
    sigma_sa: float = _f32(0.1)
    sigma_sm: float = _f32(0.1)
    speckle_mode: int = SPECKLE_GAMMA
    gamma_k: int = 4
    seed_lo: int = 0
    seed_hi: int = 0
    frame_id: int = 0
    range_norm: int = 0   # 1: each range row divided by its maximum after the gain

    def __post_init__(self):
        for f in ("r_min", "r_max", "fov_az", "fov_el", "kappa", "alpha", "gain", "sigma_phi",
                  "sigma_sa", "sigma_sm"):
            setattr(self, f, _f32(getattr(self, f)))


@dataclass
class SonarHits:
    """Structure-of-arrays hit buffer of one frame plus its reflectivity table."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    nx: np.ndarray
    ny: np.ndarray
    nz: np.ndarray
    mat: np.ndarray          # int32, < 0 = miss
    refl: np.ndarray         # float32 [n_materials]

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class SonarFrame:
    spec: SonarSpec
    hits: SonarHits


@dataclass
class WaterSpec:
    beta_d: np.ndarray       # float32 [3], the paper's beta_attn
    beta_b: np.ndarray       # float32 [3], the paper's beta_bs
    b_inf: np.ndarray        # float32 [3]


@dataclass
class CameraFrame:
    J: np.ndarray            # float32 [3, H, W] planar in-air image
    depth: np.ndarray        # float32 [H, W]
    water_row: int = 0


class Stream:
    """Uniform doubles from numpy's Philox bit generator under a 2-word key."""

    def __init__(self, *key: int):
        k = [int(v) & 0xFFFFFFFFFFFFFFFF for v in key] + [0, 0]
        self.g = np.random.Generator(np.random.Philox(key=np.array(k[:2], dtype=np.uint64)))

    def uniform(self, lo, hi, size=None):
        return lo + (hi - lo) * self.g.random(size)

    def integers(self, lo, hi_inclusive, size=None):
        u = self.g.random(size)
        return (lo + np.floor(u * (hi_inclusive - lo + 1))).astype(np.int64)

    def normal(self, size):
        n = int(np.prod(size))
        m = (n + 1) // 2
        u1 = 1.0 - self.g.random(m)          # (0, 1]
        u2 = self.g.random(m)
        rad = np.sqrt(-2.0 * np.log(u1))
        z = np.concatenate([rad * np.cos(2 * np.pi * u2), rad * np.sin(2 * np.pi * u2)])[:n]
        return z.reshape(size)


def _normals_facing(st: Stream, dx, dy, dz, cos_lo=0.5):
    """Unit normals within acos(cos_lo) of the reversed ray direction -d."""
    n = dx.shape[0]
    cg = st.uniform(cos_lo, 1.0, n)
    sg = np.sqrt(np.maximum(0.0, 1.0 - cg * cg))
    psi = st.uniform(0.0, 2 * np.pi, n)
    # orthonormal basis e1, e2 perpendicular to d: e1 = a x d for a helper
    # axis a = z (or x when d is close to z), e2 = d x e1
    ax = np.where(np.abs(dz) < 0.9, 0.0, 1.0)
    az = 1.0 - ax
    e1x = -az * dy
    e1y = az * dx - ax * dz
    e1z = ax * dy
    nrm = np.sqrt(e1x ** 2 + e1y ** 2 + e1z ** 2)
    e1x, e1y, e1z = e1x / nrm, e1y / nrm, e1z / nrm
    e2x = dy * e1z - dz * e1y
    e2y = dz * e1x - dx * e1z
    e2z = dx * e1y - dy * e1x
    nx = -cg * dx + sg * (np.cos(psi) * e1x + np.sin(psi) * e2x)
    ny = -cg * dy + sg * (np.cos(psi) * e1y + np.sin(psi) * e2y)
    nz = -cg * dz + sg * (np.cos(psi) * e1z + np.sin(psi) * e2z)
    return nx, ny, nz


def make_hits(st: Stream, spec: SonarSpec, n: int, n_materials: Optional[int] = None,
              miss_frac: float = 0.1, outside_frac: float = 0.0,
              normal_cos_lo: float = 0.5) -> SonarHits:
    """``n`` returns spread uniformly over the polar grid of ``spec``.

    A fraction ``miss_frac`` are misses (mat = -1, zero coordinates).  A
    fraction ``outside_frac`` of the hits are placed clearly outside the
    range limits, the azimuth field of view or the elevation cone.  With
    ``n_materials`` None every return has its own reflectivity (mat = k);
    otherwise ids are drawn uniformly from ``n_materials`` materials.
    Reflectivities are U[0.1, 1].
    """
    Nr, Np = spec.n_range, spec.n_azimuth
    rlo, rhi = float(spec.r_min), float(spec.r_max)
    fov, fel = float(spec.fov_az), float(spec.fov_el)
    dr = (rhi - rlo) / Nr
    dphi = fov / Np
    i = st.integers(0, Nr - 1, n)
    j = st.integers(0, Np - 1, n)
    fr = st.uniform(EDGE_MARGIN, 1.0 - EDGE_MARGIN, n)
    fp = st.uniform(EDGE_MARGIN, 1.0 - EDGE_MARGIN, n)
    r = rlo + (i + fr) * dr
    phi = -0.5 * fov + (j + fp) * dphi
    th = st.uniform(-(0.5 * fel - ELEV_MARGIN), 0.5 * fel - ELEV_MARGIN, n)

    if outside_frac > 0.0:
        u = st.g.random(n)
        kind = st.integers(0, 3, n)
        out = u < outside_frac
        far = out & (kind == 0)
        near = out & (kind == 1)
        side = out & (kind == 2)
        high = out & (kind == 3)
        r = np.where(far, rhi * st.uniform(1.01, 1.3, n), r)
        r = np.where(near, rlo * st.uniform(0.2, 0.98, n), r)
        sgn = np.where(st.g.random(n) < 0.5, -1.0, 1.0)
        side_phi = sgn * np.minimum(0.5 * fov + st.uniform(0.02, 0.5, n), np.pi - 0.05)
        phi = np.where(side & (0.5 * fov < np.pi - 0.1), side_phi, phi)
        th = np.where(high, sgn * (0.5 * fel + st.uniform(0.02, 0.3, n)), th)

    dx = np.cos(th) * np.cos(phi)
    dy = np.cos(th) * np.sin(phi)
    dz = np.sin(th)
    x, y, z = r * dx, r * dy, r * dz
    nx, ny, nz = _normals_facing(st, dx, dy, dz, normal_cos_lo)

    if n_materials is None:
        mat = np.arange(n, dtype=np.int64)
        refl = st.uniform(0.1, 1.0, n)
    else:
        mat = st.integers(0, n_materials - 1, n)
        refl = st.uniform(0.1, 1.0, n_materials)
    miss = st.g.random(n) < miss_frac
    mat = np.where(miss, -1, mat)
    zero = np.float32(0)
    f = lambda a: np.where(miss, zero, a.astype(np.float32)).astype(np.float32)
    return SonarHits(x=f(x), y=f(y), z=f(z), nx=f(nx), ny=f(ny), nz=f(nz),
                     mat=mat.astype(np.int32), refl=refl.astype(np.float32))


def make_water(st: Stream) -> WaterSpec:
    """Per-channel water parameters: beta_D ~ U[0.05, 0.6], beta_B ~ U[0.05, 0.5],
    B_inf ~ U[0, 0.3]."""
    return WaterSpec(beta_d=st.uniform(0.05, 0.6, 3).astype(np.float32),
                     beta_b=st.uniform(0.05, 0.5, 3).astype(np.float32),
                     b_inf=st.uniform(0.0, 0.3, 3).astype(np.float32))


def make_camera(st: Stream, H: int, W: int, d_lo=0.5, d_hi=30.0, water_row=0) -> CameraFrame:
    """In-air image J ~ U[0, 1] per channel and depth ~ U[d_lo, d_hi]."""
    J = st.uniform(0.0, 1.0, (3, H, W)).astype(np.float32)
    d = st.uniform(d_lo, d_hi, (H, W)).astype(np.float32)
    return CameraFrame(J=J, depth=d, water_row=water_row)


def loss_weights(key, shape):
    """Seeded N(0, 1) weights w for test losses L = <w, output>."""
    return Stream(*key).normal(shape).astype(np.float32)


# --------------------------------------------------------------------------- #
# The workloads.  Sizes follow the sensors the paper models (Oculus M750-d:  #
# 130 deg x 20 deg field of view); parameters the workloads leave open are   #
# fixed here and recorded in the design notes.                               #
# --------------------------------------------------------------------------- #

def sonar_c1(seed: int = BASE_SEED + 0) -> List[SonarFrame]:
    """Plain forward: 256 beams x 32 rays = 8192 returns, r in [0.5, 20) m,
    512 x 256 polar bins, 512 x 1024 fan, gamma speckle k = 4,
    per-return reflectivity, 10% misses."""
    st = Stream(seed, 0)
    spec = SonarSpec(r_min=0.5, r_max=20.0, n_range=512, n_azimuth=256, fan_h=512, fan_w=1024,
                     speckle_mode=SPECKLE_GAMMA, gamma_k=4, seed_lo=seed, seed_hi=0, frame_id=0)
    return [SonarFrame(spec, make_hits(st, spec, 256 * 32))]


def sonar_c2(seed: int = BASE_SEED + 1) -> List[SonarFrame]:
    """Real-time frame: 1024 beams x 128 rays = 131072 returns, r in [1, 50) m,
    1024 x 1024 bins, 1024 x 2048 fan."""
    st = Stream(seed, 0)
    spec = SonarSpec(r_min=1.0, r_max=50.0, n_range=1024, n_azimuth=1024, fan_h=1024, fan_w=2048,
                     speckle_mode=SPECKLE_GAMMA, gamma_k=4, seed_lo=seed, seed_hi=0, frame_id=0)
    return [SonarFrame(spec, make_hits(st, spec, 1024 * 128))]


def camera_c2(seed: int = BASE_SEED + 1):
    """One 1920 x 1080 RGB frame, depth U[0.5, 30] m, and its water row."""
    st = Stream(seed, 1)
    return [make_camera(st, 1080, 1920)], [make_water(st)]


def sonar_c3(seed: int = BASE_SEED + 2, n_frames: int = 256, fan: bool = True) -> List[SonarFrame]:
    """Ragged batch: per frame beams U{128..1024}, rays U{16..128}, max range
    U[10, 100] m (min 0.5 m), N_r and N_phi each U{256..1024}, fan N_r x 2 N_r,
    alpha U[0.05, 0.2], G U[0.5, 2], sigma_phi U[0.1, 0.5], sigma_sa U[0, 0.2],
    gamma speckle k = 4, frame_id = frame index."""
    frames = []
    for f in range(n_frames):
        st = Stream(seed, f)
        beams = int(st.integers(128, 1024))
        rays = int(st.integers(16, 128))
        r_max = float(st.uniform(10.0, 100.0))
        Nr = int(st.integers(256, 1024))
        Np = int(st.integers(256, 1024))
        spec = SonarSpec(r_min=0.5, r_max=r_max, n_range=Nr, n_azimuth=Np,
                         fan_h=Nr if fan else 0, fan_w=2 * Nr if fan else 0,
                         alpha=float(st.uniform(0.05, 0.2)), gain=float(st.uniform(0.5, 2.0)),
                         sigma_phi=float(st.uniform(0.1, 0.5)), sigma_sa=float(st.uniform(0.0, 0.2)),
                         speckle_mode=SPECKLE_GAMMA, gamma_k=4, seed_lo=seed, seed_hi=0, frame_id=f)
        frames.append(SonarFrame(spec, make_hits(st, spec, beams * rays)))
    return frames


def sonar_c4(seed: int = BASE_SEED + 3, n_frames: int = 32, beams: int = 512, rays: int = 64,
             n_bins: int = 512) -> List[SonarFrame]:
    """Differentiable batch: 32 frames of 512 x 64 returns, r in [0.5, 20) m,
    64 materials, 512 x 512 bins, 512 x 1024 fan, paper speckle
    (sigma_sm = 0.1), one shared parameter row."""
    st0 = Stream(seed, 1 << 20)
    refl = st0.uniform(0.1, 1.0, 64).astype(np.float32)
    frames = []
    for f in range(n_frames):
        st = Stream(seed, f)
        spec = SonarSpec(r_min=0.5, r_max=20.0, n_range=n_bins, n_azimuth=n_bins,
                         fan_h=n_bins, fan_w=2 * n_bins, speckle_mode=SPECKLE_PAPER,
                         sigma_sm=0.1, seed_lo=seed, seed_hi=0, frame_id=f)
        h = make_hits(st, spec, beams * rays, n_materials=64)
        h.refl = refl
        frames.append(SonarFrame(spec, h))
    return frames


def camera_c4(seed: int = BASE_SEED + 3, n_frames: int = 32, H: int = 540, W: int = 960):
    st0 = Stream(seed, 1 << 21)
    water = make_water(st0)
    cams = [make_camera(Stream(seed, (1 << 22) + f), H, W) for f in range(n_frames)]
    return cams, [water]


def sonar_c5(seed: int = BASE_SEED + 4, n_frames: int = 64, beams: int = 2048, rays: int = 1024,
             n_bins: int = 2048) -> List[SonarFrame]:
    """Calibration scale: 64 frames of 2048 x 1024 returns, r in [0.5, 50) m,
    2048 x 2048 bins, no fan, 64 materials, gamma speckle k = 4."""
    st0 = Stream(seed, 1 << 20)
    refl = st0.uniform(0.1, 1.0, 64).astype(np.float32)
    frames = []
    for f in range(n_frames):
        st = Stream(seed, f)
        spec = SonarSpec(r_min=0.5, r_max=50.0, n_range=n_bins, n_azimuth=n_bins,
                         speckle_mode=SPECKLE_GAMMA, gamma_k=4, seed_lo=seed, seed_hi=0,
                         frame_id=f)
        h = make_hits(st, spec, beams * rays, n_materials=64)
        h.refl = refl
        frames.append(SonarFrame(spec, h))
    return frames


# --------------------------------------------------------------------------- #
# Procedural scenes for the ray caster.  The paper's scenes (a towing tank, a  #
# pier, a mall, a wreck) are not available; a seeded seabed heightfield with   #
# box-shaped structures standing on it stands in for them.                     #
# --------------------------------------------------------------------------- #
@dataclass
class Scene:
    vertices: np.ndarray      # float32 [V, 3] world coordinates (metres, z up)
    triangles: np.ndarray     # int32 [T, 3] vertex indices; (v1 - v0) x (v2 - v0) points out of the solid
    tri_mat: np.ndarray       # int32 [T] material of each triangle
    refl: np.ndarray          # float32 [M] reflectivity of each material


@dataclass
class SonarPose:
    pos: np.ndarray           # float32 [3] sensor position (world)
    rot: np.ndarray           # float32 [3, 3] world = rot @ sensor (x forward, y left, z up)


def box_mesh(lo, hi, first_vertex=0):
    """An axis-aligned box [lo, hi] as 12 outward-facing triangles."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    v = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], np.float64)
    quads = [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (2, 3, 7, 6), (1, 2, 6, 5), (0, 4, 7, 3)]
    tris = []
    for a, b, c, d in quads:
        tris += [(a, b, c), (a, c, d)]
    return v, np.asarray(tris, np.int64) + first_vertex


def seabed_scene(seed: int = BASE_SEED + 10, n: int = 256, extent: float = 200.0, depth: float = 20.0,
                 n_materials: int = 64, n_boxes: int = 16) -> Scene:
    """A seabed heightfield of n x n vertices over [-extent/2, extent/2]^2 at
    mean depth `depth` with seeded relief (a few sinusoids, +-2.5 m), materials
    in 8 x 8 patches, and `n_boxes` axis-aligned boxes (pillars, debris)
    standing on it ahead of the origin."""
    st = Stream(seed, 0)
    xs = np.linspace(-0.5 * extent, 0.5 * extent, n)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    Z = np.full_like(X, -depth)
    for _ in range(5):
        kx, ky = st.uniform(-0.15, 0.15, 2)
        ph = st.uniform(0.0, 2 * np.pi)
        amp = st.uniform(0.2, 0.5)
        Z += amp * np.sin(kx * X + ky * Y + ph)
    verts = [np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)]
    idx = np.arange(n * n).reshape(n, n)
    v00, v10, v01, v11 = idx[:-1, :-1], idx[1:, :-1], idx[:-1, 1:], idx[1:, 1:]
    # (v00, v10, v11) and (v00, v11, v01): normals point up (+z)
    tris = [np.stack([v00, v10, v11], -1).reshape(-1, 3), np.stack([v00, v11, v01], -1).reshape(-1, 3)]
    patch = (np.minimum(idx[:-1, :-1] // n * 8 // (n - 1), 7) * 8 +
             np.minimum(idx[:-1, :-1] % n * 8 // (n - 1), 7)).reshape(-1) % n_materials
    mats = [patch, patch]
    nv = n * n
    for b in range(n_boxes):
        cx = st.uniform(8.0, 0.4 * extent)
        cy = st.uniform(-0.3 * extent, 0.3 * extent)
        hx, hy = st.uniform(0.5, 4.0, 2)
        h = st.uniform(1.0, 10.0)
        v, t = box_mesh((cx - hx, cy - hy, -depth - 3.0), (cx + hx, cy + hy, -depth + h), nv)
        verts.append(v)
        tris.append(t)
        mats.append(np.full(12, int(st.integers(0, n_materials - 1)), np.int64))
        nv += 8
    refl = st.uniform(0.1, 1.0, n_materials).astype(np.float32)
    return Scene(np.concatenate(verts).astype(np.float32), np.concatenate(tris).astype(np.int32),
                 np.concatenate(mats).astype(np.int32), refl)


def sonar_pose(height: float = 8.0, depth: float = 20.0, pitch_deg: float = 15.0, yaw_deg: float = 0.0) -> SonarPose:
    """The sensor `height` metres above the mean seabed, looking along +x
    (turned by `yaw_deg`), tilted down by `pitch_deg`."""
    p, y = np.radians(pitch_deg), np.radians(yaw_deg)
    pitch = np.array([[np.cos(p), 0.0, np.sin(p)], [0.0, 1.0, 0.0], [-np.sin(p), 0.0, np.cos(p)]])
    yaw = np.array([[np.cos(y), -np.sin(y), 0.0], [np.sin(y), np.cos(y), 0.0], [0.0, 0.0, 1.0]])
    return SonarPose(np.array([0.0, 0.0, -depth + height], np.float32), (yaw @ pitch).astype(np.float32))


def chain_and_cluster_mesh(seed: int = BASE_SEED + 15, n_chain: int = 68, n_cluster: int = 300000):
    """An adversarial mesh for hierarchy depth: n_chain triangles along +x at
    1.5^i (each 1.5 times farther and larger than the last, so a surface-area
    split peels them off about one level at a time) and n_cluster small
    triangles (corners within 0.01 of a centre in the unit cube) at the
    chain's near end.  Returns (vertices float32 [V, 3], triangles int32
    [T, 3]); coordinates stay below 2^40."""
    i = np.arange(n_chain)
    base = np.array([[1.0, 0.0, 0.0], [1.1, 0.0, 0.0], [1.0, 0.1, 0.05]])
    chain = (1.5 ** i[:, None, None] * base[None]).reshape(-1, 3)
    st = Stream(seed, 0)
    c = st.uniform(0.0, 1.0, (n_cluster, 1, 3))
    cl = (c + st.uniform(-0.01, 0.01, (n_cluster, 3, 3))).reshape(-1, 3)
    v = np.concatenate([chain, cl]).astype(np.float32)
    return v, np.arange(v.shape[0], dtype=np.int32).reshape(-1, 3)
