"""Torch-facing API: device buffers in, device images out.

PyTorch provides device memory and the current stream; every step of the
computation runs in liboceansim.so.  The autograd functions wrap the
hand-written adjoint kernels for calibration loops.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import (SONAR_GRAD_WIDTH, WATER_GRAD_WIDTH, BaroParams, CamFrame, CamOutFrame, DvlParams, RayFrame,
                   SonarFrame, UwFrame)

SONAR_PARAM_WIDTH = 8     # alpha, gain, sigma_phi, sigma_sa, sigma_sm, 3 reserved
WATER_PARAM_WIDTH = 12    # beta_d[3], beta_b[3], b_inf[3], 3 reserved


def _ptr(t: Optional[torch.Tensor]) -> int:
    return 0 if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _workspace(nbytes: int, device) -> torch.Tensor:
    # 256-byte alignment: torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


@dataclass
class SonarGeometry:
    """Host-side description of one sonar frame (grid, field of view, RNG key)."""
    r_min: float
    r_max: float
    n_range: int
    n_azimuth: int
    fov_az: float
    fov_el: float
    path_factor: float = 2.0
    fan_h: int = 0
    fan_w: int = 0
    speckle_mode: int = _lib.SPECKLE_GAMMA
    gamma_k: int = 4
    seed_lo: int = 0
    seed_hi: int = 0
    frame_id: int = 0
    param_row: int = 0
    range_norm: int = 0   # 1: each range row over its maximum after the gain (needs saved sums backward)

    @classmethod
    def from_spec(cls, spec, param_row: int = 0) -> "SonarGeometry":
        return cls(r_min=spec.r_min, r_max=spec.r_max, n_range=spec.n_range, n_azimuth=spec.n_azimuth,
                   fov_az=spec.fov_az, fov_el=spec.fov_el, path_factor=spec.kappa, fan_h=spec.fan_h,
                   fan_w=spec.fan_w, speckle_mode=spec.speckle_mode, gamma_k=spec.gamma_k,
                   seed_lo=spec.seed_lo, seed_hi=spec.seed_hi, frame_id=spec.frame_id,
                   param_row=param_row, range_norm=int(getattr(spec, "range_norm", 0)))


@dataclass
class DeviceHits:
    """Structure-of-arrays hit buffer on the device."""
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    nx: torch.Tensor
    ny: torch.Tensor
    nz: torch.Tensor
    mat: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.x.numel())

    @classmethod
    def from_host(cls, hits, device="cuda") -> "DeviceHits":
        f = lambda a, dt: torch.as_tensor(a).to(device=device, dtype=dt).contiguous()
        return cls(f(hits.x, torch.float32), f(hits.y, torch.float32), f(hits.z, torch.float32),
                   f(hits.nx, torch.float32), f(hits.ny, torch.float32), f(hits.nz, torch.float32),
                   f(hits.mat, torch.int32))


def sonar_params(rows: Sequence[dict], device="cuda") -> torch.Tensor:
    """[n_rows, 8] float32 device table of oceansim_sonar_params rows."""
    t = torch.zeros(len(rows), SONAR_PARAM_WIDTH, dtype=torch.float32)
    for r, d in enumerate(rows):
        for c, name in enumerate(_lib.SONAR_GRAD_COLUMNS):
            t[r, c] = float(d.get(name, 0.0))
    return t.to(device)


def sonar_params_from_spec(spec) -> dict:
    return {k: float(getattr(spec, k)) for k in _lib.SONAR_GRAD_COLUMNS}


def water_params(rows: Sequence, device="cuda") -> torch.Tensor:
    """[n_rows, 12] float32 device table of oceansim_water_params rows; each
    row is (beta_d[3], beta_b[3], b_inf[3])."""
    t = torch.zeros(len(rows), WATER_PARAM_WIDTH, dtype=torch.float32)
    for r, (bd, bb, bi) in enumerate(rows):
        t[r, 0:3] = torch.as_tensor(bd, dtype=torch.float32)
        t[r, 3:6] = torch.as_tensor(bb, dtype=torch.float32)
        t[r, 6:9] = torch.as_tensor(bi, dtype=torch.float32)
    return t.to(device)


def _sonar_struct(g: SonarGeometry, h: DeviceHits, polar=None, fan=None, bins=None, grad_polar=None,
                  grad_fan=None, stencil=None, saved_p=None) -> SonarFrame:
    s = SonarFrame()
    s.x, s.y, s.z = _ptr(h.x), _ptr(h.y), _ptr(h.z)
    s.nx, s.ny, s.nz = _ptr(h.nx), _ptr(h.ny), _ptr(h.nz)
    s.mat = _ptr(h.mat)
    s.n_returns = h.n
    s.r_min, s.r_max = g.r_min, g.r_max
    s.fov_az, s.fov_el = g.fov_az, g.fov_el
    s.path_factor = g.path_factor
    s.n_range, s.n_azimuth = g.n_range, g.n_azimuth
    s.fan_h, s.fan_w = g.fan_h, g.fan_w
    s.speckle_mode, s.gamma_k = g.speckle_mode, g.gamma_k
    s.param_row = g.param_row
    s.seed_lo, s.seed_hi, s.frame_id = g.seed_lo & 0xFFFFFFFF, g.seed_hi & 0xFFFFFFFF, g.frame_id & 0xFFFFFFFF
    s.polar, s.fan, s.bin_of_return = _ptr(polar), _ptr(fan), _ptr(bins)
    s.grad_polar, s.grad_fan = _ptr(grad_polar), _ptr(grad_fan)
    s.fan_stencil = _ptr(stencil)
    s.range_norm = int(g.range_norm)
    s.saved_p = _ptr(saved_p)
    return s


def fan_stencil_buffer(g: SonarGeometry, device) -> Optional[torch.Tensor]:
    """Device buffer for the saved fan stencils of a frame (None without a fan)."""
    n = _lib.oceansim_fan_stencil_size(g.fan_h, g.fan_w)
    return torch.empty(n, dtype=torch.uint8, device=device) if n else None


def render_sonar(geoms: Sequence[SonarGeometry], hits: Sequence[DeviceHits], params: torch.Tensor,
                 refl: torch.Tensor, *, polar: bool = True, fan: bool = True, bins: bool = False,
                 save_stencil: bool = False, workspace: Optional[torch.Tensor] = None) -> List[dict]:
    """Forward sonar image formation of one or many frames in one call.

    With ``save_stencil`` each frame with a fan also returns "stencil": the
    fan stencils, to hand to render_sonar_backward.  A range-normalised frame
    also returns "saved_p", the binned sums its backward needs."""
    device = params.device
    outs, structs = [], []
    for g, h in zip(geoms, hits):
        o = {}
        if polar or not (fan and g.fan_h > 0):
            o["polar"] = torch.empty(g.n_range, g.n_azimuth, dtype=torch.float32, device=device)
        if fan and g.fan_h > 0 and g.fan_w > 0:
            o["fan"] = torch.empty(g.fan_h, g.fan_w, dtype=torch.float32, device=device)
            if save_stencil:
                o["stencil"] = fan_stencil_buffer(g, device)
        if bins:
            o["bins"] = torch.empty(h.n, dtype=torch.int32, device=device)
        if g.range_norm:
            o["saved_p"] = torch.empty(g.n_range, g.n_azimuth, dtype=torch.float32, device=device)
        outs.append(o)
        structs.append(_sonar_struct(g, h, o.get("polar"), o.get("fan"), o.get("bins"),
                                     stencil=o.get("stencil"), saved_p=o.get("saved_p")))
    n_mat = int(refl.numel())
    need = _lib.oceansim_sonar_workspace_size(structs, n_mat, False)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, device)
    _lib.oceansim_sonar_render(structs, _ptr(params), int(params.shape[0]), _ptr(refl), n_mat, _ptr(ws),
                               ws.numel(), _stream(device))
    return outs


def render_sonar_backward(geoms: Sequence[SonarGeometry], hits: Sequence[DeviceHits], params: torch.Tensor,
                          refl: torch.Tensor, grad_polar: Sequence[Optional[torch.Tensor]],
                          grad_fan: Sequence[Optional[torch.Tensor]],
                          stencils: Optional[Sequence[Optional[torch.Tensor]]] = None,
                          workspace: Optional[torch.Tensor] = None,
                          saved_p: Optional[Sequence[Optional[torch.Tensor]]] = None):
    """Gradients (refl [M], params [rows, 8]) of sum <grad_polar, polar> + <grad_fan, fan>.

    ``stencils``: the fan stencils saved by the forward call (optional; without
    them the fan geometry is recomputed).  ``saved_p``: the forward's binned
    sums, required for range-normalised frames."""
    device = params.device
    stencils = stencils or [None] * len(geoms)
    saved_p = saved_p or [None] * len(geoms)
    structs = [_sonar_struct(g, h, grad_polar=gp, grad_fan=gf, stencil=sv, saved_p=sp)
               for g, h, gp, gf, sv, sp in zip(geoms, hits, grad_polar, grad_fan, stencils, saved_p)]
    n_mat = int(refl.numel())
    need = _lib.oceansim_sonar_workspace_size(structs, n_mat, True)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, device)
    g_refl = torch.empty(n_mat, dtype=torch.float32, device=device)
    g_par = torch.empty(params.shape[0], SONAR_GRAD_WIDTH, dtype=torch.float32, device=device)
    _lib.oceansim_sonar_render_backward(structs, _ptr(params), int(params.shape[0]), _ptr(refl), n_mat,
                                        _ptr(g_refl), _ptr(g_par), _ptr(ws), ws.numel(), _stream(device))
    return g_refl, g_par


def _uw_struct(J, depth, out=None, row=0, grad_out=None, grad_J=None, grad_depth=None) -> UwFrame:
    s = UwFrame()
    s.J, s.depth, s.out = _ptr(J), _ptr(depth), _ptr(out)
    s.H, s.W = int(depth.shape[-2]), int(depth.shape[-1])
    s.param_row = row
    s.grad_out, s.grad_J, s.grad_depth = _ptr(grad_out), _ptr(grad_J), _ptr(grad_depth)
    return s


def uw_form(Js: Sequence[torch.Tensor], depths: Sequence[torch.Tensor], water: torch.Tensor,
            rows: Optional[Sequence[int]] = None) -> List[torch.Tensor]:
    """Eq. (1) on planar [3, H, W] images with depths [H, W] (one launch)."""
    rows = rows or [0] * len(Js)
    outs = [torch.empty_like(J) for J in Js]
    structs = [_uw_struct(J, d, o, r) for J, d, o, r in zip(Js, depths, outs, rows)]
    need = _lib.oceansim_uw_workspace_size(structs, False)
    ws = _workspace(need, water.device) if len(Js) > 1 else None
    _lib.oceansim_uw_form(structs, _ptr(water), int(water.shape[0]), _ptr(ws), 0 if ws is None else ws.numel(),
                          _stream(water.device))
    return outs


def uw_form_backward(Js, depths, water: torch.Tensor, grad_outs, rows=None, want_image_grads=True):
    """(grad_water [rows, 9], grad_J list, grad_depth list)."""
    rows = rows or [0] * len(Js)
    gJ = [torch.empty_like(J) if want_image_grads else None for J in Js]
    gd = [torch.empty_like(d) if want_image_grads else None for d in depths]
    structs = [_uw_struct(J, d, None, r, go, a, b)
               for J, d, r, go, a, b in zip(Js, depths, rows, grad_outs, gJ, gd)]
    need = _lib.oceansim_uw_workspace_size(structs, True)
    ws = _workspace(need, water.device)
    g_w = torch.empty(water.shape[0], WATER_GRAD_WIDTH, dtype=torch.float32, device=water.device)
    _lib.oceansim_uw_form_backward(structs, _ptr(water), int(water.shape[0]), _ptr(g_w), _ptr(ws), ws.numel(),
                                   _stream(water.device))
    return g_w, gJ, gd


# --------------------------------------------------------------------------- #
# camera input conditioning and output encoding                                #
# --------------------------------------------------------------------------- #

def _cam_struct(H, W, intr, srgb=None, zdepth=None, J=None, rng=None, grad_range=None, grad_z=None) -> CamFrame:
    s = CamFrame()
    s.srgb_in, s.zdepth, s.J, s.range = _ptr(srgb), _ptr(zdepth), _ptr(J), _ptr(rng)
    s.grad_range, s.grad_zdepth = _ptr(grad_range), _ptr(grad_z)
    s.H, s.W = int(H), int(W)
    s.channels_in = int(srgb.shape[-1]) if srgb is not None else 3
    s.fx, s.fy, s.cx, s.cy = (float(v) for v in intr)
    return s


def cam_condition(srgbs: Sequence[Optional[torch.Tensor]], zdepths: Sequence[Optional[torch.Tensor]],
                  intrinsics: Sequence[Sequence[float]]):
    """Frames of uint8 sRGB [H, W, 3 or 4] and/or z-depth [H, W] (either may be
    None) -> (list of linear planar J [3, H, W] or None, list of range [H, W] or
    None), one launch per 16 frames.  intrinsics: (fx, fy, cx, cy) per frame."""
    Js, rngs, structs = [], [], []
    for srgb, z, intr in zip(srgbs, zdepths, intrinsics):
        ref = srgb if srgb is not None else z
        if ref is None:             # nothing to condition in this frame
            Js.append(None)
            rngs.append(None)
            continue
        H, W = int(ref.shape[0]), int(ref.shape[1])
        J = torch.empty(3, H, W, dtype=torch.float32, device=ref.device) if srgb is not None else None
        r = torch.empty_like(z) if z is not None else None
        Js.append(J)
        rngs.append(r)
        structs.append(_cam_struct(H, W, intr, srgb, z, J, r))
    if structs:
        dev = next(t for t in list(srgbs) + list(zdepths) if t is not None).device   # noqa: E501
        _lib.oceansim_cam_condition(structs, _stream(dev))
    return Js, rngs


def cam_condition_backward(grad_ranges: Sequence[torch.Tensor], intrinsics: Sequence[Sequence[float]]):
    """dL/d(range) [H, W] per frame -> dL/d(z-depth) [H, W] per frame."""
    gz = [torch.empty_like(g) for g in grad_ranges]
    structs = [_cam_struct(g.shape[0], g.shape[1], intr, grad_range=g, grad_z=o)
               for g, o, intr in zip(grad_ranges, gz, intrinsics)]
    if structs:
        _lib.oceansim_cam_condition_backward(structs, _stream(grad_ranges[0].device))
    return gz


def cam_encode(images: Sequence[torch.Tensor], channels_out: int = 3) -> List[torch.Tensor]:
    """Planar linear [3, H, W] float images -> uint8 sRGB [H, W, channels_out]."""
    outs, structs = [], []
    for I in images:
        H, W = int(I.shape[-2]), int(I.shape[-1])
        o = torch.empty(H, W, channels_out, dtype=torch.uint8, device=I.device)
        s = CamOutFrame()
        s.I, s.srgb_out, s.H, s.W, s.channels_out = _ptr(I), _ptr(o), H, W, channels_out
        outs.append(o)
        structs.append(s)
    if structs:
        _lib.oceansim_cam_encode(structs, _stream(images[0].device))
    return outs


# --------------------------------------------------------------------------- #
# plans                                                                       #
# --------------------------------------------------------------------------- #
def barometer(depth: torch.Tensor, p_atm: float = 101325.0, rho: float = 1025.0, g: float = 9.80665,
              sigma: float = 0.0, seed: Sequence[int] = (0, 0)) -> torch.Tensor:
    """Pressures [Pa] (float32, same shape) of depths [m] below the free
    surface (oceansim_barometer; samples numbered in C order)."""
    d = depth.contiguous()
    out = torch.empty_like(d)
    prm = BaroParams(p_atm, rho, g, sigma, int(seed[0]), int(seed[1]))
    _lib.oceansim_barometer(_ptr(d), d.numel(), prm, _ptr(out), _stream(d.device))
    return out


def dvl(t: torch.Tensor, ranges: torch.Tensor, velocity: torch.Tensor, janus_angle: float = 0.5235987755982988,
        range_min: float = 0.5, range_max: float = 80.0, min_beams: int = 3, sigma_v: float = 0.0,
        sound_speed: float = 1500.0, pings_per_output: float = 8.0, period_min: float = 0.125,
        seed: Sequence[int] = (0, 0)):
    """Janus DVL over ticks (oceansim_dvl): t [T] float64, ranges [T, N, 4],
    velocity [T, N, 3] (device) -> (velocity_out [T, N, 3] with NaN where
    there is no velocity, status [T, N] int32: 0 none, 1 velocity, 2
    dropout)."""
    t = t.contiguous()
    r = ranges.contiguous()
    v = velocity.contiguous()
    T, N = int(r.shape[0]), int(r.shape[1])
    vo = torch.empty_like(v)
    st = torch.empty(T, N, dtype=torch.int32, device=v.device)
    prm = DvlParams(janus_angle, range_min, range_max, min_beams, sigma_v, sound_speed, pings_per_output,
                    period_min, int(seed[0]), int(seed[1]))
    _lib.oceansim_dvl(_ptr(t), _ptr(r), _ptr(v), T, N, prm, _ptr(vo), _ptr(st), _stream(v.device))
    return vo, st


def _mesh_arrays(vertices, triangles, tri_mat):
    import numpy as np
    v = np.ascontiguousarray(np.asarray(vertices, dtype=np.float32).reshape(-1, 3))
    t = np.ascontiguousarray(np.asarray(triangles, dtype=np.int32).reshape(-1, 3))
    m = np.ascontiguousarray(np.asarray(tri_mat, dtype=np.int32).reshape(-1))
    if m.shape[0] != t.shape[0]:
        raise ValueError("tri_mat must have one entry per triangle")
    return v, t, m


def _info_dict(i) -> dict:
    return {k: getattr(i, k) for k, _ in i._fields_}


def scene_measure(vertices, triangles, tri_mat) -> dict:
    """Figures of the ray-casting hierarchy of a mesh, built on the host only
    (oceansim_scene_measure): triangles kept and dropped, nodes, leaves,
    depth, largest leaf, surface-area cost, device bytes."""
    v, t, m = _mesh_arrays(vertices, triangles, tri_mat)
    return _info_dict(_lib.oceansim_scene_measure(v.ctypes.data, v.shape[0], t.ctypes.data, m.ctypes.data,
                                                  t.shape[0]))


class Scene:
    """A triangle mesh in the library's ray-casting hierarchy on the current
    device (oceansim_scene_create): vertices [V, 3] float32, triangles [T, 3]
    int32, tri_mat [T] int32, host arrays (numpy or CPU tensors)."""

    def __init__(self, vertices, triangles, tri_mat):
        v, t, m = _mesh_arrays(vertices, triangles, tri_mat)
        self.handle = None
        self.handle = _lib.oceansim_scene_create(v.ctypes.data, v.shape[0], t.ctypes.data, m.ctypes.data,
                                                 t.shape[0])

    @property
    def info(self) -> dict:
        return _info_dict(_lib.oceansim_scene_get_info(self.handle))

    def close(self) -> None:
        if self.handle:
            h, self.handle = self.handle, None
            _lib.oceansim_scene_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def raycast(scene: Scene, poses: Sequence, n_beams: int, n_rays: int, fov_az: float, fov_el: float,
            t_max: float, device="cuda", out: Optional[Sequence[DeviceHits]] = None) -> List[DeviceHits]:
    """Closest hits of a beam x elevation ray pattern from each pose (pos [3],
    rot [3, 3] row-major, world = rot @ sensor + pos) against the scene
    (oceansim_raycast): one sensor-frame hit buffer (DeviceHits, return k =
    beam * n_rays + ray, material -1 for a miss) per pose, in one launch per
    16 poses on the current stream.  ``out`` reuses existing buffers."""
    import numpy as np
    n = int(n_beams) * int(n_rays)
    res = list(out) if out is not None else []
    frames = (RayFrame * max(1, len(poses)))()
    for i, (pos, rot) in enumerate(poses):
        if out is None:
            f32 = lambda: torch.empty(n, dtype=torch.float32, device=device)
            res.append(DeviceHits(f32(), f32(), f32(), f32(), f32(), f32(),
                                  torch.empty(n, dtype=torch.int32, device=device)))
        h = res[i]
        fr = frames[i]
        fr.pos[:] = [float(v) for v in np.asarray(pos, dtype=np.float64).reshape(3)]
        fr.rot[:] = [float(v) for v in np.asarray(rot, dtype=np.float64).reshape(9)]
        fr.n_beams, fr.n_rays = int(n_beams), int(n_rays)
        fr.fov_az, fr.fov_el, fr.t_max = float(fov_az), float(fov_el), float(t_max)
        for k in ("x", "y", "z", "nx", "ny", "nz", "mat"):
            setattr(fr, k, _ptr(getattr(h, k)))
    dev = res[0].x.device if res else torch.device(device)
    _lib.oceansim_raycast(scene.handle, frames, len(poses), _stream(dev))
    return res


class Plan:
    """Sonar and camera frames prepared once and launched many times
    (oceansim_plan_*): frame tables are uploaded once and, with ``graph``,
    each direction replays a captured HIP graph.

    ``sonar``: (SonarGeometry, DeviceHits) pairs; ``camera``: (J [3, H, W],
    depth [H, W], water_row) triples.  The plan allocates the outputs
    (``sonar_out[i]["polar" / "fan" / "bins"]``, ``camera_out[i]["out"]``) and,
    with ``backward``, the gradient inputs (``"grad_polar"``, ``"grad_fan"``,
    ``"grad_out"``, zero-filled) and outputs (``grad_refl``,
    ``grad_sonar_params``, ``grad_water``, and ``"grad_J"``/``"grad_depth"``
    with ``image_grads``).  Between launches the caller refills any of these
    tensors, the hits, the parameter tables and the images in place; shapes
    and buffers stay fixed."""

    def __init__(self, sonar=(), camera=(), *, sonar_params: Optional[torch.Tensor] = None,
                 refl: Optional[torch.Tensor] = None, water: Optional[torch.Tensor] = None,
                 backward: bool = False, graph: bool = False, autotune: bool = False,
                 polar: bool = True, fan: bool = True, bins: bool = False, image_grads: bool = False):
        self.handle = None
        anchor = sonar_params if sonar_params is not None else water
        self.device = anchor.device
        dev = self.device
        self.sonar_out, self.camera_out = [], []
        s_structs, c_structs = [], []
        for g, h in sonar:
            o = {}
            has_fan = fan and g.fan_h > 0 and g.fan_w > 0
            if polar or not has_fan:
                o["polar"] = torch.empty(g.n_range, g.n_azimuth, dtype=torch.float32, device=dev)
            if has_fan:
                o["fan"] = torch.empty(g.fan_h, g.fan_w, dtype=torch.float32, device=dev)
            if bins:
                o["bins"] = torch.empty(h.n, dtype=torch.int32, device=dev)
            if backward:
                if "polar" in o:
                    o["grad_polar"] = torch.zeros_like(o["polar"])
                if has_fan:
                    o["grad_fan"] = torch.zeros_like(o["fan"])
            self.sonar_out.append(o)
            s_structs.append(_sonar_struct(g, h, o.get("polar"), o.get("fan"), o.get("bins"),
                                           o.get("grad_polar"), o.get("grad_fan")))
        for J, d, row in camera:
            o = {"out": torch.empty_like(J)}
            if backward:
                o["grad_out"] = torch.zeros_like(J)
                if image_grads:
                    o["grad_J"] = torch.empty_like(J)
                    o["grad_depth"] = torch.empty_like(d)
            self.camera_out.append(o)
            c_structs.append(_uw_struct(J, d, o["out"], row, o.get("grad_out"), o.get("grad_J"),
                                        o.get("grad_depth")))
        n_mat = int(refl.numel()) if refl is not None else 0
        self.grad_refl = self.grad_sonar_params = self.grad_water = None
        if backward and sonar:
            self.grad_refl = torch.zeros(n_mat, dtype=torch.float32, device=dev)
            self.grad_sonar_params = torch.zeros(sonar_params.shape[0], SONAR_GRAD_WIDTH, dtype=torch.float32,
                                                 device=dev)
        if backward and camera:
            self.grad_water = torch.zeros(water.shape[0], WATER_GRAD_WIDTH, dtype=torch.float32, device=dev)
        flags = ((_lib.PLAN_BACKWARD if backward else 0) | (_lib.PLAN_GRAPH if graph else 0) |
                 (_lib.PLAN_AUTOTUNE if autotune else 0))
        # the plan keeps raw pointers: hold the tensors for its lifetime
        self._keep = (list(sonar), list(camera), sonar_params, refl, water)
        self.handle = _lib.oceansim_plan_create(
            s_structs, c_structs, _ptr(sonar_params), 0 if sonar_params is None else int(sonar_params.shape[0]),
            _ptr(refl), n_mat, _ptr(water), 0 if water is None else int(water.shape[0]),
            _ptr(self.grad_refl), _ptr(self.grad_sonar_params), _ptr(self.grad_water), flags, _stream(dev))

    def forward(self) -> None:
        """Enqueue the forward launches on the current stream."""
        _lib.oceansim_plan_forward(self.handle, _stream(self.device))

    def backward(self) -> None:
        """Enqueue the adjoint launches (after a forward) on the current stream."""
        _lib.oceansim_plan_backward(self.handle, _stream(self.device))

    def shape(self) -> dict:
        a = _lib.oceansim_plan_shape(self.handle)
        return {"fwd_tile_bins": a[0], "chunk": a[1], "bwd_block_bins": a[2], "graph": bool(a[3])}

    def close(self) -> None:
        if self.handle:
            _lib.oceansim_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------- #
# autograd                                                                    #
# --------------------------------------------------------------------------- #
class SonarRender(torch.autograd.Function):
    """(refl [M], params [rows, 8]) -> polar images and fans of every frame.

    Outputs: a tuple with, per frame, the polar image followed by the fan
    (when the frame has one).  Gradients flow to refl and params."""

    @staticmethod
    def forward(ctx, refl, params, geoms, hits):
        outs = render_sonar(geoms, hits, params, refl, polar=True, fan=True, save_stencil=True)
        ctx.geoms, ctx.hits = geoms, hits
        ctx.stencils = [o.get("stencil") for o in outs]
        ctx.saved_p = [o.get("saved_p") for o in outs]
        ctx.save_for_backward(refl, params)
        flat = []
        for g, o in zip(geoms, outs):
            flat.append(o["polar"])
            if "fan" in o:
                flat.append(o["fan"])
        return tuple(flat)

    @staticmethod
    def backward(ctx, *grads):
        refl, params = ctx.saved_tensors
        gp, gf, k = [], [], 0
        for g in ctx.geoms:
            gpol = grads[k]
            k += 1
            gp.append(None if gpol is None else gpol.contiguous())
            if g.fan_h > 0 and g.fan_w > 0:
                gfan = grads[k]
                k += 1
                gf.append(None if gfan is None else gfan.contiguous())
            else:
                gf.append(None)
        g_refl, g_par = render_sonar_backward(ctx.geoms, ctx.hits, params, refl, gp, gf, ctx.stencils,
                                              saved_p=ctx.saved_p)
        return g_refl, g_par, None, None


class UwForm(torch.autograd.Function):
    """(water [rows, 12], J_0, d_0, J_1, d_1, ...) -> underwater images."""

    @staticmethod
    def forward(ctx, water, rows, *images):
        Js, ds = list(images[0::2]), list(images[1::2])
        ctx.rows = rows
        ctx.save_for_backward(water, *images)
        return tuple(uw_form(Js, ds, water, rows))

    @staticmethod
    def backward(ctx, *grads):
        water, *images = ctx.saved_tensors
        Js, ds = images[0::2], images[1::2]
        gos = [torch.zeros_like(J) if g is None else g.contiguous() for g, J in zip(grads, Js)]
        g_w, gJ, gd = uw_form_backward(Js, ds, water, gos, ctx.rows, want_image_grads=True)
        gw = torch.zeros_like(water)
        gw[:, :WATER_GRAD_WIDTH] = g_w
        img_grads = []
        for a, b in zip(gJ, gd):
            img_grads += [a, b]
        return (gw, None, *img_grads)
