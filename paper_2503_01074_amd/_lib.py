"""ctypes binding of liboceansim.so: structures mirroring include/oceansim.h and
the entry points under their C names.  Argument marshalling only; every step of
the computation runs in the library's HIP kernels.  There is no fallback: if
the library is missing the import fails.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboceansim.so")

OCEANSIM_OK = 0
OCEANSIM_E_INVALID_ARG = -1
OCEANSIM_E_SHAPE = -2
OCEANSIM_E_WORKSPACE = -3
OCEANSIM_E_UNSUPPORTED = -4
OCEANSIM_E_HIP = -5
STATUS_NAMES = {0: "OK", -1: "E_INVALID_ARG", -2: "E_SHAPE", -3: "E_WORKSPACE", -4: "E_UNSUPPORTED",
                -5: "E_HIP"}

SPECKLE_OFF, SPECKLE_PAPER, SPECKLE_GAMMA = 0, 1, 2
SONAR_GRAD_WIDTH = 8
SONAR_GRAD_COLUMNS = ("alpha", "gain", "sigma_phi", "sigma_sa", "sigma_sm")
WATER_GRAD_WIDTH = 9

_P = C.c_void_p


class SonarParams(C.Structure):
    _fields_ = [("alpha", C.c_float), ("gain", C.c_float), ("sigma_phi", C.c_float),
                ("sigma_sa", C.c_float), ("sigma_sm", C.c_float), ("reserved", C.c_float * 3)]


class SonarFrame(C.Structure):
    _fields_ = [("x", _P), ("y", _P), ("z", _P), ("nx", _P), ("ny", _P), ("nz", _P), ("mat", _P),
                ("n_returns", C.c_int64),
                ("r_min", C.c_float), ("r_max", C.c_float), ("fov_az", C.c_float),
                ("fov_el", C.c_float), ("path_factor", C.c_float),
                ("n_range", C.c_int32), ("n_azimuth", C.c_int32),
                ("fan_h", C.c_int32), ("fan_w", C.c_int32),
                ("speckle_mode", C.c_int32), ("gamma_k", C.c_int32), ("param_row", C.c_int32),
                ("seed_lo", C.c_uint32), ("seed_hi", C.c_uint32), ("frame_id", C.c_uint32),
                ("polar", _P), ("fan", _P), ("bin_of_return", _P),
                ("grad_polar", _P), ("grad_fan", _P), ("fan_stencil", _P),
                ("range_norm", C.c_int32), ("saved_p", _P)]


class WaterParams(C.Structure):
    _fields_ = [("beta_d", C.c_float * 3), ("beta_b", C.c_float * 3), ("b_inf", C.c_float * 3),
                ("reserved", C.c_float * 3)]


class UwFrame(C.Structure):
    _fields_ = [("J", _P), ("depth", _P), ("out", _P), ("H", C.c_int32), ("W", C.c_int32),
                ("param_row", C.c_int32), ("grad_out", _P), ("grad_J", _P), ("grad_depth", _P)]


class CamFrame(C.Structure):
    _fields_ = [("srgb_in", _P), ("zdepth", _P), ("J", _P), ("range", _P), ("grad_range", _P),
                ("grad_zdepth", _P), ("H", C.c_int32), ("W", C.c_int32), ("channels_in", C.c_int32),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float)]


class CamOutFrame(C.Structure):
    _fields_ = [("I", _P), ("srgb_out", _P), ("H", C.c_int32), ("W", C.c_int32), ("channels_out", C.c_int32)]


class BaroParams(C.Structure):
    _fields_ = [("p_atm", C.c_double), ("rho", C.c_double), ("g", C.c_double), ("sigma", C.c_double),
                ("seed_lo", C.c_uint32), ("seed_hi", C.c_uint32)]


class DvlParams(C.Structure):
    _fields_ = [("janus_angle", C.c_double), ("range_min", C.c_double), ("range_max", C.c_double),
                ("min_beams", C.c_int32), ("sigma_v", C.c_double), ("sound_speed", C.c_double),
                ("pings_per_output", C.c_double), ("period_min", C.c_double), ("seed_lo", C.c_uint32),
                ("seed_hi", C.c_uint32)]


class SceneInfo(C.Structure):
    _fields_ = [("n_triangles", C.c_int64), ("n_dropped", C.c_int64), ("n_nodes", C.c_int64),
                ("n_leaves", C.c_int64), ("depth", C.c_int32), ("max_leaf", C.c_int32), ("sah_cost", C.c_double),
                ("device_bytes", C.c_uint64)]


class RayFrame(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("rot", C.c_float * 9), ("n_beams", C.c_int32), ("n_rays", C.c_int32),
                ("fov_az", C.c_float), ("fov_el", C.c_float), ("t_max", C.c_float)] + \
               [(k, _P) for k in ("x", "y", "z", "nx", "ny", "nz", "mat")]


class OceansimError(RuntimeError):
    def __init__(self, status: int, where: str, text: str):
        super().__init__("%s: %s (%s)" % (where, STATUS_NAMES.get(status, status), text))
        self.status = status


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError("liboceansim.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2503_01074_amd.build): %s" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    lib.oceansim_last_error.restype = C.c_char_p
    lib.oceansim_last_error.argtypes = []
    lib.oceansim_abi_version.restype = C.c_int
    lib.oceansim_abi_version.argtypes = []
    SF, UF = C.POINTER(SonarFrame), C.POINTER(UwFrame)
    sig = {
        "oceansim_sonar_workspace_size": [SF, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)],
        "oceansim_sonar_render": [SF, C.c_int32, _P, C.c_int32, _P, C.c_int32, _P, C.c_size_t, _P],
        "oceansim_sonar_render_noalloc": [SF, C.c_int32, _P, C.c_int32, _P, C.c_int32, _P],
        "oceansim_sonar_render_backward": [SF, C.c_int32, _P, C.c_int32, _P, C.c_int32, _P, _P, _P,
                                           C.c_size_t, _P],
        "oceansim_uw_workspace_size": [UF, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)],
        "oceansim_uw_form": [UF, C.c_int32, _P, C.c_int32, _P, C.c_size_t, _P],
        "oceansim_uw_form_backward": [UF, C.c_int32, _P, C.c_int32, _P, _P, C.c_size_t, _P],
        "oceansim_cam_condition": [C.POINTER(CamFrame), C.c_int32, _P],
        "oceansim_cam_condition_backward": [C.POINTER(CamFrame), C.c_int32, _P],
        "oceansim_cam_encode": [C.POINTER(CamOutFrame), C.c_int32, _P],
        "oceansim_barometer": [_P, C.c_int64, C.POINTER(BaroParams), _P, _P],
        "oceansim_dvl": [_P, _P, _P, C.c_int32, C.c_int32, C.POINTER(DvlParams), _P, _P, _P],
        "oceansim_scene_create": [_P, C.c_int64, _P, _P, C.c_int64, C.POINTER(_P)],
        "oceansim_scene_get_info": [_P, C.POINTER(SceneInfo)],
        "oceansim_scene_measure": [_P, C.c_int64, _P, _P, C.c_int64, C.POINTER(SceneInfo)],
        "oceansim_scene_destroy": [_P],
        "oceansim_raycast": [_P, C.POINTER(RayFrame), C.c_int32, _P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.oceansim_fan_stencil_size.argtypes = [C.c_int32, C.c_int32]
    lib.oceansim_fan_stencil_size.restype = C.c_size_t
    lib.oceansim_trace_enable.argtypes = [C.c_int32]
    lib.oceansim_trace_enable.restype = C.c_int
    lib.oceansim_trace_summary.argtypes = [C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
    lib.oceansim_trace_summary.restype = C.c_int
    lib.oceansim_plan_create.argtypes = [SF, C.c_int32, UF, C.c_int32, _P, C.c_int32, _P, C.c_int32, _P,
                                         C.c_int32, _P, _P, _P, C.c_int32, _P, C.POINTER(_P)]
    lib.oceansim_plan_create.restype = C.c_int
    for name in ("oceansim_plan_forward", "oceansim_plan_backward"):
        getattr(lib, name).argtypes = [_P, _P]
        getattr(lib, name).restype = C.c_int
    lib.oceansim_plan_shape.argtypes = [_P, C.POINTER(C.c_int32)]
    lib.oceansim_plan_shape.restype = C.c_int
    lib.oceansim_plan_destroy.argtypes = [_P]
    lib.oceansim_plan_destroy.restype = C.c_int
    return lib


lib = _load()

EXPORTED = ("oceansim_last_error", "oceansim_abi_version", "oceansim_sonar_workspace_size",
            "oceansim_sonar_render", "oceansim_sonar_render_noalloc", "oceansim_sonar_render_backward",
            "oceansim_uw_workspace_size",
            "oceansim_uw_form", "oceansim_uw_form_backward", "oceansim_fan_stencil_size",
            "oceansim_trace_enable", "oceansim_trace_summary", "oceansim_plan_create",
            "oceansim_plan_forward", "oceansim_plan_backward", "oceansim_plan_shape",
            "oceansim_plan_destroy", "oceansim_cam_condition", "oceansim_cam_condition_backward",
            "oceansim_cam_encode", "oceansim_barometer", "oceansim_dvl", "oceansim_scene_create",
            "oceansim_scene_get_info", "oceansim_scene_measure", "oceansim_scene_destroy", "oceansim_raycast")

PLAN_BACKWARD, PLAN_GRAPH, PLAN_AUTOTUNE = 1, 2, 4


def last_error() -> str:
    return lib.oceansim_last_error().decode()


def check(status: int, where: str) -> None:
    if status != OCEANSIM_OK:
        raise OceansimError(status, where, last_error())


def _frames(frames, cls):
    if isinstance(frames, cls):
        return C.pointer(frames), 1, frames
    arr = (cls * len(frames))(*frames)
    return arr, len(frames), arr


# --- entry points under their C names (raise OceansimError on failure) ------ #

def oceansim_abi_version() -> int:
    return lib.oceansim_abi_version()


def oceansim_sonar_workspace_size(frames, n_materials: int, with_backward: bool) -> int:
    ptr, n, _keep = _frames(frames, SonarFrame)
    out = C.c_size_t(0)
    check(lib.oceansim_sonar_workspace_size(ptr, n, n_materials, int(with_backward), C.byref(out)),
          "oceansim_sonar_workspace_size")
    return out.value


def oceansim_sonar_render(frames, params_dev: int, n_param_rows: int, refl_dev: int, n_materials: int,
                          workspace: int, workspace_bytes: int, stream: int) -> None:
    ptr, n, _keep = _frames(frames, SonarFrame)
    check(lib.oceansim_sonar_render(ptr, n, params_dev, n_param_rows, refl_dev, n_materials, workspace,
                                    workspace_bytes, stream), "oceansim_sonar_render")


def oceansim_sonar_render_noalloc(frames, params_dev: int, n_param_rows: int, refl_dev: int, n_materials: int,
                                  stream: int) -> None:
    ptr, n, _keep = _frames(frames, SonarFrame)
    check(lib.oceansim_sonar_render_noalloc(ptr, n, params_dev, n_param_rows, refl_dev, n_materials, stream),
          "oceansim_sonar_render_noalloc")


def oceansim_sonar_render_backward(frames, params_dev: int, n_param_rows: int, refl_dev: int,
                                   n_materials: int, grad_refl_dev: int, grad_params_dev: int,
                                   workspace: int, workspace_bytes: int, stream: int) -> None:
    ptr, n, _keep = _frames(frames, SonarFrame)
    check(lib.oceansim_sonar_render_backward(ptr, n, params_dev, n_param_rows, refl_dev, n_materials,
                                             grad_refl_dev, grad_params_dev, workspace, workspace_bytes,
                                             stream), "oceansim_sonar_render_backward")


def oceansim_uw_workspace_size(frames, with_backward: bool) -> int:
    ptr, n, _keep = _frames(frames, UwFrame)
    out = C.c_size_t(0)
    check(lib.oceansim_uw_workspace_size(ptr, n, int(with_backward), C.byref(out)),
          "oceansim_uw_workspace_size")
    return out.value


def oceansim_cam_condition(frames, stream: int) -> None:
    ptr, n, _keep = _frames(frames, CamFrame)
    check(lib.oceansim_cam_condition(ptr, n, stream), "oceansim_cam_condition")


def oceansim_cam_condition_backward(frames, stream: int) -> None:
    ptr, n, _keep = _frames(frames, CamFrame)
    check(lib.oceansim_cam_condition_backward(ptr, n, stream), "oceansim_cam_condition_backward")


def oceansim_cam_encode(frames, stream: int) -> None:
    ptr, n, _keep = _frames(frames, CamOutFrame)
    check(lib.oceansim_cam_encode(ptr, n, stream), "oceansim_cam_encode")


def oceansim_uw_form(frames, params_dev: int, n_param_rows: int, workspace: int, workspace_bytes: int,
                     stream: int) -> None:
    ptr, n, _keep = _frames(frames, UwFrame)
    check(lib.oceansim_uw_form(ptr, n, params_dev, n_param_rows, workspace, workspace_bytes, stream),
          "oceansim_uw_form")


def oceansim_uw_form_backward(frames, params_dev: int, n_param_rows: int, grad_params_dev: int,
                              workspace: int, workspace_bytes: int, stream: int) -> None:
    ptr, n, _keep = _frames(frames, UwFrame)
    check(lib.oceansim_uw_form_backward(ptr, n, params_dev, n_param_rows, grad_params_dev, workspace,
                                        workspace_bytes, stream), "oceansim_uw_form_backward")


def oceansim_fan_stencil_size(fan_h: int, fan_w: int) -> int:
    return int(lib.oceansim_fan_stencil_size(fan_h, fan_w))


def oceansim_trace_enable(enable: bool) -> None:
    check(lib.oceansim_trace_enable(int(enable)), "oceansim_trace_enable")


def oceansim_trace_summary() -> dict:
    """{kernel name: (calls, total microseconds)} of the traced launches."""
    need = C.c_size_t(0)
    check(lib.oceansim_trace_summary(None, 0, C.byref(need)), "oceansim_trace_summary")
    buf = C.create_string_buffer(max(1, need.value))
    check(lib.oceansim_trace_summary(buf, need.value, None), "oceansim_trace_summary")
    out = {}
    for line in buf.value.decode().splitlines():
        name, calls, us = line.split()
        out[name] = (int(calls), float(us))
    return out


def oceansim_plan_create(sonar_frames, camera_frames, sonar_params_dev: int, n_sonar_rows: int,
                         refl_dev: int, n_materials: int, water_params_dev: int, n_water_rows: int,
                         grad_refl_dev: int, grad_sonar_params_dev: int, grad_water_params_dev: int,
                         flags: int, stream: int) -> int:
    """Returns the plan handle (an opaque pointer value)."""
    sp, ns, _k1 = _frames(sonar_frames, SonarFrame) if sonar_frames else (None, 0, None)
    cp, nc, _k2 = _frames(camera_frames, UwFrame) if camera_frames else (None, 0, None)
    out = _P(None)
    check(lib.oceansim_plan_create(sp, ns, cp, nc, sonar_params_dev, n_sonar_rows, refl_dev, n_materials,
                                   water_params_dev, n_water_rows, grad_refl_dev, grad_sonar_params_dev,
                                   grad_water_params_dev, flags, stream, C.byref(out)), "oceansim_plan_create")
    return out.value


def oceansim_plan_forward(plan: int, stream: int) -> None:
    check(lib.oceansim_plan_forward(plan, stream), "oceansim_plan_forward")


def oceansim_plan_backward(plan: int, stream: int) -> None:
    check(lib.oceansim_plan_backward(plan, stream), "oceansim_plan_backward")


def oceansim_plan_shape(plan: int) -> tuple:
    shape = (C.c_int32 * 4)()
    check(lib.oceansim_plan_shape(plan, shape), "oceansim_plan_shape")
    return tuple(shape)


def oceansim_plan_destroy(plan: int) -> None:
    check(lib.oceansim_plan_destroy(plan), "oceansim_plan_destroy")


def oceansim_barometer(depth_dev: int, n: int, params: BaroParams, pressure_dev: int, stream: int) -> None:
    check(lib.oceansim_barometer(depth_dev, n, C.byref(params), pressure_dev, stream), "oceansim_barometer")


def oceansim_dvl(t_dev: int, ranges_dev: int, velocity_dev: int, n_ticks: int, n_inst: int, params: DvlParams,
                 velocity_out_dev: int, status_dev: int, stream: int) -> None:
    check(lib.oceansim_dvl(t_dev, ranges_dev, velocity_dev, n_ticks, n_inst, C.byref(params), velocity_out_dev,
                           status_dev, stream), "oceansim_dvl")


def oceansim_scene_create(vertices_host: int, n_vertices: int, triangles_host: int, tri_mat_host: int,
                          n_triangles: int) -> int:
    out = _P()
    check(lib.oceansim_scene_create(vertices_host, n_vertices, triangles_host, tri_mat_host, n_triangles,
                                    C.byref(out)), "oceansim_scene_create")
    return out.value


def oceansim_scene_get_info(scene: int) -> SceneInfo:
    info = SceneInfo()
    check(lib.oceansim_scene_get_info(scene, C.byref(info)), "oceansim_scene_get_info")
    return info


def oceansim_scene_measure(vertices_host: int, n_vertices: int, triangles_host: int, tri_mat_host: int,
                           n_triangles: int) -> SceneInfo:
    info = SceneInfo()
    check(lib.oceansim_scene_measure(vertices_host, n_vertices, triangles_host, tri_mat_host, n_triangles,
                                     C.byref(info)), "oceansim_scene_measure")
    return info


def oceansim_scene_destroy(scene: int) -> None:
    check(lib.oceansim_scene_destroy(scene), "oceansim_scene_destroy")


def oceansim_raycast(scene: int, frames, n_frames: int, stream: int) -> None:
    check(lib.oceansim_raycast(scene, frames, n_frames, stream), "oceansim_raycast")
