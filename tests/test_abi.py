"""The C-ABI library without a GPU: it loads, exports every entry point that
include/oceansim.h declares, its ctypes mirrors match the header's layout, and
invalid arguments are rejected before anything is enqueued."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oceansim.h")


def _lib():
    from paper_2503_01074_amd import _lib
    return _lib


def test_exports_every_declared_function():
    lib = _lib()
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(oceansim_[a-z_]+)\s*\(", text))
    assert declared, "no declarations found"
    so = C.CDLL(lib.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(so, name), name
    assert set(lib.EXPORTED) == declared
    assert lib.oceansim_abi_version() == 5


def test_struct_layout_matches_header():
    lib = _lib()
    structs = {
        "oceansim_sonar_params": lib.SonarParams,
        "oceansim_sonar_frame": lib.SonarFrame,
        "oceansim_water_params": lib.WaterParams,
        "oceansim_uw_frame": lib.UwFrame,
        "oceansim_cam_frame": lib.CamFrame,
        "oceansim_cam_out_frame": lib.CamOutFrame,
        "oceansim_baro_params": lib.BaroParams,
        "oceansim_dvl_params": lib.DvlParams,
        "oceansim_scene_info": lib.SceneInfo,
        "oceansim_ray_frame": lib.RayFrame,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "oceansim.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    for line in out.strip().splitlines():
        cname, field, val = line.split()
        py = structs[cname]
        if field == "sizeof":
            assert C.sizeof(py) == int(val), cname
        else:
            assert getattr(py, field).offset == int(val), (cname, field)
    assert C.sizeof(lib.SonarParams) == 32 and C.sizeof(lib.WaterParams) == 48


FAKE = 0x7F0000001000    # never dereferenced: validation fails first


def _frame(lib, **over):
    f = lib.SonarFrame()
    for k in ("x", "y", "z", "nx", "ny", "nz", "mat"):
        setattr(f, k, FAKE)
    f.n_returns = 100
    f.r_min, f.r_max = 0.5, 20.0
    f.fov_az, f.fov_el = 2.2689, 0.349
    f.path_factor = 2.0
    f.n_range, f.n_azimuth = 64, 32
    f.fan_h, f.fan_w = 32, 64
    f.speckle_mode, f.gamma_k = 2, 4
    f.param_row = 0
    f.polar = FAKE
    f.fan = FAKE
    for k, v in over.items():
        setattr(f, k, v)
    return f


CASES = [
    ("n_returns", -1, -2),
    ("x", 0, -1),
    ("mat", FAKE + 2, -1),
    ("n_range", 0, -2),
    ("n_azimuth", 0, -2),
    ("n_azimuth", 5000, -4),
    ("r_max", 0.5, -1),
    ("r_min", -1.0, -1),
    ("r_max", float("inf"), -1),
    ("fov_az", 0.0, -1),
    ("fov_az", 7.0, -1),
    ("fov_el", 0.0, -1),
    ("path_factor", -1.0, -1),
    ("path_factor", float("nan"), -1),
    ("speckle_mode", 3, -1),
    ("gamma_k", 0, -4),
    ("gamma_k", 9, -4),
    ("param_row", 1, -1),
    ("param_row", -1, -1),
    ("fan_h", -1, -2),
    ("fan_w", 0, -2),
    ("polar", FAKE + 4, -1),
    ("fan", FAKE + 8, -1),
    ("bin_of_return", FAKE + 2, -1),
]


@pytest.mark.parametrize("field,value,status", CASES)
def test_sonar_render_rejects(field, value, status):
    lib = _lib()
    f = _frame(lib, **{field: value})
    rc = lib.lib.oceansim_sonar_render(C.pointer(f), 1, FAKE, 1, FAKE, 8, FAKE, 1 << 40, None)
    assert rc == status, (field, value, rc, lib.last_error())
    assert lib.last_error()


def test_more_sonar_rejections():
    lib = _lib()
    so = lib.lib
    f = _frame(lib, polar=0, fan=0)
    assert so.oceansim_sonar_render(C.pointer(f), 1, FAKE, 1, FAKE, 8, FAKE, 1 << 40, None) == -1
    f = _frame(lib, fan_h=0, fan_w=0)     # fan output without a fan
    assert so.oceansim_sonar_render(C.pointer(f), 1, FAKE, 1, FAKE, 8, FAKE, 1 << 40, None) == -2
    f = _frame(lib, fov_az=3.5)            # a fan needs fov_az <= pi
    assert so.oceansim_sonar_render(C.pointer(f), 1, FAKE, 1, FAKE, 8, FAKE, 1 << 40, None) == -1
    f = _frame(lib)
    assert so.oceansim_sonar_render(C.pointer(f), 1, None, 1, FAKE, 8, FAKE, 1 << 40, None) == -1
    assert so.oceansim_sonar_render(C.pointer(f), 1, FAKE, 1, None, 8, FAKE, 1 << 40, None) == -1
    assert so.oceansim_sonar_render(C.pointer(f), 1, FAKE, 1, FAKE, 0, FAKE, 1 << 40, None) == -1
    assert so.oceansim_sonar_render(C.pointer(f), 1, FAKE, 0, FAKE, 8, FAKE, 1 << 40, None) == -1
    assert so.oceansim_sonar_render(None, 1, FAKE, 1, FAKE, 8, FAKE, 1 << 40, None) == -1
    assert so.oceansim_sonar_render(C.pointer(f), -1, FAKE, 1, FAKE, 8, FAKE, 1 << 40, None) == -1
    # workspace: too small, NULL, misaligned
    need = lib.oceansim_sonar_workspace_size(f, 8, False)
    assert need > 0
    assert so.oceansim_sonar_render(C.pointer(f), 1, FAKE, 1, FAKE, 8, FAKE, need - 1, None) == -3
    assert so.oceansim_sonar_render(C.pointer(f), 1, FAKE, 1, FAKE, 8, None, need, None) == -3
    assert so.oceansim_sonar_render(C.pointer(f), 1, FAKE, 1, FAKE, 8, FAKE + 16, need, None) == -3
    # backward: NULL gradient outputs, grad_fan without a fan
    ws = 1 << 40
    assert so.oceansim_sonar_render_backward(C.pointer(f), 1, FAKE, 1, FAKE, 8, None, FAKE, FAKE, ws, None) == -1
    g = _frame(lib, fan_h=0, fan_w=0, fan=0, grad_fan=FAKE)
    assert so.oceansim_sonar_render_backward(C.pointer(g), 1, FAKE, 1, FAKE, 8, FAKE, FAKE, FAKE, ws, None) == -2
    g = _frame(lib, grad_polar=FAKE + 4)
    assert so.oceansim_sonar_render_backward(C.pointer(g), 1, FAKE, 1, FAKE, 8, FAKE, FAKE, FAKE, ws, None) == -1
    # the second frame of a batch is checked too, and named in the message
    fr = (lib.SonarFrame * 2)(_frame(lib), _frame(lib, n_range=0))
    assert so.oceansim_sonar_render(fr, 2, FAKE, 1, FAKE, 8, FAKE, ws, None) == -2
    assert "frame 1" in lib.last_error()


def test_workspace_sizes_grow_with_frames():
    lib = _lib()
    a = lib.oceansim_sonar_workspace_size(_frame(lib), 8, False)
    b = lib.oceansim_sonar_workspace_size([_frame(lib), _frame(lib)], 8, False)
    c = lib.oceansim_sonar_workspace_size(_frame(lib, n_returns=10 ** 6), 8, False)
    assert b > a and c > a and a % 256 == 0
    bw = lib.oceansim_sonar_workspace_size(_frame(lib), 8, True)
    assert bw > 0


def _uw(lib, **over):
    f = lib.UwFrame()
    f.J, f.depth, f.out = FAKE, FAKE, FAKE
    f.H, f.W, f.param_row = 8, 8, 0
    for k, v in over.items():
        setattr(f, k, v)
    return f


@pytest.mark.parametrize("field,value,status", [
    ("H", 0, -2), ("W", -3, -2), ("J", 0, -1), ("depth", 0, -1), ("out", 0, -1),
    ("J", FAKE + 4, -1), ("out", FAKE + 8, -1), ("param_row", 2, -1), ("H", 1 << 20, -4)])
def test_uw_rejects(field, value, status):
    lib = _lib()
    f = _uw(lib, **{field: value})
    if field == "H" and value == 1 << 20:
        f.W = 1 << 20
    rc = lib.lib.oceansim_uw_form(C.pointer(f), 1, FAKE, 2, None, 0, None)
    assert rc == status, (field, value, rc, lib.last_error())


def test_uw_backward_rejects():
    lib = _lib()
    so = lib.lib
    f = _uw(lib)
    assert so.oceansim_uw_form_backward(C.pointer(f), 1, FAKE, 1, FAKE, FAKE, 1 << 30, None) == -1  # no grad_out
    f = _uw(lib, grad_out=FAKE, grad_J=FAKE + 4)
    assert so.oceansim_uw_form_backward(C.pointer(f), 1, FAKE, 1, FAKE, FAKE, 1 << 30, None) == -1
    f = _uw(lib, grad_out=FAKE)
    assert so.oceansim_uw_form_backward(C.pointer(f), 1, FAKE, 1, None, FAKE, 1 << 30, None) == -1
    assert so.oceansim_uw_form_backward(C.pointer(f), 1, FAKE, 1, FAKE, FAKE, 8, None) == -3


def test_range_norm_rejections():
    """range_norm must be 0 or 1; the plain backward of a range-normalised
    frame needs the forward's binned sums (checked before any device work)."""
    lib = _lib()
    so = lib.lib
    f = _frame(lib, range_norm=2)
    ws = C.c_size_t()
    assert so.oceansim_sonar_workspace_size(C.pointer(f), 1, 8, 0, C.byref(ws)) == -1
    assert "range_norm" in lib.last_error()
    g = _frame(lib, range_norm=1, polar=0, fan=0, grad_polar=FAKE)
    assert so.oceansim_sonar_render_backward(C.pointer(g), 1, FAKE, 1, FAKE, 8, FAKE, FAKE, FAKE, 1 << 30,
                                             None) == -1
    assert "saved_p" in lib.last_error()
    h = _frame(lib, range_norm=1, saved_p=FAKE + 4)
    assert so.oceansim_sonar_workspace_size(C.pointer(h), 1, 8, 0, C.byref(ws)) == -1   # misaligned


def test_plan_rejections():
    lib = _lib()
    so = lib.lib
    out = C.c_void_p(FAKE)
    good = _frame(lib, grad_fan=FAKE)
    cam = _uw(lib, grad_out=FAKE)

    def create(sonar=(good,), camera=(), sp=FAKE, rows=1, refl=FAKE, n_mat=8, wp=FAKE, wrows=1,
               g_refl=FAKE, g_sp=FAKE, g_wp=FAKE, flags=1, plan=True):
        s = (lib.SonarFrame * max(1, len(sonar)))(*sonar)
        c = (lib.UwFrame * max(1, len(camera)))(*camera)
        return so.oceansim_plan_create(s if sonar else None, len(sonar), c if camera else None, len(camera),
                                       sp, rows, refl, n_mat, wp, wrows, g_refl, g_sp, g_wp, flags, None,
                                       C.byref(out) if plan else None)

    assert create(plan=False) == -1
    assert create(sonar=(), camera=()) == -1                          # nothing to plan
    assert create(flags=8) == -1                                      # unknown flag
    assert create(sp=None) == -1 and create(refl=None) == -1
    assert create(g_refl=None) == -1 and create(g_sp=None) == -1      # backward without outputs
    assert create(sonar=(), camera=(cam,), wp=None) == -1
    assert create(sonar=(), camera=(cam,), g_wp=None) == -1
    assert out.value is None                                          # cleared on error
    assert create(sonar=(good, _frame(lib, n_range=0))) == -2
    assert "frame 1" in lib.last_error()
    assert create(sonar=(_frame(lib, param_row=3),)) == -1
    assert create(sonar=(good, _frame(lib, grad_fan=FAKE, fan=0))) == -1   # fan gradient without the fan
    assert "frame 1" in lib.last_error()
    assert create(sonar=(), camera=(_uw(lib, H=0, grad_out=FAKE),)) == -2
    assert create(sonar=(), camera=(_uw(lib),)) == -1                 # backward needs grad_out
    assert so.oceansim_plan_forward(None, None) == -1
    assert so.oceansim_plan_backward(None, None) == -1
    assert so.oceansim_plan_shape(None, (C.c_int32 * 4)()) == -1
    assert so.oceansim_plan_destroy(None) == 0


def _cam(lib, **over):
    f = lib.CamFrame()
    f.srgb_in, f.zdepth, f.J, f.range = FAKE, FAKE, FAKE, FAKE
    f.grad_range, f.grad_zdepth = FAKE, FAKE
    f.H, f.W, f.channels_in = 480, 640, 3
    f.fx, f.fy, f.cx, f.cy = 500.0, 500.0, 320.0, 240.0
    for k, v in over.items():
        setattr(f, k, v)
    return f


@pytest.mark.parametrize("over,fn,text", [
    (dict(H=-1), "fwd", "H = -1"), (dict(W=65536), "fwd", "65536"),
    (dict(channels_in=2), "fwd", "channels_in"), (dict(J=0), "fwd", "without J"),
    (dict(range=0), "fwd", "without range"), (dict(srgb_in=FAKE + 4), "fwd", "aligned"),
    (dict(fx=0.0), "fwd", "fx, fy"), (dict(cy=float("nan")), "fwd", "fx, fy"),
    (dict(fy=float("inf")), "bwd", "fx, fy"), (dict(grad_zdepth=0), "bwd", "grad_range"),
    (dict(grad_range=FAKE + 8), "bwd", "aligned"),
])
def test_cam_rejections(over, fn, text):
    """Camera conditioning validates every frame before any launch."""
    lib = _lib()
    so = lib.lib
    frames = (lib.CamFrame * 2)(_cam(lib), _cam(lib, **over))
    call = so.oceansim_cam_condition if fn == "fwd" else so.oceansim_cam_condition_backward
    assert call(frames, 2, None) in (-1, -2)
    assert text in lib.last_error() and "frame 1" in lib.last_error()


def test_cam_encode_rejections():
    lib = _lib()
    so = lib.lib
    good = lib.CamOutFrame(FAKE, FAKE, 4, 4, 3)
    for bad, text in [(lib.CamOutFrame(FAKE, FAKE, 4, 4, 5), "channels_out"),
                      (lib.CamOutFrame(0, FAKE, 4, 4, 3), "required"),
                      (lib.CamOutFrame(FAKE, FAKE + 3, 4, 4, 3), "aligned"),
                      (lib.CamOutFrame(FAKE, FAKE, 70000, 4, 3), "outside")]:
        assert so.oceansim_cam_encode((lib.CamOutFrame * 2)(good, bad), 2, None) in (-1, -2)
        assert text in lib.last_error()
    assert so.oceansim_cam_encode(None, 0, None) == 0
    assert so.oceansim_cam_encode(None, -1, None) == -1


@pytest.mark.parametrize("over, text", [({"rho": -1.0}, "rho"), ({"sigma": float("nan")}, "finite"),
                                        ({"g": float("inf")}, "finite")])
def test_barometer_rejects(over, text):
    lib = _lib()
    p = lib.BaroParams(101325.0, 1025.0, 9.80665, 0.0, 0, 0)
    for k, v in over.items():
        setattr(p, k, v)
    with pytest.raises(lib.OceansimError) as ei:
        lib.oceansim_barometer(FAKE, 10, p, FAKE, 0)
    assert ei.value.status == -1 and text in str(ei.value)
    with pytest.raises(lib.OceansimError) as ei:
        lib.oceansim_barometer(FAKE, -1, lib.BaroParams(101325.0, 1025.0, 9.8, 0.0, 0, 0), FAKE, 0)
    assert ei.value.status == -2


@pytest.mark.parametrize("over, text", [({"janus_angle": 0.0}, "janus"), ({"janus_angle": 1.6}, "janus"),
                                        ({"min_beams": 2}, "min_beams"), ({"range_max": 0.1}, "range"),
                                        ({"sound_speed": 0.0}, "sound_speed"), ({"sigma_v": -0.1}, "sigma_v")])
def test_dvl_rejects(over, text):
    lib = _lib()
    p = lib.DvlParams(0.5236, 0.5, 80.0, 3, 0.0, 1500.0, 8.0, 0.125, 0, 0)
    for k, v in over.items():
        setattr(p, k, v)
    with pytest.raises(lib.OceansimError) as ei:
        lib.oceansim_dvl(FAKE, FAKE, FAKE, 10, 10, p, FAKE, FAKE, 0)
    assert ei.value.status == -1 and text in str(ei.value)
    ok = lib.DvlParams(0.5236, 0.5, 80.0, 3, 0.0, 1500.0, 8.0, 0.125, 0, 0)
    with pytest.raises(lib.OceansimError) as ei:   # ranges must be 16-byte aligned
        lib.oceansim_dvl(FAKE, FAKE + 4, FAKE, 10, 10, ok, FAKE, FAKE, 0)
    assert ei.value.status == -1
