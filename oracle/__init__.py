"""FP64 CPU oracle for OceanSim's sonar and underwater-camera image formation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  The
arithmetic lives in ``oceansim_oracle.c`` (plain C, double precision, OpenMP);
this module only marshals numpy arrays to it with ctypes.  It imports nothing
from the GPU package.

Paper: arXiv 2503.01074, Sec. III-A.1 Eq. (1) (camera), Sec. III-A.2
Eq. (2)-(6) (sonar) and the barometer and DVL of Sec. III-A (no equations
printed: the readings are stated with each function).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oceansim_oracle.c")
_LIB = os.path.join(_HERE, "liboceansim_oracle.so")
_lock = threading.Lock()
_lib = None

SPECKLE_OFF, SPECKLE_PAPER, SPECKLE_GAMMA = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            _lib = C.CDLL(_LIB)
            _declare(_lib)
    return _lib


class _Cfg(C.Structure):
    _fields_ = [
        ("r_min", C.c_double), ("r_max", C.c_double),
        ("fov_az", C.c_double), ("fov_el", C.c_double),
        ("kappa", C.c_double), ("alpha", C.c_double), ("gain", C.c_double),
        ("sigma_phi", C.c_double), ("sigma_sa", C.c_double), ("sigma_sm", C.c_double),
        ("n_range", C.c_int32), ("n_azimuth", C.c_int32),
        ("fan_h", C.c_int32), ("fan_w", C.c_int32),
        ("speckle_mode", C.c_int32), ("gamma_k", C.c_int32),
        ("seed_lo", C.c_uint32), ("seed_hi", C.c_uint32), ("frame_id", C.c_uint32),
        ("fan_band", C.c_double),
        ("range_norm", C.c_int32),
    ]


_P = C.c_void_p


def _declare(lib):
    lib.orc_philox_many.argtypes = [C.c_int64, _P, _P, _P]
    lib.orc_philox_many.restype = None
    lib.orc_speckle_fields.argtypes = [C.POINTER(_Cfg), _P, _P]
    lib.orc_speckle_fields.restype = None
    lib.orc_fan_forward.argtypes = [C.POINTER(_Cfg), _P, _P, _P]
    lib.orc_fan_forward.restype = None
    lib.orc_fan_adjoint.argtypes = [C.POINTER(_Cfg), _P, _P]
    lib.orc_fan_adjoint.restype = None
    lib.orc_sonar_forward.argtypes = [C.POINTER(_Cfg), C.c_int64] + [_P] * 7 + [_P, C.c_int32] + [_P] * 6
    lib.orc_sonar_forward.restype = C.c_int
    lib.orc_sonar_backward.argtypes = [C.POINTER(_Cfg), C.c_int64] + [_P] * 7 + [_P, C.c_int32] + [_P] * 7
    lib.orc_sonar_backward.restype = C.c_int
    lib.orc_uw_forward.argtypes = [C.c_int64] + [_P] * 6
    lib.orc_uw_forward.restype = None
    lib.orc_uw_backward.argtypes = [C.c_int64] + [_P] * 10
    lib.orc_uw_backward.restype = None
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = C.c_int
    lib.orc_barometer.argtypes = [C.c_int64, _P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint32,
                                  C.c_uint32, _P]
    lib.orc_barometer.restype = None
    lib.orc_dvl_beam.argtypes = [C.c_int, C.c_double, _P]
    lib.orc_dvl_beam.restype = None
    lib.orc_dvl.argtypes = [C.c_int32, C.c_int32, _P, _P, _P, C.c_double, C.c_double, C.c_double, C.c_int32,
                            C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint32, C.c_uint32, _P, _P]
    lib.orc_dvl.restype = None
    lib.orc_raycast.argtypes = [C.c_int64, _P, C.c_int64, _P, _P, _P, _P, C.c_int32, C.c_int32, C.c_double,
                                C.c_double, C.c_double, C.c_double, C.c_int64, _P] + [_P] * 8
    lib.orc_raycast.restype = None


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().orc_num_threads())


@dataclass
class SonarConfig:
    """Geometry, parameters and RNG key of one sonar frame (all in FP64)."""
    r_min: float
    r_max: float
    fov_az: float
    fov_el: float
    n_range: int
    n_azimuth: int
    fan_h: int = 0
    fan_w: int = 0
    kappa: float = 2.0
    alpha: float = 0.1
    gain: float = 1.0
    sigma_phi: float = 0.25
    sigma_sa: float = 0.1
    sigma_sm: float = 0.1
    speckle_mode: int = SPECKLE_OFF
    gamma_k: int = 4
    seed_lo: int = 0
    seed_hi: int = 0
    frame_id: int = 0
    fan_band: float = 1e-6
    range_norm: int = 0

    @classmethod
    def from_spec(cls, spec, **over) -> "SonarConfig":
        """Build from any object carrying the same attribute names."""
        kw = {f: getattr(spec, f) for f in cls.__dataclass_fields__ if hasattr(spec, f)}
        kw.update(over)
        return cls(**kw)

    def _c(self) -> _Cfg:
        c = _Cfg()
        for name, _ in _Cfg._fields_:
            setattr(c, name, getattr(self, name))
        return c


def philox4x32_10(ctr, key):
    """Philox4x32-10 on rows of ctr (n,4) uint32 with keys (n,2) uint32."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    if key.shape[0] == 1 and ctr.shape[0] > 1:
        key = np.ascontiguousarray(np.repeat(key, ctr.shape[0], axis=0))
    out = np.empty_like(ctr)
    _load().orc_philox_many(ctr.shape[0], _ptr(ctr), _ptr(key), _ptr(out))
    return out


def speckle_fields(cfg: SonarConfig):
    """Additive term and multiplicative factor of every bin, [n_range, n_azimuth]."""
    add = np.empty((cfg.n_range, cfg.n_azimuth), np.float64)
    mul = np.empty_like(add)
    c = cfg._c()
    _load().orc_speckle_fields(C.byref(c), _ptr(add), _ptr(mul))
    return add, mul


def fan_forward(cfg: SonarConfig, img):
    """Fan image [fan_h, fan_w] of a polar image, plus the ambiguity mask."""
    img = _f64(img)
    fan = np.empty((cfg.fan_h, cfg.fan_w), np.float64)
    amb = np.empty((cfg.fan_h, cfg.fan_w), np.uint8)
    c = cfg._c()
    _load().orc_fan_forward(C.byref(c), _ptr(img), _ptr(fan), _ptr(amb))
    return fan, amb.astype(bool)


def fan_adjoint(cfg: SonarConfig, g_fan):
    g_fan = _f64(g_fan)
    g = np.empty((cfg.n_range, cfg.n_azimuth), np.float64)
    c = cfg._c()
    _load().orc_fan_adjoint(C.byref(c), _ptr(g_fan), _ptr(g))
    return g


def _hits(h):
    return [_f32(h.x), _f32(h.y), _f32(h.z), _f32(h.nx), _f32(h.ny), _f32(h.nz),
            np.ascontiguousarray(h.mat, dtype=np.int32)]


def sonar_forward(cfg: SonarConfig, hits, refl, with_fan: bool | None = None):
    """Everything one sonar frame produces.

    ``hits`` is any object with float32 arrays x, y, z, nx, ny, nz and int32
    mat.  Returns a dict with per-return ``intensity`` and ``bins``, the
    binned sum ``P``, the speckled polar image ``out`` and, when the config
    has a fan, ``fan`` and its ``ambiguous`` mask.
    """
    arrs = _hits(hits)
    refl = _f32(refl)
    n = arrs[0].shape[0]
    nb = (cfg.n_range, cfg.n_azimuth)
    res = {
        "intensity": np.empty(n, np.float64),
        "bins": np.empty(n, np.int32),
        "P": np.empty(nb, np.float64),
        "out": np.empty(nb, np.float64),
    }
    want_fan = (cfg.fan_h > 0 and cfg.fan_w > 0) if with_fan is None else with_fan
    if want_fan:
        res["fan"] = np.empty((cfg.fan_h, cfg.fan_w), np.float64)
        res["ambiguous"] = np.empty((cfg.fan_h, cfg.fan_w), np.uint8)
    c = cfg._c()
    _load().orc_sonar_forward(C.byref(c), n, *[_ptr(a) for a in arrs], _ptr(refl), refl.shape[0],
                              _ptr(res["intensity"]), _ptr(res["bins"]), _ptr(res["P"]),
                              _ptr(res["out"]), _ptr(res.get("fan")), _ptr(res.get("ambiguous")))
    if want_fan:
        res["ambiguous"] = res["ambiguous"].astype(bool)
    return res


SONAR_GRAD_NAMES = ("alpha", "gain", "sigma_phi", "sigma_sa", "sigma_sm")


def sonar_backward(cfg: SonarConfig, hits, refl, g_polar=None, g_fan=None, with_abs: bool = False):
    """Gradients of <g_polar, out> + <g_fan, fan>.

    Returns (g_refl [n_mat], g_par [5] in SONAR_GRAD_NAMES order,
    g_out [n_range, n_azimuth] = gradient with respect to the polar output),
    followed, with ``with_abs``, by the sums of term magnitudes of g_refl and
    g_par (the condition of each gradient sum).
    """
    arrs = _hits(hits)
    refl = _f32(refl)
    n = arrs[0].shape[0]
    g_refl = np.zeros(refl.shape[0], np.float64)
    g_par = np.zeros(5, np.float64)
    g_out = np.empty((cfg.n_range, cfg.n_azimuth), np.float64)
    a_refl = np.zeros(refl.shape[0], np.float64) if with_abs else None
    a_par = np.zeros(5, np.float64) if with_abs else None
    c = cfg._c()
    _load().orc_sonar_backward(C.byref(c), n, *[_ptr(a) for a in arrs], _ptr(refl), refl.shape[0],
                               _ptr(_f64(g_polar)), _ptr(_f64(g_fan)), _ptr(g_refl), _ptr(g_par),
                               _ptr(g_out), _ptr(a_refl), _ptr(a_par))
    if with_abs:
        return g_refl, g_par, g_out, a_refl, a_par
    return g_refl, g_par, g_out


def _water(beta_d, beta_b, b_inf):
    return [np.ascontiguousarray(np.asarray(v, np.float64).reshape(3)) for v in (beta_d, beta_b, b_inf)]


def uw_forward(J, depth, beta_d, beta_b, b_inf):
    """Eq. (1) on a planar [3, H, W] image J with depth [H, W]."""
    J = _f32(J)
    depth = _f32(depth)
    npix = depth.size
    bd, bb, bi = _water(beta_d, beta_b, b_inf)
    out = np.empty(J.shape, np.float64)
    _load().orc_uw_forward(npix, _ptr(J), _ptr(depth), _ptr(bd), _ptr(bb), _ptr(bi), _ptr(out))
    return out


UW_GRAD_NAMES = ("beta_d", "beta_b", "b_inf")


def uw_backward(J, depth, beta_d, beta_b, b_inf, g_out, want_image_grads: bool = True,
                with_abs: bool = False):
    """Gradients of <g_out, I>: (g_par [9] = beta_d[3], beta_b[3], b_inf[3], g_J, g_depth),
    followed, with ``with_abs``, by the sums of term magnitudes of g_par."""
    J = _f32(J)
    depth = _f32(depth)
    npix = depth.size
    bd, bb, bi = _water(beta_d, beta_b, b_inf)
    g_out = _f64(g_out)
    g_par = np.zeros(9, np.float64)
    a_par = np.zeros(9, np.float64) if with_abs else None
    g_J = np.empty(J.shape, np.float64) if want_image_grads else None
    g_d = np.empty(depth.shape, np.float64) if want_image_grads else None
    _load().orc_uw_backward(npix, _ptr(J), _ptr(depth), _ptr(bd), _ptr(bb), _ptr(bi), _ptr(g_out),
                            _ptr(g_par), _ptr(g_J), _ptr(g_d), _ptr(a_par))
    if with_abs:
        return g_par, g_J, g_d, a_par
    return g_par, g_J, g_d


# --------------------------------------------------------------------------- #
# Navigation sensors (Sec. III-A): barometer and DVL                          #
# --------------------------------------------------------------------------- #
@dataclass
class BaroConfig:
    """Barometer: pressure = p_atm + rho g max(depth, 0) + sigma N(0, 1)."""
    p_atm: float = 101325.0
    rho: float = 1025.0
    g: float = 9.80665
    sigma: float = 0.0
    seed_lo: int = 0
    seed_hi: int = 0


def barometer(depth, cfg: BaroConfig):
    """Pressures [Pa] of the depths [m] (any shape, flattened in C order for
    the noise counters)."""
    d = _f32(depth)
    out = np.empty(d.shape, np.float64)
    _load().orc_barometer(d.size, _ptr(d), cfg.p_atm, cfg.rho, cfg.g, cfg.sigma, cfg.seed_lo, cfg.seed_hi,
                          _ptr(out))
    return out


@dataclass
class DvlConfig:
    """Four-beam convex Janus DVL with a range-dependent rate and dropout."""
    janus: float = 30.0 * np.pi / 180.0
    range_min: float = 0.5
    range_max: float = 80.0
    min_beams: int = 3
    sigma_v: float = 0.0
    sound_speed: float = 1500.0
    pings_per_output: float = 8.0
    period_min: float = 0.125
    seed_lo: int = 0
    seed_hi: int = 0


def dvl_beams(janus: float):
    """The four unit beam directions [4, 3] (sensor frame)."""
    out = np.empty((4, 3), np.float64)
    b = np.empty(3, np.float64)
    for i in range(4):
        _load().orc_dvl_beam(i, janus, _ptr(b))
        out[i] = b
    return out


def dvl(t, ranges, vel, cfg: DvlConfig):
    """t [T] seconds, ranges [T, N, 4], vel [T, N, 3] -> (velocity [T, N, 3]
    float64 with NaN where there is none, status [T, N] int32: 0 none, 1
    velocity, 2 dropout)."""
    t = np.ascontiguousarray(t, np.float64)
    r = _f32(ranges)
    v = _f32(vel)
    T, N = r.shape[0], r.shape[1]
    out = np.empty((T, N, 3), np.float64)
    st = np.empty((T, N), np.int32)
    _load().orc_dvl(T, N, _ptr(t), _ptr(r), _ptr(v), cfg.janus, cfg.range_min, cfg.range_max, cfg.min_beams,
                    cfg.sigma_v, cfg.sound_speed, cfg.pings_per_output, cfg.period_min, cfg.seed_lo, cfg.seed_hi,
                    _ptr(out), _ptr(st))
    return out, st


# --------------------------------------------------------------------------- #
# Ray casting of the sonar's returns against a triangle mesh                  #
# --------------------------------------------------------------------------- #
def raycast(vertices, triangles, tri_mat, pos, rot, n_beams, n_rays, fov_az, fov_el, t_max, band=1e-5, sel=None):
    """Brute-force closest hits of the sonar ray pattern (see orc_raycast):
    returns a dict with x, y, z, nx, ny, nz (float64, sensor frame), mat
    (int32, -1 = miss) and ambiguous (bool), each [n_beams * n_rays], or only
    for the return indices in ``sel``."""
    vv = _f32(vertices).reshape(-1, 3)
    tt = np.ascontiguousarray(triangles, np.int32).reshape(-1, 3)
    mm = np.ascontiguousarray(tri_mat, np.int32).reshape(-1)
    p = _f32(pos).reshape(3)
    R = _f32(rot).reshape(3, 3)
    sel_a = None if sel is None else np.ascontiguousarray(sel, np.int64)
    n = int(n_beams) * int(n_rays) if sel_a is None else sel_a.shape[0]
    out = {k: np.empty(n, np.float64) for k in ("x", "y", "z", "nx", "ny", "nz")}
    out["mat"] = np.empty(n, np.int32)
    amb = np.empty(n, np.uint8)
    _load().orc_raycast(vv.shape[0], _ptr(vv), tt.shape[0], _ptr(tt), _ptr(mm), _ptr(p), _ptr(R), int(n_beams),
                        int(n_rays), float(fov_az), float(fov_el), float(t_max), float(band),
                        0 if sel_a is None else sel_a.shape[0], _ptr(sel_a),
                        *[_ptr(out[k]) for k in ("x", "y", "z", "nx", "ny", "nz", "mat")], _ptr(amb))
    out["ambiguous"] = amb.astype(bool)
    return out
