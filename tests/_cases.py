"""Small hand-built inputs shared by the oracle pins and the GPU parity tests."""
import json
import math
import os

import numpy as np

from workloads import SonarHits, SonarSpec, SPECKLE_OFF

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
DEG = math.pi / 180.0


def hit_at(r, az, el, incidence=0.0, tilt_axis=None):
    """Position at range r, azimuth az, elevation el (radians) and a unit
    normal at ``incidence`` radians from the reversed ray direction."""
    d = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    if tilt_axis is None:
        e = np.array([-math.sin(el) * math.cos(az), -math.sin(el) * math.sin(az), math.cos(el)])
    else:
        e = np.asarray(tilt_axis, float)
        e = e - e.dot(d) * d
        e = e / np.linalg.norm(e)
    n = -math.cos(incidence) * d + math.sin(incidence) * e
    return r * d, n


def build_hits(rows, refl=None):
    """rows: list of (pos[3], normal[3], mat)."""
    pos = np.array([p for p, _, _ in rows], dtype=np.float64).reshape(-1, 3)
    nrm = np.array([n for _, n, _ in rows], dtype=np.float64).reshape(-1, 3)
    mat = np.array([m for _, _, m in rows], dtype=np.int32)
    if refl is None:
        refl = np.ones(max(1, len(rows)), np.float32)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return SonarHits(x=f(pos[:, 0]), y=f(pos[:, 1]), z=f(pos[:, 2]),
                     nx=f(nrm[:, 0]), ny=f(nrm[:, 1]), nz=f(nrm[:, 2]),
                     mat=mat, refl=np.asarray(refl, np.float32))


def tiny_golden():
    """The hand-derived 3 x 4 frame of tests/golden/sonar_tiny.json."""
    with open(os.path.join(GOLDEN, "sonar_tiny.json")) as fh:
        g = json.load(fh)
    gr = g["grid"]
    spec = SonarSpec(r_min=gr["r_min"], r_max=gr["r_max"], n_range=gr["n_range"],
                     n_azimuth=gr["n_azimuth"], fov_az=gr["fov_az_deg"] * DEG,
                     fov_el=gr["fov_el_deg"] * DEG, alpha=gr["alpha"], kappa=gr["kappa"],
                     gain=gr["gain"], speckle_mode=SPECKLE_OFF)
    rows, refl, bins = [], [], []
    for k, ret in enumerate(g["returns"]):
        refl.append(ret["refl"])
        bins.append(ret["bin"])
        if ret.get("miss"):
            rows.append((np.zeros(3), np.zeros(3), -1))
            continue
        p, n = hit_at(ret["r"], ret["az_deg"] * DEG, ret["el_deg"] * DEG,
                      ret["incidence_deg"] * DEG)
        rows.append((p, n, k))
    hits = build_hits(rows, refl)
    expected = np.zeros(spec.n_range * spec.n_azimuth)
    for key, val in g["expected_polar"].items():
        if not key.startswith("_"):
            expected[int(key)] = val
    return spec, hits, np.array(bins, np.int32), expected.reshape(spec.n_range, spec.n_azimuth)


def philox_kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(t, 16) for t in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def fan_pixel_polar(spec, H, W):
    """Polar coordinates (rho, phi) of every fan pixel centre, float64 [H, W].

    Independent restatement of the fan layout for the linear-field pins: apex
    at the bottom centre, boresight up, square pixels sized so that the whole
    sector fits."""
    half = 0.5 * float(spec.fov_az)
    s = max(float(spec.r_max) / H, 2.0 * float(spec.r_max) * math.sin(half) / W)
    u = (np.arange(W) + 0.5 - 0.5 * W) * s
    v = (H - np.arange(H) - 0.5) * s
    X, Y = np.meshgrid(u, v)
    return np.hypot(X, Y), np.arctan2(-X, Y)
