"""FP64 central differences of the oracle's forward pass on the differentiable
batch (32 sonar frames of 512 x 64 returns with 64 materials, 512 x 512 bins,
512 x 1024 fans, paper speckle; 32 camera frames of 960 x 540 under one water
row), for the loss

    L = sum_f <w_polar_f, polar_f> + <w_fan_f, fan_f> + sum_c <w_c, I_c>

with the seeded N(0, 1) weights the parity tests use.  The parameters are
the sonar row (alpha, G, sigma_phi, sigma_sa, sigma_sm), eight of the 64
reflectivities and the water row (beta_D, beta_B, B_inf per channel).  No
parameter moves a return across a bin edge, so L is smooth in each of them.

Step sizes: h = 1e-5 |theta| for the sonar and water scalars (the third
derivative of exp(-2 alpha r) or exp(-beta d) relative to the first is at
most (2 r_max)^2 or d_max^2, so the truncation error stays below 1e-8
relative).  Reflectivities enter the oracle as float32: the perturbed values
are rounded to float32 and the difference quotient uses the rounded step
(L is linear in each reflectivity, so the secant is exact).
"""
import functools

import numpy as np

import oracle
from oracle import SonarConfig
import workloads as W

SONAR_KEYS = ("alpha", "gain", "sigma_phi", "sigma_sa", "sigma_sm")
REFL_SAMPLE = (0, 5, 13, 22, 31, 40, 51, 63)


def c4_inputs():
    frames = W.sonar_c4()
    cams, waters = W.camera_c4()
    gpol = [W.loss_weights((202, k), (f.spec.n_range, f.spec.n_azimuth)) for k, f in enumerate(frames)]
    gfan = [W.loss_weights((203, k), (f.spec.fan_h, f.spec.fan_w)) for k, f in enumerate(frames)]
    gout = [W.loss_weights((204, k), c.J.shape) for k, c in enumerate(cams)]
    return frames, cams, waters[0], gpol, gfan, gout


def _sonar_loss(frames, refl, gpol, gfan, over):
    tot = 0.0
    for f, a, b in zip(frames, gpol, gfan):
        res = oracle.sonar_forward(SonarConfig.from_spec(f.spec, **over), f.hits, refl)
        tot += float(np.dot(res["out"].ravel(), a.astype(np.float64).ravel()))
        tot += float(np.dot(res["fan"].ravel(), b.astype(np.float64).ravel()))
    return tot


def _camera_loss(cams, water, gout):
    tot = 0.0
    for c, g in zip(cams, gout):
        out = oracle.uw_forward(c.J, c.depth, *water)
        tot += float(np.dot(out.ravel(), g.astype(np.float64).ravel()))
    return tot


@functools.lru_cache(maxsize=1)
def c4_central_differences():
    """{"sonar": [5] (SONAR_KEYS order), "refl": {m: value}, "water": [9]}."""
    frames, cams, water, gpol, gfan, gout = c4_inputs()
    spec = frames[0].spec
    refl = frames[0].hits.refl.astype(np.float32)
    out = {"sonar": [], "refl": {}, "water": []}
    for key in SONAR_KEYS:
        theta = float(getattr(spec, key))
        h = 1e-5 * abs(theta)
        lp = _sonar_loss(frames, refl, gpol, gfan, {key: theta + h})
        lm = _sonar_loss(frames, refl, gpol, gfan, {key: theta - h})
        out["sonar"].append((lp - lm) / (2 * h))
    for m in REFL_SAMPLE:
        rp, rm = refl.copy(), refl.copy()
        rp[m] = np.float32(refl[m] * (1 + 1e-4))
        rm[m] = np.float32(refl[m] * (1 - 1e-4))
        step = float(rp[m]) - float(rm[m])
        lp = _sonar_loss(frames, rp, gpol, gfan, {})
        lm = _sonar_loss(frames, rm, gpol, gfan, {})
        out["refl"][m] = (lp - lm) / step
    base = [water.beta_d.astype(np.float64), water.beta_b.astype(np.float64), water.b_inf.astype(np.float64)]
    for p in range(3):
        for ch in range(3):
            theta = base[p][ch]
            h = 1e-5 * abs(theta)
            wp = [v.copy() for v in base]
            wm = [v.copy() for v in base]
            wp[p][ch] = theta + h
            wm[p][ch] = theta - h
            out["water"].append((_camera_loss(cams, wp, gout) - _camera_loss(cams, wm, gout)) / (2 * h))
    out["sonar"] = np.array(out["sonar"])
    out["water"] = np.array(out["water"])
    return out


def c4_oracle_gradients():
    """The oracle's analytic gradients of the same loss: (refl [64], sonar [5], water [9])."""
    frames, cams, water, gpol, gfan, gout = c4_inputs()
    refl = frames[0].hits.refl
    g_refl = np.zeros(refl.shape[0])
    g_par = np.zeros(5)
    for f, a, b in zip(frames, gpol, gfan):
        gr, gp, _ = oracle.sonar_backward(SonarConfig.from_spec(f.spec), f.hits, refl, a, b)
        g_refl += gr
        g_par += gp
    g_w = np.zeros(9)
    for c, g in zip(cams, gout):
        p, _, _ = oracle.uw_backward(c.J, c.depth, water.beta_d, water.beta_b, water.b_inf, g, False)
        g_w += p
    return g_refl, g_par, g_w
