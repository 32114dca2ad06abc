"""Pins of the oracle's navigation sensors (Sec. III-A: a barometer from the
atmospheric pressure and the water density with optional Gaussian noise; a
four-beam Janus DVL with a range-dependent rate and dropout).  Expected values
come from hydrostatics, the Janus geometry, exact recovery of a noise-free
velocity, numpy's least-squares solver, the normal law and the measurement
schedule in closed form for constant ranges."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import BaroConfig, DvlConfig


def test_barometer_hydrostatics():
    cfg = BaroConfig(p_atm=101325.0, rho=1025.0, g=9.80665)
    d = np.array([0.0, 10.0, -5.0, 1000.0, 0.5], np.float32)
    p = oracle.barometer(d, cfg)
    want = [101325.0, 101325.0 + 1025.0 * 9.80665 * 10.0, 101325.0, 101325.0 + 1025.0 * 9.80665 * 1000.0,
            101325.0 + 1025.0 * 9.80665 * 0.5]
    np.testing.assert_allclose(p, want, rtol=1e-15, atol=0)
    # the water column is linear in depth; fresh water weighs less
    p2 = oracle.barometer(np.array([20.0], np.float32), cfg)[0]
    assert p2 - cfg.p_atm == pytest.approx(2 * (p[1] - cfg.p_atm), rel=1e-15)
    fresh = oracle.barometer(np.array([10.0], np.float32), BaroConfig(rho=997.0))[0]
    assert fresh < p[1]


def test_barometer_noise_is_normal_and_reproducible():
    cfg = BaroConfig(sigma=50.0, seed_lo=11, seed_hi=3)
    d = np.full(200000, 12.5, np.float32)
    p = oracle.barometer(d, cfg)
    z = (p - (cfg.p_atm + cfg.rho * cfg.g * 12.5)) / cfg.sigma
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.std() - 1.0) < 5 / math.sqrt(2 * z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    np.testing.assert_array_equal(p, oracle.barometer(d, cfg))
    assert not np.array_equal(p, oracle.barometer(d, BaroConfig(sigma=50.0, seed_lo=12, seed_hi=3)))


def test_dvl_janus_geometry():
    for janus in (math.radians(20.0), math.radians(30.0)):
        b = oracle.dvl_beams(janus)
        np.testing.assert_allclose(np.linalg.norm(b, axis=1), 1.0, rtol=1e-15)
        np.testing.assert_allclose(b @ np.array([0.0, 0.0, -1.0]), math.cos(janus), rtol=1e-15)
        az = np.degrees(np.arctan2(b[:, 1], b[:, 0])) % 360.0
        np.testing.assert_allclose(az, [45.0, 135.0, 225.0, 315.0], atol=1e-12)
        np.testing.assert_allclose(b.sum(0), [0.0, 0.0, -4 * math.cos(janus)], atol=1e-15)


def _run(ranges, vel, cfg, dt=1.0 / 64):
    T = ranges.shape[0]
    return oracle.dvl(np.arange(T) * dt, ranges, vel, cfg)


def test_dvl_recovers_noise_free_velocity_with_three_or_four_beams():
    rs = np.random.default_rng(1)
    T, N = 1, 64
    vel = rs.normal(0, 1, (T, N, 3)).astype(np.float32)
    ranges = rs.uniform(5, 60, (T, N, 4)).astype(np.float32)
    ranges[0, N // 2:, 1] = 200.0   # beyond range_max: three beams left
    out, st = _run(ranges, vel, DvlConfig())
    assert np.all(st == 1)
    np.testing.assert_allclose(out, vel.astype(np.float64), rtol=0, atol=1e-12)


def test_dvl_dropout_and_beam_validity():
    cfg = DvlConfig(range_min=0.5, range_max=80.0, min_beams=3)
    vel = np.ones((1, 6, 3), np.float32)
    r = np.full((1, 6, 4), 10.0, np.float32)
    r[0, 0, :2] = [np.nan, np.inf]                  # two beams without a return
    r[0, 1, :3] = [0.4, -1.0, 80.5]                 # three beams out of range
    r[0, 2, :] = [0.5, 80.0, 0.5, 80.0]             # the range limits are inclusive
    r[0, 3, 0] = 90.0                               # one beam lost: three remain
    r[0, 4, :] = np.nan                             # no beam at all
    out, st = _run(r, vel, cfg)
    np.testing.assert_array_equal(st[0], [2, 2, 1, 1, 2, 1])
    assert np.all(np.isnan(out[0, [0, 1, 4]]))
    np.testing.assert_allclose(out[0, [2, 3, 5]], 1.0, atol=1e-12)
    _, st4 = _run(r, vel, DvlConfig(min_beams=4))
    np.testing.assert_array_equal(st4[0], [2, 2, 1, 2, 2, 1])


def test_dvl_least_squares_matches_library_solver():
    """With noise, the velocity is numpy's least-squares solution of the
    valid beams' along-beam equations (noise from the pinned Philox and
    Box-Muller on the cosine branch)."""
    cfg = DvlConfig(sigma_v=0.02, seed_lo=5, seed_hi=9)
    rs = np.random.default_rng(2)
    N = 40
    vel = rs.normal(0, 1, (1, N, 3)).astype(np.float32)
    r = rs.uniform(2, 70, (1, N, 4)).astype(np.float32)
    r[0, ::3, 2] = np.nan
    out, st = _run(r, vel, cfg)
    B = oracle.dvl_beams(cfg.janus)
    for n in range(N):
        ok = np.isfinite(r[0, n])
        words = [oracle.philox4x32_10(np.array([[0, n, 4, h]], np.uint32), np.array([[5, 9]], np.uint32))[0]
                 for h in (0, 1)]
        z = []
        for i in range(4):
            w = words[i // 2]
            u0 = ((int(w[2 * (i % 2)]) >> 8) + 1) / 16777216.0
            u1 = ((int(w[2 * (i % 2) + 1]) >> 8) + 1) / 16777216.0
            z.append(math.sqrt(-2 * math.log(u0)) * math.cos(2 * math.pi * u1))
        u = B @ vel[0, n].astype(np.float64) + cfg.sigma_v * np.array(z)
        x = np.linalg.lstsq(B[ok], u[ok], rcond=None)[0]
        assert st[0, n] == 1
        np.testing.assert_allclose(out[0, n], x, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("r, every", [(30.0, 21), (60.0, 41), (2.0, 8)])
def test_dvl_rate_follows_range(r, every):
    """Constant ranges r, ticks of 1/64 s: the period is max(0.125 s,
    8 * 2 r / 1500 m/s), so a measurement every ceil(period * 64) ticks."""
    T, N = 200, 3
    ranges = np.full((T, N, 4), r, np.float32)
    vel = np.zeros((T, N, 3), np.float32)
    _, st = _run(ranges, vel, DvlConfig())
    want = np.zeros(T, np.int32)
    want[::every] = 1
    for n in range(N):
        np.testing.assert_array_equal(st[:, n], want)


def test_dvl_rate_without_returns_and_after_a_gap():
    """No valid beam: the period of the maximum range (8 * 160 / 1500 s = 54.6
    ticks of 1/64 s), reported as dropouts; ranges that shrink mid-run shorten
    the period from then on."""
    T = 240
    ranges = np.full((T, 1, 4), np.nan, np.float32)
    ranges[120:] = 2.0
    _, st = _run(ranges, np.zeros((T, 1, 3), np.float32), DvlConfig())
    ticks = np.nonzero(st[:, 0])[0]
    np.testing.assert_array_equal(ticks[:3], [0, 55, 110])
    assert np.all(st[ticks[:3], 0] == 2)
    # from tick 120 the ranges give an 8-tick period, evaluated at the current
    # tick: 10 ticks have passed since tick 110, so tick 120 measures, then
    # every 8 ticks
    np.testing.assert_array_equal(ticks[3:6], [120, 128, 136])
    assert np.all(st[ticks[3:], 0] == 1)
