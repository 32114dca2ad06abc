"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test names what fixes its expected value: a published known-answer
vector, a closed form of a special case of Eq. (1)-(6), a distribution law,
an identity (energy, symmetry, adjointness) or finite differences of the
oracle's own forward pass (for the hand-derived backward pass).
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import SonarConfig
from workloads import (SPECKLE_GAMMA, SPECKLE_OFF, SPECKLE_PAPER, SonarSpec, Stream,
                       make_camera, make_hits, make_water, sonar_c1, sonar_c2)

from _cases import DEG, build_hits, fan_pixel_polar, hit_at, philox_kat, tiny_golden


# --------------------------------------------------------------------------- #
# Philox4x32-10                                                               #
# --------------------------------------------------------------------------- #
def test_philox_known_answers():
    for ctr, key, want in philox_kat():
        got = oracle.philox4x32_10(np.array([ctr]), np.array([key]))[0]
        assert [int(v) for v in got] == want


def test_philox_uniform_chi2():
    n = 1 << 18
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 1] = 7
    out = oracle.philox4x32_10(ctr, np.array([[123, 456]]))
    for w in range(4):
        hist = np.bincount((out[:, w] >> 24).astype(np.int64), minlength=256)
        chi2 = ((hist - n / 256) ** 2 / (n / 256)).sum()
        assert stats.chi2.sf(chi2, 255) > 1e-4


# --------------------------------------------------------------------------- #
# Eq. (2) and binning                                                         #
# --------------------------------------------------------------------------- #
def _cfg(spec, **kw):
    return SonarConfig.from_spec(spec, **kw)


def test_single_return_normal_incidence_closed_form():
    """A return at normal incidence gives refl * G * exp(-kappa alpha r) in its bin."""
    spec = SonarSpec(r_min=0.5, r_max=20.0, n_range=64, n_azimuth=32, alpha=0.1, gain=1.7,
                     speckle_mode=SPECKLE_OFF)
    for kappa in (2.0, 1.0):
        for r, az, el in [(3.3, 0.2, 0.05), (17.9, -1.0, -0.1), (0.77, 1.1, 0.0)]:
            p, n = hit_at(r, az, el)
            hits = build_hits([(p, n, 0)], refl=[0.6])
            res = oracle.sonar_forward(_cfg(spec, kappa=kappa), hits, hits.refl)
            rr = float(np.linalg.norm(np.float32(p).astype(np.float64)))
            want = np.float32(0.6) * np.float32(1.7) * math.exp(-kappa * np.float32(0.1) * rr)
            b = res["bins"][0]
            assert b >= 0
            assert res["out"].ravel()[b] == pytest.approx(want, rel=1e-6)
            assert np.count_nonzero(res["out"]) == 1


def test_oblique_incidence_cosine():
    spec = SonarSpec(r_min=0.5, r_max=20.0, n_range=16, n_azimuth=16, speckle_mode=SPECKLE_OFF)
    for inc in (0.0, 0.3, 1.0, 1.4):
        p, n = hit_at(5.0, 0.1, 0.0, incidence=inc)
        hits = build_hits([(p, n, 0)], refl=[1.0])
        res = oracle.sonar_forward(_cfg(spec), hits, hits.refl)
        want = math.cos(inc) * math.exp(-2 * np.float32(0.1) * 5.0)
        assert res["intensity"][0] == pytest.approx(want, rel=1e-6)
    # back-facing and zero normals return nothing but still bin
    p, n = hit_at(5.0, 0.1, 0.0, incidence=2.0)
    hits = build_hits([(p, n, 0), (p, np.zeros(3), 0)], refl=[1.0])
    res = oracle.sonar_forward(_cfg(spec), hits, hits.refl)
    assert np.all(res["intensity"] == 0.0) and np.all(res["bins"] >= 0)
    # a non-unit normal is normalised (Eq. 2 divides by |v_n|)
    p, n = hit_at(5.0, 0.1, 0.0, incidence=0.5)
    h1 = build_hits([(p, n, 0)], refl=[1.0])
    h2 = build_hits([(p, 7.5 * n, 0)], refl=[1.0])
    a = oracle.sonar_forward(_cfg(spec), h1, h1.refl)["intensity"][0]
    b = oracle.sonar_forward(_cfg(spec), h2, h2.refl)["intensity"][0]
    assert a == pytest.approx(b, rel=1e-6)


def test_tiny_golden_frame():
    spec, hits, bins, expected = tiny_golden()
    res = oracle.sonar_forward(_cfg(spec), hits, hits.refl)
    np.testing.assert_array_equal(res["bins"], bins)
    np.testing.assert_allclose(res["out"], expected, rtol=1e-6, atol=1e-12)


def test_bins_by_construction():
    """Points placed inside known cells land in exactly those cells."""
    spec = SonarSpec(r_min=1.0, r_max=50.0, n_range=1024, n_azimuth=1024, speckle_mode=SPECKLE_OFF)
    st = Stream(99, 1)
    n = 20000
    i = st.integers(0, spec.n_range - 1, n)
    j = st.integers(0, spec.n_azimuth - 1, n)
    dr = (spec.r_max - spec.r_min) / spec.n_range
    dp = spec.fov_az / spec.n_azimuth
    r = spec.r_min + (i + st.uniform(0.01, 0.99, n)) * dr
    az = -spec.fov_az / 2 + (j + st.uniform(0.01, 0.99, n)) * dp
    el = st.uniform(-0.15, 0.15, n)
    rows = []
    for k in range(n):
        p, nn = hit_at(r[k], az[k], el[k])
        rows.append((p, nn, k))
    hits = build_hits(rows, refl=np.ones(n))
    res = oracle.sonar_forward(_cfg(spec), hits, hits.refl)
    np.testing.assert_array_equal(res["bins"], (i * spec.n_azimuth + j).astype(np.int32))


def test_dropped_returns():
    spec = SonarSpec(r_min=1.0, r_max=10.0, n_range=32, n_azimuth=32, speckle_mode=SPECKLE_OFF)
    rows = []
    for r, az, el in [(0.5, 0, 0), (10.5, 0, 0), (5, 70 * DEG, 0), (5, -66 * DEG, 0),
                      (5, 0, 11 * DEG), (5, 0, -11 * DEG), (5, math.pi, 0)]:
        p, n = hit_at(r, az, el)
        rows.append((p, n, 0))
    p, n = hit_at(5, 0, 0)
    rows.append((p, n, -1))          # miss
    rows.append((p, n, 5))           # material id beyond the table
    rows.append((np.zeros(3), n, 0))  # at the origin
    hits = build_hits(rows, refl=[1.0])
    res = oracle.sonar_forward(_cfg(spec), hits, hits.refl)
    assert np.all(res["bins"] == -1)
    assert np.all(res["out"] == 0.0)


def test_energy_conservation():
    """Sum over bins of P equals the sum of the per-return closed forms."""
    spec = SonarSpec(r_min=0.5, r_max=20.0, n_range=40, n_azimuth=30, alpha=0.07, gain=1.0,
                     speckle_mode=SPECKLE_OFF)
    st = Stream(5, 5)
    n = 3000
    r = st.uniform(0.6, 19.9, n)
    az = st.uniform(-1.1, 1.1, n)
    inc = st.uniform(0.0, 1.2, n)
    refl = st.uniform(0.1, 1.0, n)
    rows = [(*hit_at(r[k], az[k], 0.0, inc[k]), k) for k in range(n)]
    hits = build_hits(rows, refl=refl)
    res = oracle.sonar_forward(_cfg(spec), hits, hits.refl)
    rr = np.sqrt(hits.x.astype(float) ** 2 + hits.y.astype(float) ** 2 + hits.z.astype(float) ** 2)
    want = (hits.refl.astype(float) * np.cos(inc) * np.exp(-2 * float(np.float32(0.07)) * rr)).sum()
    assert res["P"].sum() == pytest.approx(want, rel=1e-6)
    # many returns in one bin add up
    assert np.bincount(res["bins"], minlength=40 * 30).max() > 3


def test_generator_keeps_clear_of_edges():
    """Stored float32 hits sit >= 1e-3 cells from every bin edge (recomputed in FP64)."""
    for frame in sonar_c1() + sonar_c2():
        s, h = frame.spec, frame.hits
        hit = h.mat >= 0
        x, y, z = (a[hit].astype(np.float64) for a in (h.x, h.y, h.z))
        r = np.sqrt(x * x + y * y + z * z)
        fr = (r - s.r_min) * s.n_range / (s.r_max - s.r_min)
        fp = (np.arctan2(y, x) + s.fov_az / 2) * s.n_azimuth / s.fov_az
        for f in (fr, fp):
            frac = f - np.floor(f)
            assert np.minimum(frac, 1 - frac).min() >= 1e-3
        assert np.all(np.abs(z) < r * math.sin(s.fov_el / 2))


# --------------------------------------------------------------------------- #
# Speckle, Eq. (3)-(6)                                                        #
# --------------------------------------------------------------------------- #
def test_speckle_additive_is_rayleigh():
    """Eq. (3)-(4): with a flat beam pattern the additive term is
    R_i (1 + 0.5 sigma_sa rho) with rho ~ Rayleigh(1)."""
    sigma_sa = 0.3
    spec = SonarSpec(r_min=2.0, r_max=30.0, n_range=256, n_azimuth=512, speckle_mode=SPECKLE_GAMMA,
                     sigma_sa=sigma_sa, sigma_phi=1e30, seed_lo=11, seed_hi=22, frame_id=3)
    add, _ = oracle.speckle_fields(_cfg(spec))
    dr = (spec.r_max - spec.r_min) / spec.n_range
    ri = spec.r_min + (np.arange(spec.n_range) + 0.5) * dr
    R = (ri / spec.r_max) ** 2
    rho = (add / R[:, None] - 1.0) / (0.5 * np.float32(sigma_sa))
    ks = stats.kstest(rho.ravel(), stats.rayleigh.cdf)
    assert ks.pvalue > 1e-3
    assert rho.mean() == pytest.approx(math.sqrt(math.pi / 2), abs=5 * math.sqrt((4 - math.pi) / 2 / rho.size))
    # sigma_sa = 0 leaves the deterministic floor r_i^2 / r_max^2 of Eq. (3)
    add0, _ = oracle.speckle_fields(_cfg(spec, sigma_sa=0.0))
    np.testing.assert_allclose(add0, np.repeat(R[:, None], spec.n_azimuth, 1), rtol=1e-14)


def test_speckle_beam_pattern():
    """The azimuth factor is exp(-phi_j^2 / sigma_phi) at bin centres."""
    spec = SonarSpec(r_min=1.0, r_max=10.0, n_range=8, n_azimuth=64, speckle_mode=SPECKLE_GAMMA,
                     sigma_sa=0.2, seed_lo=1)
    a1, _ = oracle.speckle_fields(_cfg(spec, sigma_phi=0.3))
    a2, _ = oracle.speckle_fields(_cfg(spec, sigma_phi=0.7))
    dr = (spec.r_max - spec.r_min) / spec.n_range
    R = ((spec.r_min + (np.arange(8) + 0.5) * dr) / spec.r_max) ** 2
    phi = -spec.fov_az / 2 + (np.arange(64) + 0.5) * spec.fov_az / 64
    ratio = (a1 / R[:, None] - 1) / (a2 / R[:, None] - 1)
    want = np.exp(-phi ** 2 * (1 / 0.3 - 1 / 0.7))
    np.testing.assert_allclose(ratio, np.broadcast_to(want, ratio.shape), rtol=1e-10)


def test_speckle_multiplicative_laws():
    base = dict(r_min=1.0, r_max=10.0, n_range=512, n_azimuth=512, seed_lo=77, seed_hi=1)
    # Eq. (5)-(6): factor 0.5 + w_sm with w_sm ~ N(0, sigma_sm)
    spec = SonarSpec(speckle_mode=SPECKLE_PAPER, sigma_sm=0.2, **base)
    _, mul = oracle.speckle_fields(_cfg(spec))
    zs = (mul.ravel() - 0.5) / np.float32(0.2)
    assert stats.kstest(zs, stats.norm.cdf).pvalue > 1e-3
    # gamma speckle: mean 1, variance 1/k
    for k in (1, 3, 4, 8):
        spec = SonarSpec(speckle_mode=SPECKLE_GAMMA, gamma_k=k, **base)
        _, mul = oracle.speckle_fields(_cfg(spec))
        assert stats.kstest(mul.ravel(), stats.gamma(a=k, scale=1.0 / k).cdf).pvalue > 1e-3


def test_speckle_independent_across_bins_and_frames():
    spec = SonarSpec(r_min=1.0, r_max=10.0, n_range=256, n_azimuth=256, speckle_mode=SPECKLE_GAMMA,
                     sigma_sa=0.3, sigma_phi=1e30, seed_lo=5)
    a0, m0 = oracle.speckle_fields(_cfg(spec, frame_id=0))
    a1, m1 = oracle.speckle_fields(_cfg(spec, frame_id=1))
    # remove the deterministic range ramp r_i^2 / r_max^2 of Eq. (3)
    dr = (spec.r_max - spec.r_min) / spec.n_range
    R = (((spec.r_min + (np.arange(spec.n_range) + 0.5) * dr) / spec.r_max) ** 2)[:, None]
    a0, a1 = a0 / R, a1 / R
    for u, v in [(a0[:, :-1], a0[:, 1:]), (m0[:, :-1], m0[:, 1:]), (a0, a1), (m0, m1), (a0, m0)]:
        c = np.corrcoef(u.ravel(), v.ravel())[0, 1]
        assert abs(c) < 5.0 / math.sqrt(u.size)


def test_speckle_composition():
    """Eq. (5): out = Q m + a, so out(with returns) - out(empty) = G P m."""
    frame = sonar_c1()[0]
    cfg = _cfg(frame.spec, gain=float(np.float32(1.3)))
    res = oracle.sonar_forward(cfg, frame.hits, frame.hits.refl, with_fan=False)
    empty = build_hits([], refl=[1.0])
    res0 = oracle.sonar_forward(cfg, empty, empty.refl, with_fan=False)
    add, mul = oracle.speckle_fields(cfg)
    np.testing.assert_allclose(res0["out"], add, rtol=0, atol=0)
    np.testing.assert_allclose(res["out"] - res0["out"], np.float32(1.3) * res["P"] * mul,
                               rtol=1e-12, atol=1e-15)


# --------------------------------------------------------------------------- #
# Fan                                                                          #
# --------------------------------------------------------------------------- #
FAN_SPEC = SonarSpec(r_min=1.0, r_max=12.0, n_range=48, n_azimuth=40, fan_h=96, fan_w=160)


def test_fan_constant_field():
    cfg = _cfg(FAN_SPEC)
    fan, amb = oracle.fan_forward(cfg, np.full((48, 40), 2.5))
    rho, phi = fan_pixel_polar(FAN_SPEC, 96, 160)
    inside = (rho >= 1.0) & (rho <= 12.0) & (np.abs(phi) <= FAN_SPEC.fov_az / 2)
    ok = ~amb
    np.testing.assert_allclose(fan[inside & ok], 2.5, rtol=1e-14)
    assert np.all(fan[~inside & ok] == 0.0)
    assert inside.sum() > 0.3 * inside.size


def test_fan_linear_fields_are_exact():
    """Bilinear interpolation reproduces fields linear in range or azimuth."""
    cfg = _cfg(FAN_SPEC)
    dr = (12.0 - 1.0) / 48
    dp = FAN_SPEC.fov_az / 40
    ri = 1.0 + (np.arange(48) + 0.5) * dr
    pj = -FAN_SPEC.fov_az / 2 + (np.arange(40) + 0.5) * dp
    rho, phi = fan_pixel_polar(FAN_SPEC, 96, 160)
    inner = ((rho >= ri[0]) & (rho <= ri[-1]) & (phi >= pj[0]) & (phi <= pj[-1]))
    fan, amb = oracle.fan_forward(cfg, np.repeat((3.0 * ri - 1.0)[:, None], 40, 1))
    np.testing.assert_allclose(fan[inner], (3.0 * rho - 1.0)[inner], rtol=1e-12)
    fan, amb = oracle.fan_forward(cfg, np.repeat((2.0 * pj + 5.0)[None, :], 48, 0))
    np.testing.assert_allclose(fan[inner], (2.0 * phi + 5.0)[inner], rtol=1e-12)
    # clamp to edge: just inside r_min the value is that of the first row
    rim = (rho >= 1.0) & (rho < ri[0]) & (np.abs(phi) < pj[-1]) & ~amb
    fan, _ = oracle.fan_forward(cfg, np.repeat((3.0 * ri - 1.0)[:, None], 40, 1))
    assert rim.sum() > 0
    np.testing.assert_allclose(fan[rim], 3.0 * ri[0] - 1.0, rtol=1e-12)


def test_fan_mirror_symmetry_and_left_right():
    cfg = _cfg(FAN_SPEC)
    img = Stream(3, 3).uniform(0, 1, (48, 40))
    fan, _ = oracle.fan_forward(cfg, img)
    fan_m, _ = oracle.fan_forward(cfg, img[:, ::-1])
    np.testing.assert_allclose(fan[:, ::-1], fan_m, rtol=1e-12, atol=1e-15)
    # the sensor's left (positive azimuth, high column index) is drawn on the image's left
    left = np.zeros((48, 40))
    left[:, 30:] = 1.0
    fan, _ = oracle.fan_forward(cfg, left)
    assert fan[:, :80].sum() > 10 * fan[:, 80:].sum()


def test_fan_adjoint_identity():
    cfg = _cfg(FAN_SPEC)
    st = Stream(4, 4)
    x = st.uniform(-1, 1, (48, 40))
    y = st.uniform(-1, 1, (96, 160))
    fan, _ = oracle.fan_forward(cfg, x)
    gx = oracle.fan_adjoint(cfg, y)
    assert (fan * y).sum() == pytest.approx((x * gx).sum(), rel=1e-12)


def test_fan_adjoint_mirror_symmetry():
    """The transpose of the fan commutes with the left-right mirror: the fan
    gradient mirrored across the image gives the polar gradient mirrored in
    azimuth (the property that lets one operator row serve a bin and its
    mirror bin)."""
    cfg = _cfg(FAN_SPEC)
    y = Stream(4, 5).uniform(-1, 1, (96, 160))
    gx = oracle.fan_adjoint(cfg, y)
    gxm = oracle.fan_adjoint(cfg, y[:, ::-1].copy())
    np.testing.assert_allclose(gx[:, ::-1], gxm, rtol=1e-12, atol=1e-14)
    assert np.abs(gx).max() > 0


# --------------------------------------------------------------------------- #
# Camera, Eq. (1)                                                             #
# --------------------------------------------------------------------------- #
def test_uw_special_cases():
    st = Stream(8, 8)
    cam = make_camera(st, 16, 24)
    J, d = cam.J, cam.depth
    z3 = np.zeros(3)
    binf = np.array([0.1, 0.2, 0.3])
    # no water: the clear image
    np.testing.assert_array_equal(oracle.uw_forward(J, d, z3, z3, binf), J.astype(np.float64))
    # zero depth: the clear image
    np.testing.assert_allclose(oracle.uw_forward(J, np.zeros_like(d), [0.3] * 3, [0.2] * 3, binf),
                               J, rtol=0, atol=0)
    # infinite depth: the veiling light B_inf
    out = oracle.uw_forward(J, np.full_like(d, np.inf), [0.3] * 3, [0.2] * 3, binf)
    np.testing.assert_allclose(out, np.broadcast_to(binf[:, None, None], out.shape), rtol=1e-15)
    # no veiling light: pure attenuation, halving at beta_D d = ln 2
    out = oracle.uw_forward(J, np.ones_like(d), [math.log(2)] * 3, [0.2] * 3, z3)
    np.testing.assert_allclose(out, 0.5 * J.astype(np.float64), rtol=1e-15)
    # black scene: backscatter only, B_inf (1 - exp(-beta_B d))
    out = oracle.uw_forward(np.zeros_like(J), d, [0.3] * 3, [0.25] * 3, binf)
    want = binf[:, None, None] * (1 - np.exp(-0.25 * d.astype(np.float64)))[None]
    np.testing.assert_allclose(out, want, rtol=1e-13)


# --------------------------------------------------------------------------- #
# Backward passes against FP64 central differences                           #
# --------------------------------------------------------------------------- #
def _sonar_loss(spec, hits, refl, wp, wf, **over):
    cfg = _cfg(spec, **over)
    res = oracle.sonar_forward(cfg, hits, refl)
    L = (wp * res["out"]).sum()
    if wf is not None:
        L += (wf * res["fan"]).sum()
    return L


@pytest.mark.parametrize("mode", [SPECKLE_OFF, SPECKLE_PAPER, SPECKLE_GAMMA])
def test_sonar_backward_matches_central_differences(mode):
    st = Stream(21, mode)
    spec = SonarSpec(r_min=0.5, r_max=8.0, n_range=24, n_azimuth=20, fan_h=40, fan_w=64,
                     alpha=0.13, gain=1.4, sigma_phi=0.35, sigma_sa=0.15, sigma_sm=0.12,
                     speckle_mode=mode, gamma_k=4, seed_lo=9, frame_id=2)
    hits = make_hits(st, spec, 600, n_materials=6)
    refl = hits.refl.astype(np.float64)
    wp = st.normal((24, 20))
    wf = st.normal((40, 64))
    g_refl, g_par, g_out = oracle.sonar_backward(_cfg(spec), hits, hits.refl, wp, wf)

    def fd(fun, x0):
        h = 1e-6 * max(1.0, abs(x0))
        return (fun(x0 + h) - fun(x0 - h)) / (2 * h)

    names = ["alpha", "gain", "sigma_phi", "sigma_sa", "sigma_sm"]
    for k, name in enumerate(names):
        x0 = float(getattr(spec, name))
        want = fd(lambda v: _sonar_loss(spec, hits, hits.refl, wp, wf, **{name: v}), x0)
        assert g_par[k] == pytest.approx(want, rel=1e-6, abs=1e-9 * max(1.0, abs(want)))
    # reflectivity table: float32 inputs, so perturb through a float64 copy of the loss
    for m in range(6):
        def L(v):
            rf = refl.copy()
            rf[m] = v
            # the oracle takes float32 reflectivities: use a step that float32 resolves
            return _sonar_loss(spec, hits, rf.astype(np.float32), wp, wf)
        h = 2.0 ** -10
        want = (L(refl[m] + h) - L(refl[m] - h)) / (2 * h)   # exact in f32 steps; loss is linear in refl
        assert g_refl[m] == pytest.approx(want, rel=1e-6, abs=1e-9)


# --------------------------------------------------------------------------- #
# Range-wise normalisation (Sec. III-A.2, no formula given; the reading:     #
# after the gain, each range row over its maximum when that is positive)     #
# --------------------------------------------------------------------------- #
def _norm_frame(seed, n=900, mode=SPECKLE_OFF):
    st = Stream(60 + seed, mode)
    spec = SonarSpec(r_min=0.5, r_max=8.0, n_range=30, n_azimuth=24, fan_h=40, fan_w=64,
                     alpha=0.13, gain=1.4, sigma_phi=0.35, sigma_sa=0.15, sigma_sm=0.12,
                     speckle_mode=mode, gamma_k=4, seed_lo=9, frame_id=2, range_norm=1)
    hits = make_hits(st, spec, n, n_materials=6)
    return spec, hits


def _rows_emptied_and_negated(spec, hits, empty=(3, 7), negative=(5, 11)):
    """Per-return reflectivities; the returns of some rows made misses, those
    of others given negative reflectivities."""
    rows = oracle.sonar_forward(_cfg(spec, range_norm=0), hits, hits.refl)["bins"] // spec.n_azimuth
    hits.mat = np.where(np.isin(rows, empty), -1, np.arange(len(rows))).astype(np.int32)
    refl = np.abs(Stream(77, 1).uniform(0.2, 1.0, len(rows))).astype(np.float32)
    hits.refl = np.where(np.isin(rows, negative), -refl, refl).astype(np.float32)
    return hits


def test_range_norm_rows_peak_at_one():
    """Speckle off: every row with a positive maximum peaks at exactly 1 and
    keeps its shape; empty rows stay 0; the gain and a common scale of the
    reflectivities cancel."""
    spec, hits = _norm_frame(1)
    hits = _rows_emptied_and_negated(spec, hits, negative=())
    out = oracle.sonar_forward(_cfg(spec), hits, hits.refl)["out"]
    raw = oracle.sonar_forward(_cfg(spec, range_norm=0), hits, hits.refl)["out"]
    pos = raw.max(axis=1) > 0
    assert pos.sum() > 10 and (~pos).sum() > 0          # some rows are empty (returns cover part of the range)
    np.testing.assert_array_equal(out[pos].max(axis=1), 1.0)
    assert np.all(out[~pos] == 0.0)
    # each normalised row is a positive multiple of the raw row
    ratio = raw[pos].max(axis=1) / out[pos].max(axis=1)
    np.testing.assert_allclose(out[pos] * ratio[:, None], raw[pos], rtol=1e-12, atol=1e-300)
    out2 = oracle.sonar_forward(_cfg(spec, gain=3.7), hits, (hits.refl * 4.0).astype(np.float32))["out"]
    np.testing.assert_allclose(out2, out, rtol=1e-12, atol=1e-15)


def test_range_norm_leaves_negative_rows():
    """Signed reflectivities: a row whose maximum is 0 or negative is left
    as it is; the others peak at 1."""
    spec, hits = _norm_frame(2)
    hits = _rows_emptied_and_negated(spec, hits)
    out = oracle.sonar_forward(_cfg(spec), hits, hits.refl)["out"]
    raw = oracle.sonar_forward(_cfg(spec, range_norm=0), hits, hits.refl)["out"]
    neg = (raw.max(axis=1) <= 0) & (raw.min(axis=1) < 0)
    pos = raw.max(axis=1) > 0
    assert neg.sum() > 0 and pos.sum() > 0
    np.testing.assert_array_equal(out[neg], raw[neg])
    np.testing.assert_array_equal(out[pos].max(axis=1), 1.0)


@pytest.mark.parametrize("mode", [SPECKLE_OFF, SPECKLE_PAPER, SPECKLE_GAMMA])
def test_range_norm_backward_matches_central_differences(mode):
    """The subgradient at each row's maximum matches central differences
    (the maxima are unique, and the steps are too small to move them)."""
    spec, hits = _norm_frame(3, mode=mode)
    st = Stream(70, mode)
    wp = st.normal((30, 24))
    wf = st.normal((40, 64))
    refl = hits.refl.astype(np.float64)
    g_refl, g_par, _ = oracle.sonar_backward(_cfg(spec), hits, hits.refl, wp, wf)
    for k, name in enumerate(["alpha", "gain", "sigma_phi", "sigma_sa", "sigma_sm"]):
        x0 = float(getattr(spec, name))
        h = 1e-6 * max(1.0, abs(x0))
        want = (_sonar_loss(spec, hits, hits.refl, wp, wf, **{name: x0 + h}) -
                _sonar_loss(spec, hits, hits.refl, wp, wf, **{name: x0 - h})) / (2 * h)
        assert g_par[k] == pytest.approx(want, rel=1e-6, abs=1e-8 * max(1.0, abs(want)))
    # the gain cancels in every normalised row (all rows here have positive maxima or are empty)
    assert abs(g_par[1]) <= 1e-9 * np.abs(g_par).max()
    for m in range(6):
        def L(v):
            rf = refl.copy()
            rf[m] = v
            return _sonar_loss(spec, hits, rf.astype(np.float32), wp, wf)
        h = 2.0 ** -16
        want = (L(refl[m] + h) - L(refl[m] - h)) / (2 * h)
        assert g_refl[m] == pytest.approx(want, rel=1e-5, abs=1e-8 * np.abs(g_refl).max())


def test_uw_backward_matches_central_differences():
    st = Stream(31, 1)
    cam = make_camera(st, 12, 10)
    water = make_water(st)
    g = st.normal((3, 12, 10))
    bd, bb, bi = (w.astype(np.float64) for w in (water.beta_d, water.beta_b, water.b_inf))
    g_par, g_J, g_d = oracle.uw_backward(cam.J, cam.depth, bd, bb, bi, g)
    params = np.concatenate([bd, bb, bi])
    for k in range(9):
        h = 1e-6 * max(1.0, abs(params[k]))
        p1, p2 = params.copy(), params.copy()
        p1[k] += h
        p2[k] -= h
        L1 = (g * oracle.uw_forward(cam.J, cam.depth, p1[:3], p1[3:6], p1[6:])).sum()
        L2 = (g * oracle.uw_forward(cam.J, cam.depth, p2[:3], p2[3:6], p2[6:])).sum()
        assert g_par[k] == pytest.approx((L1 - L2) / (2 * h), rel=1e-7)
    # image gradients: Eq. (1) is linear in J with slope exp(-beta_D d)
    np.testing.assert_allclose(g_J, g * np.exp(-bd[:, None, None] * cam.depth.astype(float)[None]),
                               rtol=1e-14)
    # depth gradient by central differences on a few pixels; the depth is a
    # float32 input, so the step is a power of two that float32 represents
    h = 2.0 ** -9
    for (v, u) in [(0, 0), (5, 7), (11, 9)]:
        def L(dv):
            d = cam.depth.copy()
            d[v, u] = dv
            return (g * oracle.uw_forward(cam.J, d, bd, bb, bi)).sum()
        d0 = float(cam.depth[v, u])
        assert g_d[v, u] == pytest.approx((L(d0 + h) - L(d0 - h)) / (2 * h), rel=1e-5)


def test_sonar_backward_conditions_expand_the_fan():
    """The conditions of the gradients (sums of term magnitudes, the scale of
    float32 rounding) expand each bin's output gradient into its terms: the
    sigma_sa condition equals sum_b (adjoint of |g_fan| + |g_polar|)_b times
    the bin's factor R E rho / 2, which the additive field gives as
    (add - R) / sigma_sa; with a gradient that cancels within bins it exceeds
    the magnitude of the cancelled sums."""
    st = Stream(22, 1)
    spec = SonarSpec(r_min=0.5, r_max=8.0, n_range=24, n_azimuth=20, fan_h=40, fan_w=64,
                     alpha=0.13, gain=1.4, sigma_phi=0.35, sigma_sa=0.15, sigma_sm=0.12,
                     speckle_mode=SPECKLE_PAPER, seed_lo=9, frame_id=2)
    hits = make_hits(st, spec, 600, n_materials=6)
    cfg = _cfg(spec)
    wp = st.normal((24, 20))
    wf = st.normal((40, 64))
    _, g_par, g_out, a_refl, a_par = oracle.sonar_backward(cfg, hits, hits.refl, wp, wf, with_abs=True)
    add, _ = oracle.speckle_fields(cfg)
    dr = (spec.r_max - spec.r_min) / spec.n_range
    r = spec.r_min + (np.arange(spec.n_range) + 0.5) * dr
    R = (r * r / (spec.r_max * spec.r_max))[:, None]
    fsa = (add - R) / spec.sigma_sa                       # R E rho / 2 per bin
    g_abs = oracle.fan_adjoint(cfg, np.abs(wf)) + np.abs(wp)
    assert a_par[3] == pytest.approx(float((g_abs * np.abs(fsa)).sum()), rel=1e-12)
    assert a_par[3] > float(np.abs(g_out * fsa).sum())    # cancellation inside bins
    # without a fan gradient the expansion is the polar gradient itself
    _, _, g_out2, _, a_par2 = oracle.sonar_backward(cfg, hits, hits.refl, wp, None, with_abs=True)
    assert a_par2[3] == pytest.approx(float(np.abs(g_out2 * fsa).sum()), rel=1e-12)


def test_differentiable_batch_gradients_match_stored_central_differences():
    """The oracle's analytic gradients on the whole differentiable batch (32
    sonar + 32 camera frames) against FP64 central differences of its own
    forward pass, stored by tests/golden/make_c4_fd.py: 1e-7 relative."""
    import json
    import os

    import _fd
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "c4_central_differences.json")) as fh:
        fd = json.load(fh)
    g_refl, g_par, g_w = _fd.c4_oracle_gradients()
    np.testing.assert_allclose(g_par, fd["sonar"], rtol=1e-7, atol=0)
    for m, v in fd["refl"].items():
        assert g_refl[int(m)] == pytest.approx(v, rel=1e-7)
    np.testing.assert_allclose(g_w, fd["water"], rtol=1e-7, atol=0)
