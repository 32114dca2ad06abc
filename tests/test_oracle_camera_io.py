"""Pins of the camera conditioning oracle against published values, inverse
pairs and geometry (no GPU).

The sRGB transfer function is the one of IEC 61966-2-1; Eq. (1) of Sec. III-A.1
takes the line-of-sight distance d, obtained here from z-depth by pinhole
back-projection.
"""
import numpy as np
import pytest

from oracle import camera_io as cio


def test_published_srgb_values():
    # Widely tabulated values of the sRGB curves: linear 0.5 encodes to
    # 0.735357, sRGB 0.5 decodes to 0.214041 (six figures).
    assert cio.linear_to_srgb(0.5) == pytest.approx(0.735357, abs=5e-7)
    assert cio.srgb_to_linear(0.5) == pytest.approx(0.214041, abs=5e-7)
    assert cio.decode_codes(0) == 0.0
    assert cio.decode_codes(255) == pytest.approx(1.0, abs=1e-15)
    # the two segments of each curve meet at the breakpoints (to 1e-7)
    x0, y0 = 0.0031308, 0.04045
    assert 12.92 * x0 == pytest.approx(1.055 * x0 ** (1 / 2.4) - 0.055, abs=1e-7)
    assert cio.srgb_to_linear(y0) == pytest.approx(((y0 + 0.055) / 1.055) ** 2.4, abs=1e-7)


def test_inverse_pair():
    # The standard's two breakpoints (0.04045 and 12.92 * 0.0031308) differ by
    # 6.4e-8, so the pair is exact only outside that sliver of y.
    y = np.linspace(0.0, 1.0, 100001)
    off = (y < 0.0404499) | (y > 0.0404501)
    np.testing.assert_allclose(cio.linear_to_srgb(cio.srgb_to_linear(y[off])), y[off], atol=1e-12)
    np.testing.assert_allclose(cio.linear_to_srgb(cio.srgb_to_linear(y)), y, atol=5e-8)
    x = np.linspace(0.0, 1.0, 100001)
    np.testing.assert_allclose(cio.srgb_to_linear(cio.linear_to_srgb(x)), x, atol=1e-12)
    d = cio.decode_codes(np.arange(256))
    assert np.all(np.diff(d) > 0)


def test_code_round_trip():
    codes = np.arange(256, dtype=np.uint8)
    lin32 = cio.decode_codes(codes).astype(np.float32)
    np.testing.assert_array_equal(cio.encode_codes(lin32), codes)


def test_encode_is_nearest_code():
    # Brute force: the code is the one whose value lies nearest in sRGB space
    # (ties are measure zero on this grid), found by searching all 256.
    rs = np.random.default_rng(5)
    x = np.concatenate([np.linspace(0, 1, 20001), rs.uniform(0, 1, 20000)])
    y = cio.linear_to_srgb(x)
    nearest = np.argmin(np.abs(np.arange(256)[None, :] / 255.0 - y[:, None]), axis=1)
    np.testing.assert_array_equal(cio.encode_codes(x), nearest)
    special = np.array([-1.0, -0.0, 2.0, np.inf, -np.inf, np.nan])
    np.testing.assert_array_equal(cio.encode_codes(special), [0, 0, 255, 255, 0, 0])


def test_range_is_back_projected_length():
    H, W, fx, fy, cx, cy = 7, 11, 9.5, 7.25, 5.3, 2.9
    rs = np.random.default_rng(1)
    z = rs.uniform(0.5, 20.0, (H, W))
    _, r = cio.condition(zdepth=z, fx=fx, fy=fy, cx=cx, cy=cy)
    for v in range(H):
        for u in range(W):
            P = z[v, u] * np.array([(u + 0.5 - cx) / fx, (v + 0.5 - cy) / fy, 1.0])
            assert r[v, u] == pytest.approx(np.linalg.norm(P), rel=1e-14)


def test_range_inside_a_sphere():
    # A camera at the centre of a sphere of radius R sees range R everywhere:
    # z-depth is R times the z component of the unit ray.
    H, W, R = 24, 32, 3.75
    fx = fy = W / 2.0          # 90 degree horizontal field of view
    cx, cy = W / 2.0, H / 2.0
    u, v = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    d = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], -1)
    dz = d[..., 2] / np.linalg.norm(d, axis=-1)
    _, r = cio.condition(zdepth=R * dz, fx=fx, fy=fy, cx=cx, cy=cy)
    np.testing.assert_allclose(r, R, rtol=1e-14)
    # the corner pixel's ray leaves at atan(hypot(15.5, 11.5) / 16) off axis
    assert dz[0, 0] == pytest.approx(np.cos(np.arctan(np.hypot(15.5, 11.5) / 16.0)), rel=1e-14)


def test_range_principal_point_and_specials():
    z = np.array([[2.0, 0.0, np.inf, np.nan]])
    _, r = cio.condition(zdepth=z, fx=4.0, fy=4.0, cx=0.5, cy=0.5)
    assert r[0, 0] == 2.0                      # the principal point's ray is the axis
    assert r[0, 1] == 0.0 and np.isinf(r[0, 2]) and np.isnan(r[0, 3])


def test_backward_is_adjoint():
    H, W, fx, fy, cx, cy = 9, 14, 6.0, 8.0, 7.1, 4.4
    rs = np.random.default_rng(2)
    z, g = rs.normal(size=(H, W)), rs.normal(size=(H, W))
    _, r = cio.condition(zdepth=z, fx=fx, fy=fy, cx=cx, cy=cy)
    gz = cio.condition_backward(g, fx, fy, cx, cy)
    assert np.sum(g * r) == pytest.approx(np.sum(gz * z), rel=1e-12)
    # central difference of one pixel
    e = np.zeros((H, W))
    e[3, 5] = 1e-3
    rp = cio.condition(zdepth=z + e, fx=fx, fy=fy, cx=cx, cy=cy)[1]
    rm = cio.condition(zdepth=z - e, fx=fx, fy=fy, cx=cx, cy=cy)[1]
    assert (np.sum(g * rp) - np.sum(g * rm)) / 2e-3 == pytest.approx(gz[3, 5], rel=1e-9)


def test_condition_and_encode_layouts():
    rs = np.random.default_rng(3)
    img = rs.integers(0, 256, (5, 6, 4), dtype=np.uint8)
    J, _ = cio.condition(srgb=img)
    assert J.shape == (3, 5, 6)
    assert J[1, 2, 3] == cio.decode_codes(img[2, 3, 1])
    out = cio.encode(J.astype(np.float32), channels_out=4)
    np.testing.assert_array_equal(out[..., :3], img[..., :3])
    assert np.all(out[..., 3] == 255)
