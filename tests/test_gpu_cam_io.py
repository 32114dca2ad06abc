"""GPU parity of the camera input conditioning and output encoding (8-bit sRGB
around Eq. (1) of Sec. III-A.1, z-depth to line-of-sight range) against the
FP64 oracle.

Bars: decoding is exact (the library's table holds the double-precision value
rounded to the nearest float); encoding is bit-exact on any float input,
thresholds included; the range and its adjoint are within 1e-6 relative (a
handful of float roundings on a scale near 1).
"""
import numpy as np
import pytest
import torch

from oracle import camera_io as cio

pytestmark = pytest.mark.gpu

RTOL = 1e-6


def _osm():
    import paper_2503_01074_amd as osm
    return osm


def _intr(H, W, k=0):
    return (0.9 * W + 1.3 * k, 0.85 * W + 0.7 * k, 0.5 * W + 0.37, 0.5 * H - 0.21 * k)


def _depth(rs, H, W, specials=True):
    z = rs.uniform(0.2, 50.0, (H, W)).astype(np.float32)
    if specials and H * W >= 4:
        flat = z.reshape(-1)
        flat[[0, H * W // 3, H * W // 2, H * W - 1]] = [0.0, np.inf, np.nan, 1e-30]
    return z


@pytest.mark.parametrize("ch", [3, 4])
def test_decode_every_code(ch):
    osm = _osm()
    rs = np.random.default_rng(ch)
    img = np.stack([np.arange(256, dtype=np.uint8).reshape(16, 16),
                    rs.permutation(256).astype(np.uint8).reshape(16, 16),
                    (255 - np.arange(256)).astype(np.uint8).reshape(16, 16)]
                   + ([rs.integers(0, 256, (16, 16), dtype=np.uint8)] if ch == 4 else []), -1)
    (J,), (r,) = osm.cam_condition([torch.as_tensor(img).cuda()], [None], [_intr(16, 16)])
    assert r is None
    ref = cio.condition(srgb=img)[0].astype(np.float32)
    np.testing.assert_array_equal(J.cpu().numpy(), ref)


@pytest.mark.parametrize("H,W,ch", [(1, 1, 3), (3, 5, 4), (7, 13, 3), (480, 640, 4), (37, 1001, 3),
                                    (1080, 1920, 4), (2, 65535, 3)])
def test_condition_parity(H, W, ch):
    osm = _osm()
    rs = np.random.default_rng(H * 7 + W)
    img = rs.integers(0, 256, (H, W, ch), dtype=np.uint8)
    z = _depth(rs, H, W)
    intr = _intr(H, W)
    (J,), (r,) = osm.cam_condition([torch.as_tensor(img).cuda()], [torch.as_tensor(z).cuda()], [intr])
    Jr, rr = cio.condition(srgb=img, zdepth=z, fx=intr[0], fy=intr[1], cx=intr[2], cy=intr[3])
    np.testing.assert_array_equal(J.cpu().numpy(), Jr.astype(np.float32))
    np.testing.assert_allclose(r.cpu().numpy(), rr, rtol=RTOL, atol=0, equal_nan=True)


def _threshold_inputs():
    """Floats at and next to every code boundary, found with the oracle alone."""
    out = []
    up, down = np.float32(np.inf), np.float32(-np.inf)
    for j in range(1, 256):
        x = np.float32(cio.srgb_to_linear((j - 0.5) / 255.0))
        while cio.encode_codes(x) < j:
            x = np.nextafter(x, up)
        while cio.encode_codes(np.nextafter(x, down)) >= j:
            x = np.nextafter(x, down)
        out += [np.nextafter(x, down), x, np.nextafter(x, up)]
    return np.array(out, dtype=np.float32)


@pytest.mark.parametrize("H,W,ch", [(1, 1, 3), (5, 7, 4), (27, 29, 3), (480, 640, 3), (1080, 1920, 4)])
def test_encode_bit_exact(H, W, ch):
    osm = _osm()
    rs = np.random.default_rng(H + W + ch)
    I = rs.uniform(-0.1, 1.1, (3, H, W)).astype(np.float32)
    flat = I.reshape(-1)
    t = _threshold_inputs()
    n = min(t.size, flat.size)
    flat[:n] = t[:n]
    spec = np.array([np.nan, np.inf, -np.inf, -0.0, 0.0, 1.0, 2.0], dtype=np.float32)
    flat[-min(spec.size, flat.size):] = spec[:min(spec.size, flat.size)]
    (o,) = osm.cam_encode([torch.as_tensor(I).cuda()], channels_out=ch)
    np.testing.assert_array_equal(o.cpu().numpy(), cio.encode(I, channels_out=ch))


def test_encode_every_threshold():
    osm = _osm()
    t = _threshold_inputs()
    I = np.stack([t, t[::-1], np.roll(t, 7)]).reshape(3, 1, -1)
    (o,) = osm.cam_encode([torch.as_tensor(I).cuda()])
    np.testing.assert_array_equal(o.cpu().numpy(), cio.encode(I))


@pytest.mark.parametrize("H,W", [(1, 3), (9, 14), (480, 640), (1080, 1920)])
def test_backward_parity(H, W):
    osm = _osm()
    rs = np.random.default_rng(W)
    g = rs.normal(size=(H, W)).astype(np.float32)
    intr = _intr(H, W, 1)
    (gz,) = osm.cam_condition_backward([torch.as_tensor(g).cuda()], [intr])
    np.testing.assert_allclose(gz.cpu().numpy(), cio.condition_backward(g, *intr), rtol=RTOL, atol=0)


def test_batch_equals_single_and_oracle():
    """20 frames (two launches of at most 16) of mixed sizes, channel counts and
    halves: one batched call equals the per-frame calls bit for bit."""
    osm = _osm()
    rs = np.random.default_rng(11)
    shapes = [(int(rs.integers(1, 90)), int(rs.integers(1, 130))) for _ in range(20)]
    shapes[4] = (0, 17)
    imgs, zs, intrs = [], [], []
    for k, (H, W) in enumerate(shapes):
        ch = 3 + (k % 2)
        imgs.append(None if k % 5 == 2 else torch.as_tensor(rs.integers(0, 256, (H, W, ch), dtype=np.uint8)).cuda())
        zs.append(None if k % 7 == 3 else torch.as_tensor(_depth(rs, H, W)).cuda())
        intrs.append(_intr(H, W, k))
    Jb, rb = osm.cam_condition(imgs, zs, intrs)
    for k in range(20):
        Js, rsg = osm.cam_condition([imgs[k]], [zs[k]], [intrs[k]])
        if imgs[k] is not None:
            assert torch.equal(Jb[k], Js[0])
            np.testing.assert_array_equal(Jb[k].cpu().numpy(),
                                          cio.condition(srgb=imgs[k].cpu().numpy())[0].astype(np.float32))
        if zs[k] is not None:
            assert torch.equal(torch.nan_to_num(rb[k]), torch.nan_to_num(rsg[0]))
            np.testing.assert_allclose(rb[k].cpu().numpy(), cio.condition(
                zdepth=zs[k].cpu().numpy(), fx=intrs[k][0], fy=intrs[k][1], cx=intrs[k][2], cy=intrs[k][3])[1],
                rtol=RTOL, atol=0, equal_nan=True)
    gs = [torch.as_tensor(rs.normal(size=s).astype(np.float32)).cuda() for s in shapes]
    gb = osm.cam_condition_backward(gs, intrs)
    for k in range(20):
        assert torch.equal(gb[k], osm.cam_condition_backward([gs[k]], [intrs[k]])[0])
    Is = [torch.as_tensor(rs.uniform(-0.05, 1.05, (3,) + s).astype(np.float32)).cuda() for s in shapes]
    ob = osm.cam_encode(Is, channels_out=4)
    for k in range(20):
        np.testing.assert_array_equal(ob[k].cpu().numpy(), cio.encode(Is[k].cpu().numpy(), channels_out=4))


@pytest.mark.parametrize("ch", [3, 4])
def test_round_trip_full_frame(ch):
    """Decoding then encoding returns every input byte (alpha becomes 255)."""
    osm = _osm()
    rs = np.random.default_rng(ch + 40)
    img = torch.as_tensor(rs.integers(0, 256, (1080, 1920, ch), dtype=np.uint8)).cuda()
    (J,), _ = osm.cam_condition([img], [None], [_intr(1080, 1920)])
    (o,) = osm.cam_encode([J], channels_out=ch)
    assert torch.equal(o[..., :3], img[..., :3])
    if ch == 4:
        assert bool((o[..., 3] == 255).all())


def test_empty_calls():
    osm = _osm()
    assert osm.cam_condition([], [], []) == ([], [])
    z = torch.empty(0, 5, device="cuda")
    (J,), (r,) = osm.cam_condition([None], [z], [(1.0, 1.0, 0.0, 0.0)])
    assert J is None and r.shape == (0, 5)
    assert osm.cam_encode([torch.empty(3, 4, 0, device="cuda")])[0].shape == (4, 0, 3)
