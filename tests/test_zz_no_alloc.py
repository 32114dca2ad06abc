"""The allocation-free sonar forward (oceansim_sonar_render_noalloc), called
through the C ABI, against the workspace entry point oceansim_sonar_render on
the same inputs: two calls in a row, the second with a smaller input (the
scratch keeps the first call's contents), a two-frame batch (the frame table
in the scratch), and the rejection of frames that need more scratch than the
library holds.  Bins bit-exact, images to 1e-5 relative."""
import sys

import numpy as np
import pytest

import workloads as W
from _tol import assert_image_close

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _frame_bufs(osm, torch, frame):
    g = osm.SonarGeometry.from_spec(frame.spec)
    h = osm.DeviceHits.from_host(frame.hits)
    o = {"polar": torch.empty(g.n_range, g.n_azimuth, device="cuda"),
         "fan": torch.empty(g.fan_h, g.fan_w, device="cuda") if g.fan_h else None,
         "bins": torch.empty(h.n, dtype=torch.int32, device="cuda")}
    return g, h, o


def _structs(api, frames_bufs):
    return [api._sonar_struct(g, h, o["polar"], o["fan"], o["bins"]) for g, h, o in frames_bufs]


def _both(osm, torch, frames, refl):
    """Outputs of the allocation-free call and of the workspace call."""
    from paper_2503_01074_amd import _lib, api
    params = osm.sonar_params([osm.sonar_params_from_spec(frames[0].spec)])
    refl_d = torch.as_tensor(refl).cuda()
    a = [_frame_bufs(osm, torch, f) for f in frames]
    b = [_frame_bufs(osm, torch, f) for f in frames]
    sa = (_lib.SonarFrame * len(frames))(*_structs(api, a))
    sb = (_lib.SonarFrame * len(frames))(*_structs(api, b))
    stream = torch.cuda.current_stream().cuda_stream
    n_mat = int(refl_d.numel())
    _lib.oceansim_sonar_render_noalloc(sa, params.data_ptr(), 1, refl_d.data_ptr(), n_mat, stream)
    need = _lib.oceansim_sonar_workspace_size(sb, n_mat, False)
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
    _lib.oceansim_sonar_render(sb, params.data_ptr(), 1, refl_d.data_ptr(), n_mat, ws.data_ptr(), ws.numel(),
                               stream)
    torch.cuda.synchronize()
    return a, b


def _compare(a, b, what):
    for k, ((_, _, oa), (_, _, ob)) in enumerate(zip(a, b)):
        assert torch_equal(oa["bins"], ob["bins"]), "%s bins %d" % (what, k)
        assert_image_close(oa["polar"].cpu().numpy(), ob["polar"].cpu().numpy(), "%s polar %d" % (what, k))
        if oa["fan"] is not None:
            assert_image_close(oa["fan"].cpu().numpy(), ob["fan"].cpu().numpy(), "%s fan %d" % (what, k))


def torch_equal(x, y):
    import torch
    return bool(torch.equal(x, y))


def test_noalloc_matches_workspace_call_twice():
    import torch
    import paper_2503_01074_amd as osm
    _say("noalloc: the real-time frame, then a smaller frame")
    big = W.sonar_c2()
    refl_big = big[0].hits.refl
    a, b = _both(osm, torch, big, refl_big)
    _compare(a, b, "real-time frame")
    st = W.Stream(7700, 1)
    spec = W.SonarSpec(r_min=0.5, r_max=12.0, n_range=70, n_azimuth=45, fan_h=48, fan_w=90,
                       speckle_mode=W.SPECKLE_PAPER, seed_lo=5, frame_id=3)
    small = [W.SonarFrame(spec, W.make_hits(st, spec, 3000, n_materials=8))]
    a, b = _both(osm, torch, small, small[0].hits.refl)
    _compare(a, b, "small frame")


def test_noalloc_batch():
    import torch
    import paper_2503_01074_amd as osm
    _say("noalloc: a two-frame batch (frame table in the scratch)")
    st = W.Stream(7701, 1)
    specs = [W.SonarSpec(r_min=0.5, r_max=15.0, n_range=200, n_azimuth=128, fan_h=100, fan_w=200, frame_id=0),
             W.SonarSpec(r_min=1.0, r_max=30.0, n_range=97, n_azimuth=301, frame_id=1)]
    frames = [W.SonarFrame(s, W.make_hits(st, s, n, n_materials=16)) for s, n in zip(specs, [20000, 7000])]
    refl = frames[0].hits.refl
    for f in frames:
        f.hits.refl = refl
    a, b = _both(osm, torch, frames, refl)
    _compare(a, b, "batch")


def test_noalloc_rejects_frames_beyond_the_scratch():
    import torch
    import paper_2503_01074_amd as osm
    from paper_2503_01074_amd import _lib, api
    _say("noalloc: a frame that needs more scratch than the library holds is rejected")
    n = 9 << 20
    g = osm.SonarGeometry(r_min=0.5, r_max=50.0, n_range=2048, n_azimuth=2048, fov_az=2.2689, fov_el=0.349)
    h = osm.DeviceHits(*(torch.zeros(n, device="cuda") for _ in range(6)),
                       torch.full((n,), -1, dtype=torch.int32, device="cuda"))
    polar = torch.empty(2048, 2048, device="cuda")
    s = (_lib.SonarFrame * 1)(api._sonar_struct(g, h, polar))
    need = _lib.oceansim_sonar_workspace_size(s, 64, False)
    assert need > (64 << 20)
    params = osm.sonar_params([{"alpha": 0.1, "gain": 1.0, "sigma_phi": 0.25, "sigma_sa": 0.1, "sigma_sm": 0.1}])
    refl = torch.ones(64, device="cuda")
    with pytest.raises(_lib.OceansimError) as ei:
        _lib.oceansim_sonar_render_noalloc(s, params.data_ptr(), 1, refl.data_ptr(), 64,
                                           torch.cuda.current_stream().cuda_stream)
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
