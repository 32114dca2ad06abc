"""GPU parity of a backward plan's transposed fan operators (built once at
plan creation from the fan kernel's stencils; the backward gathers each polar
bin's fan gradient through them), against the FP64 oracle, on odd and
degenerate grids, mixed frames, growing gradient magnitudes and a NaN.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import SonarConfig
import workloads as W
from _tol import assert_grad_cond

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _plan_backward(frames, refl, gpol, gfan, rows=None, graph=False):
    """Plan forward + backward; gradients as float64 numpy arrays."""
    import torch
    import paper_2503_01074_amd as osm
    rows = rows or [0] * len(frames)
    geoms = [osm.SonarGeometry.from_spec(f.spec, param_row=r) for f, r in zip(frames, rows)]
    hits = [osm.DeviceHits.from_host(f.hits) for f in frames]
    row_spec = {r: f.spec for f, r in zip(frames, rows)}
    params = osm.sonar_params([osm.sonar_params_from_spec(row_spec[r]) for r in range(max(rows) + 1)])
    plan = osm.Plan(list(zip(geoms, hits)), sonar_params=params, refl=torch.as_tensor(refl).cuda(),
                    backward=True, graph=graph)
    assert plan.shape()["bwd_block_bins"] in (256, 512, 1024)
    for o, gp, gf in zip(plan.sonar_out, gpol, gfan):
        if "grad_polar" in o:
            o["grad_polar"].copy_(torch.as_tensor(gp))
        if "grad_fan" in o:
            o["grad_fan"].copy_(torch.as_tensor(gf) if gf is not None else torch.zeros_like(o["grad_fan"]))
    plan.forward()
    plan.backward()
    torch.cuda.synchronize()
    g_refl = plan.grad_refl.cpu().numpy().astype(np.float64)
    g_par = plan.grad_sonar_params.cpu().numpy().astype(np.float64)
    plan.close()
    return g_refl, g_par


def _oracle(frames, refl, gpol, gfan, rows=None):
    rows = rows or [0] * len(frames)
    n_rows = max(rows) + 1
    o_refl, c_refl = np.zeros(refl.shape[0]), np.zeros(refl.shape[0])
    o_par, c_par = np.zeros((n_rows, 5)), np.zeros((n_rows, 5))
    for f, r, gp, gf in zip(frames, rows, gpol, gfan):
        a, b, _, ca, cb = oracle.sonar_backward(SonarConfig.from_spec(f.spec), f.hits, refl, gp, gf, with_abs=True)
        o_refl += a
        c_refl += ca
        o_par[r] += b
        c_par[r] += cb
    return o_refl, o_par, c_refl, c_par


def _frame(st, Nr, Np, H, Wd, n, mode=W.SPECKLE_PAPER, frame_id=0, r_max=13.0):
    spec = W.SonarSpec(r_min=0.7, r_max=r_max, n_range=Nr, n_azimuth=Np, fan_h=H, fan_w=Wd, speckle_mode=mode,
                       gamma_k=3, sigma_sm=0.12, sigma_sa=0.15, sigma_phi=0.3, alpha=0.09, gain=1.2, seed_lo=3,
                       frame_id=frame_id)
    return W.SonarFrame(spec, W.make_hits(st, spec, n, n_materials=5))


@pytest.mark.parametrize("shape", [(37, 29, 41, 83), (1, 17, 8, 16), (23, 1, 9, 9), (60, 40, 33, 64),
                                   (300, 700, 64, 128), (24, 1, 10, 20), (2, 2, 12, 30)])
@pytest.mark.parametrize("graph", [False, True])
def test_plan_fan_transpose_vs_oracle(shape, graph):
    """Odd fan width (a centre column that is its own mirror: plain operator
    rows), even widths (mirrored rows) with an odd azimuth count (a middle
    column that is its own mirror), one range row, one or two azimuth columns,
    more bins than fan pixels."""
    Nr, Np, H, Wd = shape
    _say("plan fan transpose %s graph %s" % (shape, graph))
    st = W.Stream(8100, Nr + Np)
    frames = [_frame(st, Nr, Np, H, Wd, 3000)]
    refl = frames[0].hits.refl
    gpol = [W.loss_weights((8101, 1), (Nr, Np))]
    gfan = [W.loss_weights((8101, 2), (H, Wd))]
    g_refl, g_par = _plan_backward(frames, refl, gpol, gfan, graph=graph)
    o_refl, o_par, c_refl, c_par = _oracle(frames, refl, gpol, gfan)
    assert_grad_cond(g_refl, o_refl, c_refl, what="refl")
    assert_grad_cond(g_par[0, :5], o_par[0], c_par[0], what="params")
    assert np.all(g_par[0, 5:] == 0)


def test_plan_fan_transpose_mixed_frames_and_rows():
    """Frames with a fan, without one, and with a fan whose gradient is zero,
    on three parameter rows and all speckle modes, in one plan."""
    _say("plan fan transpose: mixed frames on three rows")
    st = W.Stream(8200, 1)
    frames = [
        _frame(st, 48, 40, 40, 72, 3000, W.SPECKLE_GAMMA, 0),
        _frame(st, 30, 24, 0, 0, 1500, W.SPECKLE_PAPER, 1),
        _frame(st, 61, 53, 51, 91, 4000, W.SPECKLE_OFF, 2, r_max=9.0),
        _frame(st, 20, 300, 64, 129, 2500, W.SPECKLE_GAMMA, 3),
    ]
    rows = [0, 1, 2, 0]
    refl = frames[0].hits.refl
    for f in frames:
        f.hits.refl = refl
    gpol = [W.loss_weights((8201, k), (f.spec.n_range, f.spec.n_azimuth)) for k, f in enumerate(frames)]
    gfan = [W.loss_weights((8202, k), (f.spec.fan_h, f.spec.fan_w)) if f.spec.fan_h else None
            for k, f in enumerate(frames)]
    gfan[2] = np.zeros((frames[2].spec.fan_h, frames[2].spec.fan_w), np.float32)
    g_refl, g_par = _plan_backward(frames, refl, gpol, gfan, rows)
    o_refl, o_par, c_refl, c_par = _oracle(frames, refl, gpol, gfan, rows)
    assert_grad_cond(g_refl, o_refl, c_refl, what="refl")
    for r in range(3):
        assert_grad_cond(g_par[r, :5], o_par[r], c_par[r], what="row %d" % r)


def test_plan_fan_transpose_growing_magnitudes():
    """A tall fan whose gradient magnitude spans nine decades down the image:
    each bin's FP64 sum keeps the small terms."""
    _say("plan fan transpose: 1400 x 2800 fan, growing gradient magnitude")
    st = W.Stream(8300, 1)
    spec = W.SonarSpec(r_min=0.5, r_max=30.0, n_range=300, n_azimuth=200, fan_h=1400, fan_w=2800,
                       alpha=0.08, gain=1.1, sigma_phi=0.3, sigma_sa=0.15, speckle_mode=W.SPECKLE_GAMMA,
                       seed_lo=5, frame_id=1)
    frames = [W.SonarFrame(spec, W.make_hits(st, spec, 20000, n_materials=16))]
    refl = frames[0].hits.refl
    ramp = np.logspace(-6, 3, spec.fan_h)[:, None]
    gfan = [(W.loss_weights((8301, 2), (spec.fan_h, spec.fan_w)) * ramp).astype(np.float32)]
    gpol = [W.loss_weights((8301, 3), (spec.n_range, spec.n_azimuth))]
    g_refl, g_par = _plan_backward(frames, refl, gpol, gfan)
    o_refl, o_par, c_refl, c_par = _oracle(frames, refl, gpol, gfan)
    assert_grad_cond(g_refl, o_refl, c_refl, what="refl")
    assert_grad_cond(g_par[0, :5], o_par[0], c_par[0], what="params")


def test_plan_fan_transpose_nan_gradient():
    """A NaN in the fan gradient reaches the same outputs as in the oracle."""
    _say("plan fan transpose: a NaN in the fan gradient")
    st = W.Stream(8400, 1)
    frames = [_frame(st, 48, 40, 40, 72, 3000, W.SPECKLE_GAMMA)]
    refl = frames[0].hits.refl
    gpol = [W.loss_weights((8401, 1), (48, 40))]
    gfan = [W.loss_weights((8401, 2), (40, 72)).copy()]
    gfan[0][20, 30] = np.nan
    g_refl, g_par = _plan_backward(frames, refl, gpol, gfan)
    o_refl, o_par, _, _ = _oracle(frames, refl, gpol, gfan)
    np.testing.assert_array_equal(np.isnan(g_refl), np.isnan(o_refl))
    np.testing.assert_array_equal(np.isnan(g_par[0, :5]), np.isnan(o_par[0]))
    assert np.isnan(o_par).any()


@pytest.mark.parametrize("n_frames,n_bins,block_bins,mixed,odd_az", [(3, 1024, 512, True, False),
                                                                      (4, 2048, 1024, True, False),
                                                                      (3, 1024, 512, False, False),
                                                                      (4, 2048, 1024, False, False),
                                                                      (3, 1024, 512, True, True),
                                                                      (4, 2048, 1024, True, True)])
def test_plan_fan_transpose_large_batches(n_frames, n_bins, block_bins, mixed, odd_az):
    """Batches of many polar bins take two or four rows per thread (the
    workgroup's wave spans then cover 128 or 256 rows and several chunks);
    even and odd fan widths alternate (mirrored and plain operator rows in one
    launch), or all widths are odd (plain rows only: the kernel without
    mirror outputs); with odd azimuth counts a thread's mirrored rows wrap
    from one range row to the next around a middle column that is its own
    mirror."""
    import paper_2503_01074_amd as osm
    _say("plan fan transpose: %d frames of %d x %d bins, mixed layouts %s, odd azimuth counts %s"
         % (n_frames, n_bins, n_bins, mixed, odd_az))
    st = W.Stream(8500 + n_bins, n_frames)
    frames = []
    for k in range(n_frames):
        spec = W.SonarSpec(r_min=0.5, r_max=12.0 + k, n_range=n_bins, n_azimuth=n_bins + 8 * k + (1 if odd_az else 0), fan_h=150 + 10 * k,
                           fan_w=300 + 21 * k if mixed else 301 + 20 * k, alpha=0.09, gain=1.2, sigma_phi=0.3, sigma_sa=0.15, sigma_sm=0.12,
                           speckle_mode=(W.SPECKLE_GAMMA, W.SPECKLE_PAPER, W.SPECKLE_OFF)[k % 3], gamma_k=3,
                           seed_lo=3, frame_id=k)
        frames.append(W.SonarFrame(spec, W.make_hits(st, spec, 3000, n_materials=5)))
    refl = frames[0].hits.refl
    for f in frames:
        f.hits.refl = refl
    gpol = [W.loss_weights((8501, k), (f.spec.n_range, f.spec.n_azimuth)) for k, f in enumerate(frames)]
    gfan = [W.loss_weights((8502, k), (f.spec.fan_h, f.spec.fan_w)) for k, f in enumerate(frames)]
    import torch
    geoms = [osm.SonarGeometry.from_spec(f.spec) for f in frames]
    hits = [osm.DeviceHits.from_host(f.hits) for f in frames]
    params = osm.sonar_params([osm.sonar_params_from_spec(frames[0].spec)])
    plan = osm.Plan(list(zip(geoms, hits)), sonar_params=params, refl=torch.as_tensor(refl).cuda(), backward=True)
    assert plan.shape()["bwd_block_bins"] == block_bins
    for o, gp, gf in zip(plan.sonar_out, gpol, gfan):
        o["grad_polar"].copy_(torch.as_tensor(gp))
        o["grad_fan"].copy_(torch.as_tensor(gf))
    plan.forward()
    plan.backward()
    torch.cuda.synchronize()
    g_refl = plan.grad_refl.cpu().numpy().astype(np.float64)
    g_par = plan.grad_sonar_params.cpu().numpy().astype(np.float64)
    plan.close()
    o_refl, o_par, c_refl, c_par = _oracle(frames, refl, gpol, gfan)
    assert_grad_cond(g_refl, o_refl, c_refl, what="refl")
    assert_grad_cond(g_par[0, :5], o_par[0], c_par[0], what="params")
