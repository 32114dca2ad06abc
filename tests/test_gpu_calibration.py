"""Sim-to-real calibration through the adjoint kernels (the use the gradients
serve; the calibration workload's shape, reduced): "real" sonar polar images
and camera images are rendered with hidden parameters; starting from
perturbed ones, Adam on the logarithms of the parameters with a mean-squared
loss recovers them.  G is held fixed (it trades off against the
reflectivities); the speckle draws use the same seed on both sides."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def test_calibration_recovers_hidden_parameters():
    import torch
    import paper_2503_01074_amd as osm
    _say("calibration: 4 sonar frames (16 materials) + 4 camera frames, 400 Adam steps")
    st = W.Stream(5150, 1)
    n_mat = 16
    hidden = {"alpha": 0.12, "sigma_phi": 0.35, "sigma_sa": 0.15}
    specs = [W.SonarSpec(r_min=0.5, r_max=12.0 + 2 * k, n_range=96, n_azimuth=64, fan_h=0, fan_w=0,
                         speckle_mode=W.SPECKLE_GAMMA, gamma_k=4, gain=1.0, seed_lo=31, frame_id=k, **hidden)
             for k in range(4)]
    hits_h = [W.make_hits(st, s, 6000, n_materials=n_mat) for s in specs]
    refl_hidden = hits_h[0].refl.astype(np.float64)
    cams = [W.make_camera(st, 48, 64) for _ in range(4)]
    water_hidden = W.make_water(st)
    dev = torch.device("cuda")

    geoms = [osm.SonarGeometry.from_spec(s) for s in specs]
    hits = [osm.DeviceHits.from_host(h, dev) for h in hits_h]
    Js = [torch.as_tensor(c.J, device=dev) for c in cams]
    ds = [torch.as_tensor(c.depth, device=dev) for c in cams]

    # the "real" images
    p_true = osm.sonar_params([dict(hidden, gain=1.0, sigma_sm=0.1)], dev)
    refl_true = torch.as_tensor(refl_hidden, dtype=torch.float32, device=dev)
    w = water_hidden
    w_true = osm.water_params([(w.beta_d, w.beta_b, w.b_inf)], dev)
    tgt_sonar = [o["polar"].clone() for o in osm.render_sonar(geoms, hits, p_true, refl_true, fan=False)]
    tgt_cam = [o.clone() for o in osm.uw_form(Js, ds, w_true)]

    # the model: a plan over the same frames; parameters start perturbed
    rng = np.random.default_rng(5151)
    start = lambda x: np.asarray(x, np.float64) * rng.uniform(0.5, 1.5, np.shape(x))
    theta = {
        "sonar": torch.tensor(np.log(start([hidden["alpha"], hidden["sigma_phi"], hidden["sigma_sa"]])),
                              device=dev, requires_grad=True),
        "refl": torch.tensor(np.log(start(refl_hidden)), device=dev, requires_grad=True),
        "water": torch.tensor(np.log(start(np.concatenate([w.beta_d, w.beta_b, w.b_inf]).astype(np.float64))),
                              device=dev, requires_grad=True),
    }
    params = osm.sonar_params([dict(hidden, gain=1.0, sigma_sm=0.1)], dev)
    refl = torch.empty(n_mat, dtype=torch.float32, device=dev)
    water = osm.water_params([(w.beta_d, w.beta_b, w.b_inf)], dev)
    plan = osm.Plan(list(zip(geoms, hits)), [(J, d, 0) for J, d in zip(Js, ds)], sonar_params=params, refl=refl,
                    water=water, backward=True, fan=False)
    opt = torch.optim.Adam(list(theta.values()), lr=0.03)
    n_s = sum(t.numel() for t in tgt_sonar)
    n_c = sum(t.numel() for t in tgt_cam)
    scale_s = 1.0 / float(sum((t.double() ** 2).sum() for t in tgt_sonar))
    scale_c = 1.0 / float(sum((t.double() ** 2).sum() for t in tgt_cam))
    first = None
    for step in range(400):
        with torch.no_grad():
            ps = theta["sonar"].exp()
            params[0, 0], params[0, 2], params[0, 3] = ps[0], ps[1], ps[2]
            refl.copy_(theta["refl"].exp())
            water[0, :9] = theta["water"].exp()
        plan.forward()
        loss = 0.0
        for o, t in zip(plan.sonar_out, tgt_sonar):
            r = o["polar"] - t
            o["grad_polar"].copy_(2.0 * scale_s * r)
            loss += scale_s * float((r.double() ** 2).sum())
        for o, t in zip(plan.camera_out, tgt_cam):
            r = o["out"] - t
            o["grad_out"].copy_(2.0 * scale_c * r)
            loss += scale_c * float((r.double() ** 2).sum())
        plan.backward()
        if first is None:
            first = loss
        with torch.no_grad():
            g = plan.grad_sonar_params[0]
            ps = theta["sonar"].exp()
            theta["sonar"].grad = torch.stack([g[0], g[2], g[3]]).double() * ps
            theta["refl"].grad = plan.grad_refl.double() * theta["refl"].exp()
            theta["water"].grad = plan.grad_water[0, :9].double() * theta["water"].exp()
        opt.step()
    torch.cuda.synchronize()
    ts = theta["sonar"].detach().exp()
    got = {"alpha": float(ts[0]), "sigma_phi": float(ts[1]),
           "sigma_sa": float(ts[2])}
    _say("loss %.3e -> %.3e; sonar %s" % (first, loss, got))
    assert loss < 1e-5 * first
    for k, v in hidden.items():
        assert abs(got[k] - v) <= 0.02 * v, (k, got[k], v)
    refl_got = theta["refl"].detach().exp().cpu().numpy()
    assert np.all(np.abs(refl_got - refl_hidden) <= 0.02 * refl_hidden), refl_got / refl_hidden
    water_got = theta["water"].detach().exp().cpu().numpy()
    water_ref = np.concatenate([w.beta_d, w.beta_b, w.b_inf]).astype(np.float64)
    assert np.all(np.abs(water_got - water_ref) <= 0.02 * water_ref), water_got / water_ref
    plan.close()
