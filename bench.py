"""Throughput of the OceanSim sonar + underwater-camera image-formation path on
one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-batched] [--no-cpu]

A step is one forward + backward pass of the whole path over the real-time
workload: one sonar frame of 1024 beams x 128 rays = 131072 returns binned on a
1024 x 1024 polar grid with gamma speckle and a 1024 x 2048 fan, plus Eq. (1)
on one 1920 x 1080 RGB frame, and the adjoints of both with respect to the
reflectivities, the sonar parameters and the water parameters.  Inputs are
seeded synthetic data already resident in device memory.

Prints one JSON line.  ``value`` is sonar returns per second through the full
step; the line also carries forward-only and batched throughputs, the roofline
of the dominant kernel (timed with HIP events on the stream it runs on) and
the FP64 oracle timed on the host's cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-range-norm", action="store_true",
                    help="skip the real-time step with the range-wise normalisation (profiler runs)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 64 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--only", choices=["c3", "c4", "c5"], default=None,
                    help="only build and run one batched leg (for profiler runs); prints no JSON line")
    ap.add_argument("--c5-frames", type=int, default=64,
                    help="sonar and camera frames of the calibration-scale leg")
    return ap.parse_args()


def copy_calibration(torch, dev):
    """A plain copy of known size: 64 MiB read, 64 MiB written per launch,
    used to scale the HBM byte counters of a profiler run."""
    n = 64 << 20
    a = torch.ones(n // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy calibration: 5 launches of a %d-byte device copy" % n)


def source_digest():
    """SHA-256 over the library sources: HBM traffic measured by a profiler
    run is used only while the kernels are those that were profiled."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2503_01074_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` (read + written) from the rocprofv3
    counter summary in profiles/, if it was taken on the current sources."""
    path = os.path.join(ROOT, "profiles", "c2_step_hbm_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else int(k["fetch_bytes"] + k["write_bytes"])


def copy_rate(torch, dev):
    """Bandwidth of a plain 64 MiB device-to-device copy (read + written
    bytes over the event-timed duration): what the memory system delivers to
    a trivial streaming kernel, for context beside the 8 TB/s peak."""
    a = torch.ones((64 << 20) // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    s = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(20):
        b.copy_(a)
    e1.record(s)
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / 20
    return round(2 * a.numel() * 4 / t / 1e9, 1)


class RealTimeStep:
    """Device buffers and prebuilt descriptors of the real-time workload."""

    def __init__(self, dev, range_norm=True):
        import torch
        import numpy as np
        import paper_2503_01074_amd as osm
        from paper_2503_01074_amd import _lib
        from paper_2503_01074_amd.api import _sonar_struct, _uw_struct
        import workloads as W

        self.torch, self.lib = torch, _lib
        frame = W.sonar_c2()[0]
        cams, waters = W.camera_c2()
        self.frame, self.cam, self.water_host = frame, cams[0], waters[0]
        spec, hits = frame.spec, frame.hits
        self.n_returns = hits.n
        self.geom = osm.SonarGeometry.from_spec(spec)
        self.hits = osm.DeviceHits.from_host(hits, dev)
        self.params = osm.sonar_params([osm.sonar_params_from_spec(spec)], dev)
        self.refl = torch.as_tensor(hits.refl, device=dev)
        self.n_mat = int(self.refl.numel())
        self.polar = torch.empty(spec.n_range, spec.n_azimuth, device=dev)
        self.fan = torch.empty(spec.fan_h, spec.fan_w, device=dev)
        self.gpol = torch.as_tensor(W.loss_weights((101, 1), (spec.n_range, spec.n_azimuth)), device=dev)
        self.gfan = torch.as_tensor(W.loss_weights((101, 2), (spec.fan_h, spec.fan_w)), device=dev)
        # training steps save the fan stencils in the forward pass for the backward pass
        self.stencil = osm.api.fan_stencil_buffer(self.geom, dev)
        self.fwd = _sonar_struct(self.geom, self.hits, self.polar, self.fan)
        self.fwd_train = _sonar_struct(self.geom, self.hits, self.polar, self.fan, stencil=self.stencil)
        self.bwd = _sonar_struct(self.geom, self.hits, grad_polar=self.gpol, grad_fan=self.gfan,
                                 stencil=self.stencil)
        self.ws_f = torch.empty(_lib.oceansim_sonar_workspace_size(self.fwd, self.n_mat, False),
                                dtype=torch.uint8, device=dev)
        self.ws_b = torch.empty(_lib.oceansim_sonar_workspace_size(self.bwd, self.n_mat, True),
                                dtype=torch.uint8, device=dev)
        self.g_refl = torch.empty(self.n_mat, device=dev)
        self.g_par = torch.empty(1, _lib.SONAR_GRAD_WIDTH, device=dev)

        H, Wd = self.cam.depth.shape
        self.npix = H * Wd
        self.J = torch.as_tensor(self.cam.J, device=dev)
        self.d = torch.as_tensor(self.cam.depth, device=dev)
        self.img = torch.empty_like(self.J)
        w = self.water_host
        self.water = osm.water_params([(w.beta_d, w.beta_b, w.b_inf)], dev)
        self.gimg = torch.as_tensor(W.loss_weights((101, 3), self.cam.J.shape), device=dev)
        self.gJ = torch.empty_like(self.J)
        self.gd = torch.empty_like(self.d)
        self.uwf = _uw_struct(self.J, self.d, self.img)
        self.uwb = _uw_struct(self.J, self.d, None, 0, self.gimg, self.gJ, self.gd)
        self.ws_u = torch.empty(max(256, _lib.oceansim_uw_workspace_size(self.uwb, True)),
                                dtype=torch.uint8, device=dev)
        self.g_w = torch.empty(1, _lib.WATER_GRAD_WIDTH, device=dev)
        self.stream = torch.cuda.current_stream(dev).cuda_stream
        self.P = lambda t: t.data_ptr()
        # the same step as a plan: frame tables uploaded once, forward and
        # backward each replayed from a captured HIP graph
        self.plans = {}
        for name, graph in (("plan", False), ("graph", True)):
            pl = osm.Plan([(self.geom, self.hits)], [(self.J, self.d, 0)], sonar_params=self.params,
                          refl=self.refl, water=self.water, backward=True, graph=graph, autotune=True,
                          image_grads=True)
            pl.sonar_out[0]["grad_polar"].copy_(self.gpol)
            pl.sonar_out[0]["grad_fan"].copy_(self.gfan)
            pl.camera_out[0]["grad_out"].copy_(self.gimg)
            self.plans[name] = pl
        if not range_norm:
            return
        # the same step with the range-wise normalisation after the gain
        import dataclasses
        pl = osm.Plan([(dataclasses.replace(self.geom, range_norm=1), self.hits)], [(self.J, self.d, 0)],
                      sonar_params=self.params, refl=self.refl, water=self.water, backward=True, autotune=True,
                      image_grads=True)
        pl.sonar_out[0]["grad_polar"].copy_(self.gpol)
        pl.sonar_out[0]["grad_fan"].copy_(self.gfan)
        pl.camera_out[0]["grad_out"].copy_(self.gimg)
        self.plans["norm"] = pl

    def sonar_forward(self, train=False):
        L, P = self.lib, self.P
        L.oceansim_sonar_render(self.fwd_train if train else self.fwd, P(self.params), 1, P(self.refl),
                                self.n_mat, P(self.ws_f), self.ws_f.numel(), self.stream)

    def sonar_backward(self):
        L, P = self.lib, self.P
        L.oceansim_sonar_render_backward(self.bwd, P(self.params), 1, P(self.refl), self.n_mat,
                                         P(self.g_refl), P(self.g_par), P(self.ws_b), self.ws_b.numel(),
                                         self.stream)

    def uw_forward(self):
        L, P = self.lib, self.P
        L.oceansim_uw_form(self.uwf, P(self.water), 1, 0, 0, self.stream)

    def uw_backward(self):
        L, P = self.lib, self.P
        L.oceansim_uw_form_backward(self.uwb, P(self.water), 1, P(self.g_w), P(self.ws_u), self.ws_u.numel(),
                                    self.stream)

    def forward(self):
        self.sonar_forward()
        self.uw_forward()

    def step(self):
        self.sonar_forward(train=True)
        self.uw_forward()
        self.sonar_backward()
        self.uw_backward()

    def plan_forward(self, name):
        self.lib.oceansim_plan_forward(self.plans[name].handle, self.stream)

    def plan_step(self, name):
        h = self.plans[name].handle
        self.lib.oceansim_plan_forward(h, self.stream)
        self.lib.oceansim_plan_backward(h, self.stream)

    def algorithmic_bytes(self):
        """Bytes each kernel must move per launch by the per-unit figures of
        the method (inputs read once, outputs written once): returns 28 B,
        polar bins 4 B, fan pixels 4 B, camera pixels 28 B forward and 44 B
        backward (with the image gradients)."""
        nb = self.geom.n_range * self.geom.n_azimuth
        npx_fan = self.geom.fan_h * self.geom.fan_w
        return {"k_bin": 28 * self.n_returns, "k_tile": 4 * nb, "k_fan": 4 * npx_fan,
                "k_tile_bwd": 4 * npx_fan + 4 * nb, "k_fant_bwd": 4 * npx_fan + 4 * nb,
                "k_ret_bwd": 28 * self.n_returns,
                # the plan's return-gather launch also carries the camera backward
                "k_ret_uw_bwd": 28 * self.n_returns + 44 * self.npix,
                "k_uw": 28 * self.npix, "k_uw_bwd": 44 * self.npix,
                # the plan's binning launch also carries the camera forward
                "k_bin_uw": 28 * self.n_returns + 28 * self.npix}


def timed(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def event_time(torch, fn, reps):
    """Average duration of fn's GPU work, from HIP events on the current stream."""
    s = torch.cuda.current_stream()
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        fn()
    b.record(s)
    b.synchronize()
    return a.elapsed_time(b) / 1e3 / reps


def median_time(torch, fn, steps, warmup, repeats=5):
    """Median over `repeats` of the mean wall-clock time of `steps` calls."""
    ts = sorted(timed(torch, fn, steps, warmup if k == 0 else 1) for k in range(repeats))
    return ts[len(ts) // 2]


def batched_legs(torch, dev, steps, only=None):
    """Ragged batch of 256 sonar frames (forward) and a differentiable batch of
    32 sonar + 32 camera frames (forward + backward): one ABI call per frame
    (plain), one call per entry point for the whole batch (batched), and a
    plan replayed from HIP graphs, with descriptors and buffers prepared
    before timing."""
    import numpy as np
    import paper_2503_01074_amd as osm
    from paper_2503_01074_amd import _lib
    from paper_2503_01074_amd.api import _sonar_struct, _uw_struct
    import workloads as W

    stream = torch.cuda.current_stream(dev).cuda_stream
    P = lambda t: t.data_ptr()
    out = {}
    reps = max(5, steps // 10)

    if only == "c4":
        return c4_leg(torch, dev, steps, out)
    frames = W.sonar_c3()
    tables, base, hits = [], 0, []
    for f in frames:
        mat = np.where(f.hits.mat >= 0, f.hits.mat + base, f.hits.mat).astype(np.int32)
        tables.append(f.hits.refl)
        base += f.hits.refl.shape[0]
        h = osm.DeviceHits.from_host(f.hits, dev)
        h.mat = torch.as_tensor(mat, device=dev)
        hits.append(h)
    refl = torch.as_tensor(np.concatenate(tables), device=dev)
    n_mat = int(refl.numel())
    geoms = [osm.SonarGeometry.from_spec(f.spec, param_row=i) for i, f in enumerate(frames)]
    params = osm.sonar_params([osm.sonar_params_from_spec(f.spec) for f in frames], dev)
    polars = [torch.empty(g.n_range, g.n_azimuth, device=dev) for g in geoms]
    fans = [torch.empty(g.fan_h, g.fan_w, device=dev) for g in geoms]
    structs = [_sonar_struct(g, h, p, q) for g, h, p, q in zip(geoms, hits, polars, fans)]
    arr = (_lib.SonarFrame * len(frames))(*structs)
    need = _lib.oceansim_sonar_workspace_size(arr, n_mat, False)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    n_ret = sum(f.hits.n for f in frames)
    n_fr = len(frames)

    def c3():
        _lib.oceansim_sonar_render(arr, P(params), n_fr, P(refl), n_mat, P(ws), need, stream)

    def c3_plain():
        for sf in structs:
            _lib.oceansim_sonar_render(sf, P(params), n_fr, P(refl), n_mat, P(ws), need, stream)

    t = median_time(torch, c3, reps, 3)
    t_plain = median_time(torch, c3_plain, max(3, reps // 4), 1)
    _lib.oceansim_trace_enable(True)
    for _ in range(3):
        c3()
    torch.cuda.synchronize()
    tr = _lib.oceansim_trace_summary()
    _lib.oceansim_trace_enable(False)
    plan = osm.Plan(list(zip(geoms, hits)), sonar_params=params, refl=refl, autotune=True)
    t_plan = median_time(torch, plan.forward, reps, 3)
    shape = plan.shape()
    plan.close()
    out["batched_c3_fwd"] = {"frames": n_fr, "returns": n_ret, "ms": t * 1e3,
                             "frames_per_s": n_fr / t, "returns_per_s": n_ret / t,
                             "plain_ms": t_plain * 1e3, "plain_frames_per_s": n_fr / t_plain,
                             "plan_ms": t_plan * 1e3, "plan_frames_per_s": n_fr / t_plan,
                             "plan_returns_per_s": n_ret / t_plan, "autotuned_shape": shape,
                             "kernels_us": {k: round(us / calls, 1) for k, (calls, us) in tr.items()}}
    log("C3 forward, 256 frames: batched call %.3f ms, one call per frame %.3f ms, autotuned plan %.3f ms %s"
        % (t * 1e3, t_plain * 1e3, t_plan * 1e3, shape))
    del hits, polars, fans, ws, arr, structs
    torch.cuda.empty_cache()
    if only == "c3":
        return out
    return c4_leg(torch, dev, steps, out)


def c4_leg(torch, dev, steps, out):
    """32 sonar + 32 camera frames, forward and forward + backward: one call
    per entry point for the whole batch, and a plan."""
    import paper_2503_01074_amd as osm
    from paper_2503_01074_amd import _lib
    from paper_2503_01074_amd.api import _sonar_struct, _uw_struct
    import workloads as W

    stream = torch.cuda.current_stream(dev).cuda_stream
    P = lambda t: t.data_ptr()
    frames = W.sonar_c4()
    cams, waters = W.camera_c4()
    refl = torch.as_tensor(frames[0].hits.refl, device=dev)
    n_mat = int(refl.numel())
    hits = [osm.DeviceHits.from_host(f.hits, dev) for f in frames]
    geoms = [osm.SonarGeometry.from_spec(f.spec, param_row=0) for f in frames]
    params = osm.sonar_params([osm.sonar_params_from_spec(frames[0].spec)], dev)
    polars = [torch.empty(g.n_range, g.n_azimuth, device=dev) for g in geoms]
    fans = [torch.empty(g.fan_h, g.fan_w, device=dev) for g in geoms]
    stencils = [osm.api.fan_stencil_buffer(g, dev) for g in geoms]
    gp = [torch.as_tensor(W.loss_weights((202, k), (g.n_range, g.n_azimuth)), device=dev)
          for k, g in enumerate(geoms)]
    gf = [torch.as_tensor(W.loss_weights((203, k), (g.fan_h, g.fan_w)), device=dev) for k, g in enumerate(geoms)]
    sf = (_lib.SonarFrame * len(frames))(*[_sonar_struct(g, h, p, q, stencil=sv) for g, h, p, q, sv in
                                           zip(geoms, hits, polars, fans, stencils)])
    sb = (_lib.SonarFrame * len(frames))(*[_sonar_struct(g, h, grad_polar=a, grad_fan=b, stencil=sv)
                                           for g, h, a, b, sv in zip(geoms, hits, gp, gf, stencils)])
    ws_f = torch.empty(_lib.oceansim_sonar_workspace_size(sf, n_mat, False), dtype=torch.uint8, device=dev)
    ws_b = torch.empty(_lib.oceansim_sonar_workspace_size(sb, n_mat, True), dtype=torch.uint8, device=dev)
    g_refl = torch.empty(n_mat, device=dev)
    g_par = torch.empty(1, _lib.SONAR_GRAD_WIDTH, device=dev)
    Js = [torch.as_tensor(c.J, device=dev) for c in cams]
    ds = [torch.as_tensor(c.depth, device=dev) for c in cams]
    imgs = [torch.empty_like(J) for J in Js]
    gi = [torch.as_tensor(W.loss_weights((204, k), c.J.shape), device=dev) for k, c in enumerate(cams)]
    gJ = [torch.empty_like(J) for J in Js]
    gd = [torch.empty_like(d) for d in ds]
    w = waters[0]
    water = osm.water_params([(w.beta_d, w.beta_b, w.b_inf)], dev)
    uf = (_lib.UwFrame * len(cams))(*[_uw_struct(J, d, o) for J, d, o in zip(Js, ds, imgs)])
    ub = (_lib.UwFrame * len(cams))(*[_uw_struct(J, d, None, 0, g, a, b) for J, d, g, a, b in
                                      zip(Js, ds, gi, gJ, gd)])
    ws_uf = torch.empty(max(256, _lib.oceansim_uw_workspace_size(uf, False)), dtype=torch.uint8, device=dev)
    ws_ub = torch.empty(max(256, _lib.oceansim_uw_workspace_size(ub, True)), dtype=torch.uint8, device=dev)
    g_w = torch.empty(1, _lib.WATER_GRAD_WIDTH, device=dev)
    n_ret = sum(f.hits.n for f in frames)
    n_fr = len(frames) + len(cams)

    def c4_fwd():
        _lib.oceansim_sonar_render(sf, P(params), 1, P(refl), n_mat, P(ws_f), ws_f.numel(), stream)
        _lib.oceansim_uw_form(uf, P(water), 1, P(ws_uf), ws_uf.numel(), stream)

    def c4_step():
        c4_fwd()
        _lib.oceansim_sonar_render_backward(sb, P(params), 1, P(refl), n_mat, P(g_refl), P(g_par), P(ws_b),
                                            ws_b.numel(), stream)
        _lib.oceansim_uw_form_backward(ub, P(water), 1, P(g_w), P(ws_ub), ws_ub.numel(), stream)

    tf = median_time(torch, c4_fwd, max(5, steps // 5), 3)
    ts = median_time(torch, c4_step, max(5, steps // 5), 3)
    plan = osm.Plan(list(zip(geoms, hits)), list(zip(Js, ds, [0] * len(cams))), sonar_params=params, refl=refl,
                    water=water, backward=True, autotune=True, image_grads=True)
    for o, a, b in zip(plan.sonar_out, gp, gf):
        o["grad_polar"].copy_(a)
        o["grad_fan"].copy_(b)
    for o, g in zip(plan.camera_out, gi):
        o["grad_out"].copy_(g)

    def c4_plan_step():
        plan.forward()
        plan.backward()
    tgf = median_time(torch, plan.forward, max(5, steps // 5), 3)
    tgs = median_time(torch, c4_plan_step, max(5, steps // 5), 3)
    shape = plan.shape()
    plan.close()
    out["batched_c4"] = {"sonar_frames": len(frames), "camera_frames": len(cams), "returns": n_ret,
                         "fwd_ms": tf * 1e3, "fwd_bwd_ms": ts * 1e3,
                         "fwd_bwd_frames_per_s": n_fr / ts, "fwd_bwd_returns_per_s": n_ret / ts,
                         "plan_fwd_ms": tgf * 1e3, "plan_fwd_bwd_ms": tgs * 1e3,
                         "plan_fwd_bwd_frames_per_s": n_fr / tgs, "plan_fwd_bwd_returns_per_s": n_ret / tgs,
                         "autotuned_shape": shape}
    log("C4 batched: fwd %.3f ms, fwd+bwd %.3f ms; autotuned plan fwd %.3f ms, fwd+bwd %.3f ms %s"
        % (tf * 1e3, ts * 1e3, tgf * 1e3, tgs * 1e3, shape))
    return out


def cpu_baseline(rt, budget_s):
    """The FP64 oracle on this host's cores over a bounded sample of the same
    workload: whole sonar frames (forward + backward) and the camera frame."""
    import numpy as np
    import oracle
    import workloads as W

    spec = rt.frame.spec
    cfg = oracle.SonarConfig.from_spec(spec)
    hits = rt.frame.hits
    gp = W.loss_weights((101, 1), (spec.n_range, spec.n_azimuth))
    gf = W.loss_weights((101, 2), (spec.fan_h, spec.fan_w))
    w = rt.water_host
    gi = W.loss_weights((101, 3), rt.cam.J.shape)
    t0 = time.perf_counter()
    n = 0
    while True:
        oracle.sonar_forward(cfg, hits, hits.refl)
        oracle.uw_forward(rt.cam.J, rt.cam.depth, w.beta_d, w.beta_b, w.b_inf)
        oracle.sonar_backward(cfg, hits, hits.refl, gp, gf)
        oracle.uw_backward(rt.cam.J, rt.cam.depth, w.beta_d, w.beta_b, w.b_inf, gi, True)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 50:
            break
    return {"value": n * hits.n / el, "unit": "returns/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d full step(s) of the real-time workload (sonar fwd+bwd, camera fwd+bwd) in %.1f s"
                      % (n, el)}


def calibration_leg(torch, dev, steps, n_frames):
    """Calibration scale: n_frames sonar frames of 2048 x 1024 returns (2048 x
    2048 bins, no fan, 64 materials, gamma speckle) and n_frames 1920 x 1080
    camera frames, forward and forward + backward through an autotuned plan
    (polar and image losses).  Four distinct sonar and camera frames are
    generated and uploaded n_frames / 4 times each (separate device buffers,
    distinct frame ids, so distinct speckle), which keeps the host-side
    generation to seconds."""
    import paper_2503_01074_amd as osm
    import workloads as W
    t0 = time.perf_counter()
    base = W.sonar_c5(n_frames=4)
    st = W.Stream(W.BASE_SEED + 4, 1 << 21)
    water_h = W.make_water(st)
    cams = [W.make_camera(W.Stream(W.BASE_SEED + 4, (1 << 22) + k), 1080, 1920) for k in range(4)]
    hits, geoms, Js, ds = [], [], [], []
    for k in range(n_frames):
        f, c = base[k % 4], cams[k % 4]
        hits.append(osm.DeviceHits.from_host(f.hits, dev))
        g = osm.SonarGeometry.from_spec(f.spec, param_row=0)
        g.frame_id = k
        geoms.append(g)
        Js.append(torch.as_tensor(c.J, device=dev))
        ds.append(torch.as_tensor(c.depth, device=dev))
    refl = torch.as_tensor(base[0].hits.refl, device=dev)
    params = osm.sonar_params([osm.sonar_params_from_spec(base[0].spec)], dev)
    water = osm.water_params([(water_h.beta_d, water_h.beta_b, water_h.b_inf)], dev)
    plan = osm.Plan(list(zip(geoms, hits)), [(J, d, 0) for J, d in zip(Js, ds)], sonar_params=params, refl=refl,
                    water=water, backward=True, autotune=True)
    gp = [torch.as_tensor(W.loss_weights((205, k), (2048, 2048)), device=dev) for k in range(4)]
    go = [torch.as_tensor(W.loss_weights((206, k), (3, 1080, 1920)), device=dev) for k in range(4)]
    for k, o in enumerate(plan.sonar_out):
        o["grad_polar"].copy_(gp[k % 4])
    for k, o in enumerate(plan.camera_out):
        o["grad_out"].copy_(go[k % 4])
    log("C5 leg: %d + %d frames prepared in %.1f s" % (n_frames, n_frames, time.perf_counter() - t0))

    def step():
        plan.forward()
        plan.backward()
    n = max(3, steps // 20)
    tf = median_time(torch, plan.forward, n, 2, 3)
    ts = median_time(torch, step, n, 2, 3)
    n_ret = sum(h.n for h in hits)
    nb = n_frames * 2048 * 2048
    npx = n_frames * 1920 * 1080
    alg_f = 28 * n_ret + 4 * nb + 28 * npx
    alg_s = alg_f + 28 * n_ret + 4 * nb + 44 * npx
    shape = plan.shape()
    log("C5 calibration scale, %d + %d frames: fwd %.3f ms (%.2f TB/s algorithmic, %.2f of 8 TB/s), fwd+bwd "
        "%.3f ms (%.2f TB/s, %.2f), %.2f G returns/s, shape %s"
        % (n_frames, n_frames, tf * 1e3, alg_f / tf / 1e12, alg_f / tf / 8e12, ts * 1e3, alg_s / ts / 1e12,
           alg_s / ts / 8e12, n_ret / ts / 1e9, shape))
    plan.close()
    return {"sonar_frames": n_frames, "camera_frames": n_frames, "returns": n_ret, "distinct_frames": 4,
            "fwd_ms": tf * 1e3, "fwd_bwd_ms": ts * 1e3, "fwd_bwd_returns_per_s": n_ret / ts,
            "fwd_alg_TBps": alg_f / tf / 1e12, "fwd_bwd_alg_TBps": alg_s / ts / 1e12,
            "fwd_bwd_hbm_frac": alg_s / ts / (HBM_PEAK_GBS * 1e9), "autotuned_shape": shape}


def camera_io_leg(torch, dev, steps):
    """8-bit sRGB and z-depth in, Eq. (1), 8-bit sRGB out on one 1920 x 1080
    RGBA frame: each entry point timed alone over `steps` launches, with its
    algorithmic bytes (conditioning 24 B/pixel: 4 B RGBA + 4 B depth in, 12 B
    J + 4 B range out; encoding 16 B: 12 B in, 4 B out; the adjoint 8 B)."""
    import paper_2503_01074_amd as osm
    H, Wd = 1080, 1920
    g = torch.Generator(device="cpu").manual_seed(7)
    img = torch.randint(0, 256, (H, Wd, 4), generator=g, dtype=torch.uint8).to(dev)
    z = (torch.rand(H, Wd, generator=g) * 20 + 0.5).to(dev)
    intr = (1662.77, 1662.77, 960.0, 540.0)     # 60 degree horizontal field of view
    water = osm.water_params([((0.35, 0.12, 0.08), (0.30, 0.15, 0.10), (0.05, 0.25, 0.35))], device=dev)
    (J,), (r,) = osm.cam_condition([img], [z], [intr])
    (I,) = osm.uw_form([J], [r], water)
    n = max(20, steps)
    s = torch.cuda.current_stream(dev)

    def timed(fn):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        for _ in range(n):
            fn()
        b.record(s)
        b.synchronize()
        return a.elapsed_time(b) / 1e3 / n

    t_c = timed(lambda: osm.cam_condition([img], [z], [intr]))
    t_u = timed(lambda: osm.uw_form([J], [r], water))
    t_e = timed(lambda: osm.cam_encode([I], channels_out=4))
    t_b = timed(lambda: osm.cam_condition_backward([r], [intr]))
    def pipeline():
        (j,), (rr,) = osm.cam_condition([img], [z], [intr])
        (ii,) = osm.uw_form([j], [rr], water)
        osm.cam_encode([ii], channels_out=4)

    t_all = timed(pipeline)
    px = H * Wd
    rate = lambda b, t: round(b * px / t / 1e9, 1)
    return {"frame": "1920x1080 RGBA8 + z-depth -> Eq. 1 -> RGBA8", "pipeline_us": round(t_all * 1e6, 2),
            "frames_per_s": round(1.0 / t_all, 1),
            "condition_us": round(t_c * 1e6, 2), "condition_GBps": rate(24, t_c),
            "uw_form_us": round(t_u * 1e6, 2), "encode_us": round(t_e * 1e6, 2), "encode_GBps": rate(16, t_e),
            "range_backward_us": round(t_b * 1e6, 2), "range_backward_GBps": rate(8, t_b)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported (the path shards by frame "
              "across GPUs, see the design notes)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        copy_calibration(torch, dev)
        return
    if args.only == "c5":
        calibration_leg(torch, dev, args.steps, args.c5_frames)
        return
    if args.only:
        legs = batched_legs(torch, dev, args.steps, only=args.only)
        log("done: %s" % ", ".join(sorted(legs)))
        return
    log("building workload")
    rt = RealTimeStep(dev, range_norm=not args.no_range_norm)

    # The step: the plan (frames prepared once, launch shapes autotuned),
    # forward + backward, K times after W warm-up steps, timed by the host
    # clock between two device synchronisations.
    log("timing %d full steps after %d warm-up" % (args.steps, args.warmup))
    headline = lambda: rt.plan_step("plan")
    t_step = timed(torch, headline, args.steps, args.warmup)
    t_fwd = timed(torch, lambda: rt.plan_forward("plan"), args.steps, args.warmup)
    log("plan: step %.3f ms, forward %.3f ms, shape %s" % (t_step * 1e3, t_fwd * 1e3, rt.plans["plan"].shape()))
    # the same step through the plain entry points (one call per entry point)
    # and through the plan's HIP graphs
    t_pstep = timed(torch, rt.step, args.steps, args.warmup)
    t_pfwd = timed(torch, rt.forward, args.steps, args.warmup)
    t_sonar_fwd = timed(torch, rt.sonar_forward, args.steps, args.warmup)
    t_gstep = timed(torch, lambda: rt.plan_step("graph"), args.steps, args.warmup)
    t_gfwd = timed(torch, lambda: rt.plan_forward("graph"), args.steps, args.warmup)
    log("plain entry points: step %.3f ms, forward %.3f ms, sonar forward %.3f ms; graph plan: step %.3f ms, "
        "forward %.3f ms" % (t_pstep * 1e3, t_pfwd * 1e3, t_sonar_fwd * 1e3, t_gstep * 1e3, t_gfwd * 1e3))
    norm = None
    if "norm" in rt.plans:
        t_nstep = timed(torch, lambda: rt.plan_step("norm"), args.steps, args.warmup)
        t_nfwd = timed(torch, lambda: rt.plan_forward("norm"), args.steps, args.warmup)
        log("with range-wise normalisation: step %.3f ms, forward %.3f ms" % (t_nstep * 1e3, t_nfwd * 1e3))
        norm = {"step_ms": t_nstep * 1e3, "returns_per_s": rt.n_returns / t_nstep, "fwd_ms": t_nfwd * 1e3}

    # per-entry-point GPU durations from events on the launch stream
    reps = max(20, args.steps)
    parts = {
        "sonar_forward": event_time(torch, rt.sonar_forward, reps),
        "sonar_backward": event_time(torch, rt.sonar_backward, reps),
        "uw_forward": event_time(torch, rt.uw_forward, reps),
        "uw_backward": event_time(torch, rt.uw_backward, reps),
    }
    # per-kernel durations: the library brackets each launch with HIP events
    # on its stream while tracing is on
    rt.lib.oceansim_trace_enable(True)
    for _ in range(reps):
        headline()
    torch.cuda.synchronize()
    trace = rt.lib.oceansim_trace_summary()
    rt.lib.oceansim_trace_enable(False)
    kern_us = {k: us / calls for k, (calls, us) in trace.items()}
    dom = max(kern_us, key=lambda k: kern_us[k] * trace[k][0])
    abytes = rt.algorithmic_bytes()
    dom_bytes = abytes.get(dom)
    achieved = dom_bytes / (kern_us[dom] * 1e-6) / 1e9 if dom_bytes else None
    roofline = {"bound": "hbm", "kernel": dom,
                "achieved": None if achieved is None else round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom), "bytes_per_launch": dom_bytes, "launch_us": round(kern_us[dom], 2)}
    kernel_table = {k: {"us": round(kern_us[k], 2), "alg_bytes": abytes.get(k),
                        "alg_GBps": round(abytes[k] / (kern_us[k] * 1e-6) / 1e9, 1) if k in abytes else None}
                    for k in sorted(kern_us, key=lambda k: -kern_us[k])}
    log("kernels (us): " + ", ".join("%s %.2f" % (k, v["us"]) for k, v in kernel_table.items()))

    extra = {}
    if not args.no_batched:
        extra = batched_legs(torch, dev, args.steps)
        extra["calibration_c5"] = calibration_leg(torch, dev, args.steps, args.c5_frames)
        extra["camera_io"] = camera_io_leg(torch, dev, args.steps)
        log("camera io: %s" % extra["camera_io"])
    cpu = None
    if not args.no_cpu:
        log("timing the FP64 oracle on the host")
        cpu = cpu_baseline(rt, args.cpu_seconds)

    line = {
        "metric": "sonar returns/s + frames/s (fwd, fwd+bwd, batched vs plain) at <=1e-5 rel err",
        "value": rt.n_returns / t_step,
        "unit": "returns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "real-time frame: 131072 sonar returns (1024 beams x 128 rays, r in [1,50) m), "
                               "1024x1024 polar bins, gamma speckle k=4, 1024x2048 fan, plus Eq. 1 on one "
                               "1920x1080 RGB frame; forward + backward",
                   "global_batch": 1, "parallelism": "none (1 GPU)"},
        "path": "plan (frames prepared once, autotuned launch shapes, camera work inside the sonar binning and return-gather launches)",
        "frames_per_s": 1.0 / t_step,
        "fwd_returns_per_s": rt.n_returns / t_fwd,
        "fwd_frames_per_s": 1.0 / t_fwd,
        "plain": {"step_ms": t_pstep * 1e3, "returns_per_s": rt.n_returns / t_pstep, "fwd_ms": t_pfwd * 1e3,
                  "sonar_fwd_only_frames_per_s": 1.0 / t_sonar_fwd},
        "graph": {"step_ms": t_gstep * 1e3, "returns_per_s": rt.n_returns / t_gstep, "fwd_ms": t_gfwd * 1e3},
        "range_norm": norm,
        "copy_GBps": copy_rate(torch, dev),
        "camera_mpx_per_s_fwd_bwd": rt.npix / t_step / 1e6,
        "entry_point_us": {k: round(v * 1e6, 2) for k, v in parts.items()},
        "kernels": kernel_table,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
