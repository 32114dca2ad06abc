"""Throughput of the OceanSim sonar + underwater-camera image-formation path on
one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-batched] [--no-cpu]

A step is one forward + backward pass of the whole path over the calibration-
scale workload: 64 sonar frames of 2048 beams x 1024 rays = 2,097,152 returns
each (range U[0.5, 50) m, 64 materials, 2048 x 2048 polar bins, gamma speckle,
no fan) and 64 RGB frames of 1920 x 1080 through Eq. (1), with the adjoints
with respect to the reflectivities, the sonar parameters and the water
parameters (polar and image losses; no image gradients).  Inputs are seeded
synthetic data already resident in device memory; the frames go through one
autotuned plan.

Prints one JSON line.  ``value`` is sonar returns per second through the full
step.  The line also carries the roofline of the dominant kernel (HIP events
on the stream the kernel is launched on), the whole step's fraction of HBM
peak, the 200-step Adam calibration at this scale, and the other workloads:
one plain frame (forward), the real-time frame (sonar + 1080p camera), the
256-frame ragged batch and the 32 + 32 differentiable batch (unbatched
forward-only against batched forward + backward), and the FP64 oracle timed on
the host's cores over a bounded sample.
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
# non-packed vector lanes: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9
C5_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "c5_step_hbm_traffic.json")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-batched", action="store_true", help="skip the other workloads and the calibration run")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 64 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--only", choices=["c2", "c3", "c4", "c5", "raycast"], default=None,
                    help="only build and run one workload (for profiler runs); prints no JSON line")
    ap.add_argument("--c5-frames", type=int, default=64,
                    help="sonar and camera frames of the calibration-scale workload")
    ap.add_argument("--calib-steps", type=int, default=200, help="Adam steps of the calibration run")
    ap.add_argument("--profile-summary", metavar="DIR", default=None,
                    help="summarise the rocprofv3 counter runs under DIR (fetch/, write/, valu/, cfetch/, "
                         "cwrite/) into the per-kernel traffic record bench.py reads; needs no GPU")
    ap.add_argument("--profile-out", default=C5_TRAFFIC_PROFILE, help="where --profile-summary writes")
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



def short_kernel_name(name):
    """'void osim::(anonymous namespace)::k_tile<Table<SonarDev>, 512>(...)' -> 'k_tile'."""
    name = name.strip().strip('"').replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):
        if ch in "<(" and depth == 0:
            cut = i
            break
    name = name[:cut]
    return name.rsplit("::", 1)[-1]


def counter_means(directory, counter):
    """Mean value of one counter per dispatch, by short kernel name, over the
    rocprofv3 counter-collection CSV files under `directory`."""
    import csv
    sums, counts = {}, {}
    for root, _, files in os.walk(directory):
        for fn in files:
            if not fn.endswith("counter_collection.csv"):
                continue
            with open(os.path.join(root, fn), newline="") as fh:
                per_dispatch = {}
                for row in csv.DictReader(fh):
                    if row["Counter_Name"] != counter:
                        continue
                    key = (row["Dispatch_Id"], short_kernel_name(row["Kernel_Name"]))
                    per_dispatch[key] = per_dispatch.get(key, 0.0) + float(row["Counter_Value"])
                for (_, k), v in per_dispatch.items():
                    sums[k] = sums.get(k, 0.0) + v
                    counts[k] = counts.get(k, 0) + 1
    return {k: sums[k] / counts[k] for k in sums}, counts


def profile_summary(directory, out_path):
    """Per-launch HBM bytes and VALU instructions of each kernel from the
    counter runs under `directory`: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) are scaled by what they read for the 64 MiB copy of
    --copy-calibration (64 MiB read and 64 MiB written per launch);
    SQ_INSTS_VALU counts wave instructions.  Writes the record bench.py reads
    (tagged with the library source digest) and prints a table."""
    copy_bytes = float(64 << 20)
    cf, _ = counter_means(os.path.join(directory, "cfetch"), "FETCH_SIZE")
    cw, _ = counter_means(os.path.join(directory, "cwrite"), "WRITE_SIZE")
    copy_name = [k for k in cf if "copyBuffer" in k or "copy" in k.lower()]
    if not copy_name:
        raise SystemExit("no copy kernel in the calibration runs")
    fetch_factor = copy_bytes / (cf[copy_name[0]] * 1024.0)
    write_factor = copy_bytes / (cw[copy_name[0]] * 1024.0)
    fetch, n = counter_means(os.path.join(directory, "fetch"), "FETCH_SIZE")
    write, _ = counter_means(os.path.join(directory, "write"), "WRITE_SIZE")
    valu, _ = counter_means(os.path.join(directory, "valu"), "SQ_INSTS_VALU")
    kernels = {}
    for k in sorted(fetch):
        if k.startswith("__amd") or k not in write:
            continue
        kernels[k] = {"fetch_bytes": fetch[k] * 1024.0 * fetch_factor, "write_bytes": write[k] * 1024.0 * write_factor,
                      "dispatches": n[k]}
        if k in valu:
            kernels[k]["valu_insts"] = valu[k]
    rec = {"source_sha256": source_digest(), "fetch_factor": fetch_factor, "write_factor": write_factor,
           "kernels": kernels}
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
    print("fetch factor %.4f, write factor %.4f (copy kernel %s)" % (fetch_factor, write_factor, copy_name[0]))
    print("| kernel | dispatches | read MB | written MB | VALU instructions (M) |")
    print("|---|---|---|---|---|")
    for k, v in kernels.items():
        print("| %s | %d | %.2f | %.2f | %s |" % (k, v["dispatches"], v["fetch_bytes"] / 1e6, v["write_bytes"] / 1e6,
                                                 "%.2f" % (v["valu_insts"] / 1e6) if "valu_insts" in v else "-"))


def measured_profile():
    """Per-kernel HBM bytes and VALU instructions per launch of the
    calibration-scale step, from the rocprofv3 counter summary in profiles/,
    if it was taken on the current sources (else None)."""
    try:
        with open(C5_TRAFFIC_PROFILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_digest():
        return None
    return rec.get("kernels", {})


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




class CalibrationScale:
    """The calibration-scale workload on the device: n_frames sonar frames of
    2048 x 1024 returns (2048 x 2048 bins, no fan, 64 materials, gamma
    speckle) and n_frames 1920 x 1080 camera frames in one autotuned backward
    plan, with seeded N(0, 1) loss gradients (polar and image losses).  Four
    distinct sonar and camera frames are generated and uploaded n_frames / 4
    times each (separate device buffers, distinct frame ids, so distinct
    speckle), which keeps the host-side generation to seconds."""

    def __init__(self, torch, dev, n_frames, autotune=True, losses=True):
        import paper_2503_01074_amd as osm
        import workloads as W
        t0 = time.perf_counter()
        self.torch = torch
        base = W.sonar_c5(n_frames=4)
        st = W.Stream(W.BASE_SEED + 4, 1 << 21)
        self.water_h = W.make_water(st)
        cams = [W.make_camera(W.Stream(W.BASE_SEED + 4, (1 << 22) + k), 1080, 1920) for k in range(4)]
        self.hits, self.geoms, self.Js, self.ds = [], [], [], []
        for k in range(n_frames):
            f, c = base[k % 4], cams[k % 4]
            self.hits.append(osm.DeviceHits.from_host(f.hits, dev))
            g = osm.SonarGeometry.from_spec(f.spec, param_row=0)
            g.frame_id = k
            self.geoms.append(g)
            self.Js.append(torch.as_tensor(c.J, device=dev))
            self.ds.append(torch.as_tensor(c.depth, device=dev))
        self.base = base
        self.refl = torch.as_tensor(base[0].hits.refl, device=dev)
        self.params = osm.sonar_params([osm.sonar_params_from_spec(base[0].spec)], dev)
        w = self.water_h
        self.water = osm.water_params([(w.beta_d, w.beta_b, w.b_inf)], dev)
        self.plan = osm.Plan(list(zip(self.geoms, self.hits)), [(J, d, 0) for J, d in zip(self.Js, self.ds)],
                             sonar_params=self.params, refl=self.refl, water=self.water, backward=True,
                             autotune=autotune)
        if losses:
            gp = [torch.as_tensor(W.loss_weights((205, k), (2048, 2048)), device=dev) for k in range(4)]
            go = [torch.as_tensor(W.loss_weights((206, k), (3, 1080, 1920)), device=dev) for k in range(4)]
            for k, o in enumerate(self.plan.sonar_out):
                o["grad_polar"].copy_(gp[k % 4])
            for k, o in enumerate(self.plan.camera_out):
                o["grad_out"].copy_(go[k % 4])
        self.n_frames = n_frames
        self.n_returns = sum(h.n for h in self.hits)
        self.n_bins = n_frames * 2048 * 2048
        self.n_px = n_frames * 1920 * 1080
        log("calibration-scale workload: %d + %d frames prepared in %.1f s, plan shape %s"
            % (n_frames, n_frames, time.perf_counter() - t0, self.plan.shape()))

    def forward(self):
        self.plan.forward()

    def step(self):
        self.plan.forward()
        self.plan.backward()

    def algorithmic_bytes(self):
        """Bytes the method must move, per launch of each kernel and per step:
        returns 28 B, polar bins 4 B out, camera pixels 28 B forward (J, d in,
        I out) and 28 B backward (dL/dI, J, d in; no image gradients); the
        sonar backward reads dL/d(polar) 4 B per bin and the returns 28 B."""
        n, nb, npx = self.n_returns, self.n_bins, self.n_px
        per_kernel = {"k_bin": 28 * n, "k_bin_uw": 28 * n + 28 * npx, "k_tile": 4 * nb, "k_uw": 28 * npx,
                      "k_tile_uw": 4 * nb + 28 * npx,
                      "k_pair_bwd": 4 * nb + 28 * n, "k_pair_uw_bwd": 4 * nb + 28 * n + 28 * npx,
                      "k_fant_bwd": 4 * nb, "k_ret_bwd": 28 * n,
                      "k_ret_uw_bwd": 28 * n + 28 * npx, "k_uw_bwd": 28 * npx}
        fwd = 28 * n + 4 * nb + 28 * npx
        bwd = 4 * nb + 28 * n + 28 * npx
        return per_kernel, fwd, bwd


def c1_leg(torch, dev, steps):
    """One plain frame (256 beams x 32 rays, 512 x 256 bins, 512 x 1024 fan):
    the forward through the plain entry point, one call per frame."""
    import paper_2503_01074_amd as osm
    from paper_2503_01074_amd import _lib
    from paper_2503_01074_amd.api import _sonar_struct
    import workloads as W
    f = W.sonar_c1()[0]
    g = osm.SonarGeometry.from_spec(f.spec)
    h = osm.DeviceHits.from_host(f.hits, dev)
    params = osm.sonar_params([osm.sonar_params_from_spec(f.spec)], dev)
    refl = torch.as_tensor(f.hits.refl, device=dev)
    polar = torch.empty(g.n_range, g.n_azimuth, device=dev)
    fan = torch.empty(g.fan_h, g.fan_w, device=dev)
    sf = _sonar_struct(g, h, polar, fan)
    n_mat = int(refl.numel())
    ws = torch.empty(max(256, _lib.oceansim_sonar_workspace_size(sf, n_mat, False)), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    P = lambda t: t.data_ptr()

    def fwd():
        _lib.oceansim_sonar_render(sf, P(params), 1, P(refl), n_mat, P(ws), ws.numel(), stream)
    t = median_time(torch, fwd, max(50, steps * 5), 10)
    tg = event_time(torch, fwd, max(50, steps * 5))
    log("C1 plain forward: %.1f us per frame (wall), %.1f us (GPU events)" % (t * 1e6, tg * 1e6))
    return {"returns": h.n, "fwd_us": t * 1e6, "fwd_gpu_us": tg * 1e6, "frames_per_s": 1.0 / t,
            "returns_per_s": h.n / t}


def c2_leg(torch, dev, steps):
    """The real-time frame (131072 returns, 1024 x 1024 bins, 1024 x 2048 fan,
    plus one 1920 x 1080 camera frame): forward + backward through the plan,
    the plain entry points and graphs, the forward alone, and the same step
    with the range-wise normalisation."""
    rt = RealTimeStep(dev, range_norm=True)
    k = max(50, steps * 5)
    t_step = timed(torch, lambda: rt.plan_step("plan"), k, 10)
    t_fwd = timed(torch, lambda: rt.plan_forward("plan"), k, 10)
    t_pstep = timed(torch, rt.step, k, 10)
    t_pfwd = timed(torch, rt.forward, k, 10)
    t_sfwd = timed(torch, rt.sonar_forward, k, 10)
    t_gstep = timed(torch, lambda: rt.plan_step("graph"), k, 10)
    t_nstep = timed(torch, lambda: rt.plan_step("norm"), k, 10)
    log("C2 real-time frame: plan step %.3f ms, forward %.3f ms; plain step %.3f ms; graph step %.3f ms; "
        "range-normalised step %.3f ms" % (t_step * 1e3, t_fwd * 1e3, t_pstep * 1e3, t_gstep * 1e3, t_nstep * 1e3))
    return {"returns": rt.n_returns, "camera_px": rt.npix, "step_ms": t_step * 1e3,
            "returns_per_s": rt.n_returns / t_step, "frames_per_s": 2.0 / t_step, "fwd_ms": t_fwd * 1e3,
            "plain_step_ms": t_pstep * 1e3, "plain_fwd_ms": t_pfwd * 1e3,
            "plain_sonar_fwd_frames_per_s": 1.0 / t_sfwd, "graph_step_ms": t_gstep * 1e3,
            "range_norm_step_ms": t_nstep * 1e3, "plan_shape": rt.plans["plan"].shape()}


def c3_leg(torch, dev, steps):
    """256 ragged sonar frames: forward only with one call per frame
    (unbatched), forward through one batched call and an autotuned plan, and
    forward + backward through the batched entry points (saved fan stencils,
    per-return reflectivities: the polar-tile backward)."""
    import numpy as np
    import paper_2503_01074_amd as osm
    from paper_2503_01074_amd import _lib
    from paper_2503_01074_amd.api import _sonar_struct
    import workloads as W
    stream = torch.cuda.current_stream(dev).cuda_stream
    P = lambda t: t.data_ptr()
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
    stencils = [osm.api.fan_stencil_buffer(g, dev) for g in geoms]
    gp = [torch.as_tensor(W.loss_weights((301, k), (g.n_range, g.n_azimuth)), device=dev)
          for k, g in enumerate(geoms)]
    gf = [torch.as_tensor(W.loss_weights((302, k), (g.fan_h, g.fan_w)), device=dev) for k, g in enumerate(geoms)]
    structs = [_sonar_struct(g, h, p, q) for g, h, p, q in zip(geoms, hits, polars, fans)]
    sf = (_lib.SonarFrame * len(frames))(*[_sonar_struct(g, h, p, q, stencil=sv) for g, h, p, q, sv in
                                           zip(geoms, hits, polars, fans, stencils)])
    sb = (_lib.SonarFrame * len(frames))(*[_sonar_struct(g, h, grad_polar=a, grad_fan=b, stencil=sv)
                                           for g, h, a, b, sv in zip(geoms, hits, gp, gf, stencils)])
    arr = (_lib.SonarFrame * len(frames))(*structs)
    need = _lib.oceansim_sonar_workspace_size(arr, n_mat, False)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    ws_f = torch.empty(_lib.oceansim_sonar_workspace_size(sf, n_mat, False), dtype=torch.uint8, device=dev)
    ws_b = torch.empty(_lib.oceansim_sonar_workspace_size(sb, n_mat, True), dtype=torch.uint8, device=dev)
    g_refl = torch.empty(n_mat, device=dev)
    g_par = torch.empty(len(frames), _lib.SONAR_GRAD_WIDTH, device=dev)
    n_ret = sum(f.hits.n for f in frames)
    n_fr = len(frames)

    def fwd_batched():
        _lib.oceansim_sonar_render(arr, P(params), n_fr, P(refl), n_mat, P(ws), need, stream)

    def fwd_unbatched():
        for s1 in structs:
            _lib.oceansim_sonar_render(s1, P(params), n_fr, P(refl), n_mat, P(ws), need, stream)

    def step_batched():
        _lib.oceansim_sonar_render(sf, P(params), n_fr, P(refl), n_mat, P(ws_f), ws_f.numel(), stream)
        _lib.oceansim_sonar_render_backward(sb, P(params), n_fr, P(refl), n_mat, P(g_refl), P(g_par), P(ws_b),
                                            ws_b.numel(), stream)

    reps = max(5, steps // 2)
    t_b = median_time(torch, fwd_batched, reps, 3)
    t_u = median_time(torch, fwd_unbatched, max(3, reps // 4), 1)
    t_s = median_time(torch, step_batched, reps, 3)
    plan = osm.Plan(list(zip(geoms, hits)), sonar_params=params, refl=refl, autotune=True)
    t_p = median_time(torch, plan.forward, reps, 3)
    shape = plan.shape()
    plan.close()
    log("C3 ragged batch, 256 frames: unbatched forward %.3f ms, batched forward %.3f ms, plan forward %.3f ms, "
        "batched forward + backward %.3f ms" % (t_u * 1e3, t_b * 1e3, t_p * 1e3, t_s * 1e3))
    return {"frames": n_fr, "returns": n_ret, "unbatched_fwd_ms": t_u * 1e3,
            "unbatched_fwd_frames_per_s": n_fr / t_u, "batched_fwd_ms": t_b * 1e3,
            "batched_fwd_frames_per_s": n_fr / t_b, "plan_fwd_ms": t_p * 1e3, "plan_fwd_frames_per_s": n_fr / t_p,
            "plan_fwd_returns_per_s": n_ret / t_p, "batched_fwd_bwd_ms": t_s * 1e3,
            "batched_fwd_bwd_frames_per_s": n_fr / t_s, "autotuned_shape": shape}


def c4_leg(torch, dev, steps):
    """32 sonar + 32 camera frames: forward only with one call per frame
    (unbatched), and forward + backward through the batched entry points and
    through an autotuned plan."""
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
    s1 = [_sonar_struct(g, h, p, q) for g, h, p, q in zip(geoms, hits, polars, fans)]
    sf = (_lib.SonarFrame * len(frames))(*[_sonar_struct(g, h, p, q, stencil=sv) for g, h, p, q, sv in
                                           zip(geoms, hits, polars, fans, stencils)])
    sb = (_lib.SonarFrame * len(frames))(*[_sonar_struct(g, h, grad_polar=a, grad_fan=b, stencil=sv)
                                           for g, h, a, b, sv in zip(geoms, hits, gp, gf, stencils)])
    ws_1 = torch.empty(_lib.oceansim_sonar_workspace_size(s1[0], n_mat, False), dtype=torch.uint8, device=dev)
    ws_f = torch.empty(_lib.oceansim_sonar_workspace_size(sf, n_mat, False), dtype=torch.uint8, device=dev)
    ws_b = torch.empty(_lib.oceansim_sonar_workspace_size(sb, n_mat, True), dtype=torch.uint8, device=dev)
    g_refl = torch.empty(n_mat, device=dev)
    g_par = torch.empty(1, _lib.SONAR_GRAD_WIDTH, device=dev)
    Js = [torch.as_tensor(c.J, device=dev) for c in cams]
    ds = [torch.as_tensor(c.depth, device=dev) for c in cams]
    imgs = [torch.empty_like(J) for J in Js]
    gi = [torch.as_tensor(W.loss_weights((204, k), c.J.shape), device=dev) for k, c in enumerate(cams)]
    w = waters[0]
    water = osm.water_params([(w.beta_d, w.beta_b, w.b_inf)], dev)
    u1 = [_uw_struct(J, d, o) for J, d, o in zip(Js, ds, imgs)]
    uf = (_lib.UwFrame * len(cams))(*u1)
    ub = (_lib.UwFrame * len(cams))(*[_uw_struct(J, d, None, 0, g) for J, d, g in zip(Js, ds, gi)])
    ws_uf = torch.empty(max(256, _lib.oceansim_uw_workspace_size(uf, False)), dtype=torch.uint8, device=dev)
    ws_ub = torch.empty(max(256, _lib.oceansim_uw_workspace_size(ub, True)), dtype=torch.uint8, device=dev)
    g_w = torch.empty(1, _lib.WATER_GRAD_WIDTH, device=dev)
    n_ret = sum(f.hits.n for f in frames)
    n_fr = len(frames) + len(cams)

    def fwd_unbatched():
        for s in s1:
            _lib.oceansim_sonar_render(s, P(params), 1, P(refl), n_mat, P(ws_1), ws_1.numel(), stream)
        for u in u1:
            _lib.oceansim_uw_form(u, P(water), 1, P(ws_uf), ws_uf.numel(), stream)

    def step_batched():
        _lib.oceansim_sonar_render(sf, P(params), 1, P(refl), n_mat, P(ws_f), ws_f.numel(), stream)
        _lib.oceansim_uw_form(uf, P(water), 1, P(ws_uf), ws_uf.numel(), stream)
        _lib.oceansim_sonar_render_backward(sb, P(params), 1, P(refl), n_mat, P(g_refl), P(g_par), P(ws_b),
                                            ws_b.numel(), stream)
        _lib.oceansim_uw_form_backward(ub, P(water), 1, P(g_w), P(ws_ub), ws_ub.numel(), stream)

    reps = max(5, steps // 2)
    t_u = median_time(torch, fwd_unbatched, reps, 3)
    t_s = median_time(torch, step_batched, reps, 3)
    plan = osm.Plan(list(zip(geoms, hits)), list(zip(Js, ds, [0] * len(cams))), sonar_params=params, refl=refl,
                    water=water, backward=True, autotune=True)
    for o, a, b in zip(plan.sonar_out, gp, gf):
        o["grad_polar"].copy_(a)
        o["grad_fan"].copy_(b)
    for o, g in zip(plan.camera_out, gi):
        o["grad_out"].copy_(g)

    def plan_step():
        plan.forward()
        plan.backward()
    t_pf = median_time(torch, plan.forward, reps, 3)
    t_ps = median_time(torch, plan_step, reps, 3)
    shape = plan.shape()
    plan.close()
    log("C4 differentiable batch, 32 + 32 frames: unbatched forward %.3f ms; batched forward + backward %.3f ms; "
        "plan forward %.3f ms, forward + backward %.3f ms %s"
        % (t_u * 1e3, t_s * 1e3, t_pf * 1e3, t_ps * 1e3, shape))
    return {"sonar_frames": len(frames), "camera_frames": len(cams), "returns": n_ret,
            "unbatched_fwd_ms": t_u * 1e3, "unbatched_fwd_frames_per_s": n_fr / t_u,
            "batched_fwd_bwd_ms": t_s * 1e3, "batched_fwd_bwd_frames_per_s": n_fr / t_s,
            "plan_fwd_ms": t_pf * 1e3, "plan_fwd_bwd_ms": t_ps * 1e3, "plan_fwd_bwd_frames_per_s": n_fr / t_ps,
            "plan_fwd_bwd_returns_per_s": n_ret / t_ps, "autotuned_shape": shape}


def calibration_run(torch, dev, n_frames, n_steps):
    """Sim-to-real calibration at scale: the targets are rendered with hidden
    parameters (sonar alpha, sigma_phi, sigma_sa, the 64 reflectivities; the
    water row), then Adam (learning rate 1e-2, on the logarithms of the
    parameters) starts from hidden x U[0.5, 1.5] and minimises the mean
    squared error of all polar and camera images through the plan's adjoints.
    G is held fixed (it trades off against the reflectivities); both sides use
    the same speckle draws."""
    import numpy as np
    cs = CalibrationScale(torch, dev, n_frames, autotune=True, losses=False)
    plan = cs.plan
    base = cs.base[0].spec
    hidden_sonar = np.array([base.alpha, base.sigma_phi, base.sigma_sa], np.float64)
    hidden_refl = cs.refl.double().cpu().numpy()
    w = cs.water_h
    hidden_water = np.concatenate([w.beta_d, w.beta_b, w.b_inf]).astype(np.float64)
    t0 = time.perf_counter()
    plan.forward()
    tgt_s = [o["polar"].clone() for o in plan.sonar_out]
    tgt_c = [o["out"].clone() for o in plan.camera_out]
    rng = np.random.default_rng(250301074)
    hidden = (hidden_sonar, hidden_refl, hidden_water)
    starts = [np.asarray(v, np.float64) * rng.uniform(0.5, 1.5, np.shape(v)) for v in hidden]
    start_err = max(float(np.max(np.abs(a - b) / np.abs(b))) for a, b in zip(starts, hidden))
    theta = [torch.tensor(np.log(v), device=dev, requires_grad=True) for v in starts]
    opt = torch.optim.Adam(theta, lr=1e-2)
    scale_s = 1.0 / float(sum((t.double() ** 2).sum() for t in tgt_s))
    scale_c = 1.0 / float(sum((t.double() ** 2).sum() for t in tgt_c))
    loss_dev = torch.zeros((), dtype=torch.float64, device=dev)
    first = None
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for step in range(n_steps):
        with torch.no_grad():
            ps = theta[0].exp()
            cs.params[0, 0], cs.params[0, 2], cs.params[0, 3] = ps[0], ps[1], ps[2]
            cs.refl.copy_(theta[1].exp())
            cs.water[0, :9] = theta[2].exp()
        plan.forward()
        loss_dev.zero_()
        for o, t in zip(plan.sonar_out, tgt_s):
            r = o["polar"] - t
            torch.mul(r, 2.0 * scale_s, out=o["grad_polar"])
            loss_dev += scale_s * torch.dot(r.view(-1), r.view(-1)).double()
        for o, t in zip(plan.camera_out, tgt_c):
            r = o["out"] - t
            torch.mul(r, 2.0 * scale_c, out=o["grad_out"])
            loss_dev += scale_c * torch.dot(r.view(-1), r.view(-1)).double()
        plan.backward()
        if first is None:
            first = float(loss_dev)
        with torch.no_grad():
            g = plan.grad_sonar_params[0]
            theta[0].grad = torch.stack([g[0], g[2], g[3]]).double() * theta[0].exp()
            theta[1].grad = plan.grad_refl.double() * theta[1].exp()
            theta[2].grad = plan.grad_water[0, :9].double() * theta[2].exp()
        opt.step()
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t1
    last = float(loss_dev)
    got = [t.detach().exp().cpu().numpy() for t in theta]
    rel = lambda a, b: np.abs(a - b) / np.abs(b)
    names = ["alpha", "sigma_phi", "sigma_sa"]
    res = {"sonar_frames": n_frames, "camera_frames": n_frames, "steps": n_steps, "optimizer": "Adam lr 1e-2 on log parameters",
           "loss_first": first, "loss_last": last, "loss_reduction": last / first if first else None,
           "loop_s": t_loop, "ms_per_adam_step": t_loop / n_steps * 1e3,
           "rel_err": {**{n: float(v) for n, v in zip(names, rel(got[0], hidden_sonar))},
                       "refl_max": float(rel(got[1], hidden_refl).max()),
                       "refl_median": float(np.median(rel(got[1], hidden_refl))),
                       "beta_d": [float(v) for v in rel(got[2][:3], hidden_water[:3])],
                       "beta_b": [float(v) for v in rel(got[2][3:6], hidden_water[3:6])],
                       "b_inf": [float(v) for v in rel(got[2][6:], hidden_water[6:])]},
           "start_rel_err_max": start_err}
    log("calibration run, %d + %d frames, %d Adam steps in %.2f s (%.2f ms per step): loss %.3e -> %.3e; "
        "relative errors %s" % (n_frames, n_frames, n_steps, t_loop, t_loop / n_steps * 1e3, first, last,
                                res["rel_err"]))
    plan.close()
    return res


def nav_leg(torch, dev, steps):
    """The navigation sensors: the DVL over 512 ticks for 65536 instances
    (vehicles or Monte Carlo runs) with ranges drawn over [0, 100] m, and the
    barometer over 16 M depth samples, with noise."""
    import paper_2503_01074_amd as osm
    g = torch.Generator(device="cpu").manual_seed(11)
    T, N = 512, 65536
    t = torch.cumsum(torch.full((T,), 0.01, dtype=torch.float64), 0).to(dev)
    ranges = (torch.rand(T, N, 4, generator=g) * 100.0).to(dev)
    vel = torch.randn(T, N, 3, generator=g).to(dev)
    depth = (torch.rand(1 << 24, generator=g) * 500.0).to(dev)
    reps = max(5, steps // 2)
    t_dvl = event_time(torch, lambda: osm.dvl(t, ranges, vel, sigma_v=0.01, seed=(1, 2)), reps)
    t_baro = event_time(torch, lambda: osm.barometer(depth, sigma=20.0, seed=(3, 4)), reps)
    log("navigation sensors: DVL %d ticks x %d instances %.1f us (%.2f G updates/s); barometer %d samples "
        "%.1f us" % (T, N, t_dvl * 1e6, T * N / t_dvl / 1e9, depth.numel(), t_baro * 1e6))
    return {"dvl_ticks": T, "dvl_instances": N, "dvl_us": t_dvl * 1e6, "dvl_updates_per_s": T * N / t_dvl,
            "dvl_GBps": round(T * N * (16 + 12 + 12 + 4) / t_dvl / 1e9, 1),
            "barometer_samples": depth.numel(), "barometer_us": t_baro * 1e6,
            "barometer_samples_per_s": depth.numel() / t_baro,
            "barometer_GBps": round(depth.numel() * 8 / t_baro / 1e9, 1)}


def kernel_us(torch, fn, reps):
    """Per-kernel device time of fn (library event tracing): {name: (launches per call, us per call)}."""
    from paper_2503_01074_amd import _lib
    fn()
    torch.cuda.synchronize()
    _lib.oceansim_trace_enable(True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    tr = _lib.oceansim_trace_summary()
    _lib.oceansim_trace_enable(False)
    return {k: (calls / reps, us / reps) for k, (calls, us) in tr.items()}


def raycast_leg(torch, dev, steps):
    """Ray casting of the sonar's returns against the seabed scene (a 256 x 256
    height field over 200 m with 16 boxes: 130242 triangles): the real-time
    pattern (1024 beams x 128 rays over 130 x 20 degrees, 50 m) from one pose,
    and 64 poses of the calibration-scale pattern (2048 x 1024 rays) in one
    call.  Then the sonar forward at real-time settings (1024 x 1024 bins, a
    1024 x 2048 fan, gamma speckle) on the cast returns against the same
    number of uniformly drawn returns: binning structured (beam-ordered)
    input."""
    import math
    import paper_2503_01074_amd as osm
    import workloads as W
    s = W.seabed_scene()
    t0 = time.perf_counter()
    scene = osm.Scene(s.vertices, s.triangles, s.tri_mat)
    t_build = time.perf_counter() - t0
    info = scene.info
    fa, fe = math.radians(130.0), math.radians(20.0)
    pose = W.sonar_pose()
    rt = osm.raycast(scene, [(pose.pos, pose.rot)], 1024, 128, fa, fe, 50.0, device=dev)
    reps = max(10, steps)
    k_rt = kernel_us(torch, lambda: osm.raycast(scene, [(pose.pos, pose.rot)], 1024, 128, fa, fe, 50.0, out=rt),
                     reps)
    t_rt = k_rt["k_raycast"][1] * 1e-6
    hit_rt = float((rt[0].mat >= 0).float().mean())
    poses = [W.sonar_pose(height=4.0 + 8.0 * (i % 8) / 7, pitch_deg=5.0 + 25.0 * (i // 8) / 7,
                          yaw_deg=-60.0 + 120.0 * i / 63) for i in range(64)]
    pp = [(p.pos, p.rot) for p in poses]
    big = osm.raycast(scene, pp, 2048, 1024, fa, fe, 50.0, device=dev)
    k_big = kernel_us(torch, lambda: osm.raycast(scene, pp, 2048, 1024, fa, fe, 50.0, out=big), 3)
    t_big = k_big["k_raycast"][1] * 1e-6
    n_big = 64 * 2048 * 1024
    hit_big = float(sum((h.mat >= 0).sum().item() for h in big) / n_big)
    del big
    torch.cuda.empty_cache()
    log("ray casting: scene of %d triangles built in %.0f ms (depth %d, SAH cost %.1f); 1024 x 128 rays %.1f us "
        "(%.2f G rays/s, %.0f%% hit); 64 x 2048 x 1024 rays %.2f ms (%.2f G rays/s, %.0f%% hit)"
        % (info["n_triangles"], t_build * 1e3, info["depth"], info["sah_cost"], t_rt * 1e6,
           131072 / t_rt / 1e9, 100 * hit_rt, t_big * 1e3, n_big / t_big / 1e9, 100 * hit_big))

    # the sonar forward on the cast returns against uniformly drawn ones
    frame = W.sonar_c2()[0]
    spec = frame.spec
    geom = osm.SonarGeometry.from_spec(spec)
    params = osm.sonar_params([osm.sonar_params_from_spec(spec)], dev)
    rnd = osm.DeviceHits.from_host(frame.hits, dev)
    refl_rnd = torch.as_tensor(frame.hits.refl, device=dev)
    refl_scn = torch.as_tensor(s.refl, device=dev)
    ws = torch.empty(1 << 26, dtype=torch.uint8, device=dev)
    f_cast = kernel_us(torch, lambda: osm.render_sonar([geom], [rt[0]], params, refl_scn, workspace=ws), reps)
    f_rnd = kernel_us(torch, lambda: osm.render_sonar([geom], [rnd], params, refl_rnd, workspace=ws), reps)
    sum_us = lambda d: sum(v[1] for v in d.values())
    log("sonar forward at real-time settings: cast returns %.1f us, uniform returns %.1f us"
        % (sum_us(f_cast), sum_us(f_rnd)))
    scene.close()
    return {"scene_triangles": info["n_triangles"], "bvh_build_ms": round(t_build * 1e3, 1),
            "bvh_depth": info["depth"], "bvh_sah_cost": round(info["sah_cost"], 2),
            "bvh_device_bytes": info["device_bytes"],
            "real_time_rays": 131072, "real_time_us": round(t_rt * 1e6, 2),
            "real_time_rays_per_s": 131072 / t_rt, "real_time_hit_frac": round(hit_rt, 3),
            "calibration_rays": n_big, "calibration_ms": round(t_big * 1e3, 3),
            "calibration_rays_per_s": n_big / t_big, "calibration_hit_frac": round(hit_big, 3),
            "sonar_fwd_cast_returns_us": {k: round(v[1], 2) for k, v in f_cast.items()},
            "sonar_fwd_uniform_returns_us": {k: round(v[1], 2) for k, v in f_rnd.items()}}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(budget_s):
    """The FP64 oracle on this host's cores over a bounded sample of the
    calibration-scale workload: whole frames (one 2,097,152-return sonar frame
    forward + backward and one 1920 x 1080 camera frame forward + backward) for
    about `budget_s` seconds, scaled to returns per second."""
    import oracle
    import workloads as W
    frame = W.sonar_c5(n_frames=1)[0]
    cam = W.make_camera(W.Stream(W.BASE_SEED + 4, 1 << 22), 1080, 1920)
    w = W.make_water(W.Stream(W.BASE_SEED + 4, 1 << 21))
    spec = frame.spec
    cfg = oracle.SonarConfig.from_spec(spec)
    hits = frame.hits
    gp = W.loss_weights((205, 0), (spec.n_range, spec.n_azimuth))
    gi = W.loss_weights((206, 0), cam.J.shape)
    t0 = time.perf_counter()
    n = 0
    while True:
        oracle.sonar_forward(cfg, hits, hits.refl)
        oracle.uw_forward(cam.J, cam.depth, w.beta_d, w.beta_b, w.b_inf)
        oracle.sonar_backward(cfg, hits, hits.refl, gp, None)
        oracle.uw_backward(cam.J, cam.depth, w.beta_d, w.beta_b, w.b_inf, gi, False)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 20:
            break
    return {"value": n * hits.n / el, "unit": "returns/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": "%d sonar frame(s) of the calibration-scale workload (2,097,152 returns, 2048 x 2048 bins, "
                      "forward + backward) each with one 1920 x 1080 camera frame (forward + backward) in %.1f s; "
                      "a full step is 64 of each" % (n, el)}


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
    if args.profile_summary:
        profile_summary(args.profile_summary, args.profile_out)
        return
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
    if args.only == "c2":
        c2_leg(torch, dev, args.steps)
        return
    if args.only == "c3":
        c3_leg(torch, dev, args.steps)
        return
    if args.only == "c4":
        c4_leg(torch, dev, args.steps)
        return
    if args.only == "raycast":
        raycast_leg(torch, dev, args.steps)
        return
    from paper_2503_01074_amd import _lib

    cs = CalibrationScale(torch, dev, args.c5_frames)
    if args.only == "c5":
        t = timed(torch, cs.step, args.steps, args.warmup)
        log("calibration-scale step: %.3f ms" % (t * 1e3))
        return

    # The step: forward + backward of all frames through the plan, K times
    # after W warm-up steps, timed by the host clock between two device
    # synchronisations.
    log("timing %d full steps after %d warm-up" % (args.steps, args.warmup))
    t_step = timed(torch, cs.step, args.steps, args.warmup)
    t_fwd = timed(torch, cs.forward, args.steps, args.warmup)
    log("calibration-scale step %.3f ms, forward %.3f ms" % (t_step * 1e3, t_fwd * 1e3))

    # per-kernel durations: the library brackets each launch with HIP events
    # on its stream while tracing is on
    reps = max(5, args.steps // 2)
    _lib.oceansim_trace_enable(True)
    for _ in range(reps):
        cs.step()
    torch.cuda.synchronize()
    trace = _lib.oceansim_trace_summary()
    _lib.oceansim_trace_enable(False)
    kern_us = {k: us / calls for k, (calls, us) in trace.items()}
    dom = max(kern_us, key=lambda k: kern_us[k] * trace[k][0])
    abytes, fwd_bytes, bwd_bytes = cs.algorithmic_bytes()
    prof = measured_profile()
    dom_bytes = abytes.get(dom)
    achieved = dom_bytes / (kern_us[dom] * 1e-6) / 1e9 if dom_bytes else None
    traffic = None
    valu_frac = None
    if prof and dom in prof:
        traffic = int(prof[dom]["fetch_bytes"] + prof[dom]["write_bytes"])
        if prof[dom].get("valu_insts"):
            valu_frac = round(prof[dom]["valu_insts"] * 64 / (kern_us[dom] * 1e-6) / VALU_PEAK_LANE_OPS, 4)
    roofline = {"bound": "hbm", "kernel": dom,
                "achieved": None if achieved is None else round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "bytes_per_launch": dom_bytes, "launch_us": round(kern_us[dom], 2),
                "valu_frac": valu_frac}
    kernel_table = {}
    for k in sorted(kern_us, key=lambda k: -kern_us[k] * trace[k][0]):
        row = {"calls_per_step": trace[k][0] / reps, "us": round(kern_us[k], 2), "alg_bytes": abytes.get(k),
               "alg_GBps": round(abytes[k] / (kern_us[k] * 1e-6) / 1e9, 1) if k in abytes else None}
        if prof and k in prof:
            row["traffic_bytes"] = int(prof[k]["fetch_bytes"] + prof[k]["write_bytes"])
            if prof[k].get("valu_insts"):
                row["valu_frac"] = round(prof[k]["valu_insts"] * 64 / (kern_us[k] * 1e-6) / VALU_PEAK_LANE_OPS, 3)
        kernel_table[k] = row
    log("kernels (us per launch): " + ", ".join("%s %.1f" % (k, v["us"]) for k, v in kernel_table.items()))
    step_bytes = fwd_bytes + bwd_bytes
    n_ret = cs.n_returns
    n_frames = cs.n_frames
    shape = cs.plan.shape()
    cs.plan.close()
    del cs
    torch.cuda.empty_cache()

    extra = {}
    if not args.no_batched:
        extra["calibration_c5_adam"] = calibration_run(torch, dev, args.c5_frames, args.calib_steps)
        torch.cuda.empty_cache()
        extra["plain_c1"] = c1_leg(torch, dev, args.steps)
        extra["real_time_c2"] = c2_leg(torch, dev, args.steps)
        torch.cuda.empty_cache()
        extra["batched_c3"] = c3_leg(torch, dev, args.steps)
        torch.cuda.empty_cache()
        extra["batched_c4"] = c4_leg(torch, dev, args.steps)
        torch.cuda.empty_cache()
        extra["camera_io"] = camera_io_leg(torch, dev, args.steps)
        extra["navigation"] = nav_leg(torch, dev, args.steps)
        extra["ray_casting"] = raycast_leg(torch, dev, args.steps)
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu:
        log("timing the FP64 oracle on the host")
        cpu = cpu_baseline(args.cpu_seconds)

    line = {
        "metric": "sonar returns/s + frames/s (fwd, fwd+bwd, batched vs plain) at <=1e-5 rel err",
        "value": n_ret / t_step,
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
        "config": {"workload": "calibration scale: %d sonar frames x 2,097,152 returns (2048 beams x 1024 rays, "
                               "r in [0.5,50) m, 64 materials, gamma speckle k=4), 2048x2048 polar bins, no fan, "
                               "plus Eq. 1 on %d RGB frames of 1920x1080; forward + backward (polar and image "
                               "losses) through one autotuned plan" % (n_frames, n_frames),
                   "global_batch": 2 * n_frames, "parallelism": "none (1 GPU)"},
        "path": "plan (frames prepared once, autotuned launch shapes; backward from the forward's material pairs)",
        "frames_per_s": 2 * n_frames / t_step,
        "fwd_ms": t_fwd * 1e3,
        "fwd_returns_per_s": n_ret / t_fwd,
        "fwd_frames_per_s": 2 * n_frames / t_fwd,
        "step_alg_bytes": step_bytes,
        "step_hbm_frac": round(step_bytes / t_step / (HBM_PEAK_GBS * 1e9), 4),
        "fwd_hbm_frac": round(fwd_bytes / t_fwd / (HBM_PEAK_GBS * 1e9), 4),
        "autotuned_shape": shape,
        "copy_GBps": copy_rate(torch, dev),
        "kernels": kernel_table,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
