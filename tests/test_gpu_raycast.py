"""GPU parity of the ray caster (the returns of Sec. III-A.2 come from ray
tracing the scene) against the oracle's brute-force FP64 caster, through the
C ABI.

Bar: on every ray the oracle does not flag as ambiguous (band 1e-4: a hit
within 1e-4 barycentric units of a triangle edge, two surfaces closer than
1e-4 t, a sliver, a grazing hit) the material id is bit-exact; the hit point
agrees within 1e-5 of the hit distance (single-precision Moller-Trumbore
against the double-precision signed-volume test: both round the same
float32 vertices); the unit normal within 1e-5.  (The oracle also flags rays
that pass within the band of an edge of a triangle they miss in front of
their hit, and hits within the band of the casting distance.)  The full-size case (1024 x 128 rays, the
real-time sonar pattern, against the 130 k-triangle seabed) is compared on a
sample of 1024 rays the oracle casts one by one."""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

FOV_AZ, FOV_EL = math.radians(130.0), math.radians(20.0)
BAND = 1e-4


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def _gpu(scene, poses, nb, nr, t_max, fov_az=FOV_AZ, fov_el=FOV_EL):
    import torch
    import paper_2503_01074_amd as osm
    hits = osm.raycast(scene, [(p.pos, p.rot) for p in poses], nb, nr, fov_az, fov_el, t_max)
    torch.cuda.synchronize()
    return [{k: getattr(h, k).cpu().numpy() for k in ("x", "y", "z", "nx", "ny", "nz", "mat")} for h in hits]


def _compare(got, want, t_max, sel=None):
    """Parity on the rays the oracle decides; returns how many were compared."""
    g = {k: (v if sel is None else v[sel]) for k, v in got.items()}
    pw = np.stack([want["x"], want["y"], want["z"]], 1)
    t_o = np.linalg.norm(pw, axis=1)
    ok = ~want["ambiguous"]
    np.testing.assert_array_equal(g["mat"][ok], want["mat"][ok])
    hit = ok & (want["mat"] >= 0)
    pg = np.stack([g["x"], g["y"], g["z"]], 1).astype(np.float64)
    err = np.linalg.norm(pg[hit] - pw[hit], axis=1)
    assert np.all(err <= 1e-5 * np.maximum(t_o[hit], 1.0)), float(np.max(err / np.maximum(t_o[hit], 1.0)))
    ng = np.stack([g["nx"], g["ny"], g["nz"]], 1).astype(np.float64)
    nw = np.stack([want["nx"], want["ny"], want["nz"]], 1)
    assert np.all(np.abs(ng[hit] - nw[hit]) <= 1e-5)
    miss = ok & (want["mat"] < 0)
    for k in ("x", "y", "z", "nx", "ny", "nz"):
        assert np.all(g[k][miss] == 0.0)
    return int(ok.sum()), int((~ok).sum())


def _oracle(s, pose, nb, nr, t_max, sel=None, fov_az=FOV_AZ, fov_el=FOV_EL):
    return oracle.raycast(s.vertices, s.triangles, s.tri_mat, pose.pos, pose.rot, nb, nr, fov_az, fov_el, t_max,
                          band=BAND, sel=sel)


def test_small_seabed_every_ray():
    import paper_2503_01074_amd as osm
    _say("ray cast: small seabed (32 x 32 grid, 4 boxes), 128 x 32 rays, every ray")
    s = W.seabed_scene(seed=W.BASE_SEED + 11, n=32, extent=120.0, n_boxes=4)
    pose = W.sonar_pose(height=6.0, pitch_deg=18.0)
    sc = osm.Scene(s.vertices, s.triangles, s.tri_mat)
    got = _gpu(sc, [pose], 128, 32, 60.0)[0]
    want = _oracle(s, pose, 128, 32, 60.0)
    n_ok, n_amb = _compare(got, want, 60.0)
    assert n_ok > 0.9 * 128 * 32 and (want["mat"] >= 0).sum() > 1000
    _say("compared %d rays, %d ambiguous" % (n_ok, n_amb))


@pytest.mark.parametrize("yaw, pitch, height", [(0.0, 15.0, 8.0), (37.0, 30.0, 4.0), (-120.0, 5.0, 12.0)])
def test_full_size_seabed_sampled(yaw, pitch, height):
    import paper_2503_01074_amd as osm
    _say("ray cast: seabed 256 x 256 + 16 boxes, 1024 x 128 rays, yaw %g pitch %g height %g" % (yaw, pitch, height))
    s = W.seabed_scene()
    pose = W.sonar_pose(height=height, pitch_deg=pitch, yaw_deg=yaw)
    sc = osm.Scene(s.vertices, s.triangles, s.tri_mat)
    assert sc.info["n_triangles"] == s.triangles.shape[0] and sc.info["depth"] <= 32
    got = _gpu(sc, [pose], 1024, 128, 50.0)[0]
    rs = np.random.default_rng(abs(int(yaw * 10)) + 7)
    sel = np.concatenate([rs.choice(1024 * 128, 1000, replace=False), [0, 127, 128, 1024 * 128 - 1]])
    want = _oracle(s, pose, 1024, 128, 50.0, sel=sel)
    n_ok, _ = _compare(got, want, 50.0, sel=sel)
    assert n_ok > 900
    # every return lies within the casting distance; misses are exactly zero
    t = np.sqrt(got["x"].astype(np.float64) ** 2 + got["y"] ** 2 + got["z"] ** 2)
    assert np.all(t[got["mat"] >= 0] <= 50.0 * (1 + 1e-6)) and np.all(t[got["mat"] < 0] == 0.0)
    assert np.all(np.abs(np.sqrt(got["nx"].astype(np.float64) ** 2 + got["ny"] ** 2 + got["nz"] ** 2)
                         [got["mat"] >= 0] - 1.0) < 1e-5)


def test_closed_forms_plane_and_wall():
    import paper_2503_01074_amd as osm
    _say("ray cast: plane below, wall ahead")
    sq = np.array([[-500, -500, -5], [500, -500, -5], [500, 500, -5], [-500, 500, -5]], np.float32)
    sc = osm.Scene(sq, np.array([[0, 1, 2], [0, 2, 3]], np.int32), np.array([7, 7], np.int32))
    ident = W.SonarPose(np.zeros(3, np.float32), np.eye(3, dtype=np.float32))
    g = _gpu(sc, [ident], 16, 8, 1000.0)[0]
    az = np.repeat(-0.5 * FOV_AZ + (np.arange(16) + 0.5) * FOV_AZ / 16, 8)
    el = np.tile(-0.5 * FOV_EL + (np.arange(8) + 0.5) * FOV_EL / 8, 16)
    down = el < 0
    tt = 5.0 / -np.sin(el[down])
    np.testing.assert_allclose(g["z"][down], -5.0, rtol=2e-6)
    np.testing.assert_allclose(g["x"][down], tt * np.cos(el[down]) * np.cos(az[down]), rtol=2e-6, atol=2e-5)
    assert np.all(g["mat"][down] == 7) and np.all(g["mat"][~down] == -1)
    np.testing.assert_allclose(g["nz"][down], 1.0, rtol=1e-6)
    assert np.all(g["nx"][down] == 0.0) and np.all(g["ny"][down] == 0.0)
    # beyond the casting distance: a miss
    g = _gpu(sc, [ident], 16, 8, 50.0)[0]
    np.testing.assert_array_equal(g["mat"][down], np.where(tt <= 50.0, 7, -1))
    assert 0 < (g["mat"] == 7).sum() < down.sum()
    bv, bt = W.box_mesh((10.0, -60.0, -60.0), (12.0, 60.0, 60.0))
    sc = osm.Scene(bv.astype(np.float32), bt.astype(np.int32), np.full(12, 3, np.int32))
    g = _gpu(sc, [ident], 16, 8, 1000.0)[0]
    np.testing.assert_allclose(g["x"], 10.0, rtol=2e-6)
    np.testing.assert_allclose(g["nx"], -1.0, rtol=1e-6)
    assert np.all(g["mat"] == 3)


def test_batched_poses_equal_single_casts_bitwise():
    import paper_2503_01074_amd as osm
    _say("ray cast: 19 poses in one call (two launches) against one at a time")
    s = W.seabed_scene(seed=W.BASE_SEED + 12, n=64, extent=150.0, n_boxes=6)
    sc = osm.Scene(s.vertices, s.triangles, s.tri_mat)
    poses = [W.sonar_pose(height=3.0 + 0.5 * i, pitch_deg=5.0 + 2.0 * i, yaw_deg=-90.0 + 10.0 * i)
             for i in range(19)]
    batch = _gpu(sc, poses, 96, 40, 70.0)
    for i, p in enumerate(poses):
        one = _gpu(sc, [p], 96, 40, 70.0)[0]
        for k in one:
            np.testing.assert_array_equal(batch[i][k], one[k])
    # bitwise repeatable
    again = _gpu(sc, poses[:3], 96, 40, 70.0)
    for i in range(3):
        for k in again[i]:
            np.testing.assert_array_equal(again[i][k], batch[i][k])


def test_ragged_patterns_in_one_call():
    import torch
    import paper_2503_01074_amd as osm
    from paper_2503_01074_amd import _lib
    _say("ray cast: ragged patterns (1 x 1, 7 x 3, 300 x 17) in one call")
    s = W.seabed_scene(seed=W.BASE_SEED + 13, n=48, extent=100.0, n_boxes=3)
    sc = osm.Scene(s.vertices, s.triangles, s.tri_mat)
    pose = W.sonar_pose(height=5.0, pitch_deg=12.0)
    shapes = [(1, 1), (7, 3), (300, 17)]
    frames = (_lib.RayFrame * 3)()
    outs = []
    for i, (nb, nr) in enumerate(shapes):
        n = nb * nr
        o = {k: torch.full((n,), 7.0, device="cuda") for k in ("x", "y", "z", "nx", "ny", "nz")}
        o["mat"] = torch.full((n,), 99, dtype=torch.int32, device="cuda")
        outs.append(o)
        fr = frames[i]
        fr.pos[:] = [float(v) for v in pose.pos]
        fr.rot[:] = [float(v) for v in pose.rot.reshape(-1)]
        fr.n_beams, fr.n_rays, fr.fov_az, fr.fov_el, fr.t_max = nb, nr, FOV_AZ, FOV_EL, 45.0
        for k in o:
            setattr(fr, k, o[k].data_ptr())
    _lib.oceansim_raycast(sc.handle, frames, 3, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    for (nb, nr), o in zip(shapes, outs):
        want = _oracle(s, pose, nb, nr, 45.0)
        _compare({k: v.cpu().numpy() for k, v in o.items()}, want, 45.0)


def test_empty_and_degenerate_scenes_miss_everywhere():
    import paper_2503_01074_amd as osm
    _say("ray cast: empty scene, needles only")
    ident = W.SonarPose(np.zeros(3, np.float32), np.eye(3, dtype=np.float32))
    sc = osm.Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), np.zeros(0, np.int32))
    g = _gpu(sc, [ident], 8, 4, 100.0)[0]
    assert np.all(g["mat"] == -1) and np.all(g["x"] == 0.0)
    # a needle 10 m long and 1e-7 m wide straight ahead: dropped at build
    nv = np.array([[5.0, -5e-8, -5.0], [5.0, 0.0, 5.0], [5.0, 5e-8, -5.0]], np.float32)
    sc = osm.Scene(nv, np.array([[0, 1, 2]], np.int32), np.array([1], np.int32))
    assert sc.info["n_dropped"] == 1 and sc.info["n_triangles"] == 0
    g = _gpu(sc, [ident], 8, 4, 100.0)[0]
    assert np.all(g["mat"] == -1)


def test_raycast_validation_through_the_abi():
    import torch
    import paper_2503_01074_amd as osm
    from paper_2503_01074_amd import _lib
    _say("ray cast: argument validation")
    s = W.seabed_scene(seed=W.BASE_SEED + 14, n=8, extent=20.0, n_boxes=1)
    sc = osm.Scene(s.vertices, s.triangles, s.tri_mat)
    m = torch.empty(4, dtype=torch.int32, device="cuda")
    fr = (_lib.RayFrame * 1)()
    fr[0].rot[:] = [1, 0, 0, 0, 1, 0, 0, 0, 1]
    fr[0].n_beams, fr[0].n_rays, fr[0].fov_az, fr[0].fov_el, fr[0].t_max = 2, 2, 1.0, 0.2, 10.0
    fr[0].mat = m.data_ptr()
    st = torch.cuda.current_stream().cuda_stream
    assert _lib.lib.oceansim_raycast(sc.handle, fr, 1, st) == 0
    for field, val, code in (("t_max", 0.0, -1), ("t_max", float("inf"), -1), ("fov_el", 3.5, -1),
                             ("fov_az", -0.1, -1), ("n_rays", -1, -2)):
        old = getattr(fr[0], field)
        setattr(fr[0], field, val)
        assert _lib.lib.oceansim_raycast(sc.handle, fr, 1, st) == code, field
        setattr(fr[0], field, old)
    fr[0].mat = None
    assert _lib.lib.oceansim_raycast(sc.handle, fr, 1, st) == -1
    fr[0].mat = m.data_ptr() + 2
    assert _lib.lib.oceansim_raycast(sc.handle, fr, 1, st) == -1
    assert _lib.lib.oceansim_raycast(None, fr, 1, st) == -1
    torch.cuda.synchronize()


def test_deepest_hierarchy_full_stack():
    import paper_2503_01074_amd as osm
    _say("ray cast: chain + cluster mesh (depth 32), sensor below the cluster looking up")
    v, t = W.chain_and_cluster_mesh()
    m = (np.arange(t.shape[0]) % 61).astype(np.int32)
    sc = osm.Scene(v, t, m)
    assert sc.info["depth"] == 32
    s = W.Scene(v, t, m, np.ones(61, np.float32))
    # sensor x axis pointing up (+z), 3 m below the unit cube's centre
    up = np.array([[0.0, 0.0, -1.0], [0.0, 1.0, 0.0], [1.0, 0.0, 0.0]], np.float32)
    pose = W.SonarPose(np.array([0.5, 0.5, -3.0], np.float32), up)
    fa, fe = math.radians(16.0), math.radians(16.0)   # the footprint stays inside the cluster
    got = _gpu(sc, [pose], 64, 32, 20.0, fov_az=fa, fov_el=fe)[0]
    sel = np.random.default_rng(3).choice(64 * 32, 400, replace=False)
    want = _oracle(s, pose, 64, 32, 20.0, sel=sel, fov_az=fa, fov_el=fe)
    n_ok, _ = _compare(got, want, 20.0, sel=sel)
    assert n_ok > 300 and (want["mat"] >= 0).sum() > 300
