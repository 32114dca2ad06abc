"""Pins of the oracle's ray caster (the returns of Sec. III-A.2 come from the
renderer's ray tracing): closed-form hits on planes and boxes, a tessellated
sphere bounded by the analytic sphere, invariance under a rigid motion of
scene and sensor together, independence of triangle order, the nearest of
two surfaces, and subsets of returns."""
import math

import numpy as np

import oracle
import workloads as W

FOV_AZ, FOV_EL = math.radians(130.0), math.radians(20.0)


def _pattern(nb, nr):
    az = -0.5 * FOV_AZ + (np.arange(nb) + 0.5) * FOV_AZ / nb
    el = -0.5 * FOV_EL + (np.arange(nr) + 0.5) * FOV_EL / nr
    A, E = np.meshgrid(az, el, indexing="ij")
    return A.ravel(), E.ravel()


def _square(z, half, mat, up=True):
    v = np.array([[-half, -half, z], [half, -half, z], [half, half, z], [-half, half, z]], np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]] if up else [[0, 2, 1], [0, 3, 2]], np.int32)
    return v, t, np.full(2, mat, np.int32)


def _cast(v, t, m, pos=(0, 0, 0), rot=np.eye(3), nb=16, nr=8, t_max=1000.0, sel=None):
    return oracle.raycast(v, t, m, np.asarray(pos, np.float32), np.asarray(rot, np.float32), nb, nr, FOV_AZ, FOV_EL,
                          t_max, sel=sel)


def test_plane_below_closed_form():
    v, t, m = _square(-5.0, 500.0, 7)
    h = _cast(v, t, m)
    az, el = _pattern(16, 8)
    down = el < 0
    tt = 5.0 / -np.sin(el[down])
    np.testing.assert_allclose(h["z"][down], -5.0, rtol=1e-12)
    np.testing.assert_allclose(h["x"][down], tt * np.cos(el[down]) * np.cos(az[down]), rtol=1e-12)
    np.testing.assert_allclose(h["y"][down], tt * np.cos(el[down]) * np.sin(az[down]), rtol=1e-12, atol=1e-12)
    assert np.all(h["mat"][down] == 7) and np.all(h["mat"][~down] == -1)
    n = np.stack([h["nx"], h["ny"], h["nz"]], 1)[down]
    np.testing.assert_allclose(n, np.broadcast_to([0.0, 0.0, 1.0], n.shape), atol=1e-15)
    assert np.all(h["x"][~down] == 0.0)
    # beyond the casting distance: a miss
    far = _cast(v, t, m, t_max=100.0)
    np.testing.assert_array_equal(far["mat"][down], np.where(tt <= 100.0, 7, -1))


def test_wall_ahead_closed_form_and_outward_normal():
    bv, bt = W.box_mesh((10.0, -60.0, -60.0), (12.0, 60.0, 60.0))
    h = _cast(bv.astype(np.float32), bt.astype(np.int32), np.full(12, 3, np.int32))
    az, el = _pattern(16, 8)
    tt = 10.0 / (np.cos(el) * np.cos(az))
    np.testing.assert_allclose(h["x"], 10.0, rtol=1e-12)
    np.testing.assert_allclose(np.hypot(np.hypot(h["x"], h["y"]), h["z"]), tt, rtol=1e-12)
    n = np.stack([h["nx"], h["ny"], h["nz"]], 1)
    np.testing.assert_allclose(n, np.broadcast_to([-1.0, 0.0, 0.0], n.shape), atol=1e-15)
    assert np.all(h["mat"] == 3)


def test_sphere_tessellation_lies_within_the_sphere():
    c, rad = np.array([15.0, 0.0, 0.0]), 3.0
    nlat, nlon = 24, 48
    th = np.linspace(0, np.pi, nlat + 1)
    ph = np.linspace(0, 2 * np.pi, nlon + 1)[:-1]
    verts = [c + rad * np.array([np.sin(a) * np.cos(b), np.sin(a) * np.sin(b), np.cos(a)]) for a in th for b in ph]
    tris = []
    for i in range(nlat):
        for j in range(nlon):
            a, b = i * nlon + j, i * nlon + (j + 1) % nlon
            cc, d = (i + 1) * nlon + j, (i + 1) * nlon + (j + 1) % nlon
            tris += [(a, cc, d), (a, d, b)]
    v = np.asarray(verts, np.float32)
    t = np.asarray(tris, np.int32)
    h = _cast(v, t, np.zeros(len(tris), np.int32), nb=64, nr=32)
    az, el = _pattern(64, 32)
    d = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], 1)
    # analytic sphere: |t d - c| = rad
    bq = d @ c
    disc = bq ** 2 - (c @ c - rad ** 2)
    hit = h["mat"] >= 0
    assert np.all(disc[hit] >= -1e-9), "a hit outside the sphere's shadow"
    t_sph = bq[hit] - np.sqrt(np.maximum(disc[hit], 0.0))
    p = np.stack([h["x"], h["y"], h["z"]], 1)[hit]
    t_poly = np.linalg.norm(p, axis=1)
    assert np.all(t_poly >= t_sph - 1e-6)
    r_hit = np.linalg.norm(p - c, axis=1)
    inner = rad * math.cos(math.pi / nlat) * math.cos(math.pi / nlon)   # the polyhedron's inner bound
    assert np.all(r_hit <= rad + 1e-5) and np.all(r_hit >= inner - 1e-5)
    # rays well inside the sphere's shadow all hit
    assert np.all(hit[disc > 0.2 * rad ** 2])


def test_rigid_motion_of_scene_and_sensor():
    s = W.seabed_scene(seed=5, n=24, extent=60.0, n_boxes=3)
    pose = W.sonar_pose(height=6.0, pitch_deg=20.0)
    a = _cast(s.vertices, s.triangles, s.tri_mat, pose.pos, pose.rot, nb=32, nr=8)
    yaw = math.radians(37.0)
    Rz = np.array([[math.cos(yaw), -math.sin(yaw), 0], [math.sin(yaw), math.cos(yaw), 0], [0, 0, 1]])
    shift = np.array([3.0, -2.0, 0.5])
    v2 = (s.vertices.astype(np.float64) @ Rz.T + shift).astype(np.float32)
    b = _cast(v2, s.triangles, s.tri_mat, (Rz @ pose.pos.astype(np.float64) + shift).astype(np.float32),
              (Rz @ pose.rot.astype(np.float64)).astype(np.float32), nb=32, nr=8)
    ok = ~(a["ambiguous"] | b["ambiguous"])
    np.testing.assert_array_equal(a["mat"][ok], b["mat"][ok])
    for k in ("x", "y", "z", "nx", "ny", "nz"):
        np.testing.assert_allclose(a[k][ok], b[k][ok], rtol=1e-4, atol=1e-4)


def test_order_nearest_and_subsets():
    v1, t1, m1 = _square(-5.0, 2000.0, 1)
    v2, t2, m2 = _square(-8.0, 2000.0, 2)
    v = np.concatenate([v2, v1])
    t = np.concatenate([t2, t1 + 4])
    m = np.concatenate([m2, m1])
    h = _cast(v, t, m)
    _, el = _pattern(16, 8)
    assert np.all(h["mat"][el < 0] == 1)
    # triangle order does not matter
    perm = np.array([3, 1, 0, 2])
    h2 = _cast(v, t[perm], m[perm])
    for k in ("x", "y", "z", "mat"):
        np.testing.assert_array_equal(h[k], h2[k])
    # a subset of returns is the same as those returns of the full cast
    sel = np.array([5, 0, 77, 127, 64])
    hs = _cast(v, t, m, sel=sel)
    for k in ("x", "y", "z", "nx", "ny", "nz", "mat"):
        np.testing.assert_array_equal(hs[k], h[k][sel])


def test_ambiguity_flags_shared_edges_slivers_and_grazing():
    # sensor x axis pointing straight down: the one ray of a 1 x 1 pattern
    down = np.array([[0.0, 0.0, 1.0], [0.0, 1.0, 0.0], [-1.0, 0.0, 0.0]])
    v, t, m = _square(-5.0, 50.0, 4)
    one = oracle.raycast(v, t, m, np.zeros(3, np.float32), down.astype(np.float32), 1, 1, 0.0, 0.0, 100.0)
    # the hit (0, 0, -5) lies on the square's diagonal, the edge both triangles share
    assert one["mat"][0] == 4 and one["ambiguous"][0]
    np.testing.assert_allclose([one["x"][0], one["y"][0], one["z"][0]], [5.0, 0.0, 0.0], rtol=1e-15)
    off = oracle.raycast(v, t, m, np.array([3.0, -7.0, 0.0], np.float32), down.astype(np.float32), 1, 1, 0.0, 0.0,
                         100.0)
    assert off["mat"][0] == 4 and not off["ambiguous"][0]
    # a small triangle in front of the square whose edge the ray passes 1e-6 m
    # beside: a near miss, flagged; 1e-3 m beside: decided
    for gap, flagged in ((1e-6, True), (1e-3, False)):
        tv = np.array([[3.0 + gap, -8.0, -2.0], [3.0 + gap, -6.0, -2.0], [4.0, -7.0, -2.0]], np.float32)
        vv = np.concatenate([v, tv])
        tt = np.concatenate([t, [[4, 5, 6]]]).astype(np.int32)
        mm = np.concatenate([m, [8]]).astype(np.int32)
        nm = oracle.raycast(vv, tt, mm, np.array([3.0, -7.0, 0.0], np.float32), down.astype(np.float32), 1, 1, 0.0,
                            0.0, 100.0)
        assert nm["mat"][0] == 4 and bool(nm["ambiguous"][0]) == flagged
    # a hit just inside the casting distance is flagged; well inside it is not
    lim = oracle.raycast(v, t, m, np.array([3.0, -7.0, 0.0], np.float32), down.astype(np.float32), 1, 1, 0.0, 0.0,
                         5.00001)
    assert lim["mat"][0] == 4 and lim["ambiguous"][0]
    # and a square just beyond it: a miss, flagged
    lim = oracle.raycast(v, t, m, np.array([3.0, -7.0, 0.0], np.float32), down.astype(np.float32), 1, 1, 0.0, 0.0,
                         4.99999)
    assert lim["mat"][0] == -1 and lim["ambiguous"][0]
    # a needle 10 m long and 1e-7 m wide under the ray: hit, flagged as a sliver
    sv = np.array([[-5.0, -5e-8, -5.0], [5.0, 0.0, -5.0], [-5.0, 5e-8, -5.0]], np.float32)
    st = np.array([[0, 1, 2]], np.int32)
    h = oracle.raycast(sv, st, np.array([9], np.int32), np.zeros(3, np.float32), down.astype(np.float32), 1, 1,
                       0.0, 0.0, 100.0)
    assert h["mat"][0] == 9 and h["ambiguous"][0]
    # the same needle beside the ray: a clean miss
    h = oracle.raycast(sv, st, np.array([9], np.int32), np.array([0.0, 1e-3, 0.0], np.float32),
                       down.astype(np.float32), 1, 1, 0.0, 0.0, 100.0)
    assert h["mat"][0] == -1
    # a wall through (20, 0, 0) turned 1e-4 degrees out of the ray's vertical plane: grazing, flagged
    tg = math.tan(math.radians(1e-4))
    wv = np.array([[-50.0, -70.0 * tg, -50.0], [100.0, 80.0 * tg, -50.0], [20.0, 0.0, 50.0]], np.float32)
    gh = _cast(wv, np.array([[0, 1, 2]], np.int32), np.array([2], np.int32), nb=1, nr=1)
    assert gh["mat"][0] == 2 and gh["ambiguous"][0]
    assert abs(gh["x"][0] - 20.0) < 0.1
