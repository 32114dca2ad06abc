// Ray casting of the imaging sonar's returns on gfx950 (Sec. III-A.2 of
// arXiv 2503.01074 obtains the returns by ray tracing the scene): closest
// hits of a beam x elevation ray pattern against a triangle mesh in a binary
// bounding-volume hierarchy (built on the host, bvh.cpp).
//
//   k_raycast  one thread per ray.  Stack-based ordered traversal: an inner
//              node holds both child boxes (one 64-byte fetch tests both), the
//              nearer child is taken first and the other deferred on a
//              per-thread stack in LDS (thread-minor, so a wave's stack
//              accesses are conflict-free); leaves hold at most 8 triangles,
//              each tested with the Moller-Trumbore algorithm in single
//              precision.  The hit point is written as t times the
//              sensor-frame direction, the normal as R^T of the hit
//              triangle's unit normal: the return buffers the sonar image
//              formation reads.
//
// Several poses go in one launch (grid.y = pose); their descriptors travel in
// the kernel arguments, so a cast allocates nothing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/oceansim.h"
#include "device.hpp"
#include "host.hpp"
#include "launch.hpp"
#include "scene.hpp"

struct oceansim_scene {
    int device = 0;
    osim::BvhNode *nodes = nullptr;
    osim::BvhTri *tris = nullptr;
    int root = 0;
    int empty = 1;
    oceansim_scene_info info{};
};

namespace osim {
namespace {

constexpr int kRayThreads = 128;
constexpr int kRayFramesPerLaunch = 16;
constexpr float kSlabWiden = 1.00000036f;   // 1 + 2 gamma_3, gamma_n = n eps / (1 - n eps), eps = 2^-24

struct RayFrameDev {
    float o[3];
    float R[9];
    float az0, daz, el0, del, t_max;
    int nb, nr, n;
    gptr<float> x, y, z, nx, ny, nz;
    gptr<int> mat;
};

struct RayGroup {
    RayFrameDev f[kRayFramesPerLaunch];
};
static_assert(sizeof(RayGroup) <= 3072, "ray-cast kernel arguments");

__device__ __forceinline__ float4 ld4(gptr<const float4> p) { return gload(p); }

template <int NT>
__global__ __launch_bounds__(NT) void k_raycast(RayGroup g, gptr<const float4> nodes, gptr<const float4> tris,
                                                int root, int empty) {
    __shared__ int stk[kBvhMaxDepth * NT];
    const RayFrameDev &f = g.f[blockIdx.y];
    const int tid = threadIdx.x;
    const int k = blockIdx.x * NT + tid;
    if (k >= f.n) return;
    const int b = k / f.nr;
    const int r = k - b * f.nr;
    const float az = f.az0 + ((float)b + 0.5f) * f.daz;
    const float el = f.el0 + ((float)r + 0.5f) * f.del;
    float sa, ca, se, ce;
    sincosf(az, &sa, &ca);
    sincosf(el, &se, &ce);
    const float s0 = ce * ca, s1 = ce * sa, s2 = se;   // sensor frame
    const float d0 = f.R[0] * s0 + f.R[1] * s1 + f.R[2] * s2;
    const float d1 = f.R[3] * s0 + f.R[4] * s1 + f.R[5] * s2;
    const float d2 = f.R[6] * s0 + f.R[7] * s1 + f.R[8] * s2;
    const float o0 = f.o[0], o1 = f.o[1], o2 = f.o[2];
    // reciprocal direction; a zero component becomes a tiny one of its sign
    // (the box margins make that harmless), keeping the slab products finite
    auto safe = [](float v) { return fabsf(v) > kMinDirComponent ? v : copysignf(kMinDirComponent, v); };
    const float i0 = 1.0f / safe(d0), i1 = 1.0f / safe(d1), i2 = 1.0f / safe(d2);

    float tbest = f.t_max;
    int hit = -1;
    // Entry distance of a box when the ray meets it before tbest, else +inf.
    // The slab distances are (plane - origin) / direction, each off by at most
    // about two roundings; widening the far end by 1 + 2 gamma_3 (Ize, Robust
    // BVH Ray Traversal, JCGT 2013) keeps the test conservative, including
    // for boxes of zero thickness.
    auto slab = [&](float lx, float ly, float lz, float hx, float hy, float hz) {
        const float ax = (lx - o0) * i0, bx = (hx - o0) * i0;
        const float ay = (ly - o1) * i1, by = (hy - o1) * i1;
        const float az_ = (lz - o2) * i2, bz = (hz - o2) * i2;
        const float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az_, bz), 0.0f));
        const float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az_, bz), tbest));
        return tn <= tf * kSlabWiden ? tn : INFINITY;
    };

    int ref = root;
    int sp = 0;
    if (!empty) {
        while (true) {
            if (ref >= 0) {
                const gptr<const float4> nd = nodes + 4LL * ref;
                const float4 a = ld4(nd), bq = ld4(nd + 1), c = ld4(nd + 2);
                const int4 rr = gload((gptr<const int4>)(nd + 3));
                const float t0 = slab(a.x, a.y, a.z, a.w, bq.x, bq.y);
                const float t1 = slab(bq.z, bq.w, c.x, c.y, c.z, c.w);
                const bool h0 = t0 < INFINITY, h1 = t1 < INFINITY;
                if (h0 && h1) {
                    const bool swap = t1 < t0;
                    ref = swap ? rr.y : rr.x;
                    stk[sp * NT + tid] = swap ? rr.x : rr.y;
                    ++sp;
                    continue;
                }
                if (h0 || h1) {
                    ref = h0 ? rr.x : rr.y;
                    continue;
                }
            } else {
                const int code = ~ref;
                const int first = code >> kLeafShift;
                const int cnt = (code & (kLeafMax - 1)) + 1;
                for (int i = 0; i < cnt; ++i) {
                    const gptr<const float4> tp = tris + 3LL * (first + i);
                    const float4 A = ld4(tp), E1 = ld4(tp + 1), E2 = ld4(tp + 2);
                    // Moller-Trumbore: p = d x e2, det = e1 . p
                    const float p0 = d1 * E2.z - d2 * E2.y;
                    const float p1 = d2 * E2.x - d0 * E2.z;
                    const float p2 = d0 * E2.y - d1 * E2.x;
                    const float det = E1.x * p0 + E1.y * p1 + E1.z * p2;
                    const float inv = 1.0f / det;
                    const float q0 = o0 - A.x, q1 = o1 - A.y, q2 = o2 - A.z;
                    const float u = (q0 * p0 + q1 * p1 + q2 * p2) * inv;
                    const float c0 = q1 * E1.z - q2 * E1.y;
                    const float c1 = q2 * E1.x - q0 * E1.z;
                    const float c2 = q0 * E1.y - q1 * E1.x;
                    const float v = (d0 * c0 + d1 * c1 + d2 * c2) * inv;
                    const float t = (E2.x * c0 + E2.y * c1 + E2.z * c2) * inv;
                    if (det != 0.0f && u >= 0.0f && v >= 0.0f && u + v <= 1.0f && t > 0.0f && t <= tbest &&
                        (hit < 0 || t < tbest)) {
                        tbest = t;
                        hit = first + i;
                    }
                }
            }
            if (sp == 0) break;
            --sp;
            ref = stk[sp * NT + tid];
        }
    }
    float px = 0.0f, py = 0.0f, pz = 0.0f, wx = 0.0f, wy = 0.0f, wz = 0.0f;
    int m = -1;
    if (hit >= 0) {
        const gptr<const float4> tp = tris + 3LL * hit;
        const float4 A = ld4(tp), E1 = ld4(tp + 1), E2 = ld4(tp + 2);
        const float n0 = E1.y * E2.z - E1.z * E2.y;
        const float n1 = E1.z * E2.x - E1.x * E2.z;
        const float n2 = E1.x * E2.y - E1.y * E2.x;
        const float il = 1.0f / sqrtf(n0 * n0 + n1 * n1 + n2 * n2);
        const float w0 = n0 * il, w1 = n1 * il, w2 = n2 * il;
        wx = f.R[0] * w0 + f.R[3] * w1 + f.R[6] * w2;
        wy = f.R[1] * w0 + f.R[4] * w1 + f.R[7] * w2;
        wz = f.R[2] * w0 + f.R[5] * w1 + f.R[8] * w2;
        px = tbest * s0;
        py = tbest * s1;
        pz = tbest * s2;
        m = __float_as_int(A.w);
    }
    if (f.x) f.x[k] = px;
    if (f.y) f.y[k] = py;
    if (f.z) f.z[k] = pz;
    if (f.nx) f.nx[k] = wx;
    if (f.ny) f.ny[k] = wy;
    if (f.nz) f.nz[k] = wz;
    f.mat[k] = m;
}

bool finite_all(const float *v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

bool aligned4(const void *p) { return ((uintptr_t)p & 3u) == 0; }

}  // namespace
}  // namespace osim

using namespace osim;
using host::fail;
using host::hip_fail;
using host::ok;

extern "C" {

int oceansim_scene_create(const float *vertices, int64_t n_vertices, const int32_t *triangles,
                          const int32_t *tri_mat, int64_t n_triangles, oceansim_scene **scene) {
    if (!scene) return fail(OCEANSIM_E_INVALID_ARG, "scene is NULL");
    *scene = nullptr;
    BvhBuild B;
    int rc = build_bvh(vertices, n_vertices, triangles, tri_mat, n_triangles, B);
    if (rc != OCEANSIM_OK) return rc;
    oceansim_scene *s = new (std::nothrow) oceansim_scene();
    if (!s) {
        free_bvh(B);
        return fail(OCEANSIM_E_HIP, "host memory for the scene");
    }
    hipError_t e = hipGetDevice(&s->device);
    s->root = B.root;
    s->empty = B.empty ? 1 : 0;
    s->info = B.info;
    if (e == hipSuccess && !B.empty) {
        e = hipMalloc((void **)&s->nodes, sizeof(BvhNode) * (size_t)std::max(1LL, B.n_nodes));
        if (e == hipSuccess) e = hipMalloc((void **)&s->tris, sizeof(BvhTri) * (size_t)B.n_tris);
        if (e == hipSuccess && B.n_nodes)
            e = hipMemcpy(s->nodes, B.nodes, sizeof(BvhNode) * (size_t)B.n_nodes, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->tris, B.tris, sizeof(BvhTri) * (size_t)B.n_tris, hipMemcpyHostToDevice);
    }
    free_bvh(B);
    if (e != hipSuccess) {
        if (s->nodes) (void)hipFree(s->nodes);
        if (s->tris) (void)hipFree(s->tris);
        delete s;
        return hip_fail(e, "scene upload");
    }
    *scene = s;
    return ok();
}

int oceansim_scene_measure(const float *vertices, int64_t n_vertices, const int32_t *triangles,
                           const int32_t *tri_mat, int64_t n_triangles, oceansim_scene_info *info) {
    if (!info) return fail(OCEANSIM_E_INVALID_ARG, "info is NULL");
    BvhBuild B;
    const int rc = build_bvh(vertices, n_vertices, triangles, tri_mat, n_triangles, B);
    if (rc == OCEANSIM_OK) *info = B.info;
    free_bvh(B);
    return rc;
}

int oceansim_scene_get_info(const oceansim_scene *scene, oceansim_scene_info *info) {
    if (!scene || !info) return fail(OCEANSIM_E_INVALID_ARG, "scene or info is NULL");
    *info = scene->info;
    return ok();
}

int oceansim_scene_destroy(oceansim_scene *scene) {
    if (!scene) return ok();
    hipError_t e = hipSuccess;
    if (scene->nodes || scene->tris) {
        int cur = 0;
        e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != scene->device) e = hipSetDevice(scene->device);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (scene->nodes) (void)hipFree(scene->nodes);
        if (scene->tris) (void)hipFree(scene->tris);
        if (cur != scene->device) (void)hipSetDevice(cur);
    }
    delete scene;
    return e == hipSuccess ? ok() : hip_fail(e, "scene destroy");
}

int oceansim_raycast(const oceansim_scene *scene, const oceansim_ray_frame *frames, int32_t n_frames,
                     void *stream) {
    if (!scene) return fail(OCEANSIM_E_INVALID_ARG, "scene is NULL");
    if (n_frames < 0) return fail(OCEANSIM_E_SHAPE, "n_frames < 0");
    if (n_frames == 0) return ok();
    if (!frames) return fail(OCEANSIM_E_INVALID_ARG, "frames is NULL");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != scene->device)
        return fail(OCEANSIM_E_INVALID_ARG, "the scene lives on device %d, the current device is %d", scene->device,
                    dev);
    std::vector<RayFrameDev> fd;
    fd.reserve((size_t)n_frames);
    for (int i = 0; i < n_frames; ++i) {
        const oceansim_ray_frame &q = frames[i];
        if (q.n_beams < 0 || q.n_rays < 0) return fail(OCEANSIM_E_SHAPE, "frame %d: negative beam or ray count", i);
        const long long n = (long long)q.n_beams * q.n_rays;
        if (n > 0x7fffffffLL) return fail(OCEANSIM_E_UNSUPPORTED, "frame %d: more than 2^31 - 1 rays", i);
        if (!(q.fov_az >= 0.0f && q.fov_az <= 6.2831855f))
            return fail(OCEANSIM_E_INVALID_ARG, "frame %d: fov_az must be in [0, 2pi]", i);
        if (!(q.fov_el >= 0.0f && q.fov_el < 3.1415927f))
            return fail(OCEANSIM_E_INVALID_ARG, "frame %d: fov_el must be in [0, pi)", i);
        if (!(q.t_max > 0.0f && std::isfinite(q.t_max)))
            return fail(OCEANSIM_E_INVALID_ARG, "frame %d: t_max must be finite and > 0", i);
        if (!finite_all(q.pos, 3) || !finite_all(q.rot, 9))
            return fail(OCEANSIM_E_INVALID_ARG, "frame %d: non-finite pose", i);
        for (int a = 0; a < 3; ++a)
            if (std::fabs(q.pos[a]) > kMaxCoord)
                return fail(OCEANSIM_E_UNSUPPORTED, "frame %d: sensor position beyond 2^40", i);
        if (n == 0) continue;
        if (!q.mat) return fail(OCEANSIM_E_INVALID_ARG, "frame %d: mat is NULL", i);
        const void *outs[7] = {q.x, q.y, q.z, q.nx, q.ny, q.nz, q.mat};
        for (auto p : outs)
            if (!aligned4(p)) return fail(OCEANSIM_E_INVALID_ARG, "frame %d: misaligned output", i);
        RayFrameDev d;
        for (int a = 0; a < 3; ++a) d.o[a] = q.pos[a];
        for (int a = 0; a < 9; ++a) d.R[a] = q.rot[a];
        d.az0 = -0.5f * q.fov_az;
        d.daz = (float)((double)q.fov_az / q.n_beams);
        d.el0 = -0.5f * q.fov_el;
        d.del = (float)((double)q.fov_el / q.n_rays);
        d.t_max = q.t_max;
        d.nb = q.n_beams;
        d.nr = q.n_rays;
        d.n = (int)n;
        d.x = gcast(q.x);
        d.y = gcast(q.y);
        d.z = gcast(q.z);
        d.nx = gcast(q.nx);
        d.ny = gcast(q.ny);
        d.nz = gcast(q.nz);
        d.mat = gcast(q.mat);
        fd.push_back(d);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const gptr<const float4> nodes = gcast(reinterpret_cast<const float4 *>(scene->nodes));
    const gptr<const float4> tris = gcast(reinterpret_cast<const float4 *>(scene->tris));
    for (size_t g0 = 0; g0 < fd.size(); g0 += kRayFramesPerLaunch) {
        RayGroup grp;
        std::memset(&grp, 0, sizeof grp);
        const int cnt = (int)std::min<size_t>(kRayFramesPerLaunch, fd.size() - g0);
        int max_n = 0;
        for (int j = 0; j < cnt; ++j) {
            grp.f[j] = fd[g0 + j];
            max_n = std::max(max_n, grp.f[j].n);
        }
        const unsigned blocks = (unsigned)((max_n + kRayThreads - 1) / kRayThreads);
        OSIM_LAUNCH("k_raycast", k_raycast<kRayThreads>, dim3(blocks, (unsigned)cnt), dim3(kRayThreads), 0, st,
                    grp, nodes, tris, scene->root, scene->empty);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "ray-cast launch");
    }
    return ok();
}

}  // extern "C"
