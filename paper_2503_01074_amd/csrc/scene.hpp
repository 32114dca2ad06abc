// Device layout of a ray-casting scene (internal to the library): a binary
// bounding-volume hierarchy whose nodes hold the boxes of both children, and
// the triangles in leaf order.
#pragma once

#include <cstdint>

#include "../../include/oceansim.h"

namespace osim {

// Child references.  ref >= 0: an inner node (index into the node array);
// ref < 0: a leaf, ~ref = (first triangle << 3) | (triangles - 1).
constexpr int kLeafMax = 8;
constexpr int kLeafShift = 3;
constexpr int kMaxSceneTriangles = 1 << 28;
// Deepest leaf (root at depth 0).  A traversal keeps at most one deferred
// child per level on its stack, so this is also the stack depth.
constexpr int kBvhMaxDepth = 32;
// Largest coordinate magnitude of a vertex or a sensor position (2^40 m):
// the triangle test's triple products then stay below 2^126 and the slab
// products below 2^101, finite in float32 (a direction component below 2^-60
// in magnitude is cast as 2^-60 of its sign).
constexpr float kMaxCoord = 1099511627776.0f;
constexpr float kMinDirComponent = 8.67361737988403547e-19f;

__host__ __device__ inline int leaf_ref(int first, int count) { return ~((first << kLeafShift) | (count - 1)); }

// 64 bytes: child 0 box, child 1 box, the two references.
struct alignas(16) BvhNode {
    float lo0[3], hi0[3], lo1[3], hi1[3];
    int32_t ref[2];
    int32_t pad[2];
};
static_assert(sizeof(BvhNode) == 64, "node layout");

// 48 bytes: v0 with the material id in the fourth word, then the two edges
// e1 = v1 - v0 and e2 = v2 - v0.
struct alignas(16) BvhTri {
    float v0[3];
    int32_t mat;
    float e1[3];
    float pad1;
    float e2[3];
    float pad2;
};
static_assert(sizeof(BvhTri) == 48, "triangle layout");

// Host-side result of a build.
struct BvhBuild {
    int root = 0;       // reference of the root (a leaf for tiny meshes)
    bool empty = true;  // no triangle kept: every ray misses
    BvhNode *nodes = nullptr;
    long long n_nodes = 0;
    BvhTri *tris = nullptr;
    long long n_tris = 0;
    oceansim_scene_info info{};
};

// Builds the hierarchy (binned surface-area heuristic) into host arrays
// owned by `out` (released by free_bvh).  Returns an oceansim_status and sets
// the library's last error on failure.
int build_bvh(const float *vertices, long long n_vertices, const int32_t *triangles, const int32_t *tri_mat,
              long long n_triangles, BvhBuild &out);
void free_bvh(BvhBuild &b);

}  // namespace osim
