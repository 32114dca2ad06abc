// Host build of the ray-casting hierarchy: a binary BVH over the mesh's
// triangles by the binned surface-area heuristic, laid out for the gfx950
// traversal kernel (both child boxes in the parent, triangles in leaf order
// as v0 and the two edges).
//
// Boxes are computed in double precision from the float32 vertices, rounded
// outwards to float32 and widened by 2^-22 of their own coordinate
// magnitude; the traversal's slab test widens its far distance by the
// rounding bound of its arithmetic, so that no box is rejected on rounding
// alone.  Depth is bounded by kBvhMaxDepth: a node whose heuristic split
// could not finish within the bound is split at the object median instead.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "host.hpp"
#include "scene.hpp"

namespace osim {

using host::fail;
using host::ok;

namespace {

constexpr int kBins = 16;
constexpr double kCostNode = 1.0;   // relative cost of a node visit against a triangle test

struct Box {
    double lo[3] = {INFINITY, INFINITY, INFINITY};
    double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void grow(const double *p) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], p[a]);
            hi[a] = std::max(hi[a], p[a]);
        }
    }
    void grow(const Box &b) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], b.lo[a]);
            hi[a] = std::max(hi[a], b.hi[a]);
        }
    }
    bool valid() const { return lo[0] <= hi[0]; }
    double area() const {
        if (!valid()) return 0.0;
        const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

struct Prim {
    Box box;
    double c[3];   // box centre
    int tri;       // index into the kept triangles
};

struct Builder {
    std::vector<Prim> prims;
    std::vector<BvhNode> nodes;
    std::vector<int> order;   // kept-triangle index per leaf slot
    int depth = 0, max_leaf = 0;
    long long n_leaves = 0;
    double sah = 0.0;         // sum over nodes of area * cost, divided by the root area at the end

    // Levels an object-median subtree of n primitives needs below its root.
    static int median_levels(int n) {
        int lv = 0;
        for (long long cap = kLeafMax; cap < n; cap *= 2) ++lv;
        return lv;
    }

    Box bounds(int b, int e) const {
        Box r;
        for (int i = b; i < e; ++i) r.grow(prims[i].box);
        return r;
    }

    // The box in float32, rounded outwards and widened by 2^-22 of its
    // largest coordinate magnitude: the stored triangles' second and third
    // corners (v0 + the float32 edges) may lie an ulp outside the box of the
    // original corners.
    static void store_box(const Box &b, float *lo, float *hi) {
        double m = 0.0;
        for (int a = 0; a < 3; ++a) m = std::max({m, std::fabs(b.lo[a]), std::fabs(b.hi[a])});
        const double pad = std::ldexp(m, -22);
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::nextafter((float)(b.lo[a] - pad), -INFINITY);
            hi[a] = std::nextafter((float)(b.hi[a] + pad), INFINITY);
        }
    }

    int make_leaf(int b, int e, int d) {
        for (int i = b; i < e; ++i) order.push_back(prims[i].tri);
        depth = std::max(depth, d);
        max_leaf = std::max(max_leaf, e - b);
        ++n_leaves;
        sah += bounds(b, e).area() * (e - b);
        return leaf_ref((int)order.size() - (e - b), e - b);
    }

    // Best binned split of prims[b, e): axis, bin boundary and cost (in units
    // of the node's area); false if the centres do not spread.
    bool sah_split(int b, int e, const Box &nb, int &axis, double &where, double &cost) const {
        Box cb;
        for (int i = b; i < e; ++i) cb.grow(prims[i].c);
        cost = INFINITY;
        for (int a = 0; a < 3; ++a) {
            const double ext = cb.hi[a] - cb.lo[a];
            if (!(ext > 0.0)) continue;
            Box bin[kBins];
            int cnt[kBins] = {};
            const double scale = kBins / ext;
            for (int i = b; i < e; ++i) {
                int k = (int)((prims[i].c[a] - cb.lo[a]) * scale);
                k = std::min(std::max(k, 0), kBins - 1);
                ++cnt[k];
                bin[k].grow(prims[i].box);
            }
            double right_area[kBins];
            int right_cnt[kBins];
            Box acc;
            int n = 0;
            for (int k = kBins - 1; k > 0; --k) {
                acc.grow(bin[k]);
                n += cnt[k];
                right_area[k] = acc.area();
                right_cnt[k] = n;
            }
            Box left;
            int nl = 0;
            for (int k = 1; k < kBins; ++k) {
                left.grow(bin[k - 1]);
                nl += cnt[k - 1];
                if (nl == 0 || right_cnt[k] == 0) continue;
                const double c = left.area() * nl + right_area[k] * right_cnt[k];
                if (c < cost) {
                    cost = c;
                    axis = a;
                    where = cb.lo[a] + k / scale;
                }
            }
        }
        if (!std::isfinite(cost)) return false;
        cost = kCostNode + cost / std::max(nb.area(), 1e-300);
        return true;
    }

    int build(int b, int e, int d) {
        const int n = e - b;
        const Box nb = bounds(b, e);
        const bool median = d + median_levels(n) >= kBvhMaxDepth;
        int mid = -1;
        if (!median) {
            int axis = 0;
            double where = 0.0, cost = 0.0;
            const bool can = sah_split(b, e, nb, axis, where, cost);
            if (n <= kLeafMax && (!can || cost >= (double)n)) return make_leaf(b, e, d);
            if (can) {
                auto it = std::partition(prims.begin() + b, prims.begin() + e,
                                         [&](const Prim &p) { return p.c[axis] < where; });
                mid = (int)(it - prims.begin());
                if (mid == b || mid == e) mid = -1;
            }
        } else if (n <= kLeafMax) {
            return make_leaf(b, e, d);
        }
        if (mid < 0) {
            // object median along the widest spread of the centres
            Box cb;
            for (int i = b; i < e; ++i) cb.grow(prims[i].c);
            int axis = 0;
            for (int a = 1; a < 3; ++a)
                if (cb.hi[a] - cb.lo[a] > cb.hi[axis] - cb.lo[axis]) axis = a;
            mid = b + n / 2;
            std::nth_element(prims.begin() + b, prims.begin() + mid, prims.begin() + e,
                             [axis](const Prim &p, const Prim &q) {
                                 return p.c[axis] < q.c[axis] || (p.c[axis] == q.c[axis] && p.tri < q.tri);
                             });
        }
        const int id = (int)nodes.size();
        nodes.emplace_back();
        sah += nb.area() * kCostNode;
        const int r0 = build(b, mid, d + 1);
        const int r1 = build(mid, e, d + 1);
        BvhNode &nd = nodes[id];
        store_box(bounds(b, mid), nd.lo0, nd.hi0);
        store_box(bounds(mid, e), nd.lo1, nd.hi1);
        nd.ref[0] = r0;
        nd.ref[1] = r1;
        nd.pad[0] = nd.pad[1] = 0;
        return id;
    }
};

}  // namespace

int build_bvh(const float *vertices, long long n_vertices, const int32_t *triangles, const int32_t *tri_mat,
              long long n_triangles, BvhBuild &out) {
    out = BvhBuild{};
    if (n_vertices < 0 || n_triangles < 0) return fail(OCEANSIM_E_SHAPE, "negative vertex or triangle count");
    if (n_triangles > 0 && (!vertices || !triangles || !tri_mat))
        return fail(OCEANSIM_E_INVALID_ARG, "NULL vertex, triangle or material array");
    if (n_triangles > kMaxSceneTriangles)
        return fail(OCEANSIM_E_UNSUPPORTED, "more than 2^28 triangles");
    for (long long i = 0; i < 3 * n_vertices; ++i) {
        if (!std::isfinite(vertices[i])) return fail(OCEANSIM_E_INVALID_ARG, "vertex %lld is not finite", i / 3);
        if (std::fabs(vertices[i]) > kMaxCoord)
            return fail(OCEANSIM_E_UNSUPPORTED, "vertex %lld: coordinates beyond 2^40", i / 3);
    }
    Builder B;
    B.prims.reserve((size_t)n_triangles);
    std::vector<long long> kept;
    kept.reserve((size_t)n_triangles);
    for (long long f = 0; f < n_triangles; ++f) {
        double v[3][3];
        for (int j = 0; j < 3; ++j) {
            const int32_t idx = triangles[3 * f + j];
            if (idx < 0 || idx >= n_vertices)
                return fail(OCEANSIM_E_INVALID_ARG, "triangle %lld: vertex index %d outside [0, %lld)", f, idx,
                            n_vertices);
            for (int a = 0; a < 3; ++a) v[j][a] = vertices[3LL * idx + a];
        }
        double e1[3], e2[3], e3[3];
        for (int a = 0; a < 3; ++a) {
            e1[a] = v[1][a] - v[0][a];
            e2[a] = v[2][a] - v[0][a];
            e3[a] = v[2][a] - v[1][a];
        }
        const double n0 = e1[1] * e2[2] - e1[2] * e2[1];
        const double n1 = e1[2] * e2[0] - e1[0] * e2[2];
        const double n2 = e1[0] * e2[1] - e1[1] * e2[0];
        const double l2 = std::max({e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2],
                                    e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2],
                                    e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2]});
        const double nl = std::sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        if (!(nl >= std::ldexp(l2, -20)) || l2 == 0.0) continue;   // needle or point
        Prim p;
        for (int j = 0; j < 3; ++j) p.box.grow(v[j]);
        for (int a = 0; a < 3; ++a) p.c[a] = 0.5 * (p.box.lo[a] + p.box.hi[a]);
        p.tri = (int)kept.size();
        kept.push_back(f);
        B.prims.push_back(p);
    }
    const long long n_kept = (long long)kept.size();
    out.info.n_triangles = n_kept;
    out.info.n_dropped = n_triangles - n_kept;
    if (n_kept == 0) {
        out.empty = true;
        return ok();
    }
    B.nodes.reserve((size_t)std::max(1LL, n_kept / 2));
    B.order.reserve((size_t)n_kept);
    const double root_area = B.bounds(0, (int)n_kept).area();
    out.root = B.build(0, (int)n_kept, 0);
    if (B.depth > kBvhMaxDepth) return fail(OCEANSIM_E_UNSUPPORTED, "hierarchy deeper than %d levels", kBvhMaxDepth);
    out.empty = false;
    out.n_nodes = (long long)B.nodes.size();
    out.n_tris = n_kept;
    out.nodes = static_cast<BvhNode *>(std::malloc(sizeof(BvhNode) * std::max(1LL, out.n_nodes)));
    out.tris = static_cast<BvhTri *>(std::malloc(sizeof(BvhTri) * (size_t)n_kept));
    if (!out.nodes || !out.tris) {
        free_bvh(out);
        return fail(OCEANSIM_E_HIP, "host memory for the hierarchy");
    }
    if (out.n_nodes) std::memcpy(out.nodes, B.nodes.data(), sizeof(BvhNode) * (size_t)out.n_nodes);
    for (long long s = 0; s < n_kept; ++s) {
        const long long f = kept[(size_t)B.order[(size_t)s]];
        const float *V[3];
        for (int j = 0; j < 3; ++j) V[j] = vertices + 3LL * triangles[3 * f + j];
        BvhTri &t = out.tris[s];
        for (int a = 0; a < 3; ++a) {
            t.v0[a] = V[0][a];
            t.e1[a] = (float)((double)V[1][a] - V[0][a]);
            t.e2[a] = (float)((double)V[2][a] - V[0][a]);
        }
        t.mat = tri_mat[f];
        t.pad1 = t.pad2 = 0.0f;
    }
    out.info.n_nodes = out.n_nodes;
    out.info.n_leaves = B.n_leaves;
    out.info.depth = B.depth;
    out.info.max_leaf = B.max_leaf;
    out.info.sah_cost = root_area > 0.0 ? B.sah / root_area : 0.0;
    out.info.device_bytes = (uint64_t)(sizeof(BvhNode) * out.n_nodes + sizeof(BvhTri) * n_kept);
    return ok();
}

void free_bvh(BvhBuild &b) {
    std::free(b.nodes);
    std::free(b.tris);
    b.nodes = nullptr;
    b.tris = nullptr;
}

}  // namespace osim
