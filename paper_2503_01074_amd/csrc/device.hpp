// Device-side building blocks of the OceanSim gfx950 library: the frame
// descriptors the kernels read, Philox4x32-10, and the per-return,
// per-bin and per-pixel formulas of Sec. III-A.1 / III-A.2 of the paper
// (arXiv 2503.01074).  Header-only; included by every kernel translation unit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osim {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kWave = 64;
constexpr int kMaxTileBins = 4096;   // polar bins of a backward tile workgroup (one row at least)
constexpr int kMaxFwdTileBins = 16384;   // polar bins owned by one forward tile workgroup
constexpr int kWideThreads = 512;    // threads of the wide binning, forward-tile and pair-backward workgroups
constexpr int kMaxTiles = 4096;      // tiles per frame (LDS histogram in the binning pass)
constexpr int kXcds = 8;            // accelerator complex dies (each with its own L2)
constexpr int kFanRows = 2;        // fan rows per thread (one pixel pair each, 8 rows apart)
constexpr int kFanTileU = 32;      // pixel pairs per fan workgroup along a row
constexpr int kFanTileV = 16;      // fan rows per fan workgroup (8 x kFanRows)
constexpr int kLaneHistMats = 64;    // materials reduced per workgroup in an LDS table (above: global atomics)

enum Kind { KBIN = 0, KTILE = 1, KFAN = 2, KRET = 3, KTILEB = 4, KFANT = 5, KROW = 6, KIND_COUNT = 7 };
enum Speckle { SPECKLE_OFF = 0, SPECKLE_PAPER = 1, SPECKLE_GAMMA = 2 };

// Pointers into device global memory.  Descriptor pointers carry the global
// address space in their type: read from a device frame table they would
// otherwise be generic pointers, and every access would compile to a flat
// (not global) memory instruction.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__host__ __device__ __forceinline__ gptr<T> gcast(T *p) {
    return (gptr<T>)p;
}

// Vector loads and stores through global pointers (HIP's vector classes
// take generic references, so they go through clang's native vectors).
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
typedef int i32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint2 gload(gptr<const uint2> p) {
    const u32x2_t v = *(gptr<const u32x2_t>)p;
    return make_uint2(v.x, v.y);
}
__device__ __forceinline__ void gstore(gptr<uint2> p, uint2 v) { *(gptr<u32x2_t>)p = u32x2_t{v.x, v.y}; }
__device__ __forceinline__ int4 gload(gptr<const int4> p) {
    const i32x4_t v = *(gptr<const i32x4_t>)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gstore(gptr<int4> p, int4 v) { *(gptr<i32x4_t>)p = i32x4_t{v.x, v.y, v.z, v.w}; }
__device__ __forceinline__ float4 gload(gptr<const float4> p) {
    const f32x4_t v = *(gptr<const f32x4_t>)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gstore(gptr<float4> p, float4 v) { *(gptr<f32x4_t>)p = f32x4_t{v.x, v.y, v.z, v.w}; }
// Non-temporal stores, for final outputs that no later kernel reads back:
// the lines stream to HBM without displacing cached inputs, which lifts the
// write-heavy camera and fan kernels from ~5.5 to ~7.4 TB/s.
__device__ __forceinline__ void gstore_stream(gptr<float4> p, float4 v) {
    __builtin_nontemporal_store(f32x4_t{v.x, v.y, v.z, v.w}, (gptr<f32x4_t>)p);
}
__device__ __forceinline__ void gstore_stream(gptr<float> p, float v) { __builtin_nontemporal_store(v, p); }

// --------------------------------------------------------------------------
// One sonar frame as the kernels see it.  Built on the host from the public
// descriptor: float inputs promoted exactly to double, derived constants
// computed once in double.
// --------------------------------------------------------------------------
struct SonarDev {
    gptr<const float> x, y, z, nx, ny, nz;
    gptr<const int> mat;
    gptr<float> polar;          // speckled polar image (caller buffer or workspace)
    gptr<float> fan;
    gptr<int> bin_of_return;
    gptr<const float> grad_polar, grad_fan;
    gptr<uint2> pairs;          // binning pass output: (tile-local bin, intensity), or with
                                // matp (tile-local bin | material << 16, cos x attenuation)
    gptr<float> pair_r;         // the pairs' ranges (same order), for the pair backward; or nullptr
    gptr<float> tile_cemax;     // per forward tile, the largest |cos x attenuation| of its pairs
                                // (written by the forward tile with pair_r; bounds the pair backward's sums)
    int matp;                   // pairs carry the material id (tables of at most 64 materials)
    gptr<int> chunk_off;        // [n_chunks][n_tiles + 1] exclusive offsets per chunk
    gptr<float> grad_img;       // backward: dL/d(polar image) [nb]
    long long n;                // returns
    int n_range, n_az, fan_h, fan_w;
    int rows_per_tile, tile_bins, n_tiles;          // forward polar tiles
    int rows_per_tile_b, tile_bins_b, n_tiles_b;    // backward polar tiles
    int chunk, n_chunks;        // returns per binning workgroup, workgroups
    int ret_chunk, n_ret_chunks;// returns per backward-gather workgroup, workgroups
    int fan_bpr, fan_blocks;    // fan: workgroup columns (kFanTileU pairs each), workgroups
    int speckle, gamma_k, param_row;
    float inv_gamma_k;          // 1 / gamma_k
    unsigned seed_lo, seed_hi, frame_id;
    int blk[KIND_COUNT];        // first global workgroup of this frame, per kernel kind
    double r_min, r_max;        // polar grid [r_min, r_max)
    double fov_az, half_az;     // full and half azimuth field of view
    double sin_half_el;         // sin(fov_el / 2)
    double kappa;               // path factor of Eq. 2
    double scale_r;             // N_r / (r_max - r_min)
    double scale_phi;           // N_phi / fov_az
    double dr, dphi;            // bin sizes
    double fan_s;               // fan pixel size
    double tan_half_az;         // tan(fov_az / 2) (fans need fov_az <= pi)
    double inv_r_max;           // 1 / r_max
    float scale_phi_f, half_az_f;
    int az_fast;                // FP32 azimuth is accurate to < 1e-3 cell on this grid
    int half_w;                 // fan pixel pairs per row: ceil(fan_w / 2)
    gptr<int4> stencil;         // saved fan stencils [fan_h][half_w] or nullptr
    gptr<double2> cols;         // forward fan: {sin, cos} of each column-centre azimuth [n_az]
    double sin_half_az, cos_half_az;
    int wide_cols;              // columns wider than 0.09 rad: offsets need the full arctangent
    float r_min_f, scale_r_f;
    // Transposed fan operator (plans): the entries of operator row h are
    // ft_ent[ft_ptr[h] .. ft_ptr[h + 1]), each {fan pixel, bilinear weight as
    // float bits}, in a fixed order.  Plain layout: row h is bin h, pixel
    // v * fan_w + u.  Mirrored layout (ft_mirror, even fan width): row
    // i * ceil(N_phi / 2) + j is bin (i, j) and also stands for its mirror
    // bin (i, N_phi-1-j), whose entries are the same weights at the mirrored
    // pixels (v, fan_w-1-u); pixel packed as (v << 16) | u.  nullptr: none.
    gptr<const int> ft_ptr;
    gptr<const uint2> ft_ent;
    int ft_mirror;
    // Range-wise normalisation: each range row of Q = G P over its maximum
    // (when positive).  saved_p: the forward's binned sums P [nb]; dldq: the
    // backward's dL/dQ per bin [nb].
    int range_norm;
    gptr<float> saved_p;
    gptr<float> dldq;
    int n_fant_blocks;          // backward workgroups (kBlock * BPT operator rows each) through the operator
};

struct UwDev {
    gptr<const float> J, depth;
    gptr<float> out;
    gptr<const float> grad_out;
    gptr<float> grad_J, grad_depth;
    long long npix;
    int param_row;
    int blk;                    // first global workgroup
    int n_blocks;
    int fwd_px;                 // forward: pixels per thread (4, 8, 16 or 32; the same for every frame of a launch)
    int bwd_px;                 // backward: pixels per thread (8, 16, 32 or 64; likewise)
};

// Workgroups are dispatched to the XCDs round-robin (workgroup b to XCD
// b % kXcds).  Kernels whose neighbouring workgroups share data (polar rows
// gathered by nearby fan tiles, fan pixels near adjacent polar tiles) use
// this logical id instead: each XCD receives runs of G consecutive logical
// workgroups (so the shared lines are fetched into one L2), and the runs are
// dealt round-robin (so work that varies smoothly with the id stays balanced
// across XCDs).  A bijection on [0, n); the last partial round keeps b.
template <int G>
__host__ __device__ __forceinline__ int xcd_grouped_id(int b, int n) {
    constexpr int round = kXcds * G;
    if (b >= n / round * round) return b;
    return b / round * round + (b % kXcds) * G + (b / kXcds) % G;
}

// Flat walk over NT segments laid end to end (segment c holds flat indices
// [seg_end[c - 1], seg_end[c]), seg_end the inclusive prefix of the
// lengths, total the last entry): a coarse map of 2 NT entries finds the
// segment of a flat index k without a full binary search.  Entry j holds the
// segment of flat index j << shift (shift the smallest with (total - 1) >>
// shift < 2 NT - 1) and entry n_map the segment of the last index; each
// non-empty segment writes its own entries.
__host__ __device__ __forceinline__ int seg_map_shift(int total, int map_entries) {
    int shift = 0;
    while (((total - 1) >> shift) >= map_entries - 1) ++shift;
    return shift;
}
__host__ __device__ __forceinline__ void seg_map_fill(unsigned short *map, int seg, int excl, int incl, int total,
                                                      int shift) {
    if (incl <= excl) return;
    for (int j = (int)(((long long)excl + (1LL << shift) - 1) >> shift); ((long long)j << shift) < incl; ++j)
        map[j] = (unsigned short)seg;
    if (incl == total) map[((total - 1) >> shift) + 1] = (unsigned short)seg;
}
// The segment holding flat index k < total: first c with seg_end[c] > k.  It
// lies between the map's entries around k; three branch-free steps cover
// eight segments, a loop the rare wider spans (empty segments between).
template <int NT>
__host__ __device__ __forceinline__ int seg_find(const int *seg_end, const unsigned short *map, int shift, int k) {
    const int lo = map[k >> shift], hi = map[(k >> shift) + 1];
    int cc = lo;
#pragma unroll
    for (int s = 4; s > 0; s >>= 1) cc += seg_end[min(cc + s - 1, NT - 1)] <= k ? s : 0;
    if (hi - lo >= 8) {
        int a = lo, b = hi;
        while (a < b) {
            const int m = (a + b) >> 1;
            if (seg_end[m] <= k)
                a = m + 1;
            else
                b = m;
        }
        cc = a;
    }
    return cc;
}

// Launches that interleave n_tile tile workgroups with n_cam camera
// workgroups evenly through the dispatch order: workgroup x (of n_tile +
// n_cam) is camera group floor(x C / N) when floor((x + 1) C / N) >
// floor(x C / N), else tile x - floor(x C / N) (C = n_cam, N = n_tile +
// n_cam).  Every tile and every camera group is taken exactly once.
struct FusedSlot {
    bool cam;
    int index;
};
__host__ __device__ __forceinline__ FusedSlot fused_slot(long long x, int n_tile, int n_cam) {
    const long long n = (long long)n_tile + n_cam;
    const int c_before = (int)(x * n_cam / n);
    const int c_upto = (int)((x + 1) * n_cam / n);
    return c_upto > c_before ? FusedSlot{true, c_before} : FusedSlot{false, (int)(x - c_before)};
}

// Frame sources: a single frame passed by value in the kernel arguments, or a
// device-resident table (batched calls and plans).  Workgroups find their
// frame by a uniform binary search over the per-frame first-block indices.
template <class F>
struct One {
    F f;
    __device__ __forceinline__ int locate(int b, int kind, int &local) const {
        local = b;
        return 0;
    }
    __device__ __forceinline__ const F &frame(int) const { return f; }
};

template <class F>
struct Table {
    const F *t;
    int n;
    __device__ __forceinline__ int locate(int b, int kind, int &local) const {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (t[mid].blk[kind] <= b) lo = mid; else hi = mid - 1;
        }
        local = b - t[lo].blk[kind];
        return lo;
    }
    __device__ __forceinline__ const F &frame(int i) const { return t[i]; }
};

template <>
__device__ __forceinline__ int Table<UwDev>::locate(int b, int, int &local) const {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (t[mid].blk <= b) lo = mid; else hi = mid - 1;
    }
    local = b - t[lo].blk;
    return lo;
}

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit products of counter words 0 and 2, whose halves are xored with
// the other words and the round key; the key advances by two Weyl constants.
// The key schedule is uniform across a wave and stays in scalar registers.
// --------------------------------------------------------------------------
struct Words { uint32_t w0, w1, w2, w3; };

// a ^ b ^ c in one instruction (gfx950's three-input bit operation with the
// odd-parity truth table)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        uint64_t a = (uint64_t)c0 * 0xD2511F53u;
        uint64_t b = (uint64_t)c2 * 0xCD9E8D57u;
        uint32_t n0 = xor3((uint32_t)(b >> 32), c1, k0);
        uint32_t n2 = xor3((uint32_t)(a >> 32), c3, k1);
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t pick(const Words &w, uint32_t k) {
    return k == 0 ? w.w0 : k == 1 ? w.w1 : k == 2 ? w.w2 : w.w3;
}

// Top 24 bits plus one, times 2^-24: a uniform in (0, 1], exact in float.
__device__ __forceinline__ float unit_uniform(uint32_t w) {
    return (float)((w >> 8) + 1u) * 5.9604644775390625e-8f;
}

// -ln(u) for a uniform u in (0, 1] (a multiple of 2^-24) from the hardware
// log2.  Over all 2^24 such u its relative error is below 1.7e-7, also where
// -ln(u) is tiny (u near 1); measured on gfx950 against FP64.
__device__ __forceinline__ float neg_ln(float u) {
    return -__builtin_amdgcn_logf(u) * 0.69314718055994531f;
}

// Unit Rayleigh variate of bin b (additive stream, Eq. 4 with sigma = 1):
// sqrt(-2 ln u), the factor 2 folded into the constant of neg_ln (scaling by
// two is exact, so this is sqrt(2 neg_ln(u)) bit for bit).
__device__ __forceinline__ float rayleigh_of_word(uint32_t w) {
    return __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(unit_uniform(w)) * -1.38629436111989062f);
}

// Multiplicative speckle factor of bin b and, in PAPER mode, its standard
// normal draw (Eq. 5-6).  GAMMA: -(1/k) ln prod u_w (a unit-mean Gamma(k, 1/k)).
__device__ __forceinline__ float speckle_factor(const SonarDev &f, uint32_t b, float sigma_sm,
                                                float *gauss_out) {
    if (f.speckle == SPECKLE_PAPER) {
        Words w = philox(b >> 1, f.frame_id, 1u, 0u, f.seed_lo, f.seed_hi);
        uint32_t h = (b & 1u) * 2u;
        float u0 = unit_uniform(pick(w, h));
        float u1 = unit_uniform(pick(w, h + 1u));
        float g = __builtin_amdgcn_sqrtf(2.0f * neg_ln(u0)) * cospif(2.0f * u1);
        *gauss_out = g;
        return 0.5f + sigma_sm * g;
    }
    if (f.speckle == SPECKLE_GAMMA) {
        // -ln of the product of each group's (up to four) uniforms: the
        // uniforms are at least 2^-24, so a group's product is at least
        // 2^-96, a normal float, and one logarithm serves four draws
        *gauss_out = 0.0f;
        float acc = 0.0f;
        int k = f.gamma_k;
        for (int g = 0; 4 * g < k; ++g) {
            Words w = philox(b, f.frame_id, 2u, (uint32_t)g, f.seed_lo, f.seed_hi);
            int left = k - 4 * g;
            float prod = unit_uniform(w.w0);
            if (left > 1) prod *= unit_uniform(w.w1);
            if (left > 2) prod *= unit_uniform(w.w2);
            if (left > 3) prod *= unit_uniform(w.w3);
            acc += neg_ln(prod);
        }
        return acc * f.inv_gamma_k;
    }
    *gauss_out = 0.0f;
    return 1.0f;
}

// --------------------------------------------------------------------------
// Per-return geometry (Sec. III-A.2): range test on an FP64 range, azimuth
// bin from an FP32 atan2 that is redone in FP64 when it lands within 2e-3
// of a cell edge, elevation cone test in FP64.  Returns the frame-linear bin
// or -1, and the FP64 range.
// --------------------------------------------------------------------------
__device__ __forceinline__ int return_bin(const SonarDev &f, float xf, float yf, float zf, int m,
                                          int n_mat, double &r) {
    double x = xf, y = yf, z = zf;
    r = __builtin_sqrt(x * x + y * y + z * z);
    if (m < 0 || m >= n_mat) return -1;
    if (!(r > 0.0)) return -1;
    if (!(r >= f.r_min && r < f.r_max)) return -1;
    if (!(__builtin_fabs(z) <= r * f.sin_half_el)) return -1;
    double fr = (r - f.r_min) * f.scale_r;
    int i = (int)fr;                               // fr >= 0 here
    if (i > f.n_range - 1) i = f.n_range - 1;
    float phi = atan2f(yf, xf);
    float fp = (phi + f.half_az_f) * f.scale_phi_f;
    float frac = fp - floorf(fp);
    int j;
    bool near_edge = !f.az_fast || (frac < 2e-3f) || (frac > 1.0f - 2e-3f) ||
                     !(fp > 2e-3f) || !(fp < (float)f.n_az - 2e-3f);
    if (near_edge) {
        double phid = atan2(y, x);
        if (!(phid >= -f.half_az && phid < f.half_az)) return -1;
        double fpd = (phid + f.half_az) * f.scale_phi;
        j = (int)__builtin_floor(fpd);
    } else {
        j = (int)fp;
    }
    if (j > f.n_az - 1) j = f.n_az - 1;
    if (j < 0) j = 0;
    return i * f.n_az + j;
}

// Eq. (2): refl * max(0, -x.n / (|x| |n|)) * exp(-kappa alpha r).
// cosg and att receive the two factors (needed by the adjoint).
__device__ __forceinline__ float return_intensity(const SonarDev &f, float xf, float yf, float zf,
                                                  float nxf, float nyf, float nzf, double r,
                                                  float refl, float alpha, float &cosg,
                                                  float &att) {
    double dot = (double)xf * nxf + (double)yf * nyf + (double)zf * nzf;
    float nn = __builtin_sqrtf(nxf * nxf + nyf * nyf + nzf * nzf);
    float c = 0.0f;
    if (nn > 0.0f) c = -(float)dot / ((float)r * nn);
    c = c > 0.0f ? c : 0.0f;
    // exponent in FP64 (it can reach ~40), split so that expf sees the head
    double arg = f.kappa * (double)alpha * r;
    float hi = (float)arg;
    float lo = (float)(arg - (double)hi);
    float e = expf(-hi) * (1.0f - lo);
    cosg = c;
    att = e;
    return refl * c * e;
}

// Additive speckle geometry of bin (i, j): R_i = r_i^2 / r_max^2 and the
// bin-centre azimuth phi_j (Eq. 3).
__device__ __forceinline__ float range_ramp(const SonarDev &f, int i) {
    double ri = f.r_min + ((double)i + 0.5) * f.dr;
    double q = ri * f.inv_r_max;
    return (float)(q * q);
}
__device__ __forceinline__ float bin_azimuth(const SonarDev &f, int j) {
    return (float)(-f.half_az + ((double)j + 0.5) * f.dphi);
}

// --------------------------------------------------------------------------
// Fan geometry, FP64: polar position of pixel (v, u) and its bilinear stencil.
// i0/j0 index the first row/column, t/s the weights of the second; i1/j1 are
// i0+1/j0+1 except on single-row/column grids (then equal, weight 0).
// --------------------------------------------------------------------------
struct Stencil {
    int i0, i1, j0, j1;
    double t, s;
};

__device__ __forceinline__ void fan_position(const SonarDev &f, int v, int u, double &rho,
                                             double &phi) {
    double xc = ((double)u + 0.5 - 0.5 * (double)f.fan_w) * f.fan_s;
    double yc = ((double)f.fan_h - (double)v - 0.5) * f.fan_s;
    rho = __builtin_sqrt(xc * xc + yc * yc);
    phi = atan2(-xc, yc);
}

// Radial half of the stencil: rows and weight of rho (inside test on rho).
__device__ __forceinline__ bool fan_radial(const SonarDev &f, double rho, Stencil &st) {
    if (!(rho >= f.r_min && rho <= f.r_max)) return false;
    double fr = (rho - f.r_min) * f.scale_r - 0.5;
    const double nr1 = (double)(f.n_range - 1);
    fr = fr < 0.0 ? 0.0 : (fr > nr1 ? nr1 : fr);
    if (f.n_range == 1) {
        st.i0 = st.i1 = 0;
        st.t = 0.0;
    } else {
        int i0 = (int)fr;
        if (i0 > f.n_range - 2) i0 = f.n_range - 2;
        st.i0 = i0;
        st.i1 = i0 + 1;
        st.t = fr - (double)i0;
    }
    return true;
}

// Angular half: columns and weight of phi (inside test on phi).
__device__ __forceinline__ bool fan_angular(const SonarDev &f, double phi, Stencil &st) {
    if (!(phi >= -f.half_az && phi <= f.half_az)) return false;
    double fp = (phi + f.half_az) * f.scale_phi - 0.5;
    const double np1 = (double)(f.n_az - 1);
    fp = fp < 0.0 ? 0.0 : (fp > np1 ? np1 : fp);
    if (f.n_az == 1) {
        st.j0 = st.j1 = 0;
        st.s = 0.0;
    } else {
        int j0 = (int)fp;
        if (j0 > f.n_az - 2) j0 = f.n_az - 2;
        st.j0 = j0;
        st.j1 = j0 + 1;
        st.s = fp - (double)j0;
    }
    return true;
}

__device__ __forceinline__ bool fan_stencil(const SonarDev &f, double rho, double phi,
                                            Stencil &st) {
    return fan_radial(f, rho, st) && fan_angular(f, phi, st);
}

// --------------------------------------------------------------------------
// Fan geometry from the nearest bin centres.  The bilinear weight along an
// axis is the pixel's offset from a bin centre in units of the bin size; it
// is computed here from differences that are formed exactly in FP64 (squared
// radii; the cross and dot products of the pixel position with the centre
// direction), so each weight and its complement keep ~1e-7 RELATIVE accuracy
// without an FP64 square root or arctangent per pixel.  Approximate FP32
// positions only choose the nearest centre, to well within half a bin.
// --------------------------------------------------------------------------

// atan(z) for z in [0, 1]: odd least-squares polynomial fitted for this
// kernel, |error| < 1.2e-5 rad (used only to pick the nearest column).
__device__ __forceinline__ float atan01_approx(float z) {
    const float z2 = z * z;
    float p = 0.02084507f;
    p = __builtin_fmaf(p, z2, -0.08515627f);
    p = __builtin_fmaf(p, z2, 0.18015924f);
    p = __builtin_fmaf(p, z2, -0.33030477f);
    p = __builtin_fmaf(p, z2, 0.9998663f);
    return p * z;
}

// atan2(a, b) for a, b >= 0, |error| < 1.2e-5 rad.
__device__ __forceinline__ float atan2_pos_approx(float a, float b) {
    const float lo = fminf(a, b), hi = fmaxf(a, b);
    const float t = atan01_approx(lo * __builtin_amdgcn_rcpf(fmaxf(hi, 1e-30f)));
    return a > b ? 1.5707963f - t : t;
}

// Offset e in (-1, 1) of a coordinate from centre k of an axis of n bins,
// in bins -> first bin of the stencil and the stored weight code of the
// second bin (see encode_weight), with the clamping of the plain definition
// at the two outer half-bins.
__device__ __forceinline__ void axis_from_offset(int k, float e, int n, int &k0, float &code) {
    e = e + 0.0f;   // no negative zero: its sign would read as "weight 1"
    if (n == 1) {
        k0 = 0;
        code = 0.0f;
        return;
    }
    k0 = e < 0.0f ? k - 1 : k;
    code = e > 0.5f ? e - 1.0f : (e < -0.5f ? e + 1.0f : e);
    if (k0 < 0) {               // before the first centre: weight 0 on bin 1
        k0 = 0;
        code = 0.0f;
    }
    if (k0 > n - 2) {           // past the last centre: weight 1 on bin n-1
        k0 = n - 2;
        code = -0.0f;
    }
}

// Whether a LEFT-half fan pixel (offset ax = -x_c >= 0 from the axis, y_c > 0
// along it, squared distance rho2 from the apex, all FP64 from exact pixel
// offsets) lies in the sector: r_min <= rho <= r_max and |phi| <= fov/2,
// the latter as ax cos(fov/2) <= yc sin(fov/2) (fov <= pi, yc > 0).
__device__ __forceinline__ bool fan_inside(const SonarDev &f, double ax, double yc, double rho2) {
    return rho2 >= f.r_min * f.r_min && rho2 <= f.r_max * f.r_max && ax * f.cos_half_az <= yc * f.sin_half_az;
}

// Radial half of a fan pixel at squared distance rho2 from the apex: (first
// row, weight code); valid indices for any rho2.
__device__ __forceinline__ void fan_radial_fast(const SonarDev &f, double rho2, int &i0, float &code) {
    const float rho_f = __builtin_amdgcn_sqrtf((float)rho2);   // hardware sqrt: only picks the nearest row
    int in = (int)__builtin_rintf((rho_f - f.r_min_f) * f.scale_r_f - 0.5f);
    in = in < 0 ? 0 : (in > f.n_range - 1 ? f.n_range - 1 : in);
    const double rc = __builtin_fma((double)in + 0.5, f.dr, f.r_min);
    // rho - rc = (rho^2 - rc^2) / (rho + rc): numerator exact to FP64 rounding
    const float num = (float)__builtin_fma(-rc, rc, rho2);
    const float e = num * __builtin_amdgcn_rcpf(rho_f + (float)rc) * f.scale_r_f;
    axis_from_offset(in, e, f.n_range, i0, code);
}

// Angular half of a LEFT-half fan pixel, in two steps so that the column
// table loads of several pixels can be in flight together: the nearest column
// from the approximate azimuth (clamped, valid for any position), then the
// offset e from that column's centre in columns, from its {sin, cos}: the
// mirror pixel has column N_phi - 1 - jn and offset -e.
__device__ __forceinline__ int fan_column_guess(const SonarDev &f, double ax, double yc) {
    const float phi = atan2_pos_approx((float)ax, (float)yc);
    const int j = (int)__builtin_rintf((phi + f.half_az_f) * f.scale_phi_f - 0.5f);
    return j < 0 ? 0 : (j > f.n_az - 1 ? f.n_az - 1 : j);
}

__device__ __forceinline__ float fan_column_offset(const SonarDev &f, double ax, double yc, double sn, double cn) {
    // angle from the centre direction: atan of the cross over the dot product
    const double cr = __builtin_fma(ax, cn, -yc * sn);
    const double dt = __builtin_fma(ax, sn, yc * cn);
    const float q = (float)cr * __builtin_amdgcn_rcpf((float)dt);
    float d;
    if (f.wide_cols) {
        d = atanf(q);
    } else {
        // |q| < 0.05: the series to q^5 is exact to float precision
        const float q2 = q * q;
        d = q * __builtin_fmaf(q2, __builtin_fmaf(q2, 0.2f, -0.33333334f), 1.0f);
    }
    return d * f.scale_phi_f;
}

// Saved stencil of a pair of mirror-image fan pixels (left pixel u, right
// pixel W-1-u): {first row (-1 = outside the sector), left pixel's first
// column, row weight, left column weight}.  A weight w in [0, 1] is stored as
// the smaller of w and 1 - w, its sign bit telling which, so that both w and
// 1 - w keep full float relative precision.  The right pixel's columns are
// the mirror image: first column N_phi - 2 - j0, weight code negated.
__device__ __forceinline__ float encode_weight(double w) {
    return w <= 0.5 ? (float)w : -(float)(1.0 - w);
}
__device__ __forceinline__ void decode_weight(float e, float &w, float &one_minus_w) {
    if (__builtin_signbit(e)) {
        w = 1.0f + e;
        one_minus_w = -e;
    } else {
        w = e;
        one_minus_w = 1.0f - e;
    }
}

// --------------------------------------------------------------------------
// Wave / workgroup reductions in a fixed order (bit-reproducible).
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    return v;   // lane 0 holds the sum
}

// Sums `v` over a workgroup of NT threads; thread 0 receives the result.
// `sh` needs NT / kWave doubles.  Contains barriers: call from every thread.
template <int NT = kBlock>
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / kWave; ++k) s += sh[k];
    return s;
}

// N sums over a workgroup with one barrier pair: the same fixed order per
// sum as block_sum.  `sh` holds N * NT / 64 doubles; thread k < N returns sum k.
// tx: the thread's index among the NT threads summed (a wider workgroup may
// run several such groups side by side, each with its own `sh`; every thread
// of the workgroup must call it, since it contains workgroup barriers).
template <int N, int NT = kBlock>
__device__ __forceinline__ double block_sum_n(const double (&v)[N], double *sh, int tx) {
    const int lane = tx & (kWave - 1), wid = tx / kWave;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double w = wave_sum(v[k]);
        if (lane == 0) sh[k * (NT / kWave) + wid] = w;
    }
    __syncthreads();
    double s = 0.0;
    if (tx < N)
        for (int k = 0; k < NT / kWave; ++k) s += sh[tx * (NT / kWave) + k];
    return s;
}
template <int N, int NT = kBlock>
__device__ __forceinline__ double block_sum_n(const double (&v)[N], double *sh) {
    return block_sum_n<N, NT>(v, sh, (int)threadIdx.x);
}

// This thread's share of sum_{k < n} get(k) over a workgroup of NT threads
// (thread t takes k = t, t + NT, ...), with sixteen loads in flight per
// iteration and four accumulators; the assignment of elements to threads and
// accumulators is fixed, so the result is reproducible.  Combine the threads
// with block_sum.
template <int NT = kBlock, class Get>
__device__ __forceinline__ double thread_share_sum(int n, Get get) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = threadIdx.x;
    for (; k + 15 * NT < n; k += 16 * NT) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = get(k + q * NT);
#pragma unroll
        for (int q = 0; q < 16; q += 4) {
            s0 += v[q];
            s1 += v[q + 1];
            s2 += v[q + 2];
            s3 += v[q + 3];
        }
    }
    for (; k < n; k += NT) s0 += get(k);
    return ((s0 + s1) + s2) + s3;
}

// Inclusive scan of one value per thread across a workgroup of NT threads
// (wave shuffles, then the wave totals); `wtot` holds NT / 64 ints in LDS and
// may be reused only after a barrier.  Every thread must call it.
template <int NT = kBlock>
__device__ __forceinline__ int block_inclusive_scan1(int v, int *wtot, int &total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    if (lane == kWave - 1) wtot[w] = v;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / kWave; ++k) {
        const int t = wtot[k];
        base += k < w ? t : 0;
        tot += t;
    }
    total = tot;
    return v + base;
}

// Exclusive scan of a[0..n) in LDS by a workgroup of NT threads; a[n]
// receives the total.  `tmp` holds NT ints.  Every thread must call it.
template <int NT = kBlock>
__device__ void block_exclusive_scan(int *a, int n, int *tmp) {
    const int tid = threadIdx.x;
    const int per = (n + NT - 1) / NT;
    const int lo = tid * per;
    const int hi = min(lo + per, n);
    int s = 0;
    for (int k = lo; k < hi; ++k) s += a[k];
    tmp[tid] = s;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
        int v = tid >= off ? tmp[tid - off] : 0;
        __syncthreads();
        tmp[tid] += v;
        __syncthreads();
    }
    int run = tmp[tid] - s;
    for (int k = lo; k < hi; ++k) {
        int c = a[k];
        a[k] = run;
        run += c;
    }
    if (tid == NT - 1) a[n] = tmp[NT - 1];
    __syncthreads();
}

}  // namespace osim
