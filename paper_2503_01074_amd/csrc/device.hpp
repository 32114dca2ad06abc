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
constexpr int kMaxTileBins = 4096;   // polar bins owned by one tile workgroup (one row at least)
constexpr int kMaxTiles = 4096;      // tiles per frame (LDS histogram in the binning pass)
constexpr int kLaneHistMats = 64;    // materials reduced with lane-private LDS histograms

enum Kind { KBIN = 0, KTILE = 1, KFAN = 2, KRET = 3, KTILEB = 4, KIND_COUNT = 5 };
enum Speckle { SPECKLE_OFF = 0, SPECKLE_PAPER = 1, SPECKLE_GAMMA = 2 };

// --------------------------------------------------------------------------
// One sonar frame as the kernels see it.  Built on the host from the public
// descriptor: float inputs promoted exactly to double, derived constants
// computed once in double.
// --------------------------------------------------------------------------
struct SonarDev {
    const float *x, *y, *z, *nx, *ny, *nz;
    const int *mat;
    float *polar;               // speckled polar image (caller buffer or workspace)
    float *fan;
    int *bin_of_return;
    const float *grad_polar, *grad_fan;
    uint2 *pairs;               // binning pass output: (tile-local bin, intensity)
    int *chunk_off;             // [n_chunks][n_tiles + 1] exclusive offsets per chunk
    float *grad_img;            // backward: dL/d(polar image) [nb]
    long long n;                // returns
    int n_range, n_az, fan_h, fan_w;
    int rows_per_tile, tile_bins, n_tiles;          // forward polar tiles
    int rows_per_tile_b, tile_bins_b, n_tiles_b;    // backward polar tiles
    int chunk, n_chunks;        // returns per binning workgroup, workgroups
    int ret_chunk, n_ret_chunks;// returns per backward-gather workgroup, workgroups
    int fan_bpr, fan_blocks;    // fan: workgroups per pixel row, total
    int speckle, gamma_k, param_row;
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
    int4 *stencil;              // saved fan stencils [fan_h][half_w] or nullptr
};

struct UwDev {
    const float *J, *depth;
    float *out;
    const float *grad_out;
    float *grad_J, *grad_depth;
    long long npix;
    int param_row;
    int blk;                    // first global workgroup
    int n_blocks;
};

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

__device__ __forceinline__ Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        uint64_t a = (uint64_t)c0 * 0xD2511F53u;
        uint64_t b = (uint64_t)c2 * 0xCD9E8D57u;
        uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
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

// Unit Rayleigh variate of bin b (additive stream, Eq. 4 with sigma = 1).
__device__ __forceinline__ float rayleigh_of_word(uint32_t w) {
    return __builtin_amdgcn_sqrtf(2.0f * neg_ln(unit_uniform(w)));
}

// Multiplicative speckle factor of bin b and, in PAPER mode, its standard
// normal draw (Eq. 5-6).  GAMMA: -(1/k) sum ln u_w (a unit-mean Gamma(k, 1/k)).
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
        *gauss_out = 0.0f;
        float acc = 0.0f;
        int k = f.gamma_k;
        for (int g = 0; 4 * g < k; ++g) {
            Words w = philox(b, f.frame_id, 2u, (uint32_t)g, f.seed_lo, f.seed_hi);
            int left = k - 4 * g;
            acc += neg_ln(unit_uniform(w.w0));
            if (left > 1) acc += neg_ln(unit_uniform(w.w1));
            if (left > 2) acc += neg_ln(unit_uniform(w.w2));
            if (left > 3) acc += neg_ln(unit_uniform(w.w3));
        }
        return acc / (float)k;
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
