// Sonar image formation kernels for gfx950 (Sec. III-A.2 of arXiv 2503.01074).
//
// Forward, per frame:
//   k_bin   one workgroup per chunk of returns: Eq. (2) intensity and bin of
//           every return, then an LDS counting sort of the chunk by polar tile
//           (a tile is a block of whole range rows).  Writes the chunk's
//           (tile-local bin, intensity) pairs grouped by tile and the chunk's
//           per-tile offsets.  No global atomics.
//   k_tile  one workgroup per polar tile: gathers the tile's pairs from every
//           chunk and sums them into an LDS histogram (binning by summation),
//           then applies the gain and the speckle of Eq. (3)-(6) per bin and
//           streams the tile out row-major.
//   k_fan   one thread per mirror pair of fan pixels: FP64 polar coordinates,
//           bilinear interpolation of the polar image.
// Backward, per frame:
//   k_tile_bwd  one workgroup per polar tile: transpose of the fan as a gather
//               of the fan pixels whose stencil touches the tile, accumulated
//               in LDS in 64-bit fixed point (order-independent, so the sums
//               are bit-reproducible), plus the polar gradient; adjoint of the
//               additive speckle term (sigma_phi, sigma_sa partial sums).
//   k_ret_bwd   one workgroup per chunk of returns: adjoint of binning as a
//               gather of the bin gradient at each return, then of gain,
//               multiplicative speckle and Eq. (2) (alpha, gain, sigma_sm and
//               reflectivity partial sums).
#include "device.hpp"
#include "launch.hpp"

namespace osim {

// ---------------------------------------------------------------------------
// Exclusive scan of a[0..n) in LDS by one workgroup; a[n] receives the total.
// `tmp` holds kBlock ints.  Every thread must call it.
// ---------------------------------------------------------------------------
__device__ void block_exclusive_scan(int *a, int n, int *tmp) {
    const int tid = threadIdx.x;
    const int per = (n + kBlock - 1) / kBlock;
    const int lo = tid * per;
    const int hi = min(lo + per, n);
    int s = 0;
    for (int k = lo; k < hi; ++k) s += a[k];
    tmp[tid] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the kBlock partial sums
    for (int off = 1; off < kBlock; off <<= 1) {
        int v = tid >= off ? tmp[tid - off] : 0;
        __syncthreads();
        tmp[tid] += v;
        __syncthreads();
    }
    int run = tmp[tid] - s;   // exclusive prefix of this thread's segment
    for (int k = lo; k < hi; ++k) {
        int c = a[k];
        a[k] = run;
        run += c;
    }
    if (tid == kBlock - 1) a[n] = tmp[kBlock - 1];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// k_bin
// ---------------------------------------------------------------------------
template <class Src, int R>
__global__ __launch_bounds__(kBlock) void k_bin(Src src, const oceansim_sonar_params *params,
                                                const float *refl, int n_mat) {
    extern __shared__ int4 lds_raw[];
    int local;
    const int fi = src.locate(blockIdx.x, KBIN, local);
    const SonarDev &f = src.frame(fi);
    const int tid = threadIdx.x;
    const int n_tiles = f.n_tiles;
    int *hist = reinterpret_cast<int *>(lds_raw);                    // n_tiles + 1
    __shared__ int scan_tmp[kBlock];
    uint2 *stage = reinterpret_cast<uint2 *>(hist + ((n_tiles + 1 + 3) & ~3));  // R * kBlock

    const float alpha = params[f.param_row].alpha;
    const long long base = (long long)local * (R * kBlock);

    for (int t = tid; t <= n_tiles; t += kBlock) hist[t] = 0;
    __syncthreads();

    int tile[R], rank[R];
    uint32_t lbin[R];
    float inten[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const long long k = base + (long long)q * kBlock + tid;
        tile[q] = -1;
        if (k < f.n) {
            const float xf = f.x[k], yf = f.y[k], zf = f.z[k];
            const int m = f.mat[k];
            double r;
            const int b = return_bin(f, xf, yf, zf, m, n_mat, r);
            if (f.bin_of_return) f.bin_of_return[k] = b;
            if (b >= 0) {
                float cosg, att;
                inten[q] = return_intensity(f, xf, yf, zf, f.nx[k], f.ny[k], f.nz[k], r, refl[m],
                                            alpha, cosg, att);
                const int i = b / f.n_az;
                const int t = i / f.rows_per_tile;
                tile[q] = t;
                lbin[q] = (uint32_t)(b - t * f.tile_bins);
                rank[q] = atomicAdd(&hist[t], 1);
            }
        }
    }
    __syncthreads();
    block_exclusive_scan(hist, n_tiles, scan_tmp);

    int *off = f.chunk_off + (long long)local * (n_tiles + 1);
    for (int t = tid; t <= n_tiles; t += kBlock) off[t] = hist[t];
#pragma unroll
    for (int q = 0; q < R; ++q)
        if (tile[q] >= 0)
            stage[hist[tile[q]] + rank[q]] = make_uint2(lbin[q], __float_as_uint(inten[q]));
    __syncthreads();
    const int total = hist[n_tiles];
    uint2 *dst = f.pairs + base;
    for (int k = tid; k < total; k += kBlock) dst[k] = stage[k];
}

// ---------------------------------------------------------------------------
// k_tile
// ---------------------------------------------------------------------------
template <class Src>
__global__ __launch_bounds__(kBlock) void k_tile(Src src, const oceansim_sonar_params *params) {
    extern __shared__ int4 lds_raw[];
    float *acc = reinterpret_cast<float *>(lds_raw);
    int tile;
    const int fi = src.locate(blockIdx.x, KTILE, tile);
    const SonarDev &f = src.frame(fi);
    const int tid = threadIdx.x;
    const long long nb = (long long)f.n_range * f.n_az;
    const long long b_lo = (long long)tile * f.tile_bins;
    const long long b_hi = min(b_lo + (long long)f.tile_bins, nb);
    const int nbins = (int)(b_hi - b_lo);

    for (int k = tid; k < nbins; k += kBlock) acc[k] = 0.0f;
    __syncthreads();

    // binning by summation: every chunk's segment for this tile
    const int stride = f.n_tiles + 1;
    for (int c = tid; c < f.n_chunks; c += kBlock) {
        const int *off = f.chunk_off + (long long)c * stride + tile;
        const int s = off[0], e = off[1];
        const uint2 *p = f.pairs + (long long)c * f.chunk;
        for (int k = s; k < e; ++k) {
            const uint2 q = p[k];
            if (q.x < (uint32_t)nbins) atomicAdd(&acc[q.x], __uint_as_float(q.y));
        }
    }
    __syncthreads();

    const oceansim_sonar_params pr = params[f.param_row];
    const float G = pr.gain;
    // groups of four consecutive frame-linear bins share one additive Philox call
    const long long q_first = b_lo >> 2, q_last = (b_hi - 1) >> 2;
    for (long long q = q_first + tid; q <= q_last; q += kBlock) {
        const long long b0 = q << 2;
        float P[4], out[4];
        bool in[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const long long b = b0 + w;
            in[w] = b >= b_lo && b < b_hi;
            P[w] = in[w] ? acc[b - b_lo] : 0.0f;
        }
        if (f.speckle == SPECKLE_OFF) {
#pragma unroll
            for (int w = 0; w < 4; ++w) out[w] = G * P[w];
        } else {
            const Words wd = philox((uint32_t)q, f.frame_id, 0u, 0u, f.seed_lo, f.seed_hi);
            int i = (int)(b0 / f.n_az);
            int j = (int)(b0 - (long long)i * f.n_az);
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const float R = range_ramp(f, i);
                const float phi = bin_azimuth(f, j);
                const float E = expf(-(phi * phi) / pr.sigma_phi);
                const float rho = rayleigh_of_word(pick(wd, (uint32_t)w));
                const float add = R * (1.0f + 0.5f * E * (pr.sigma_sa * rho));
                float m = 0.0f, gz;
                if (P[w] != 0.0f) m = speckle_factor(f, (uint32_t)(b0 + w), pr.sigma_sm, &gz);
                out[w] = (G * P[w]) * m + add;
                if (++j == f.n_az) { j = 0; ++i; }
            }
        }
        if (in[0] && in[3]) {
            *reinterpret_cast<float4 *>(f.polar + b0) = make_float4(out[0], out[1], out[2], out[3]);
        } else {
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (in[w]) f.polar[b0 + w] = out[w];
        }
    }
}

// ---------------------------------------------------------------------------
// k_fan: pixel u (left half, x <= 0) and its mirror W-1-u share rho and |phi|.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fan_sample(const SonarDev &f, const float *img, double rho,
                                            double phi) {
    Stencil st;
    if (!fan_stencil(f, rho, phi, st)) return 0.0f;
    const long long r0 = (long long)st.i0 * f.n_az, r1 = (long long)st.i1 * f.n_az;
    const double a = img[r0 + st.j0], b = img[r0 + st.j1];
    const double c = img[r1 + st.j0], d = img[r1 + st.j1];
    const double t = st.t, s = st.s;
    return (float)((1.0 - t) * (1.0 - s) * a + (1.0 - t) * s * b + t * (1.0 - s) * c + t * s * d);
}

// Polar position of left-half pixel (v, u): rho and the azimuth |phi| >= 0.
__device__ __forceinline__ void fan_left(const SonarDev &f, int v, int u, double &rho,
                                         double &phi_pos) {
    const double ax = (0.5 * (double)f.fan_w - (double)u - 0.5) * f.fan_s;   // = -x_c >= 0
    const double yc = ((double)f.fan_h - (double)v - 0.5) * f.fan_s;
    rho = __builtin_sqrt(ax * ax + yc * yc);
    phi_pos = atan2(ax, yc);
}

template <class Src>
__global__ __launch_bounds__(kBlock) void k_fan(Src src) {
    int local;
    const int fi = src.locate(blockIdx.x, KFAN, local);
    const SonarDev &f = src.frame(fi);
    const int v = local / f.fan_bpr;
    const int u = (local - v * f.fan_bpr) * kBlock + threadIdx.x;
    const int half_w = (f.fan_w + 1) >> 1;
    if (u >= half_w) return;
    double rho, phi;
    fan_left(f, v, u, rho, phi);
    float *row = f.fan + (long long)v * f.fan_w;
    row[u] = fan_sample(f, f.polar, rho, phi);
    const int um = f.fan_w - 1 - u;
    if (um != u) row[um] = fan_sample(f, f.polar, rho, -phi);
}

// ---------------------------------------------------------------------------
// k_tile_bwd
// ---------------------------------------------------------------------------
constexpr int kRowBatch = 1024;

// Left-half pixel interval [ua, ub] of fan row v whose centres may lie within
// radial distance [rlo, rhi] of the apex and inside the sector (with a
// one-pixel margin; the exact stencil test decides membership).
__device__ __forceinline__ void row_interval(const SonarDev &f, int v, double rlo, double rhi,
                                             int &ua, int &ub) {
    const double s = f.fan_s;
    const double y = ((double)f.fan_h - (double)v - 0.5) * s;
    ua = 1;
    ub = 0;
    if (y > rhi) return;
    double xo = __builtin_sqrt(rhi * rhi - y * y);
    if (f.half_az < 1.5707963267948966) {
        const double xs = y * f.tan_half_az + s;
        xo = xo < xs ? xo : xs;
    }
    const double xi = rlo > y ? __builtin_sqrt(rlo * rlo - y * y) : 0.0;
    if (xi > xo) return;
    // left half: x in [-xo, -xi]  ->  u = x / s + W/2 - 1/2
    const double c = 0.5 * (double)f.fan_w - 0.5;
    double a = -xo / s + c, b = -xi / s + c;
    int half_w = (f.fan_w + 1) >> 1;
    int lo = (int)__builtin_floor(a) - 1, hi = (int)__builtin_ceil(b) + 1;
    lo = lo < 0 ? 0 : lo;
    hi = hi > half_w - 1 ? half_w - 1 : hi;
    ua = lo;
    ub = hi;
}

template <class Src>
__global__ __launch_bounds__(kBlock) void k_tile_bwd(Src src, const oceansim_sonar_params *params,
                                                     double *part, int *part_row,
                                                     float *grad_refl_zero, int n_mat_zero) {
    extern __shared__ int4 lds_raw[];
    long long *acc = reinterpret_cast<long long *>(lds_raw);
    __shared__ int row_u0[kRowBatch];
    __shared__ int row_pre[kRowBatch + 1];
    __shared__ unsigned poison[kMaxTileBins / 32];
    __shared__ double red[kBlock / kWave];
    __shared__ int scan_tmp[kBlock];
    __shared__ double sh_scale;

    int tile;
    const int fi = src.locate(blockIdx.x, KTILE, tile);
    const SonarDev &f = src.frame(fi);
    const int tid = threadIdx.x;

    // the atomic reflectivity path (many materials) accumulates into a zeroed table
    if (grad_refl_zero)
        for (int k = blockIdx.x * kBlock + tid; k < n_mat_zero; k += gridDim.x * kBlock)
            grad_refl_zero[k] = 0.0f;

    const long long nb = (long long)f.n_range * f.n_az;
    const long long b_lo = (long long)tile * f.tile_bins;
    const long long b_hi = min(b_lo + (long long)f.tile_bins, nb);
    const int nbins = (int)(b_hi - b_lo);
    const int ia = tile * f.rows_per_tile;
    const int ib = min(ia + f.rows_per_tile, f.n_range);

    for (int k = tid; k < nbins; k += kBlock) acc[k] = 0;
    for (int k = tid; k < (nbins + 31) / 32; k += kBlock) poison[k] = 0u;
    if (tid == 0) sh_scale = 0.0;
    __syncthreads();

    const bool have_fan = f.grad_fan != nullptr && f.fan_h > 0 && f.fan_w > 0;
    if (have_fan) {
        const double s = f.fan_s;
        double rlo = f.r_min + ((double)ia - 0.5) * f.dr - s;
        double rhi = f.r_min + ((double)ib + 0.5) * f.dr + s;
        rlo = rlo < 0.0 ? 0.0 : rlo;
        const double rmax_s = f.r_max + s;
        rhi = rhi > rmax_s ? rmax_s : rhi;
        const double ymin = rlo * cos(f.half_az < 1.5707963267948966 ? f.half_az : 1.5707963267948966) - s;
        const double ymax = rhi + s;
        const double H = (double)f.fan_h;
        int v_lo = (int)__builtin_floor(H - 0.5 - ymax / s);
        int v_hi = (int)__builtin_ceil(H - 0.5 - (ymin > 0.0 ? ymin : 0.0) / s);
        v_lo = v_lo < 0 ? 0 : v_lo;
        v_hi = v_hi > f.fan_h - 1 ? f.fan_h - 1 : v_hi;
        const int W = f.fan_w;

        // two passes over the candidate pixels: the largest |gradient| fixes
        // the fixed-point scale, then the stencil contributions are added
        for (int pass = 0; pass < 2; ++pass) {
            double local_max = 0.0, local_cnt = 0.0;
            for (int vb = v_lo; vb <= v_hi; vb += kRowBatch) {
                const int nrows = min(kRowBatch, v_hi - vb + 1);
                __syncthreads();
                for (int rr = tid; rr < nrows; rr += kBlock) {
                    int ua, ub;
                    row_interval(f, vb + rr, rlo, rhi, ua, ub);
                    row_u0[rr] = ua;
                    row_pre[rr] = ub >= ua ? ub - ua + 1 : 0;
                }
                __syncthreads();
                block_exclusive_scan(row_pre, nrows, scan_tmp);
                const int total = row_pre[nrows];
                for (int idx = tid; idx < total; idx += kBlock) {
                    int lo = 0, hi = nrows - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (row_pre[mid] <= idx) lo = mid; else hi = mid - 1;
                    }
                    const int v = vb + lo;
                    const int u = row_u0[lo] + (idx - row_pre[lo]);
                    const int um = W - 1 - u;
                    const float *grow = f.grad_fan + (long long)v * W;
                    const float g0 = grow[u];
                    const float g1 = um != u ? grow[um] : 0.0f;
                    if (pass == 0) {
                        const double a0 = __builtin_fabs((double)g0), a1 = __builtin_fabs((double)g1);
                        // a non-finite gradient poisons only its own stencil
                        // (handled in pass 1), so leave it out of the scale
                        if (a0 == a0 && a0 <= 1.7976931348623157e308 && a0 > local_max) local_max = a0;
                        if (a1 == a1 && a1 <= 1.7976931348623157e308 && a1 > local_max) local_max = a1;
                        local_cnt += 2.0;
                        continue;
                    }
                    const double scale = sh_scale;
                    double rho, phi;
                    fan_left(f, v, u, rho, phi);
                    for (int side = 0; side < 2; ++side) {
                        if (side == 1 && um == u) break;
                        const float g = side == 0 ? g0 : g1;
                        if (g == 0.0f) continue;
                        Stencil st;
                        if (!fan_stencil(f, rho, side == 0 ? phi : -phi, st)) continue;
                        if (st.i1 < ia || st.i0 >= ib) continue;
                        const bool finite = __builtin_isfinite(g);
                        const double gd = (double)g;
                        const int ii[2] = {st.i0, st.i1};
                        const int jj[2] = {st.j0, st.j1};
                        const double wr[2] = {1.0 - st.t, st.t};
                        const double wc[2] = {1.0 - st.s, st.s};
#pragma unroll
                        for (int a = 0; a < 2; ++a) {
                            if (ii[a] < ia || ii[a] >= ib) continue;
                            if (a == 1 && ii[1] == ii[0]) continue;
#pragma unroll
                            for (int c = 0; c < 2; ++c) {
                                if (c == 1 && jj[1] == jj[0]) continue;
                                const int lb = (ii[a] - ia) * f.n_az + jj[c];
                                const double w = wr[a] * wc[c];
                                if (!finite) {
                                    atomicOr(&poison[lb >> 5], 1u << (lb & 31));
                                    continue;
                                }
                                const long long qv = __double2ll_rn(w * gd * scale);
                                if (qv != 0)
                                    atomicAdd(reinterpret_cast<unsigned long long *>(&acc[lb]),
                                              (unsigned long long)qv);
                            }
                        }
                    }
                }
            }
            if (pass == 0) {
                // workgroup max of |g| and of the candidate count
                double mx = local_max;
                for (int off = 32; off > 0; off >>= 1) {
                    const double o = __shfl_down(mx, off, kWave);
                    mx = o > mx ? o : mx;
                }
                const double cnt = block_sum(local_cnt, red);   // thread 0
                __syncthreads();
                if ((tid & (kWave - 1)) == 0) red[tid / kWave] = mx;
                __syncthreads();
                if (tid == 0) {
                    double m = 0.0;
                    for (int k = 0; k < kBlock / kWave; ++k) m = red[k] > m ? red[k] : m;
                    // |sum| <= cnt * max < 2^62 after scaling
                    double sc = 0.0;
                    if (m > 0.0) {
                        int e;
                        frexp(m * (cnt > 1.0 ? cnt : 1.0), &e);
                        sc = ldexp(1.0, 61 - e);
                    }
                    sh_scale = sc;
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }

    // epilogue: fixed point -> float, plus the polar gradient; adjoint of Eq. (3)-(4)
    const oceansim_sonar_params pr = params[f.param_row];
    const double inv_scale = (have_fan && sh_scale > 0.0) ? 1.0 / sh_scale : 0.0;
    double g_sphi = 0.0, g_ssa = 0.0;
    const long long q_first = b_lo >> 2, q_last = (b_hi - 1) >> 2;
    for (long long q = q_first + tid; q <= q_last; q += kBlock) {
        const long long b0 = q << 2;
        Words wd{0u, 0u, 0u, 0u};
        if (f.speckle != SPECKLE_OFF) wd = philox((uint32_t)q, f.frame_id, 0u, 0u, f.seed_lo, f.seed_hi);
        int i = (int)(b0 / f.n_az);
        int j = (int)(b0 - (long long)i * f.n_az);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const long long b = b0 + w;
            if (b >= b_lo && b < b_hi) {
                const int lb = (int)(b - b_lo);
                double g = (double)acc[lb] * inv_scale;
                if (poison[lb >> 5] & (1u << (lb & 31))) g = __builtin_nan("");
                if (f.grad_polar) g += (double)f.grad_polar[b];
                f.grad_img[b] = (float)g;
                if (f.speckle != SPECKLE_OFF) {
                    const double R = (double)range_ramp(f, i);
                    const double phi = (double)bin_azimuth(f, j);
                    const double E = (double)expf(-((float)phi * (float)phi) / pr.sigma_phi);
                    const double rho = (double)rayleigh_of_word(pick(wd, (uint32_t)w));
                    // d add / d sigma_sa and d add / d sigma_phi of Eq. (3)-(4)
                    g_ssa += g * R * 0.5 * E * rho;
                    g_sphi += g * R * 0.5 * (double)pr.sigma_sa * rho * E * (phi * phi) /
                              ((double)pr.sigma_phi * (double)pr.sigma_phi);
                }
            }
            if (++j == f.n_az) { j = 0; ++i; }
        }
    }
    const double s_phi = block_sum(g_sphi, red);
    const double s_sa = block_sum(g_ssa, red);
    if (tid == 0) {
        const int slot = blockIdx.x;
        double *p = part + (long long)slot * 5;
        p[0] = 0.0;
        p[1] = 0.0;
        p[2] = s_phi;
        p[3] = s_sa;
        p[4] = 0.0;
        part_row[slot] = f.param_row;
    }
}

// ---------------------------------------------------------------------------
// k_ret_bwd
// ---------------------------------------------------------------------------
template <class Src, int R>
__global__ __launch_bounds__(kBlock) void k_ret_bwd(Src src, const oceansim_sonar_params *params,
                                                    const float *refl, int n_mat, double *part,
                                                    int *part_row, int slot_base,
                                                    double *refl_part, float *grad_refl_atomic) {
    extern __shared__ int4 lds_raw[];
    // thread-private reflectivity columns [n_mat][kBlock] (small tables); the
    // same memory later serves the workgroup reductions
    float *hist = reinterpret_cast<float *>(lds_raw);
    double *red = reinterpret_cast<double *>(lds_raw);
    int local;
    const int fi = src.locate(blockIdx.x, KRET, local);
    const SonarDev &f = src.frame(fi);
    const int tid = threadIdx.x;
    const bool lane_hist = refl_part != nullptr;

    if (lane_hist)
        for (int k = tid; k < n_mat * kBlock; k += kBlock) hist[k] = 0.0f;
    __syncthreads();

    const oceansim_sonar_params pr = params[f.param_row];
    const float G = pr.gain;
    double g_alpha = 0.0, g_gain = 0.0, g_ssm = 0.0;
    const long long base = (long long)local * (R * kBlock);
#pragma unroll 4
    for (int q = 0; q < R; ++q) {
        const long long k = base + (long long)q * kBlock + tid;
        if (k >= f.n) break;
        const float xf = f.x[k], yf = f.y[k], zf = f.z[k];
        const int m = f.mat[k];
        double r;
        const int b = return_bin(f, xf, yf, zf, m, n_mat, r);
        if (b < 0) continue;
        float cosg, att;
        const float I = return_intensity(f, xf, yf, zf, f.nx[k], f.ny[k], f.nz[k], r, refl[m],
                                         pr.alpha, cosg, att);
        const float gI_t = f.grad_img[b];          // dL / d(polar image) at this return's bin
        float z = 0.0f;
        const float mult = speckle_factor(f, (uint32_t)b, pr.sigma_sm, &z);
        const double gIt = (double)gI_t;
        const double gI = (double)G * (double)mult * gIt;   // dL / dI_k
        g_alpha += gI * (double)I * (-f.kappa * r);
        g_gain += gIt * (double)mult * (double)I;
        g_ssm += gIt * (double)G * (double)I * (double)z;
        const float gr = (float)(gI * (double)cosg * (double)att);
        if (lane_hist)
            hist[m * kBlock + tid] += gr;
        else
            atomicAdd(&grad_refl_atomic[m], gr);
    }
    if (lane_hist) {
        __syncthreads();
        // fixed order: threads 0..255 of each material column
        for (int mm = tid; mm < n_mat; mm += kBlock) {
            double s = 0.0;
            const float *h = hist + mm * kBlock;
            for (int l = 0; l < kBlock; ++l) s += (double)h[l];
            refl_part[(long long)blockIdx.x * n_mat + mm] = s;
        }
    }
    __syncthreads();
    const double sa = block_sum(g_alpha, red);
    const double sg = block_sum(g_gain, red);
    const double sm = block_sum(g_ssm, red);
    const int slot = slot_base + blockIdx.x;
    if (tid == 0) {
        double *p = part + (long long)slot * 5;
        p[0] = sa;
        p[1] = sg;
        p[2] = 0.0;
        p[3] = 0.0;
        p[4] = sm;
        part_row[slot] = f.param_row;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <class Src>
static hipError_t launch_fwd(const Src &src, const SonarGrid &g, const oceansim_sonar_params *params,
                             const float *refl, int n_mat, hipStream_t st) {
    if (g.bin_blocks > 0) {
        const size_t lds = (size_t)((g.max_tiles + 1 + 3) & ~3) * 4 + (size_t)g.chunk * 8;
        switch (g.chunk / kBlock) {
            case 4: hipLaunchKernelGGL((k_bin<Src, 4>), dim3(g.bin_blocks), dim3(kBlock), lds, st, src, params, refl, n_mat); break;
            case 8: hipLaunchKernelGGL((k_bin<Src, 8>), dim3(g.bin_blocks), dim3(kBlock), lds, st, src, params, refl, n_mat); break;
            case 16: hipLaunchKernelGGL((k_bin<Src, 16>), dim3(g.bin_blocks), dim3(kBlock), lds, st, src, params, refl, n_mat); break;
            default: return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_tile<Src>), dim3(g.tile_blocks), dim3(kBlock), (size_t)g.max_tile_bins * 4, st,
                       src, params);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g.fan_blocks > 0) {
        hipLaunchKernelGGL((k_fan<Src>), dim3(g.fan_blocks), dim3(kBlock), 0, st, src);
        e = hipGetLastError();
    }
    return e;
}

template <class Src>
static hipError_t launch_bwd(const Src &src, const SonarGrid &g, const oceansim_sonar_params *params,
                             const float *refl, int n_mat, double *part, int *part_row,
                             double *refl_part, float *grad_refl, hipStream_t st) {
    const bool lane_hist = n_mat <= kLaneHistMats;
    hipLaunchKernelGGL((k_tile_bwd<Src>), dim3(g.tile_blocks), dim3(kBlock), (size_t)g.max_tile_bins * 8, st,
                       src, params, part, part_row, lane_hist ? (float *)nullptr : grad_refl, n_mat);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g.ret_blocks > 0) {
        size_t lds = lane_hist ? (size_t)n_mat * kBlock * 4 : 0;
        if (lds < (size_t)(kBlock / kWave) * 8) lds = (size_t)(kBlock / kWave) * 8;
        double *rp = lane_hist ? refl_part : nullptr;
        float *ga = lane_hist ? nullptr : grad_refl;
        switch (g.ret_chunk / kBlock) {
            case 4: hipLaunchKernelGGL((k_ret_bwd<Src, 4>), dim3(g.ret_blocks), dim3(kBlock), lds, st, src, params, refl, n_mat, part, part_row, g.tile_blocks, rp, ga); break;
            case 8: hipLaunchKernelGGL((k_ret_bwd<Src, 8>), dim3(g.ret_blocks), dim3(kBlock), lds, st, src, params, refl, n_mat, part, part_row, g.tile_blocks, rp, ga); break;
            case 16: hipLaunchKernelGGL((k_ret_bwd<Src, 16>), dim3(g.ret_blocks), dim3(kBlock), lds, st, src, params, refl, n_mat, part, part_row, g.tile_blocks, rp, ga); break;
            default: return hipErrorInvalidValue;
        }
        e = hipGetLastError();
    }
    return e;
}

hipError_t sonar_forward_one(const SonarDev &f, const SonarGrid &g, const oceansim_sonar_params *params,
                             const float *refl, int n_mat, hipStream_t st) {
    return launch_fwd(One<SonarDev>{f}, g, params, refl, n_mat, st);
}
hipError_t sonar_forward_table(const SonarDev *t, int n, const SonarGrid &g,
                               const oceansim_sonar_params *params, const float *refl, int n_mat,
                               hipStream_t st) {
    return launch_fwd(Table<SonarDev>{t, n}, g, params, refl, n_mat, st);
}
hipError_t sonar_backward_one(const SonarDev &f, const SonarGrid &g, const oceansim_sonar_params *params,
                              const float *refl, int n_mat, double *part, int *part_row,
                              double *refl_part, float *grad_refl, hipStream_t st) {
    return launch_bwd(One<SonarDev>{f}, g, params, refl, n_mat, part, part_row, refl_part, grad_refl, st);
}
hipError_t sonar_backward_table(const SonarDev *t, int n, const SonarGrid &g,
                                const oceansim_sonar_params *params, const float *refl, int n_mat,
                                double *part, int *part_row, double *refl_part, float *grad_refl,
                                hipStream_t st) {
    return launch_bwd(Table<SonarDev>{t, n}, g, params, refl, n_mat, part, part_row, refl_part, grad_refl, st);
}

}  // namespace osim
