// Underwater colour image formation, Eq. (1) of arXiv 2503.01074 (Sec. III-A.1),
// and its adjoint, for gfx950.
//
//   I_c = J_c exp(-beta_D,c d) + B_inf,c (1 - exp(-beta_B,c d))
//
// A pure streaming kernel: 28 bytes per pixel forward (J, d in; I out), read
// and written as float4 on planar [3][H][W] images, 16 pixels per thread.
// The backward kernel reduces the nine parameter gradients per workgroup in
// FP64 and a fixed order; the final per-row sum is reduce_rows.
#include "device.hpp"
#include "launch.hpp"

namespace osim {

struct Water {
    float bd[3], bb[3], bi[3];
};

__device__ __forceinline__ Water load_water(const oceansim_water_params *p, int row) {
    Water w;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        w.bd[c] = p[row].beta_d[c];
        w.bb[c] = p[row].beta_b[c];
        w.bi[c] = p[row].b_inf[c];
    }
    return w;
}

// beta * d, taken as 0 when beta = 0 (so an infinite depth leaves the term alone)
__device__ __forceinline__ float bdprod(float beta, float d) { return beta == 0.0f ? 0.0f : beta * d; }

__device__ __forceinline__ float uw_pixel(float J, float d, float bd, float bb, float bi) {
    const float T = expf(-bdprod(bd, d));
    const float S1 = -expm1f(-bdprod(bb, d));
    return J * T + bi * S1;
}

template <class Src>
__global__ __launch_bounds__(kBlock) void k_uw(Src src, const oceansim_water_params *params) {
    int local;
    const int fi = src.locate(blockIdx.x, 0, local);
    const UwDev &f = src.frame(fi);
    const Water w = load_water(params, f.param_row);
    const long long npix = f.npix;
    const long long p0 = (long long)local * kUwPixelsPerBlock;
    const bool vec = (npix & 3) == 0;
#pragma unroll
    for (int it = 0; it < kUwPixelsPerBlock / (kBlock * 4); ++it) {
        const long long p = p0 + ((long long)it * kBlock + threadIdx.x) * 4;
        if (p >= npix) break;
        if (vec) {
            const float4 d = *reinterpret_cast<const float4 *>(f.depth + p);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float4 J = *reinterpret_cast<const float4 *>(f.J + c * npix + p);
                float4 o;
                o.x = uw_pixel(J.x, d.x, w.bd[c], w.bb[c], w.bi[c]);
                o.y = uw_pixel(J.y, d.y, w.bd[c], w.bb[c], w.bi[c]);
                o.z = uw_pixel(J.z, d.z, w.bd[c], w.bb[c], w.bi[c]);
                o.w = uw_pixel(J.w, d.w, w.bd[c], w.bb[c], w.bi[c]);
                *reinterpret_cast<float4 *>(f.out + c * npix + p) = o;
            }
        } else {
            for (long long q = p; q < p + 4 && q < npix; ++q) {
                const float d = f.depth[q];
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    f.out[c * npix + q] = uw_pixel(f.J[c * npix + q], d, w.bd[c], w.bb[c], w.bi[c]);
            }
        }
    }
}

// Adjoint of Eq. (1) at one pixel and channel; accumulates the parameter
// gradients and returns dL/dJ, adding this channel's share of dL/dd.
__device__ __forceinline__ float uw_pixel_bwd(float g, float J, float d, float bd, float bb, float bi,
                                              double acc[9], int c, float &gd) {
    const float T = expf(-bdprod(bd, d));
    const float S = expf(-bdprod(bb, d));
    const float S1 = -expm1f(-bdprod(bb, d));
    // the d-weighted terms vanish where T or S does (0 * inf := 0)
    if (T != 0.0f) acc[c] += (double)(g * (-J * T * d));
    if (S != 0.0f) acc[3 + c] += (double)(g * (bi * S * d));
    acc[6 + c] += (double)(g * S1);
    gd += g * (-bd * J * T + bi * bb * S);
    return g * T;
}

template <class Src>
__global__ __launch_bounds__(kBlock) void k_uw_bwd(Src src, const oceansim_water_params *params,
                                                   double *part, int *part_row) {
    __shared__ double red[kBlock / kWave];
    int local;
    const int fi = src.locate(blockIdx.x, 0, local);
    const UwDev &f = src.frame(fi);
    const Water w = load_water(params, f.param_row);
    const long long npix = f.npix;
    const long long p0 = (long long)local * kUwPixelsPerBlock;
    const bool vec = (npix & 3) == 0;
    double acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.0;
    for (int it = 0; it < kUwPixelsPerBlock / (kBlock * 4); ++it) {
        const long long p = p0 + ((long long)it * kBlock + threadIdx.x) * 4;
        if (p >= npix) break;
        if (vec) {
            const float4 d = *reinterpret_cast<const float4 *>(f.depth + p);
            float4 gdv = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float4 J = *reinterpret_cast<const float4 *>(f.J + c * npix + p);
                const float4 g = *reinterpret_cast<const float4 *>(f.grad_out + c * npix + p);
                float4 gj;
                gj.x = uw_pixel_bwd(g.x, J.x, d.x, w.bd[c], w.bb[c], w.bi[c], acc, c, gdv.x);
                gj.y = uw_pixel_bwd(g.y, J.y, d.y, w.bd[c], w.bb[c], w.bi[c], acc, c, gdv.y);
                gj.z = uw_pixel_bwd(g.z, J.z, d.z, w.bd[c], w.bb[c], w.bi[c], acc, c, gdv.z);
                gj.w = uw_pixel_bwd(g.w, J.w, d.w, w.bd[c], w.bb[c], w.bi[c], acc, c, gdv.w);
                if (f.grad_J) *reinterpret_cast<float4 *>(f.grad_J + c * npix + p) = gj;
            }
            if (f.grad_depth) *reinterpret_cast<float4 *>(f.grad_depth + p) = gdv;
        } else {
            for (long long q = p; q < p + 4 && q < npix; ++q) {
                const float d = f.depth[q];
                float gd = 0.0f;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float gj = uw_pixel_bwd(f.grad_out[c * npix + q], f.J[c * npix + q], d,
                                                  w.bd[c], w.bb[c], w.bi[c], acc, c, gd);
                    if (f.grad_J) f.grad_J[c * npix + q] = gj;
                }
                if (f.grad_depth) f.grad_depth[q] = gd;
            }
        }
    }
    double tot[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) tot[k] = block_sum(acc[k], red);
    if (threadIdx.x == 0) {
        double *o = part + (long long)blockIdx.x * 9;
#pragma unroll
        for (int k = 0; k < 9; ++k) o[k] = tot[k];
        part_row[blockIdx.x] = f.param_row;
    }
}

hipError_t uw_forward_one(const UwDev &f, int blocks, const oceansim_water_params *params, hipStream_t st) {
    OSIM_LAUNCH("k_uw", (k_uw<One<UwDev>>), dim3(blocks), dim3(kBlock), 0, st, One<UwDev>{f}, params);
    return hipGetLastError();
}
hipError_t uw_forward_table(const UwDev *t, int n, int blocks, const oceansim_water_params *params,
                            hipStream_t st) {
    OSIM_LAUNCH("k_uw", (k_uw<Table<UwDev>>), dim3(blocks), dim3(kBlock), 0, st, Table<UwDev>{t, n}, params);
    return hipGetLastError();
}
hipError_t uw_backward_one(const UwDev &f, int blocks, const oceansim_water_params *params, double *part,
                           int *part_row, hipStream_t st) {
    OSIM_LAUNCH("k_uw_bwd", (k_uw_bwd<One<UwDev>>), dim3(blocks), dim3(kBlock), 0, st, One<UwDev>{f}, params,
                       part, part_row);
    return hipGetLastError();
}
hipError_t uw_backward_table(const UwDev *t, int n, int blocks, const oceansim_water_params *params,
                             double *part, int *part_row, hipStream_t st) {
    OSIM_LAUNCH("k_uw_bwd", (k_uw_bwd<Table<UwDev>>), dim3(blocks), dim3(kBlock), 0, st, Table<UwDev>{t, n},
                       params, part, part_row);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed-order reductions of per-workgroup partial sums.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_reduce_rows(const double *part, const int *row, int n_slots,
                                                        int width, float *out, int out_stride) {
    __shared__ double red[kBlock / kWave];
    const int r = blockIdx.x / out_stride, c = blockIdx.x % out_stride;
    double s = 0.0;
    if (c < width)
        for (int k = threadIdx.x; k < n_slots; k += kBlock)
            if (row[k] == r) s += part[(long long)k * width + c];
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) out[(long long)r * out_stride + c] = c < width ? (float)tot : 0.0f;
}

__global__ __launch_bounds__(kBlock) void k_reduce_cols(const double *part, int n_slots, int width,
                                                        float *out) {
    __shared__ double red[kBlock / kWave];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int k = threadIdx.x; k < n_slots; k += kBlock) s += part[(long long)k * width + c];
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) out[c] = (float)tot;
}

hipError_t reduce_rows(const double *part, const int *row, int n_slots, int width, int n_rows, float *out,
                       int out_stride, hipStream_t st) {
    OSIM_LAUNCH("k_reduce_rows", k_reduce_rows, dim3(n_rows * out_stride), dim3(kBlock), 0, st, part, row, n_slots,
                       width, out, out_stride);
    return hipGetLastError();
}

hipError_t reduce_cols(const double *part, int n_slots, int width, float *out, hipStream_t st) {
    OSIM_LAUNCH("k_reduce_cols", k_reduce_cols, dim3(width), dim3(kBlock), 0, st, part, n_slots, width, out);
    return hipGetLastError();
}

}  // namespace osim
