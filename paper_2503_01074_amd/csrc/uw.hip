// Underwater colour image formation, Eq. (1) of arXiv 2503.01074 (Sec. III-A.1),
// and its adjoint, for gfx950: the camera kernels and the fixed-order
// reductions of per-workgroup partial sums.
//
// A pure streaming kernel: 28 bytes per pixel forward (J, d in; I out), read
// and written as float4 on planar [3][H][W] images.  The backward kernel
// reduces the nine parameter gradients per workgroup in FP64 and a fixed
// order; the final per-row sum is reduce_rows.
#include "uw_body.hpp"

namespace osim {

template <class Src>
__global__ __launch_bounds__(kBlock) void k_uw(Src src, const oceansim_water_params *params) {
    uw_fwd_block<Src, kBlock>(src, params, blockIdx.x);
}

template <class Src>
__global__ __launch_bounds__(kBlock) void k_uw_bwd(Src src, const oceansim_water_params *params,
                                                   double *part, int *part_row) {
    __shared__ double red9[9 * (kBlock / kWave)];
    uw_bwd_block<Src, kBlock>(src, params, part, part_row, blockIdx.x, gridDim.x, red9);
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
    if (c < width) {
        // column c of the column-major partials, slots of row r
        const double *a = part + (long long)c * n_slots;
        s = thread_share_sum(n_slots, [&](int k) {
            const double v = a[k];   // both loads issued; the row decides
            return row[k] == r ? v : 0.0;
        });
    }
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) out[(long long)r * out_stride + c] = c < width ? (float)tot : 0.0f;
}

__global__ __launch_bounds__(kBlock) void k_reduce_cols(const double *part, int n_slots, int width,
                                                        float *out) {
    __shared__ double red[kBlock / kWave];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int k = threadIdx.x; k < n_slots; k += kBlock) s += part[(long long)c * n_slots + k];
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
