// Underwater colour image formation, Eq. (1) of arXiv 2503.01074 (Sec. III-A.1),
// and its adjoint, for gfx950: the camera kernels and the fixed-order
// reductions of per-workgroup partial sums.
//
// A pure streaming kernel: 28 bytes per pixel forward (J, d in; I out), read
// and written as float4 on planar [3][H][W] images.  The backward kernel
// reduces the nine parameter gradients per workgroup in FP64 and a fixed
// order; the final per-row sum is reduce_rows.
#include "reduce_body.hpp"
#include "uw_body.hpp"

namespace osim {

template <class Src>
__global__ __launch_bounds__(kBlock) void k_uw(Src src, const oceansim_water_params *params) {
    uw_fwd_block<Src, kBlock>(src, params, blockIdx.x, threadIdx.x);
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
__global__ __launch_bounds__(kBlock) void k_reduce_rows(RowsReduce a) {
    __shared__ double red[kBlock / kWave];
    rows_reduce_block(a, blockIdx.x, red);
}

// The sonar reduction's workgroups, then the row-keyed reduction's.
__global__ __launch_bounds__(kBlock) void k_reduce_pair(SonarReduce s, RowsReduce r) {
    __shared__ double red[kBlock / kWave];
    if ((int)blockIdx.x < s.blocks)
        sonar_reduce_block(s, blockIdx.x, red);
    else
        rows_reduce_block(r, blockIdx.x - s.blocks, red);
}

static RowsReduce rows_args(const double *part, const int *row, int n_slots, int width, int n_rows, float *out,
                            int out_stride) {
    RowsReduce a;
    a.part = part;
    a.row = row;
    a.n_slots = n_slots;
    a.width = width;
    a.out = out;
    a.out_stride = out_stride;
    a.blocks = n_rows * out_stride;
    return a;
}

hipError_t reduce_rows(const double *part, const int *row, int n_slots, int width, int n_rows, float *out,
                       int out_stride, hipStream_t st) {
    const RowsReduce a = rows_args(part, row, n_slots, width, n_rows, out, out_stride);
    OSIM_LAUNCH("k_reduce_rows", k_reduce_rows, dim3(a.blocks), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t reduce_pair(const SonarReduce &s, const RowsReduce &r, hipStream_t st) {
    OSIM_LAUNCH("k_reduce_pair", k_reduce_pair, dim3(s.blocks + r.blocks), dim3(kBlock), 0, st, s, r);
    return hipGetLastError();
}


}  // namespace osim
