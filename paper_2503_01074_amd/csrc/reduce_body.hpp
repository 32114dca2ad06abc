// Fixed-order reductions of per-workgroup partial sums, one workgroup per
// output value.  Shared by the sonar and camera backward launches and by the
// plan, which reduces both in one launch.
#pragma once
#include "device.hpp"
#include "launch.hpp"

namespace osim {

// grad_params[r][c] (c < 5) from the slots of the frames using parameter row
// r: tile and return-chunk partials, column-major part[c * n_slots + slot],
// slot rows after the five columns; then one workgroup per material for the
// small reflectivity tables (refl_part column-major [n_mat][ret_slots]).
__device__ __forceinline__ void sonar_reduce_block(const SonarReduce &a, int b, double *red) {
    if (b < a.n_rows * OCEANSIM_SONAR_GRAD_WIDTH) {
        const int r = b / OCEANSIM_SONAR_GRAD_WIDTH, c = b % OCEANSIM_SONAR_GRAD_WIDTH;
        double s = 0.0;
        if (c < 5) {
            const double *col = a.part + (long long)c * a.n_slots;
            const int *row = reinterpret_cast<const int *>(a.part + 5LL * a.n_slots);
            s = thread_share_sum(a.n_slots, [&](int k) {
                const double v = col[k];   // both loads issued; the row decides
                return row[k] == r ? v : 0.0;
            });
        }
        const double tot = block_sum(s, red);
        if (threadIdx.x == 0) a.grad_params[b] = (float)tot;
    } else {
        const int m = b - a.n_rows * OCEANSIM_SONAR_GRAD_WIDTH;
        const double *col = a.refl_part ? a.refl_part + (long long)m * a.ret_slots : nullptr;
        const double s = col ? thread_share_sum(a.ret_slots, [&](int k) { return col[k]; }) : 0.0;
        const double tot = block_sum(s, red);
        if (threadIdx.x == 0) a.grad_refl[m] = (float)tot;
    }
}

// out[r * out_stride + c] = sum over slots s with row[s] == r of
// part[c * n_slots + s] (c < width; the other columns are written 0).
__device__ __forceinline__ void rows_reduce_block(const RowsReduce &a, int b, double *red) {
    const int r = b / a.out_stride, c = b % a.out_stride;
    double s = 0.0;
    if (c < a.width) {
        const double *col = a.part + (long long)c * a.n_slots;
        s = thread_share_sum(a.n_slots, [&](int k) {
            const double v = col[k];
            return a.row[k] == r ? v : 0.0;
        });
    }
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) a.out[(long long)r * a.out_stride + c] = c < a.width ? (float)tot : 0.0f;
}

}  // namespace osim
