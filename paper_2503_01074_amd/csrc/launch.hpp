// Host-side launchers of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/oceansim.h"
#include "device.hpp"

namespace osim {

// Event tracing of kernel launches (see oceansim_trace_enable): while tracing
// is on, a TraceScope brackets one launch with events on its stream.
bool trace_active();
void trace_record(const char *name, hipStream_t st, hipEvent_t *a, hipEvent_t *b);
void trace_commit(const char *name, hipStream_t st, hipEvent_t a, hipEvent_t b);
// While set (per thread), launches are being captured into a graph and are not traced.
void set_capturing(bool on);

struct TraceScope {
    const char *name;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    bool on;
    TraceScope(const char *n, hipStream_t s) : name(n), st(s), on(trace_active()) {
        if (on) trace_record(name, st, &a, &b);
    }
    ~TraceScope() {
        if (on) trace_commit(name, st, a, b);
    }
};

#define OSIM_LAUNCH(NAME, ...)                   \
    do {                                         \
        ::osim::TraceScope osim_ts_(NAME, st);   \
        hipLaunchKernelGGL(__VA_ARGS__);         \
    } while (0)

// Launch geometry of one sonar call (all frames).
struct SonarGrid {
    int bin_blocks;      // binning workgroups over all frames
    int tile_blocks;     // forward polar-tile workgroups over all frames
    int tile_b_blocks;   // backward polar-tile workgroups over all frames
    int fan_blocks;      // fan workgroups over all frames
    int ret_blocks;      // backward return-gather workgroups over all frames
    int chunk;           // returns per binning workgroup (256 * R)
    int ret_chunk;       // returns per return-gather workgroup (256 * R)
    int max_tiles;       // largest forward tile count of a frame
    int max_tile_bins;   // largest forward tile of a frame, in bins
    int max_tile_bins_b; // largest backward tile of a frame, in bins
    int all_saved;       // every frame with a fan gradient has saved fan stencils
    int max_n_az;        // widest polar grid of a frame (azimuth cells)
    int fant_blocks;     // backward workgroups of kBlock * fant_bpt bins over all frames (transposed fan operator)
    int fant_bpt;        // bins per thread of those workgroups: 1, 2 or 4
    int use_fant;        // backward through the frames' transposed fan operators instead of polar tiles
    int fant_mirror;     // some frame's operator has the mirrored layout
    int row_blocks;      // backward: one workgroup per range row of the range-normalised frames
    int max_rows_per_tile;   // forward: widest tile (rows) of a range-normalised frame; 0: none
    int pair_bwd;        // backward from the forward's material pairs (k_pair_bwd, one workgroup per forward tile)
    int wide_col_regs;   // every frame's n_azimuth divides 4 * kWideThreads: in a wide tile each thread
                         // keeps the same four columns, so their beam-pattern factors live in registers
};

constexpr int kBwdThreads = 512;   // threads of a backward polar-tile workgroup

// Camera frames carried along in the forward binning launch of a plan
// with both kinds of frames: device frame table, workgroups (kBlock threads
// each) and the water parameters.
struct UwCompanion {
    const UwDev *table = nullptr;
    int n = 0;
    int blocks = 0;
    const oceansim_water_params *params = nullptr;
};

// Camera frames whose backward rides along in the return-gather launch of a
// plan's sonar backward: device frame table, workgroups (kBlock threads
// each), water parameters and the partial-sum buffers of the camera backward.
struct UwBwdCompanion {
    const UwDev *table = nullptr;
    int n = 0;
    int blocks = 0;
    const oceansim_water_params *params = nullptr;
    double *part = nullptr;
    int *part_row = nullptr;
};

hipError_t sonar_forward_one(const SonarDev &f, const SonarGrid &g, const oceansim_sonar_params *params,
                             const float *refl, int n_mat, hipStream_t st);
hipError_t sonar_forward_table(const SonarDev *t, int n, const SonarGrid &g,
                               const oceansim_sonar_params *params, const float *refl, int n_mat,
                               hipStream_t st, const UwCompanion *uw = nullptr);
// The saved fan stencils of the frames of a forward table (column tables,
// then the fan kernel's geometry alone: no image is read or written).
hipError_t sonar_fan_stencils_table(const SonarDev *t, int n, const SonarGrid &g, hipStream_t st);

// Arguments of the fixed-order reduction that ends a sonar backward launch
// (`blocks` workgroups: n_rows * 8 parameter sums, then n_mat reflectivity
// sums when the small-table path is used).
struct SonarReduce {
    const double *part = nullptr;
    int n_slots = 0, n_rows = 0;
    float *grad_params = nullptr;
    const double *refl_part = nullptr;
    int ret_slots = 0, n_mat = 0;
    float *grad_refl = nullptr;
    int blocks = 0;
};
// Arguments of a row-keyed reduction (n_rows * out_stride workgroups).
struct RowsReduce {
    const double *part = nullptr;
    const int *row = nullptr;
    int n_slots = 0, width = 0;
    float *out = nullptr;
    int out_stride = 0;
    int blocks = 0;
};

// Backward: partial sums into part (column-major [5][tile and return
// workgroups]) and refl_part (column-major [n_mat][return workgroups], small
// tables), reduced in a fixed order into grad_params [n_rows][8] and
// grad_refl [n_mat].  With `defer`, the reduction is not launched: its
// arguments are returned there for a later reduce_pair.  With `uwb`, the
// camera backward of those frames is launched too (in the return-gather
// launch when its LDS allows, else right after it).
hipError_t sonar_backward_one(const SonarDev &f, const SonarGrid &g, const oceansim_sonar_params *params,
                              int n_rows, const float *refl, int n_mat, double *part, double *refl_part,
                              float *grad_params, float *grad_refl, hipStream_t st);
hipError_t sonar_backward_table(const SonarDev *t, int n, const SonarGrid &g,
                                const oceansim_sonar_params *params, int n_rows, const float *refl,
                                int n_mat, double *part, double *refl_part, float *grad_params,
                                float *grad_refl, hipStream_t st, SonarReduce *defer = nullptr,
                                const UwBwdCompanion *uwb = nullptr);

// Camera pixels per thread, chosen per launch from the batch's size: the
// smallest count for small batches, doubled up to the largest while every CU
// still gets kUwMinBlocks / 256 workgroups.  Fewer, longer workgroups pay
// where camera workgroups share a launch with sonar tiles, since each holds
// the tiles' LDS while it waits on memory (at calibration scale the fused
// tile and camera launch went from 1890 to 1570 us going from 4 to 32
// pixels per thread).  The backward's per-workgroup partial sums are
// amortised over at least 8 pixels per thread.
constexpr int kUwFwdMinPixelsPerThread = 4;
constexpr int kUwFwdMaxPixelsPerThread = 32;
constexpr int kUwBwdMinPixelsPerThread = 8;
constexpr int kUwBwdMaxPixelsPerThread = 32;
constexpr long long kUwMinBlocks = 4096;

hipError_t uw_forward_one(const UwDev &f, int blocks, const oceansim_water_params *params, hipStream_t st);
hipError_t uw_forward_table(const UwDev *t, int n, int blocks, const oceansim_water_params *params,
                            hipStream_t st);
hipError_t uw_backward_one(const UwDev &f, int blocks, const oceansim_water_params *params, double *part,
                           int *part_row, hipStream_t st);
hipError_t uw_backward_table(const UwDev *t, int n, int blocks, const oceansim_water_params *params,
                             double *part, int *part_row, hipStream_t st);

// out[r * out_stride + c] = sum over slots s with row[s] == r of part[c * n_slots + s]
// (c < width; columns width..out_stride-1 are written 0), in a fixed order.
hipError_t reduce_rows(const double *part, const int *row, int n_slots, int width, int n_rows,
                       float *out, int out_stride, hipStream_t st);
// A deferred sonar reduction and a row-keyed reduction in one launch (the
// same per-output order as launching them apart, so the same bits).
hipError_t reduce_pair(const SonarReduce &s, const RowsReduce &r, hipStream_t st);

}  // namespace osim
