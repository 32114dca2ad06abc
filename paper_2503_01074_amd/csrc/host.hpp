// Host-side planning shared by the plain entry points and plans (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/oceansim.h"
#include "device.hpp"
#include "launch.hpp"

namespace osim {
namespace host {

constexpr size_t kWsAlign = 256;

// Launch-shape knobs; 0 = the built-in heuristic.
struct Tuning {
    int fwd_tile_bins = 0;   // forward polar tile size target (bins, whole rows)
    int chunk = 0;           // returns per binning / return-gather workgroup (512..4096)
    int bwd_tile_bins = 0;   // backward polar tile size target (bins, whole rows)
    int fant_bpt = 0;        // bins per thread through the transposed fan operators (1, 2, 4; 0: by size)
};

struct SonarPlan {
    std::vector<SonarDev> dev;
    SonarGrid grid{};
    size_t bytes = 0;
    // workspace offsets
    size_t off_table = 0;
    std::vector<size_t> off_pairs, off_chunk_off, off_polar, off_grad_img, off_cols;
    std::vector<size_t> off_pair_r;   // ranges of the pairs (forward of a pair-backward plan)
    std::vector<size_t> off_cemax;    // per-tile largest |cos x attenuation| (same)
    std::vector<size_t> off_dldq;   // range-normalised frames' dL/dQ (backward)
    size_t off_part = 0, off_refl_part = 0;
    int n_slots = 0;
};

struct UwPlan {
    std::vector<UwDev> dev;
    int blocks = 0;
    size_t bytes = 0, off_table = 0, off_part = 0, off_part_row = 0;
};

// Layout of a frame's transposed fan operator in a backward plan: 0 none (no
// fan gradient), 1 one row per polar bin, 2 mirrored: with an even fan width
// the fan's left and right halves are exact mirror images (pixel (v, u) and
// (v, W-1-u) take mirrored stencils with bit-identical weights), so the bins
// of the first ceil(N_phi / 2) columns carry the entries and bin (i, N_phi-1-j)
// reads those of (i, j) at the mirrored pixels: half the operator bytes.
// Pixels are then packed as (v << 16) | u, hence the 16-bit limits.
inline int fan_operator_layout(const oceansim_sonar_frame &f) {
    if (!f.fan || !f.grad_fan || f.fan_h <= 0 || f.fan_w <= 0) return 0;
    return (f.fan_w % 2 == 0 && f.fan_w <= 65535 && f.fan_h <= 65535) ? 2 : 1;
}

int fail(int code, const char *fmt, ...);
int ok();
int hip_fail(hipError_t e, const char *what);

// force_table: reserve a device frame table even for a single frame (plans
// always launch from tables; the plain entry points pass one frame by value).
// pair_mode (plans): the backward runs from the forward's material pairs
// (k_pair_bwd): the forward keeps the pairs' ranges, the backward takes one
// workgroup per forward tile and operator rows only for frames with a fan
// gradient; link_pairs then points the backward frames at the forward's pairs.
int plan_sonar(const oceansim_sonar_frame *frames, int n_frames, int n_param_rows, int n_mat, bool backward,
               SonarPlan &P, const Tuning *tune, bool force_table = false, bool pair_mode = false);
// Whether a plan over these frames can take the pair backward: material
// tables of at most 64 entries and no range-wise normalisation.
bool pair_backward_ok(const oceansim_sonar_frame *frames, int n_frames, int n_mat);
// Backward frames of a pair-backward plan read the pairs, offsets and ranges
// of the forward frames (after both are carved).
void link_pairs(SonarPlan &bwd, const SonarPlan &fwd);
void carve_sonar(SonarPlan &P, char *ws, bool backward);
int check_ws(void *ws, size_t have, size_t need);
// threads: workgroup size of the kernel that runs the camera frames (the
// camera kernels' own, or that of a sonar kernel carrying them along).
int plan_uw(const oceansim_uw_frame *frames, int n_frames, int n_param_rows, bool backward, UwPlan &P,
            bool force_table = false, int threads = kBlock);

template <class T>
hipError_t upload_table(const std::vector<T> &v, char *ws, size_t off, hipStream_t st) {
    return hipMemcpyAsync(ws + off, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st);
}

}  // namespace host
}  // namespace osim
