// C ABI of the OceanSim gfx950 library: argument validation, launch planning,
// workspace carving and dispatch.  See include/oceansim.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <atomic>
#include <mutex>

#include "../../include/oceansim.h"
#include "device.hpp"
#include "launch.hpp"
#include "host.hpp"

using namespace osim;

namespace osim {
namespace host {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() {
    g_err.clear();
    return OCEANSIM_OK;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(OCEANSIM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

namespace {
bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }
size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
constexpr long long kMaxReturns = (1LL << 31) - 1;
constexpr int kMaxFanSide = 32768;
}  // namespace

// --------------------------------------------------------------------------
// Sonar planning
// --------------------------------------------------------------------------

int check_frame(const oceansim_sonar_frame &fr, int idx, int n_param_rows, bool backward) {
    if (fr.n_returns < 0) return fail(OCEANSIM_E_SHAPE, "frame %d: n_returns < 0", idx);
    if (fr.n_returns > kMaxReturns)
        return fail(OCEANSIM_E_UNSUPPORTED, "frame %d: more than 2^31-1 returns", idx);
    if (fr.n_returns > 0 && (!fr.x || !fr.y || !fr.z || !fr.nx || !fr.ny || !fr.nz || !fr.mat))
        return fail(OCEANSIM_E_INVALID_ARG, "frame %d: NULL return buffer", idx);
    const void *rp[7] = {fr.x, fr.y, fr.z, fr.nx, fr.ny, fr.nz, fr.mat};
    for (auto p : rp)
        if (!aligned(p, 4)) return fail(OCEANSIM_E_INVALID_ARG, "frame %d: misaligned return buffer", idx);
    if (fr.n_range < 1 || fr.n_azimuth < 1)
        return fail(OCEANSIM_E_SHAPE, "frame %d: n_range and n_azimuth must be >= 1", idx);
    if (fr.n_azimuth > kMaxTileBins)
        return fail(OCEANSIM_E_UNSUPPORTED, "frame %d: n_azimuth > %d", idx, kMaxTileBins);
    if ((long long)fr.n_range * fr.n_azimuth > (long long)kMaxTiles * kMaxTileBins)
        return fail(OCEANSIM_E_UNSUPPORTED, "frame %d: more than %d polar bins", idx,
                    kMaxTiles * kMaxTileBins);
    if (!(std::isfinite(fr.r_min) && std::isfinite(fr.r_max) && fr.r_min >= 0.0f && fr.r_max > fr.r_min))
        return fail(OCEANSIM_E_INVALID_ARG, "frame %d: need finite 0 <= r_min < r_max", idx);
    if (!(fr.fov_az > 0.0f && fr.fov_az <= 6.2831855f))
        return fail(OCEANSIM_E_INVALID_ARG, "frame %d: fov_az must be in (0, 2pi]", idx);
    if (!(fr.fov_el > 0.0f && fr.fov_el <= 3.1415927f))
        return fail(OCEANSIM_E_INVALID_ARG, "frame %d: fov_el must be in (0, pi]", idx);
    if (!(std::isfinite(fr.path_factor) && fr.path_factor >= 0.0f))
        return fail(OCEANSIM_E_INVALID_ARG, "frame %d: path_factor must be finite and >= 0", idx);
    if (fr.speckle_mode < OCEANSIM_SPECKLE_OFF || fr.speckle_mode > OCEANSIM_SPECKLE_GAMMA)
        return fail(OCEANSIM_E_INVALID_ARG, "frame %d: unknown speckle_mode %d", idx, fr.speckle_mode);
    if (fr.speckle_mode == OCEANSIM_SPECKLE_GAMMA && (fr.gamma_k < 1 || fr.gamma_k > 8))
        return fail(OCEANSIM_E_UNSUPPORTED, "frame %d: gamma_k must be an integer in 1..8", idx);
    if (fr.param_row < 0 || fr.param_row >= n_param_rows)
        return fail(OCEANSIM_E_INVALID_ARG, "frame %d: param_row %d outside [0, %d)", idx, fr.param_row,
                    n_param_rows);
    if (fr.range_norm != 0 && fr.range_norm != 1)
        return fail(OCEANSIM_E_INVALID_ARG, "frame %d: range_norm must be 0 or 1", idx);
    if (!aligned(fr.saved_p, 16)) return fail(OCEANSIM_E_INVALID_ARG, "frame %d: saved_p must be 16-byte aligned", idx);
    const bool has_fan = fr.fan_h != 0 || fr.fan_w != 0;
    if (has_fan) {
        if (fr.fan_h < 1 || fr.fan_w < 1 || fr.fan_h > kMaxFanSide || fr.fan_w > kMaxFanSide)
            return fail(OCEANSIM_E_SHAPE, "frame %d: fan size must be 0x0 or in 1..%d", idx, kMaxFanSide);
        if (!(fr.fov_az <= 3.1415927f))
            return fail(OCEANSIM_E_INVALID_ARG, "frame %d: a fan needs fov_az <= pi", idx);
    }
    if (!backward) {
        if (!fr.polar && !fr.fan)
            return fail(OCEANSIM_E_INVALID_ARG, "frame %d: polar and fan outputs are both NULL", idx);
        if (fr.fan && !has_fan) return fail(OCEANSIM_E_SHAPE, "frame %d: fan output given but fan is 0x0", idx);
        if (!aligned(fr.polar, 16) || !aligned(fr.fan, 16))
            return fail(OCEANSIM_E_INVALID_ARG, "frame %d: polar/fan must be 16-byte aligned", idx);
        if (!aligned(fr.bin_of_return, 4))
            return fail(OCEANSIM_E_INVALID_ARG, "frame %d: misaligned bin_of_return", idx);
        if (fr.fan_stencil && !fr.fan)
            return fail(OCEANSIM_E_INVALID_ARG, "frame %d: fan_stencil is written with the fan output only", idx);
    } else {
        if (fr.grad_fan && !has_fan)
            return fail(OCEANSIM_E_SHAPE, "frame %d: grad_fan given but fan is 0x0", idx);
        if (!aligned(fr.grad_polar, 16) || !aligned(fr.grad_fan, 16))
            return fail(OCEANSIM_E_INVALID_ARG, "frame %d: grad_polar/grad_fan must be 16-byte aligned", idx);
    }
    if (fr.fan_stencil && !has_fan)
        return fail(OCEANSIM_E_SHAPE, "frame %d: fan_stencil given but fan is 0x0", idx);
    if (!aligned(fr.fan_stencil, 16))
        return fail(OCEANSIM_E_INVALID_ARG, "frame %d: fan_stencil must be 16-byte aligned", idx);
    return OCEANSIM_OK;
}

int pow2_at_least(long long v) {
    int p = 1;
    while (p < v && p < (1 << 30)) p <<= 1;
    return p;
}

int plan_sonar(const oceansim_sonar_frame *frames, int n_frames, int n_param_rows, int n_mat, bool backward,
               SonarPlan &P, const Tuning *tune, bool force_table, bool pair_mode) {
    if (n_frames < 0) return fail(OCEANSIM_E_INVALID_ARG, "n_frames < 0");
    if (n_frames > 0 && !frames) return fail(OCEANSIM_E_INVALID_ARG, "frames is NULL");
    if (n_mat < 1) return fail(OCEANSIM_E_INVALID_ARG, "n_materials must be >= 1");
    if (n_param_rows < 1) return fail(OCEANSIM_E_INVALID_ARG, "n_param_rows must be >= 1");
    P.dev.assign(n_frames, SonarDev{});
    int max_tiles = 1, max_tile_bins = 1, max_tile_bins_b = 1;
    long long total_nb = 0, total_n = 0;
    for (int i = 0; i < n_frames; ++i) {
        int rc = check_frame(frames[i], i, n_param_rows, backward);
        if (rc) return rc;
        total_nb += (long long)frames[i].n_range * frames[i].n_azimuth;
        total_n += frames[i].n_returns;
    }
    // Forward tiles: aim at ~512 tile workgroups per call or more, with
    // 1024..4096 bins each; a tile holds whole range rows.  Backward tiles:
    // up to 2048 bins (their pixel work grows with the tile's radial extent).
    long long tb_target = std::min<long long>(kMaxTileBins, std::max<long long>(1024, total_nb / 512));
    if (tune && tune->fwd_tile_bins > 0) tb_target = std::min(tune->fwd_tile_bins, kMaxFwdTileBins);
    const int tb_b = (tune && tune->bwd_tile_bins > 0) ? std::min(tune->bwd_tile_bins, kMaxTileBins) : 2048;
    for (int i = 0; i < n_frames; ++i) {
        const oceansim_sonar_frame &fr = frames[i];
        SonarDev &d = P.dev[i];
        int rpt = std::max(1, std::min(fr.n_range, (int)(tb_target / fr.n_azimuth)));
        int n_tiles = (fr.n_range + rpt - 1) / rpt;
        while (n_tiles > kMaxTiles && (rpt + 1) * fr.n_azimuth <= kMaxFwdTileBins) {
            ++rpt;
            n_tiles = (fr.n_range + rpt - 1) / rpt;
        }
        if (n_tiles > kMaxTiles) return fail(OCEANSIM_E_UNSUPPORTED, "frame %d: too many polar rows", i);
        d.rows_per_tile = rpt;
        d.tile_bins = rpt * fr.n_azimuth;
        d.n_tiles = n_tiles;
        const int rpt_b = std::max(1, std::min(fr.n_range, tb_b / fr.n_azimuth));
        d.rows_per_tile_b = rpt_b;
        d.tile_bins_b = rpt_b * fr.n_azimuth;
        d.n_tiles_b = (fr.n_range + rpt_b - 1) / rpt_b;
        max_tiles = std::max(max_tiles, n_tiles);
        max_tile_bins = std::max(max_tile_bins, d.tile_bins);
        max_tile_bins_b = std::max(max_tile_bins_b, d.tile_bins_b);
    }
    // Returns per binning workgroup: enough workgroups to fill the chip, while
    // the per-(chunk, tile) offset table stays below ~2 entries per return.
    int chunk = std::min(4096, std::max(512, pow2_at_least(total_n / 1024)));
    auto table_entries = [&](int ch) {
        long long e = 0;
        for (int i = 0; i < n_frames; ++i)
            e += (frames[i].n_returns + ch - 1) / ch * (long long)(P.dev[i].n_tiles + 1);
        return e;
    };
    while (chunk < 4096 && table_entries(chunk) > 2 * total_n + (1 << 20)) chunk *= 2;
    if (tune && tune->chunk > 0) chunk = tune->chunk;
    // the return-gather workgroups (256 threads) take at most 4096 returns
    const int ret_chunk = std::min(chunk, 4096);
    P.grid.chunk = chunk;
    P.grid.ret_chunk = ret_chunk;
    P.grid.max_tiles = max_tiles;
    P.grid.max_tile_bins = max_tile_bins;
    P.grid.max_tile_bins_b = max_tile_bins_b;
    P.grid.max_n_az = 1;
    P.grid.wide_col_regs = 1;
    for (int i = 0; i < n_frames; ++i) {
        P.grid.max_n_az = std::max(P.grid.max_n_az, frames[i].n_azimuth);
        if ((4 * kWideThreads) % frames[i].n_azimuth != 0) P.grid.wide_col_regs = 0;
    }

    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = round_up(off + bytes, kWsAlign);
        return o;
    };
    P.off_table = (n_frames > 1 || force_table) ? take(sizeof(SonarDev) * std::max(1, n_frames)) : 0;
    P.off_pairs.assign(n_frames, 0);
    P.off_chunk_off.assign(n_frames, 0);
    P.off_polar.assign(n_frames, (size_t)-1);
    P.off_cols.assign(n_frames, (size_t)-1);
    P.off_grad_img.assign(n_frames, (size_t)-1);
    P.off_pair_r.assign(n_frames, (size_t)-1);
    P.off_cemax.assign(n_frames, (size_t)-1);
    int bin_blocks = 0, tile_blocks = 0, tile_b_blocks = 0, fan_blocks = 0, ret_blocks = 0, fant_blocks = 0;
    int row_blocks = 0, max_rows_per_tile = 0;   // range-wise normalisation
    P.off_dldq.assign(n_frames, (size_t)-1);
    // Bins per thread through the transposed fan operators: one while the
    // workgroups fit the chip a few times over; more for large batches, where
    // the per-workgroup costs (frame lookup, pointer loads, partial sums) add up.
    int fant_bpt = total_nb >= (16LL << 20) ? 4 : (total_nb >= (2LL << 20) ? 2 : 1);
    if (tune && (tune->fant_bpt == 1 || tune->fant_bpt == 2 || tune->fant_bpt == 4)) fant_bpt = tune->fant_bpt;
    for (int i = 0; i < n_frames; ++i) {
        const oceansim_sonar_frame &fr = frames[i];
        SonarDev &d = P.dev[i];
        const long long nb = (long long)fr.n_range * fr.n_azimuth;
        d.n = fr.n_returns;
        d.n_range = fr.n_range;
        d.n_az = fr.n_azimuth;
        d.fan_h = fr.fan_h;
        d.fan_w = fr.fan_w;
        d.chunk = chunk;
        d.n_chunks = (int)((fr.n_returns + chunk - 1) / chunk);
        d.ret_chunk = ret_chunk;
        d.n_ret_chunks = (int)((fr.n_returns + ret_chunk - 1) / ret_chunk);
        d.matp = n_mat <= kLaneHistMats ? 1 : 0;
        d.half_w = (fr.fan_w + 1) / 2;
        d.fan_bpr = (d.half_w + kFanTileU - 1) / kFanTileU;
        d.stencil = gcast(static_cast<int4 *>(fr.fan_stencil));
        const bool fan_out = fr.fan_h > 0 && fr.fan_w > 0 && (backward ? true : fr.fan != nullptr);
        d.fan_blocks = (!backward && fan_out) ? (fr.fan_h + kFanTileV - 1) / kFanTileV * d.fan_bpr : 0;
        d.speckle = fr.speckle_mode;
        d.gamma_k = fr.gamma_k;
        d.inv_gamma_k = fr.gamma_k > 0 ? 1.0f / (float)fr.gamma_k : 1.0f;
        d.param_row = fr.param_row;
        d.seed_lo = fr.seed_lo;
        d.seed_hi = fr.seed_hi;
        d.frame_id = fr.frame_id;
        d.blk[KBIN] = bin_blocks;
        d.blk[KTILE] = tile_blocks;
        d.blk[KFAN] = fan_blocks;
        d.blk[KRET] = ret_blocks;
        d.blk[KTILEB] = tile_b_blocks;
        d.blk[KFANT] = fant_blocks;
        d.ft_mirror = backward && fan_operator_layout(fr) == 2 ? 1 : 0;
        const long long op_rows = d.ft_mirror ? (long long)fr.n_range * ((fr.n_azimuth + 1) / 2) : nb;
        // the pair backward reads the polar gradient of frames without a
        // transposed fan operator directly: operator rows for the others only
        const bool fant_rows = backward && (!pair_mode || fan_operator_layout(fr) != 0);
        d.n_fant_blocks = fant_rows ? (int)((op_rows + kBlock * fant_bpt - 1) / (kBlock * fant_bpt)) : 0;
        fant_blocks += d.n_fant_blocks;
        bin_blocks += d.n_chunks;
        tile_blocks += d.n_tiles;
        tile_b_blocks += d.n_tiles_b;
        fan_blocks += d.fan_blocks;
        ret_blocks += d.n_ret_chunks;
        // geometry in double
        d.r_min = fr.r_min;
        d.r_max = fr.r_max;
        d.fov_az = fr.fov_az;
        d.half_az = 0.5 * (double)fr.fov_az;
        d.sin_half_el = std::sin(0.5 * (double)fr.fov_el);
        d.kappa = fr.path_factor;
        d.scale_r = (double)fr.n_range / ((double)fr.r_max - (double)fr.r_min);
        d.scale_phi = (double)fr.n_azimuth / (double)fr.fov_az;
        d.dr = ((double)fr.r_max - (double)fr.r_min) / fr.n_range;
        d.inv_r_max = 1.0 / (double)fr.r_max;
        d.dphi = (double)fr.fov_az / fr.n_azimuth;
        if (fr.fan_h > 0 && fr.fan_w > 0) {
            const double s1 = (double)fr.r_max / fr.fan_h;
            const double s2 = 2.0 * (double)fr.r_max * std::sin(d.half_az) / fr.fan_w;
            d.fan_s = s1 > s2 ? s1 : s2;
            d.tan_half_az = std::tan(std::min(d.half_az, 1.5707963267948966));
        }
        d.sin_half_az = std::sin(d.half_az);
        d.cos_half_az = std::cos(d.half_az);
        d.r_min_f = fr.r_min;
        d.scale_r_f = (float)d.scale_r;
        d.cols = nullptr;
        // offsets from a column centre reach half a column plus the error of
        // the approximate azimuth; the short arctangent series needs |q| < 0.05
        d.wide_cols = d.dphi > 0.09 ? 1 : 0;
        d.scale_phi_f = (float)d.scale_phi;
        d.half_az_f = (float)d.half_az;
        // FP32 azimuth error, in cells, is below ~3.3e-7 N_phi (see return_bin)
        d.az_fast = (3.5e-7 * fr.n_azimuth < 1e-3) ? 1 : 0;
        // pointers
        d.x = gcast(fr.x); d.y = gcast(fr.y); d.z = gcast(fr.z);
        d.nx = gcast(fr.nx); d.ny = gcast(fr.ny); d.nz = gcast(fr.nz);
        d.mat = gcast(fr.mat);
        d.polar = gcast(fr.polar);
        d.fan = gcast(fr.fan);
        d.bin_of_return = gcast(fr.bin_of_return);
        d.grad_polar = gcast(fr.grad_polar);
        d.grad_fan = gcast(fr.grad_fan);
        d.range_norm = fr.range_norm;
        d.saved_p = gcast(fr.saved_p);
        d.blk[KROW] = row_blocks;
        if (backward && fr.range_norm) row_blocks += fr.n_range;
        if (fr.range_norm) max_rows_per_tile = std::max(max_rows_per_tile, d.rows_per_tile);
        if (!backward) {
            P.off_pairs[i] = take(sizeof(uint2) * (size_t)d.n_chunks * chunk);
            P.off_chunk_off[i] = take(sizeof(int) * (size_t)d.n_chunks * (d.n_tiles + 1));
            if (!fr.polar) P.off_polar[i] = take(sizeof(float) * (size_t)nb);
            if (d.fan_blocks > 0) P.off_cols[i] = take(sizeof(double) * 2 * (size_t)fr.n_azimuth);
            if (pair_mode) {
                P.off_pair_r[i] = take(sizeof(float) * (size_t)d.n_chunks * chunk);
                P.off_cemax[i] = take(sizeof(float) * (size_t)d.n_tiles);
            }
        } else {
            if (d.n_fant_blocks > 0 || !pair_mode) P.off_grad_img[i] = take(sizeof(float) * (size_t)nb);
            if (fr.range_norm) P.off_dldq[i] = take(sizeof(float) * (size_t)nb);
        }
    }
    P.grid.bin_blocks = bin_blocks;
    P.grid.row_blocks = row_blocks;
    P.grid.max_rows_per_tile = max_rows_per_tile;
    P.grid.tile_blocks = tile_blocks;
    P.grid.fan_blocks = fan_blocks;
    P.grid.ret_blocks = ret_blocks;
    P.grid.tile_b_blocks = tile_b_blocks;
    P.grid.fant_blocks = fant_blocks;
    P.grid.fant_bpt = fant_bpt;
    P.grid.use_fant = 0;
    P.grid.pair_bwd = backward && pair_mode ? 1 : 0;
    P.grid.fant_mirror = 0;
    for (const SonarDev &d : P.dev) P.grid.fant_mirror |= d.ft_mirror;
    P.grid.all_saved = 1;
    for (int i = 0; i < n_frames; ++i)
        if (frames[i].grad_fan && !frames[i].fan_stencil) P.grid.all_saved = 0;
    if (backward) {
        // slots for either backward decomposition of the polar gradient
        // (the pair backward: operator rows, then one slot per forward tile)
        P.n_slots = pair_mode ? fant_blocks + tile_blocks : std::max(tile_b_blocks, fant_blocks) + ret_blocks + row_blocks;
        // five FP64 partial sums per slot (column-major), then the slot's parameter row
        P.off_part = take((sizeof(double) * 5 + sizeof(int)) * (size_t)std::max(1, P.n_slots));
        if (n_mat <= kLaneHistMats)
            P.off_refl_part = take(sizeof(double) * (size_t)std::max(1, pair_mode ? tile_blocks : ret_blocks) * n_mat);
    }
    P.bytes = std::max<size_t>(off, kWsAlign);
    return OCEANSIM_OK;
}

bool pair_backward_ok(const oceansim_sonar_frame *frames, int n_frames, int n_mat) {
    if (n_mat > kLaneHistMats) return false;
    for (int i = 0; i < n_frames; ++i)
        if (frames[i].range_norm) return false;
    return true;
}

void link_pairs(SonarPlan &bwd, const SonarPlan &fwd) {
    for (size_t i = 0; i < bwd.dev.size() && i < fwd.dev.size(); ++i) {
        bwd.dev[i].pairs = fwd.dev[i].pairs;
        bwd.dev[i].chunk_off = fwd.dev[i].chunk_off;
        bwd.dev[i].pair_r = fwd.dev[i].pair_r;
        bwd.dev[i].tile_cemax = fwd.dev[i].tile_cemax;
    }
}

void carve_sonar(SonarPlan &P, char *ws, bool backward) {
    for (size_t i = 0; i < P.dev.size(); ++i) {
        SonarDev &d = P.dev[i];
        if (!backward) {
            d.pairs = gcast(reinterpret_cast<uint2 *>(ws + P.off_pairs[i]));
            d.chunk_off = gcast(reinterpret_cast<int *>(ws + P.off_chunk_off[i]));
            if (P.off_polar[i] != (size_t)-1) d.polar = gcast(reinterpret_cast<float *>(ws + P.off_polar[i]));
            if (P.off_cols[i] != (size_t)-1) d.cols = gcast(reinterpret_cast<double2 *>(ws + P.off_cols[i]));
            if (P.off_pair_r[i] != (size_t)-1) d.pair_r = gcast(reinterpret_cast<float *>(ws + P.off_pair_r[i]));
            if (P.off_cemax[i] != (size_t)-1) d.tile_cemax = gcast(reinterpret_cast<float *>(ws + P.off_cemax[i]));
        } else {
            if (P.off_grad_img[i] != (size_t)-1) d.grad_img = gcast(reinterpret_cast<float *>(ws + P.off_grad_img[i]));
            if (P.off_dldq[i] != (size_t)-1) d.dldq = gcast(reinterpret_cast<float *>(ws + P.off_dldq[i]));
        }
    }
}

int check_ws(void *ws, size_t have, size_t need) {
    if (need > have)
        return fail(OCEANSIM_E_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", have, need);
    if (!ws) return fail(OCEANSIM_E_WORKSPACE, "workspace is NULL");
    if (!aligned(ws, kWsAlign)) return fail(OCEANSIM_E_WORKSPACE, "workspace must be 256-byte aligned");
    return OCEANSIM_OK;
}

// --------------------------------------------------------------------------
// Camera planning
// --------------------------------------------------------------------------

int plan_uw(const oceansim_uw_frame *frames, int n_frames, int n_param_rows, bool backward, UwPlan &P,
            bool force_table, int threads) {
    if (n_frames < 0) return fail(OCEANSIM_E_INVALID_ARG, "n_frames < 0");
    if (n_frames > 0 && !frames) return fail(OCEANSIM_E_INVALID_ARG, "frames is NULL");
    if (n_param_rows < 1) return fail(OCEANSIM_E_INVALID_ARG, "n_param_rows must be >= 1");
    P.dev.assign(n_frames, UwDev{});
    int blocks = 0;
    // pixels per thread from the batch's size (the same for all frames)
    long long total_px = 0;
    for (int i = 0; i < n_frames; ++i)
        if (frames[i].H > 0 && frames[i].W > 0) total_px += (long long)frames[i].H * frames[i].W;
    int fwd_px = kUwFwdMinPixelsPerThread, bwd_px = kUwBwdMinPixelsPerThread;
    while (fwd_px < kUwFwdMaxPixelsPerThread && total_px / ((long long)threads * fwd_px * 2) >= kUwMinBlocks)
        fwd_px *= 2;
    while (bwd_px < kUwBwdMaxPixelsPerThread && total_px / ((long long)threads * bwd_px * 2) >= kUwMinBlocks)
        bwd_px *= 2;
    for (int i = 0; i < n_frames; ++i) {
        const oceansim_uw_frame &fr = frames[i];
        if (fr.H < 1 || fr.W < 1) return fail(OCEANSIM_E_SHAPE, "camera frame %d: H and W must be >= 1", i);
        const long long npix = (long long)fr.H * fr.W;
        if (npix * 3 > kMaxReturns)
            return fail(OCEANSIM_E_UNSUPPORTED, "camera frame %d: image too large", i);
        if (fr.param_row < 0 || fr.param_row >= n_param_rows)
            return fail(OCEANSIM_E_INVALID_ARG, "camera frame %d: param_row %d outside [0, %d)", i,
                        fr.param_row, n_param_rows);
        if (!fr.J || !fr.depth) return fail(OCEANSIM_E_INVALID_ARG, "camera frame %d: NULL J or depth", i);
        if (!backward && !fr.out) return fail(OCEANSIM_E_INVALID_ARG, "camera frame %d: NULL out", i);
        if (backward && !fr.grad_out) return fail(OCEANSIM_E_INVALID_ARG, "camera frame %d: NULL grad_out", i);
        const void *ps[6] = {fr.J, fr.depth, fr.out, fr.grad_out, fr.grad_J, fr.grad_depth};
        for (auto p : ps)
            if (!aligned(p, 16))
                return fail(OCEANSIM_E_INVALID_ARG, "camera frame %d: image buffers must be 16-byte aligned", i);
        UwDev &d = P.dev[i];
        d.J = gcast(fr.J);
        d.depth = gcast(fr.depth);
        d.out = gcast(fr.out);
        d.grad_out = gcast(fr.grad_out);
        d.grad_J = gcast(fr.grad_J);
        d.grad_depth = gcast(fr.grad_depth);
        d.npix = npix;
        d.param_row = fr.param_row;
        d.fwd_px = fwd_px;
        d.bwd_px = bwd_px;
        const long long ppb = (long long)threads * (backward ? bwd_px : fwd_px);
        d.n_blocks = (int)((npix + ppb - 1) / ppb);
        d.blk = blocks;
        blocks += d.n_blocks;
    }
    P.blocks = blocks;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = round_up(off + bytes, kWsAlign);
        return o;
    };
    P.off_table = (n_frames > 1 || force_table) ? take(sizeof(UwDev) * std::max(1, n_frames)) : 0;
    if (backward) {
        P.off_part = take(sizeof(double) * 9 * (size_t)std::max(1, blocks));
        P.off_part_row = take(sizeof(int) * (size_t)std::max(1, blocks));
    }
    P.bytes = off;
    return OCEANSIM_OK;
}

}  // namespace host
}  // namespace osim

namespace {
// --------------------------------------------------------------------------
// Kernel-launch tracing
// --------------------------------------------------------------------------
struct TraceRec {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_trace_mu;
std::atomic<bool> g_trace_on{false};
std::vector<TraceRec> g_trace;

}  // namespace

namespace osim {
namespace {
thread_local bool t_capturing = false;   // launches being captured into a graph are not traced
}  // namespace

void set_capturing(bool on) { t_capturing = on; }
bool trace_active() { return g_trace_on.load(std::memory_order_relaxed) && !t_capturing; }
void trace_record(const char *, hipStream_t st, hipEvent_t *a, hipEvent_t *b) {
    if (hipEventCreate(a) != hipSuccess) { *a = *b = nullptr; return; }
    if (hipEventCreate(b) != hipSuccess) { (void)hipEventDestroy(*a); *a = *b = nullptr; return; }
    (void)hipEventRecord(*a, st);
}
void trace_commit(const char *name, hipStream_t st, hipEvent_t a, hipEvent_t b) {
    if (!a) return;
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_trace_mu);
    g_trace.push_back(TraceRec{name, a, b});
}
}  // namespace osim

using namespace osim::host;

extern "C" {

int oceansim_trace_enable(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_trace_mu);
    if (enable) {
        for (auto &r : g_trace) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        g_trace.clear();
    }
    g_trace_on.store(enable != 0);
    return ok();
}

int oceansim_trace_summary(char *buf, size_t len, size_t *needed) {
    std::lock_guard<std::mutex> lk(g_trace_mu);
    std::vector<std::pair<std::string, std::pair<long, double>>> agg;
    for (auto &r : g_trace) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(e, "trace event");
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e, "trace event");
        auto it = std::find_if(agg.begin(), agg.end(), [&](auto &p) { return p.first == r.name; });
        if (it == agg.end()) agg.push_back({r.name, {1, ms * 1e3}});
        else { it->second.first += 1; it->second.second += ms * 1e3; }
    }
    std::string out;
    char line[256];
    for (auto &p : agg) {
        snprintf(line, sizeof line, "%s %ld %.3f\n", p.first.c_str(), p.second.first, p.second.second);
        out += line;
    }
    if (needed) *needed = out.size() + 1;
    if (buf && len > 0) {
        size_t n = std::min(len - 1, out.size());
        memcpy(buf, out.data(), n);
        buf[n] = 0;
    }
    return ok();
}

size_t oceansim_fan_stencil_size(int32_t fan_h, int32_t fan_w) {
    if (fan_h <= 0 || fan_w <= 0) return 0;
    return (size_t)fan_h * (size_t)((fan_w + 1) / 2) * 16;
}

const char *oceansim_last_error(void) { return g_err.c_str(); }

int oceansim_abi_version(void) { return OCEANSIM_ABI_VERSION; }

int oceansim_sonar_workspace_size(const oceansim_sonar_frame *frames, int32_t n_frames, int32_t n_materials,
                                  int32_t with_backward, size_t *bytes) {
    if (!bytes) return fail(OCEANSIM_E_INVALID_ARG, "bytes is NULL");
    SonarPlan P;
    // the row count is not known here: accept any row index for sizing
    int rc = plan_sonar(frames, n_frames, 0x7fffffff, n_materials, with_backward != 0, P, nullptr);
    if (rc) return rc;
    *bytes = P.bytes;
    return ok();
}

}  // extern "C"

namespace {

// The sonar forward of planned frames into a checked workspace.
int render_planned(SonarPlan &P, int32_t n_frames, const oceansim_sonar_params *params_dev, const float *refl_dev,
                   int32_t n_materials, void *workspace, size_t workspace_bytes, void *stream) {
    int rc = check_ws(workspace, workspace_bytes, P.bytes);
    if (rc) return rc;
    char *ws = static_cast<char *>(workspace);
    carve_sonar(P, ws, false);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (n_frames == 1) {
        e = sonar_forward_one(P.dev[0], P.grid, params_dev, refl_dev, n_materials, st);
    } else {
        e = upload_table(P.dev, ws, P.off_table, st);
        if (e != hipSuccess) return hip_fail(e, "frame table upload");
        e = sonar_forward_table(reinterpret_cast<const SonarDev *>(ws + P.off_table), n_frames, P.grid,
                                params_dev, refl_dev, n_materials, st);
    }
    if (e != hipSuccess) return hip_fail(e, "sonar forward launch");
    return ok();
}

// Scratch memory of the allocation-free sonar forward: a file-scope device
// array (one copy per GPU, held until the process ends).  Host code reaches
// it only through the address hipGetSymbolAddress returns for the current
// device, kept per device.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kMaxScratchDevices = 64;
__device__ __align__(256) char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

int scratch_of_current_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(OCEANSIM_E_UNSUPPORTED, "device %d: the allocation-free entry point serves devices 0..%d", dev,
                    kMaxScratchDevices - 1);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "scratch address");
        if (!p) return fail(OCEANSIM_E_HIP, "scratch address is NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return OCEANSIM_OK;
}

}  // namespace

extern "C" {

int oceansim_sonar_render(const oceansim_sonar_frame *frames, int32_t n_frames,
                          const oceansim_sonar_params *params_dev, int32_t n_param_rows, const float *refl_dev,
                          int32_t n_materials, void *workspace, size_t workspace_bytes, void *stream) {
    if (!params_dev) return fail(OCEANSIM_E_INVALID_ARG, "params_dev is NULL");
    if (!refl_dev) return fail(OCEANSIM_E_INVALID_ARG, "refl_dev is NULL");
    SonarPlan P;
    int rc = plan_sonar(frames, n_frames, n_param_rows, n_materials, false, P, nullptr);
    if (rc) return rc;
    if (n_frames == 0) return ok();
    return render_planned(P, n_frames, params_dev, refl_dev, n_materials, workspace, workspace_bytes, stream);
}

int oceansim_sonar_render_noalloc(const oceansim_sonar_frame *frames, int32_t n_frames,
                                  const oceansim_sonar_params *params_dev, int32_t n_param_rows,
                                  const float *refl_dev, int32_t n_materials, void *stream) {
    if (!params_dev) return fail(OCEANSIM_E_INVALID_ARG, "params_dev is NULL");
    if (!refl_dev) return fail(OCEANSIM_E_INVALID_ARG, "refl_dev is NULL");
    SonarPlan P;
    int rc = plan_sonar(frames, n_frames, n_param_rows, n_materials, false, P, nullptr);
    if (rc) return rc;
    if (n_frames == 0) return ok();
    if (P.bytes > kNoAllocScratchBytes)
        return fail(OCEANSIM_E_UNSUPPORTED,
                    "these frames need %zu bytes of scratch; the allocation-free entry point has %zu (use "
                    "oceansim_sonar_render with a workspace)", P.bytes, kNoAllocScratchBytes);
    void *ws = nullptr;
    rc = scratch_of_current_device(&ws);
    if (rc) return rc;
    return render_planned(P, n_frames, params_dev, refl_dev, n_materials, ws, kNoAllocScratchBytes, stream);
}

int oceansim_sonar_render_backward(const oceansim_sonar_frame *frames, int32_t n_frames,
                                   const oceansim_sonar_params *params_dev, int32_t n_param_rows,
                                   const float *refl_dev, int32_t n_materials, float *grad_refl_dev,
                                   float *grad_params_dev, void *workspace, size_t workspace_bytes,
                                   void *stream) {
    if (!params_dev) return fail(OCEANSIM_E_INVALID_ARG, "params_dev is NULL");
    if (!refl_dev) return fail(OCEANSIM_E_INVALID_ARG, "refl_dev is NULL");
    if (!grad_refl_dev || !grad_params_dev) return fail(OCEANSIM_E_INVALID_ARG, "gradient output is NULL");
    if (!aligned(grad_refl_dev, 4) || !aligned(grad_params_dev, 4))
        return fail(OCEANSIM_E_INVALID_ARG, "misaligned gradient output");
    SonarPlan P;
    int rc = plan_sonar(frames, n_frames, n_param_rows, n_materials, true, P, nullptr);
    if (rc) return rc;
    for (int i = 0; i < n_frames; ++i)
        if (frames[i].range_norm && !frames[i].saved_p)
            return fail(OCEANSIM_E_INVALID_ARG, "frame %d: range_norm needs the forward's saved_p", i);
    rc = check_ws(workspace, workspace_bytes, P.bytes);
    if (rc) return rc;
    char *ws = static_cast<char *>(workspace);
    carve_sonar(P, ws, true);
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *part = reinterpret_cast<double *>(ws + P.off_part);
    const bool lane_hist = n_materials <= kLaneHistMats;
    double *refl_part = lane_hist ? reinterpret_cast<double *>(ws + P.off_refl_part) : nullptr;
    hipError_t e = hipSuccess;
    if (n_frames <= 1) {
        SonarDev empty{};
        e = sonar_backward_one(n_frames == 1 ? P.dev[0] : empty, P.grid, params_dev, n_param_rows, refl_dev,
                               n_materials, part, refl_part, grad_params_dev, grad_refl_dev, st);
    } else {
        e = upload_table(P.dev, ws, P.off_table, st);
        if (e != hipSuccess) return hip_fail(e, "frame table upload");
        e = sonar_backward_table(reinterpret_cast<const SonarDev *>(ws + P.off_table), n_frames, P.grid,
                                 params_dev, n_param_rows, refl_dev, n_materials, part, refl_part,
                                 grad_params_dev, grad_refl_dev, st);
    }
    if (e != hipSuccess) return hip_fail(e, "sonar backward launch");
    return ok();
}

int oceansim_uw_workspace_size(const oceansim_uw_frame *frames, int32_t n_frames, int32_t with_backward,
                               size_t *bytes) {
    if (!bytes) return fail(OCEANSIM_E_INVALID_ARG, "bytes is NULL");
    UwPlan P;
    std::vector<oceansim_uw_frame> tmp(frames, frames + std::max(0, n_frames));
    for (auto &f : tmp) f.param_row = 0;   // sizing does not depend on rows
    int rc = plan_uw(frames ? tmp.data() : nullptr, n_frames, 1, with_backward != 0, P);
    if (rc) return rc;
    *bytes = P.bytes;
    return ok();
}

int oceansim_uw_form(const oceansim_uw_frame *frames, int32_t n_frames, const oceansim_water_params *params_dev,
                     int32_t n_param_rows, void *workspace, size_t workspace_bytes, void *stream) {
    if (!params_dev) return fail(OCEANSIM_E_INVALID_ARG, "params_dev is NULL");
    UwPlan P;
    int rc = plan_uw(frames, n_frames, n_param_rows, false, P);
    if (rc) return rc;
    if (n_frames == 0 || P.blocks == 0) return ok();
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (n_frames == 1) {
        e = uw_forward_one(P.dev[0], P.blocks, params_dev, st);
    } else {
        rc = check_ws(workspace, workspace_bytes, P.bytes);
        if (rc) return rc;
        char *ws = static_cast<char *>(workspace);
        e = upload_table(P.dev, ws, P.off_table, st);
        if (e != hipSuccess) return hip_fail(e, "frame table upload");
        e = uw_forward_table(reinterpret_cast<const UwDev *>(ws + P.off_table), n_frames, P.blocks, params_dev, st);
    }
    if (e != hipSuccess) return hip_fail(e, "uw_form launch");
    return ok();
}

int oceansim_uw_form_backward(const oceansim_uw_frame *frames, int32_t n_frames,
                              const oceansim_water_params *params_dev, int32_t n_param_rows,
                              float *grad_params_dev, void *workspace, size_t workspace_bytes, void *stream) {
    if (!params_dev) return fail(OCEANSIM_E_INVALID_ARG, "params_dev is NULL");
    if (!grad_params_dev) return fail(OCEANSIM_E_INVALID_ARG, "grad_params_dev is NULL");
    UwPlan P;
    int rc = plan_uw(frames, n_frames, n_param_rows, true, P);
    if (rc) return rc;
    rc = check_ws(workspace, workspace_bytes, P.bytes);
    if (rc) return rc;
    char *ws = static_cast<char *>(workspace);
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *part = reinterpret_cast<double *>(ws + P.off_part);
    int *part_row = reinterpret_cast<int *>(ws + P.off_part_row);
    hipError_t e = hipSuccess;
    if (n_frames == 1 && P.blocks > 0) {
        e = uw_backward_one(P.dev[0], P.blocks, params_dev, part, part_row, st);
    } else if (n_frames > 1 && P.blocks > 0) {
        e = upload_table(P.dev, ws, P.off_table, st);
        if (e != hipSuccess) return hip_fail(e, "frame table upload");
        e = uw_backward_table(reinterpret_cast<const UwDev *>(ws + P.off_table), n_frames, P.blocks, params_dev,
                              part, part_row, st);
    }
    if (e != hipSuccess) return hip_fail(e, "uw_form backward launch");
    e = reduce_rows(part, part_row, P.blocks, 9, n_param_rows, grad_params_dev, OCEANSIM_WATER_GRAD_WIDTH, st);
    if (e != hipSuccess) return hip_fail(e, "water gradient reduction");
    return ok();
}

}  // extern "C"
