// Navigation sensors of Sec. III-A of arXiv 2503.01074 on gfx950: the
// barometer (pressure from the atmospheric pressure and the water density,
// optional Gaussian noise) and the four-beam Janus DVL (range-dependent
// measurement rate, dropout when too few beams return).  The paper prints no
// equations for either; the readings are stated in include/oceansim.h.
//
//   k_baro  one pressure per sample (elementwise, four samples per thread).
//   k_dvl   one thread per instance (a vehicle or a Monte Carlo run), walking
//           its ticks in order: the measurement schedule carries the time of
//           the last measurement from tick to tick.  Inputs are tick-major
//           ([tick][instance]), so the loads of a tick are coalesced across
//           the threads of a wave.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/oceansim.h"
#include "device.hpp"
#include "host.hpp"
#include "launch.hpp"

namespace osim {
namespace {

constexpr int kNavThreads = 256;
constexpr int kBaroPerThread = 4;

// Standard normal from two words of a Philox block: Box-Muller, cosine branch.
__device__ __forceinline__ float gauss_of_words(uint32_t w0, uint32_t w1) {
    return __builtin_amdgcn_sqrtf(2.0f * neg_ln(unit_uniform(w0))) * cospif(2.0f * unit_uniform(w1));
}

struct BaroDev {
    double p_atm, rho_g, sigma;
    uint32_t seed_lo, seed_hi;
};

__global__ __launch_bounds__(kNavThreads) void k_baro(gptr<const float> depth, long long n, BaroDev p,
                                                      gptr<float> pressure) {
    const long long k0 = ((long long)blockIdx.x * kNavThreads * kBaroPerThread) + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kBaroPerThread; ++u) {
        const long long k = k0 + (long long)u * kNavThreads;
        if (k >= n) return;
        const double d = (double)depth[k];
        double z = 0.0;
        if (p.sigma != 0.0) {
            const Words w = philox((uint32_t)k, (uint32_t)((unsigned long long)k >> 32), 3u, 0u, p.seed_lo, p.seed_hi);
            z = (double)gauss_of_words(w.w0, w.w1);
        }
        // the water column above the sensor (none above the surface)
        const double column = d > 0.0 ? p.rho_g * d : 0.0;
        pressure[k] = (float)(p.p_atm + column + p.sigma * z);
    }
}

struct DvlDev {
    double beam[4][3];          // unit beam directions (sensor frame)
    double range_min, range_max;
    double sigma_v;
    double pings_per_output, sound_speed, period_min;
    int min_beams;
    uint32_t seed_lo, seed_hi;
};

__global__ __launch_bounds__(kNavThreads) void k_dvl(gptr<const double> t, gptr<const float4> ranges,
                                                     gptr<const float> vel, int n_ticks, int n_inst, DvlDev p,
                                                     gptr<float> vout, gptr<int> status) {
    const int n = blockIdx.x * kNavThreads + threadIdx.x;
    if (n >= n_inst) return;
    double t_last = 0.0;
    bool have_last = false;
    // the next tick's inputs are loaded while this tick is processed (the
    // ticks of one instance are sequential; past the last tick the loads
    // re-read it)
    float4 r4n = gload((gptr<const float4>)(ranges + n));
    float vn0 = vel[3LL * n], vn1 = vel[3LL * n + 1], vn2 = vel[3LL * n + 2];
    for (int k = 0; k < n_ticks; ++k) {
        const long long row = (long long)k * n_inst + n;
        const float4 r4 = r4n;
        const double v0 = vn0, v1 = vn1, v2 = vn2;
        {
            const long long nrow = (long long)(k + 1 < n_ticks ? k + 1 : k) * n_inst + n;
            r4n = gload((gptr<const float4>)(ranges + nrow));
            vn0 = vel[3 * nrow];
            vn1 = vel[3 * nrow + 1];
            vn2 = vel[3 * nrow + 2];
        }
        const float r[4] = {r4.x, r4.y, r4.z, r4.w};
        bool ok[4];
        int nv = 0;
        double r_ref = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double ri = (double)r[i];
            ok[i] = __builtin_isfinite(ri) && ri >= p.range_min && ri <= p.range_max;
            if (ok[i]) {
                ++nv;
                r_ref = ri > r_ref ? ri : r_ref;
            }
        }
        if (nv == 0) r_ref = p.range_max;
        // ping period of the current altitude: two-way travel of the farthest
        // valid beam times the pings averaged into one output
        double period = p.pings_per_output * 2.0 * r_ref / p.sound_speed;
        period = period < p.period_min ? p.period_min : period;
        const double tk = t[k];
        const bool due = !have_last || (tk - t_last >= period);
        gptr<float> vo = vout + 3 * row;
        if (!due || nv < p.min_beams) {
            vo[0] = vo[1] = vo[2] = __builtin_nanf("");
            status[row] = due ? 2 : 0;
            if (due) {
                have_last = true;
                t_last = tk;
            }
            continue;
        }
        have_last = true;
        t_last = tk;
        // normal equations over the valid beams: A x = B^T u, A = sum b b^T
        Words w01{0u, 0u, 0u, 0u}, w23{0u, 0u, 0u, 0u};
        if (p.sigma_v != 0.0) {
            w01 = philox((uint32_t)k, (uint32_t)n, 4u, 0u, p.seed_lo, p.seed_hi);
            w23 = philox((uint32_t)k, (uint32_t)n, 4u, 1u, p.seed_lo, p.seed_hi);
        }
        double a00 = 0.0, a01 = 0.0, a02 = 0.0, a11 = 0.0, a12 = 0.0, a22 = 0.0;
        double q0 = 0.0, q1 = 0.0, q2 = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (!ok[i]) continue;
            const double *b = p.beam[i];
            double z = 0.0;
            if (p.sigma_v != 0.0) {
                const Words &w = i < 2 ? w01 : w23;
                z = (double)gauss_of_words(pick(w, 2u * (i & 1)), pick(w, 2u * (i & 1) + 1u));
            }
            const double u = b[0] * v0 + b[1] * v1 + b[2] * v2 + p.sigma_v * z;   // along-beam Doppler velocity
            a00 += b[0] * b[0];
            a01 += b[0] * b[1];
            a02 += b[0] * b[2];
            a11 += b[1] * b[1];
            a12 += b[1] * b[2];
            a22 += b[2] * b[2];
            q0 += b[0] * u;
            q1 += b[1] * u;
            q2 += b[2] * u;
        }
        // x = adj(A) q / det(A) for the symmetric A
        const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
        const double c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
        const double inv_det = 1.0 / (a00 * c00 + a01 * c01 + a02 * c02);
        vo[0] = (float)((c00 * q0 + c01 * q1 + c02 * q2) * inv_det);
        vo[1] = (float)((c01 * q0 + c11 * q1 + c12 * q2) * inv_det);
        vo[2] = (float)((c02 * q0 + c12 * q1 + c22 * q2) * inv_det);
        status[row] = 1;
    }
}

bool aligned_to(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace
}  // namespace osim

using namespace osim;
using namespace osim::host;

extern "C" {

int oceansim_barometer(const float *depth_dev, int64_t n, const oceansim_baro_params *params, float *pressure_dev,
                       void *stream) {
    if (!params) return fail(OCEANSIM_E_INVALID_ARG, "params is NULL");
    if (n < 0) return fail(OCEANSIM_E_SHAPE, "n < 0");
    if (n > 0 && (!depth_dev || !pressure_dev)) return fail(OCEANSIM_E_INVALID_ARG, "NULL buffer");
    if (!aligned_to(depth_dev, 4) || !aligned_to(pressure_dev, 4))
        return fail(OCEANSIM_E_INVALID_ARG, "misaligned buffer");
    const oceansim_baro_params &q = *params;
    if (!(std::isfinite(q.p_atm) && std::isfinite(q.rho) && std::isfinite(q.g) && std::isfinite(q.sigma) &&
          q.rho >= 0.0 && q.g >= 0.0 && q.sigma >= 0.0))
        return fail(OCEANSIM_E_INVALID_ARG, "barometer parameters must be finite, rho, g and sigma >= 0");
    if (n == 0) return ok();
    BaroDev p{q.p_atm, q.rho * q.g, q.sigma, q.seed_lo, q.seed_hi};
    const long long per_block = (long long)kNavThreads * kBaroPerThread;
    const long long blocks = (n + per_block - 1) / per_block;
    if (blocks > 0x7fffffffLL) return fail(OCEANSIM_E_UNSUPPORTED, "too many samples");
    hipStream_t st = static_cast<hipStream_t>(stream);
    OSIM_LAUNCH("k_baro", k_baro, dim3((unsigned)blocks), dim3(kNavThreads), 0, st, gcast(depth_dev), (long long)n,
                p, gcast(pressure_dev));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "barometer launch");
}

int oceansim_dvl(const double *t_dev, const float *ranges_dev, const float *velocity_dev, int32_t n_ticks,
                 int32_t n_inst, const oceansim_dvl_params *params, float *velocity_out_dev, int32_t *status_dev,
                 void *stream) {
    if (!params) return fail(OCEANSIM_E_INVALID_ARG, "params is NULL");
    if (n_ticks < 0 || n_inst < 0) return fail(OCEANSIM_E_SHAPE, "n_ticks and n_inst must be >= 0");
    if ((long long)n_ticks * n_inst == 0) return ok();
    if (!t_dev || !ranges_dev || !velocity_dev || !velocity_out_dev || !status_dev)
        return fail(OCEANSIM_E_INVALID_ARG, "NULL buffer");
    if (!aligned_to(t_dev, 8) || !aligned_to(ranges_dev, 16) || !aligned_to(velocity_dev, 4) ||
        !aligned_to(velocity_out_dev, 4) || !aligned_to(status_dev, 4))
        return fail(OCEANSIM_E_INVALID_ARG, "misaligned buffer (ranges 16-byte, times 8-byte aligned)");
    const oceansim_dvl_params &q = *params;
    if (!(q.janus_angle > 0.0 && q.janus_angle < 1.5707963267948966))
        return fail(OCEANSIM_E_INVALID_ARG, "janus_angle must be in (0, pi/2)");
    if (!(std::isfinite(q.range_min) && std::isfinite(q.range_max) && q.range_min >= 0.0 &&
          q.range_max >= q.range_min))
        return fail(OCEANSIM_E_INVALID_ARG, "need finite 0 <= range_min <= range_max");
    if (q.min_beams != 3 && q.min_beams != 4)
        return fail(OCEANSIM_E_INVALID_ARG, "min_beams must be 3 or 4 (a velocity needs three beams)");
    if (!(std::isfinite(q.sigma_v) && q.sigma_v >= 0.0 && q.sound_speed > 0.0 && std::isfinite(q.sound_speed) &&
          q.pings_per_output > 0.0 && std::isfinite(q.pings_per_output) && q.period_min >= 0.0 &&
          std::isfinite(q.period_min)))
        return fail(OCEANSIM_E_INVALID_ARG, "sigma_v, sound_speed, pings_per_output, period_min out of range");
    DvlDev p;
    for (int i = 0; i < 4; ++i) {
        const double psi = 0.7853981633974483 + 1.5707963267948966 * i;
        p.beam[i][0] = std::sin(q.janus_angle) * std::cos(psi);
        p.beam[i][1] = std::sin(q.janus_angle) * std::sin(psi);
        p.beam[i][2] = -std::cos(q.janus_angle);
    }
    p.range_min = q.range_min;
    p.range_max = q.range_max;
    p.sigma_v = q.sigma_v;
    p.pings_per_output = q.pings_per_output;
    p.sound_speed = q.sound_speed;
    p.period_min = q.period_min;
    p.min_beams = q.min_beams;
    p.seed_lo = q.seed_lo;
    p.seed_hi = q.seed_hi;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int blocks = (n_inst + kNavThreads - 1) / kNavThreads;
    OSIM_LAUNCH("k_dvl", k_dvl, dim3(blocks), dim3(kNavThreads), 0, st, gcast(t_dev),
                gcast(reinterpret_cast<const float4 *>(ranges_dev)), gcast(velocity_dev), (int)n_ticks, (int)n_inst,
                p, gcast(velocity_out_dev), gcast(status_dev));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : hip_fail(e, "dvl launch");
}

}  // extern "C"
