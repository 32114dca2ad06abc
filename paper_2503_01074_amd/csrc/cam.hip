// Camera input conditioning and output encoding for gfx950 (Sec. III-A.1):
// 8-bit sRGB in and out around Eq. (1), and z-depth turned into the
// line-of-sight distance that Eq. (1) attenuates with, plus that conversion's
// adjoint.
//
// Pure streaming kernels, four consecutive pixels per thread: the byte image
// moves as dwords (RGB: three per four pixels, RGBA: one dwordx4), planar
// float images as float4 when the plane size is a multiple of four, depth
// always as float4.  Decoding is one LDS table lookup per channel; encoding
// takes a first-guess code from the float's exponent and top mantissa bits
// and one comparison with the next of 255 LDS thresholds that reproduce the
// double-precision rounding decision exactly (srgb_tables.hpp), so no power
// function runs on the GPU.  Up to kCamBatch frames travel by value in the
// kernel arguments: no workspace, no table upload.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/oceansim.h"
#include "host.hpp"
#include "launch.hpp"
#include "srgb_tables.hpp"

namespace osim {
namespace {

constexpr int kCamBatch = 16;
constexpr int kCamBlock = 256;
constexpr int kPix = 4;                       // pixels per thread
constexpr int kMaxCamBlocks = (1 << 24) - 1;  // grid limit: 2^32 work-items

struct CamDev {
    const uint8_t *srgb;
    const float *src;   // forward: z-depth; backward: dL/d(range)
    float *J;
    float *dst;         // forward: range; backward: dL/dz
    unsigned hw;        // H * W (< 2^32 with H, W <= 65535)
    int W, ch;
    float ifx, ify, cx, cy;
    int block0;         // first workgroup of this frame in the launch
};
struct CamBatch {
    int n;
    CamDev f[kCamBatch];
};
struct OutDev {
    const float *I;
    uint8_t *out;
    unsigned hw;
    int ch;
    int block0;
};
struct OutBatch {
    int n;
    OutDev f[kCamBatch];
};

// The frame of this workgroup: uniform selects over constant kernel-argument
// offsets (no dynamically indexed copy of the batch).
template <class Batch, class Dev>
__device__ __forceinline__ Dev frame_of(const Batch &B) {
    Dev f = B.f[0];
#pragma unroll
    for (int k = 1; k < kCamBatch; ++k)
        if (k < B.n && (int)blockIdx.x >= B.f[k].block0) f = B.f[k];
    return f;
}

__device__ __forceinline__ unsigned byte_of(const uint32_t *w, int i) { return (w[i >> 2] >> (8 * (i & 3))) & 255u; }

// BWD = false: decode srgb into J (when present) and scale z-depth into range
// (when present).  BWD = true: scale dL/d(range) into dL/dz.
template <bool BWD>
__global__ __launch_bounds__(kCamBlock) void k_cam_cond(CamBatch B) {
    __shared__ float dec[256];
    const CamDev f = frame_of<CamBatch, CamDev>(B);
    if (!BWD && f.srgb) {
        dec[threadIdx.x] = kSrgbDecode[threadIdx.x];
        __syncthreads();
    }
    const unsigned p = ((unsigned)(blockIdx.x - f.block0) * kCamBlock + threadIdx.x) * kPix;
    if (p >= f.hw) return;
    const bool full = f.hw - p >= (unsigned)kPix;

    if (f.src) {
        float z[kPix];
        if (full) {
            const float4 t = *reinterpret_cast<const float4 *>(f.src + p);
            z[0] = t.x, z[1] = t.y, z[2] = t.z, z[3] = t.w;
        } else {
#pragma unroll
            for (int k = 0; k < kPix; ++k) z[k] = p + k < f.hw ? f.src[p + k] : 0.f;
        }
        unsigned v = p / (unsigned)f.W, u = p - v * (unsigned)f.W;
#pragma unroll
        for (int k = 0; k < kPix; ++k) {
            const float a = ((float)u + 0.5f - f.cx) * f.ifx;
            const float b = ((float)v + 0.5f - f.cy) * f.ify;
            z[k] *= sqrtf(1.f + a * a + b * b);
            if (++u == (unsigned)f.W) u = 0, ++v;
        }
        if (full) {
            *reinterpret_cast<float4 *>(f.dst + p) = make_float4(z[0], z[1], z[2], z[3]);
        } else {
#pragma unroll
            for (int k = 0; k < kPix; ++k)
                if (p + k < f.hw) f.dst[p + k] = z[k];
        }
    }

    if (!BWD && f.srgb) {
        unsigned c[kPix][3];
        if (full && f.ch == 3) {
            const uint32_t *w = reinterpret_cast<const uint32_t *>(f.srgb + (size_t)p * 3);
            const uint32_t ws[3] = {w[0], w[1], w[2]};
#pragma unroll
            for (int k = 0; k < kPix; ++k)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) c[k][ch] = byte_of(ws, 3 * k + ch);
        } else if (full) {
            const uint4 t = *reinterpret_cast<const uint4 *>(f.srgb + (size_t)p * 4);
            const uint32_t ws[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int k = 0; k < kPix; ++k)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) c[k][ch] = byte_of(ws, 4 * k + ch);
        } else {
#pragma unroll
            for (int k = 0; k < kPix; ++k)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch)
                    c[k][ch] = p + k < f.hw ? f.srgb[(size_t)(p + k) * f.ch + ch] : 0u;
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float *plane = f.J + (size_t)ch * f.hw;
            if (full && (f.hw & 3u) == 0) {
                *reinterpret_cast<float4 *>(plane + p) =
                    make_float4(dec[c[0][ch]], dec[c[1][ch]], dec[c[2][ch]], dec[c[3][ch]]);
            } else {
#pragma unroll
                for (int k = 0; k < kPix; ++k)
                    if (p + k < f.hw) plane[p + k] = dec[c[k][ch]];
            }
        }
    }
}

static_assert(kSrgbGuessSpan == 1 && kSrgbGuessN % 4 == 0, "one threshold comparison after the guess");

__global__ __launch_bounds__(kCamBlock) void k_cam_encode(OutBatch B) {
    __shared__ float thr[257];                      // thr[256] = +inf: the guess may be 255
    __shared__ uint32_t guess_w[kSrgbGuessN / 4];   // the first-guess codes, four per word
    const OutDev f = frame_of<OutBatch, OutDev>(B);
    thr[threadIdx.x] = kSrgbThreshold[threadIdx.x];
    if (threadIdx.x == 0) thr[256] = __builtin_inff();
    for (int k = threadIdx.x; k < kSrgbGuessN / 4; k += kCamBlock)
        guess_w[k] = (uint32_t)kSrgbGuess[4 * k] | (uint32_t)kSrgbGuess[4 * k + 1] << 8 |
                     (uint32_t)kSrgbGuess[4 * k + 2] << 16 | (uint32_t)kSrgbGuess[4 * k + 3] << 24;
    __syncthreads();
    const unsigned char *guess = reinterpret_cast<const unsigned char *>(guess_w);
    const unsigned p = ((unsigned)(blockIdx.x - f.block0) * kCamBlock + threadIdx.x) * kPix;
    if (p >= f.hw) return;
    const bool full = f.hw - p >= (unsigned)kPix;

    uint32_t c[kPix][3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float *plane = f.I + (size_t)ch * f.hw;
        float x[kPix];
        if (full && (f.hw & 3u) == 0) {
            const float4 t = *reinterpret_cast<const float4 *>(plane + p);
            x[0] = t.x, x[1] = t.y, x[2] = t.z, x[3] = t.w;
        } else {
#pragma unroll
            for (int k = 0; k < kPix; ++k) x[k] = p + k < f.hw ? plane[p + k] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < kPix; ++k) {
            // the number of thresholds x reaches (NaN reaches none): below
            // 2^-13 none, from 1 on all 255; between, the code of x's bucket
            // (exponent and top seven mantissa bits) and one more comparison
            const float xv = x[k];
            int idx = (int)(__float_as_uint(xv) >> 16) - (kSrgbGuessE0 << 7);
            idx = idx < 0 ? 0 : (idx > kSrgbGuessN - 1 ? kSrgbGuessN - 1 : idx);
            unsigned q = guess[idx];
            q += xv >= thr[q + 1] ? 1u : 0u;
            c[k][ch] = xv >= 1.0f ? 255u : (xv >= 0x1p-13f ? q : 0u);
        }
    }
    if (full && f.ch == 3) {
        uint32_t w[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < kPix; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) w[(3 * k + ch) >> 2] |= c[k][ch] << (8 * ((3 * k + ch) & 3));
        uint32_t *o = reinterpret_cast<uint32_t *>(f.out + (size_t)p * 3);
        o[0] = w[0], o[1] = w[1], o[2] = w[2];
    } else if (full) {
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < kPix; ++k) w[k] = c[k][0] | c[k][1] << 8 | c[k][2] << 16 | 0xff000000u;
        *reinterpret_cast<uint4 *>(f.out + (size_t)p * 4) = make_uint4(w[0], w[1], w[2], w[3]);
    } else {
#pragma unroll
        for (int k = 0; k < kPix; ++k) {
            if (p + k >= f.hw) continue;
            uint8_t *o = f.out + (size_t)(p + k) * f.ch;
            o[0] = (uint8_t)c[k][0], o[1] = (uint8_t)c[k][1], o[2] = (uint8_t)c[k][2];
            if (f.ch == 4) o[3] = 255;
        }
    }
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

int blocks_for(unsigned hw) {
    const unsigned long long quads = (hw + (unsigned long long)kPix - 1) / kPix;
    return (int)((quads + kCamBlock - 1) / kCamBlock);
}

int check_shape(int H, int W, int i) {
    if (H < 0 || W < 0 || H > 65535 || W > 65535)
        return host::fail(OCEANSIM_E_SHAPE, "frame %d: H = %d, W = %d outside 0..65535", i, H, W);
    return OCEANSIM_OK;
}

int check_intrinsics(const oceansim_cam_frame &f, int i) {
    if (!std::isfinite(f.fx) || !std::isfinite(f.fy) || f.fx == 0.f || f.fy == 0.f || !std::isfinite(f.cx) ||
        !std::isfinite(f.cy))
        return host::fail(OCEANSIM_E_INVALID_ARG, "frame %d: fx, fy must be finite and nonzero, cx, cy finite", i);
    return OCEANSIM_OK;
}

int check_cam(const oceansim_cam_frame &f, int i, bool bwd) {
    int rc = check_shape(f.H, f.W, i);
    if (rc) return rc;
    if (f.H == 0 || f.W == 0) return OCEANSIM_OK;   // an empty frame needs no buffers
    if (bwd) {
        if (!f.grad_range || !f.grad_zdepth)
            return host::fail(OCEANSIM_E_INVALID_ARG, "frame %d: grad_range and grad_zdepth are required", i);
        if (!aligned16(f.grad_range) || !aligned16(f.grad_zdepth))
            return host::fail(OCEANSIM_E_INVALID_ARG, "frame %d: gradient buffers must be 16-byte aligned", i);
        return check_intrinsics(f, i);
    }
    if (f.srgb_in) {
        if (f.channels_in != 3 && f.channels_in != 4)
            return host::fail(OCEANSIM_E_INVALID_ARG, "frame %d: channels_in = %d (3 or 4)", i, f.channels_in);
        if (!f.J) return host::fail(OCEANSIM_E_INVALID_ARG, "frame %d: srgb_in given without J", i);
        if (!aligned16(f.srgb_in) || !aligned16(f.J))
            return host::fail(OCEANSIM_E_INVALID_ARG, "frame %d: srgb_in and J must be 16-byte aligned", i);
    }
    if (f.zdepth) {
        if (!f.range) return host::fail(OCEANSIM_E_INVALID_ARG, "frame %d: zdepth given without range", i);
        if (!aligned16(f.zdepth) || !aligned16(f.range))
            return host::fail(OCEANSIM_E_INVALID_ARG, "frame %d: zdepth and range must be 16-byte aligned", i);
        return check_intrinsics(f, i);
    }
    return OCEANSIM_OK;
}

// Validates every frame first, then launches in batches of at most kCamBatch
// frames and kMaxCamBlocks workgroups.
int cam_condition(const oceansim_cam_frame *frames, int n_frames, void *stream, bool bwd) {
    if (n_frames < 0) return host::fail(OCEANSIM_E_INVALID_ARG, "n_frames < 0");
    if (n_frames > 0 && !frames) return host::fail(OCEANSIM_E_INVALID_ARG, "frames is NULL");
    for (int i = 0; i < n_frames; ++i) {
        int rc = check_cam(frames[i], i, bwd);
        if (rc) return rc;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    CamBatch B{};
    int blocks = 0;
    auto flush = [&]() -> hipError_t {
        if (B.n == 0) return hipSuccess;
        if (bwd)
            OSIM_LAUNCH("k_cam_cond_bwd", (k_cam_cond<true>), dim3(blocks), dim3(kCamBlock), 0, st, B);
        else
            OSIM_LAUNCH("k_cam_cond", (k_cam_cond<false>), dim3(blocks), dim3(kCamBlock), 0, st, B);
        B = CamBatch{};
        blocks = 0;
        return hipGetLastError();
    };
    for (int i = 0; i < n_frames; ++i) {
        const oceansim_cam_frame &f = frames[i];
        const unsigned hw = (unsigned)f.H * (unsigned)f.W;
        const int nb = blocks_for(hw);
        const bool work = hw > 0 && (bwd || f.srgb_in || f.zdepth);
        if (!work) continue;
        if (B.n == kCamBatch || blocks + nb > kMaxCamBlocks) {
            hipError_t e = flush();
            if (e != hipSuccess) return host::hip_fail(e, "camera conditioning launch");
        }
        CamDev &d = B.f[B.n++];
        d.srgb = bwd ? nullptr : f.srgb_in;
        d.src = bwd ? f.grad_range : f.zdepth;
        d.J = f.J;
        d.dst = bwd ? f.grad_zdepth : f.range;
        d.hw = hw;
        d.W = f.W;
        d.ch = f.channels_in;
        d.ifx = (float)(1.0 / (double)f.fx);
        d.ify = (float)(1.0 / (double)f.fy);
        d.cx = f.cx;
        d.cy = f.cy;
        d.block0 = blocks;
        blocks += nb;
    }
    hipError_t e = flush();
    if (e != hipSuccess) return host::hip_fail(e, "camera conditioning launch");
    return host::ok();
}

}  // namespace
}  // namespace osim

using namespace osim;

extern "C" int oceansim_cam_condition(const oceansim_cam_frame *frames, int32_t n_frames, void *stream) {
    return cam_condition(frames, n_frames, stream, false);
}

extern "C" int oceansim_cam_condition_backward(const oceansim_cam_frame *frames, int32_t n_frames, void *stream) {
    return cam_condition(frames, n_frames, stream, true);
}

extern "C" int oceansim_cam_encode(const oceansim_cam_out_frame *frames, int32_t n_frames, void *stream) {
    if (n_frames < 0) return host::fail(OCEANSIM_E_INVALID_ARG, "n_frames < 0");
    if (n_frames > 0 && !frames) return host::fail(OCEANSIM_E_INVALID_ARG, "frames is NULL");
    for (int i = 0; i < n_frames; ++i) {
        const oceansim_cam_out_frame &f = frames[i];
        int rc = check_shape(f.H, f.W, i);
        if (rc) return rc;
        if (f.channels_out != 3 && f.channels_out != 4)
            return host::fail(OCEANSIM_E_INVALID_ARG, "frame %d: channels_out = %d (3 or 4)", i, f.channels_out);
        if (f.H == 0 || f.W == 0) continue;
        if (!f.I || !f.srgb_out) return host::fail(OCEANSIM_E_INVALID_ARG, "frame %d: I and srgb_out are required", i);
        if (!aligned16(f.I) || !aligned16(f.srgb_out))
            return host::fail(OCEANSIM_E_INVALID_ARG, "frame %d: I and srgb_out must be 16-byte aligned", i);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    OutBatch B{};
    int blocks = 0;
    auto flush = [&]() -> hipError_t {
        if (B.n == 0) return hipSuccess;
        OSIM_LAUNCH("k_cam_encode", k_cam_encode, dim3(blocks), dim3(kCamBlock), 0, st, B);
        B = OutBatch{};
        blocks = 0;
        return hipGetLastError();
    };
    for (int i = 0; i < n_frames; ++i) {
        const oceansim_cam_out_frame &f = frames[i];
        const unsigned hw = (unsigned)f.H * (unsigned)f.W;
        if (hw == 0) continue;
        const int nb = blocks_for(hw);
        if (B.n == kCamBatch || blocks + nb > kMaxCamBlocks) {
            hipError_t e = flush();
            if (e != hipSuccess) return host::hip_fail(e, "camera encoding launch");
        }
        OutDev &d = B.f[B.n++];
        d.I = f.I;
        d.out = f.srgb_out;
        d.hw = hw;
        d.ch = f.channels_out;
        d.block0 = blocks;
        blocks += nb;
    }
    hipError_t e = flush();
    if (e != hipSuccess) return host::hip_fail(e, "camera encoding launch");
    return host::ok();
}
