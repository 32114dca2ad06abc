// Underwater colour image formation, Eq. (1) of arXiv 2503.01074 (Sec. III-A.1),
// and its adjoint: per-pixel formulas and the work of one workgroup, shared
// by the camera kernels and by the sonar kernels that carry camera frames
// along in the same launch (internal).
//
//   I_c = J_c exp(-beta_D,c d) + B_inf,c (1 - exp(-beta_B,c d))
#pragma once

#include <type_traits>

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

// e^x for x <= 0 (also -inf and NaN): the hardware 2^y, with the product
// x log2(e) carried to ~2^-48 relative in y + lo so that its rounding does
// not reach the result (a few ulp over the whole range, against the plain
// 2^(x log2 e), whose error grows with |x|).  Below 2^-150 the result is 0.
__device__ __forceinline__ float exp_nonpos(float x) {
    const float kLog2eHi = 1.44269502f;          // log2(e) rounded to float
    const float kLog2eLo = 1.92596299e-8f;       // log2(e) - kLog2eHi
    const float y = x * kLog2eHi;
    if (y < -150.0f) return 0.0f;
    const float lo = __builtin_fmaf(x, kLog2eHi, -y) + x * kLog2eLo;
    return __builtin_amdgcn_exp2f(y) * __builtin_fmaf(lo, 0.693147182f, 1.0f);
}

// 1 - e^-x for x >= 0, given e = e^-x: the difference where it loses at most
// two bits (x > 1/4), else the Taylor series of -expm1(-x) to x^7 (its
// remainder is below 2e-9 relative there).  Both are evaluated and one is
// selected: a branch here splits the unrolled pixel loop into divergent
// blocks and keeps every pixel's intermediates live across them.
__device__ __forceinline__ float one_minus_exp_neg(float x, float e) {
    float p = 1.0f / 5040.0f;
    p = __builtin_fmaf(p, x, -1.0f / 720.0f);
    p = __builtin_fmaf(p, x, 1.0f / 120.0f);
    p = __builtin_fmaf(p, x, -1.0f / 24.0f);
    p = __builtin_fmaf(p, x, 1.0f / 6.0f);
    p = __builtin_fmaf(p, x, -0.5f);
    p = __builtin_fmaf(p, x, 1.0f);
    const float near = p * x;
    const float far = 1.0f - e;
    return x > 0.25f ? far : near;
}

__device__ __forceinline__ float uw_pixel(float J, float d, float bd, float bb, float bi) {
    const float T = exp_nonpos(-bdprod(bd, d));
    const float xb = bdprod(bb, d);
    const float S1 = one_minus_exp_neg(xb, exp_nonpos(-xb));
    return J * T + bi * S1;
}

// The full-size camera block body: KIT float4 groups per thread from pixel
// p0 on, two groups' loads in flight at a time.
template <int NT, int KIT>
__device__ __forceinline__ void uw_fwd_groups(gptr<const float> __restrict__ Jp, gptr<const float> __restrict__ Dp,
                                              gptr<float> __restrict__ Op, long long npix, long long p0, int tx,
                                              const Water &w) {
    constexpr int KH = KIT < 2 ? KIT : 2;
#pragma unroll
    for (int i0 = 0; i0 < KIT; i0 += KH) {
        float4 d[KH], J[KH][3];
#pragma unroll
        for (int h = 0; h < KH; ++h) {
            const long long p = p0 + ((long long)(i0 + h) * NT + tx) * 4;
            d[h] = gload((gptr<const float4>)(Dp + p));
#pragma unroll
            for (int c = 0; c < 3; ++c) J[h][c] = gload((gptr<const float4>)(Jp + c * npix + p));
        }
#pragma unroll
        for (int h = 0; h < KH; ++h) {
            const long long p = p0 + ((long long)(i0 + h) * NT + tx) * 4;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float4 o;
                o.x = uw_pixel(J[h][c].x, d[h].x, w.bd[c], w.bb[c], w.bi[c]);
                o.y = uw_pixel(J[h][c].y, d[h].y, w.bd[c], w.bb[c], w.bi[c]);
                o.z = uw_pixel(J[h][c].z, d[h].z, w.bd[c], w.bb[c], w.bi[c]);
                o.w = uw_pixel(J[h][c].w, d[h].w, w.bd[c], w.bb[c], w.bi[c]);
                gstore_stream((gptr<float4>)(Op + c * npix + p), o);
            }
        }
    }
}

// Workgroup `bid` (of NT threads, this thread being `tx` of them) of a
// forward launch over the frames of src: f.fwd_px pixels per thread (4, 8,
// 16 or 32, the same for every frame of the launch), as float4 groups.  No
// barrier: a wider workgroup may run several of these blocks side by side.
template <class Src, int NT>
__device__ __forceinline__ void uw_fwd_block(const Src &src, const oceansim_water_params *params, int bid,
                                             int tx) {
    int local;
    const int fi = src.locate(bid, 0, local);
    const UwDev f = src.frame(fi);
    const Water w = load_water(params, f.param_row);
    const long long npix = f.npix;
    const int px = f.fwd_px;
    const long long p0 = (long long)local * NT * px;
    // restrict-qualified views (the output never aliases the inputs), so the
    // loads of a group can be in flight before the previous group's stores
    const gptr<const float> __restrict__ Jp = f.J;
    const gptr<const float> __restrict__ Dp = f.depth;
    const gptr<float> __restrict__ Op = f.out;
    if ((npix & 3) == 0 && p0 + (long long)NT * px <= npix) {
        switch (px) {
            case 32: uw_fwd_groups<NT, 8>(Jp, Dp, Op, npix, p0, tx, w); break;
            case 16: uw_fwd_groups<NT, 4>(Jp, Dp, Op, npix, p0, tx, w); break;
            case 8: uw_fwd_groups<NT, 2>(Jp, Dp, Op, npix, p0, tx, w); break;
            default: uw_fwd_groups<NT, 1>(Jp, Dp, Op, npix, p0, tx, w); break;
        }
        return;
    }
    // ragged tail (or an image whose size is not a multiple of 4): per pixel
    for (int it = 0; it < px / 4; ++it) {
        const long long p = p0 + ((long long)it * NT + tx) * 4;
        for (long long q = p; q < p + 4 && q < npix; ++q) {
            const float d = Dp[q];
#pragma unroll
            for (int c = 0; c < 3; ++c)
                gstore_stream(Op + c * npix + q, uw_pixel(Jp[c * npix + q], d, w.bd[c], w.bb[c], w.bi[c]));
        }
    }
}

// e^x for x <= 0 as the hardware 2^(x log2 e) with the product rounded to
// float: within about 1e-6 relative over x in [-20, 0], which the adjoint's
// tolerance leaves room for (the forward image keeps exp_nonpos).
__device__ __forceinline__ float exp_nonpos_adj(float x) { return __builtin_amdgcn_exp2f(x * 1.44269502f); }

// Adjoint of Eq. (1) at one pixel and channel; accumulates the parameter
// gradients and returns dL/dJ, adding this channel's share of dL/dd.
// 1 - e^-x for x >= 0 as one_minus_exp_neg, the series to x^5 (below 1/4
// its remainder is under 1.4e-6 relative, within the adjoint's tolerance
// like exp_nonpos_adj; the forward image keeps the series to x^7).
__device__ __forceinline__ float one_minus_exp_neg_adj(float x, float e) {
    float p = 1.0f / 120.0f;
    p = __builtin_fmaf(p, x, -1.0f / 24.0f);
    p = __builtin_fmaf(p, x, 1.0f / 6.0f);
    p = __builtin_fmaf(p, x, -0.5f);
    p = __builtin_fmaf(p, x, 1.0f);
    const float near = p * x;
    const float far = 1.0f - e;
    return x > 0.25f ? far : near;
}

__device__ __forceinline__ float uw_pixel_bwd(float g, float J, float d, float bd, float bb, float bi,
                                              float acc[9], int c, float &gd) {
    const float T = exp_nonpos_adj(-bdprod(bd, d));
    const float xb = bdprod(bb, d);
    const float S = exp_nonpos_adj(-xb);
    const float S1 = one_minus_exp_neg_adj(xb, S);
    // the d-weighted terms vanish where T or S does (0 * inf := 0)
    if (T != 0.0f) acc[c] += g * (-J * T * d);
    if (S != 0.0f) acc[3 + c] += g * (bi * S * d);
    acc[6 + c] += g * S1;
    gd += g * (-bd * J * T + bi * bb * S);
    return g * T;
}

// The full-size camera backward block body: KIT float4 groups per thread
// from pixel p0 on, two groups' loads in flight at a time (for KIT > 2 an
// empty asm statement taking the running sums as operands ends each pair of
// groups, so the next pair's loads are not hoisted above it).  IMG: image
// gradients are written (GJ or GD set); without, their terms are not formed.
template <int NT, int KIT, bool IMG>
__device__ __forceinline__ void uw_bwd_groups(gptr<const float> __restrict__ Jp, gptr<const float> __restrict__ Dp,
                                              gptr<const float> __restrict__ Gp, gptr<float> __restrict__ GJ,
                                              gptr<float> __restrict__ GD, long long npix, long long p0, int tx,
                                              const Water &w, float (&acc)[9]) {
#pragma unroll
    for (int i0 = 0; i0 < KIT; i0 += 2) {
        float4 d[2], J[2][3], g[2][3];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const long long p = p0 + ((long long)(i0 + h) * NT + tx) * 4;
            d[h] = gload((gptr<const float4>)(Dp + p));
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                J[h][c] = gload((gptr<const float4>)(Jp + c * npix + p));
                g[h][c] = gload((gptr<const float4>)(Gp + c * npix + p));
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const long long p = p0 + ((long long)(i0 + h) * NT + tx) * 4;
            float4 gdv = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float4 gj;
                gj.x = uw_pixel_bwd(g[h][c].x, J[h][c].x, d[h].x, w.bd[c], w.bb[c], w.bi[c], acc, c, gdv.x);
                gj.y = uw_pixel_bwd(g[h][c].y, J[h][c].y, d[h].y, w.bd[c], w.bb[c], w.bi[c], acc, c, gdv.y);
                gj.z = uw_pixel_bwd(g[h][c].z, J[h][c].z, d[h].z, w.bd[c], w.bb[c], w.bi[c], acc, c, gdv.z);
                gj.w = uw_pixel_bwd(g[h][c].w, J[h][c].w, d[h].w, w.bd[c], w.bb[c], w.bi[c], acc, c, gdv.w);
                if (IMG && GJ) gstore_stream((gptr<float4>)(GJ + c * npix + p), gj);
            }
            if (IMG && GD) gstore_stream((gptr<float4>)(GD + p), gdv);
        }
        if (i0 + 2 < KIT)
            __asm__ volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]),
                             "+v"(acc[5]), "+v"(acc[6]), "+v"(acc[7]), "+v"(acc[8])::"memory");
    }
}

// Workgroup `bid` (of NT threads, this thread being `tx` of them) of a
// backward launch: f.bwd_px pixels per thread, as float4 groups: with 8
// pixels per thread and PINNED = false, both groups' loads in flight
// together; otherwise one channel of one group at a time (PINNED: the
// register budget of launches shared with sonar tiles); the nine parameter partial sums of the workgroup go to
// part[c * n_slots + bid] (FP64, fixed order) and its parameter row to
// part_row[bid].  `red9` is LDS of 9 * NT / 64 doubles.  Contains workgroup
// barriers: in a wider workgroup that runs several such blocks side by side,
// every thread calls it, those of a block past the last with active = false
// (no pixels, nothing written).
template <class Src, int NT, bool PINNED = false>
__device__ __forceinline__ void uw_bwd_block(const Src &src, const oceansim_water_params *params, double *part,
                                             int *part_row, int bid, int n_slots, double *red9,
                                             int tx = (int)threadIdx.x, bool active = true) {
    // per-thread partial sums in FP32 (|error| <= ~5e-7 of the sum of the
    // magnitudes per group of pixels), then FP64 across threads and workgroups
    float acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.0f;
    int row = 0;
    if (active) {
        int local;
        const int fi = src.locate(bid, 0, local);
        const UwDev f = src.frame(fi);
        row = f.param_row;
        const Water w = load_water(params, f.param_row);
        const long long npix = f.npix;
        const int px = f.bwd_px;
        const int n_it = px / 4;   // even
        const long long p0 = (long long)local * NT * px;
        const gptr<const float> __restrict__ Jp = f.J;
        const gptr<const float> __restrict__ Dp = f.depth;
        const gptr<const float> __restrict__ Gp = f.grad_out;
        const gptr<float> __restrict__ GJ = f.grad_J;
        const gptr<float> __restrict__ GD = f.grad_depth;
        if ((npix & 3) == 0 && p0 + (long long)NT * px <= npix) {
            // without image gradients (GJ and GD null) the code is compiled
            // without them, so their terms are not formed
            const bool img = GJ || GD;
            if (!PINNED && n_it == 2) {
                if (img)
                    uw_bwd_groups<NT, 2, true>(Jp, Dp, Gp, GJ, GD, npix, p0, tx, w, acc);
                else
                    uw_bwd_groups<NT, 2, false>(Jp, Dp, Gp, GJ, GD, npix, p0, tx, w, acc);
            } else {
                // one channel at a time: the empty asm statements take the
                // running sums as operands, so each channel's arithmetic is
                // done before the next channel's loads are issued
                auto channels = [&](auto with_img) __attribute__((always_inline)) {
                    constexpr bool IMG = decltype(with_img)::value;
#pragma unroll 1
                    for (int it = 0; it < n_it; ++it) {
                        const long long p = p0 + ((long long)it * NT + tx) * 4;
                        const float4 d = gload((gptr<const float4>)(Dp + p));
                        float4 gdv = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const float4 J = gload((gptr<const float4>)(Jp + c * npix + p));
                            const float4 g = gload((gptr<const float4>)(Gp + c * npix + p));
                            float4 gj;
                            gj.x = uw_pixel_bwd(g.x, J.x, d.x, w.bd[c], w.bb[c], w.bi[c], acc, c, gdv.x);
                            gj.y = uw_pixel_bwd(g.y, J.y, d.y, w.bd[c], w.bb[c], w.bi[c], acc, c, gdv.y);
                            gj.z = uw_pixel_bwd(g.z, J.z, d.z, w.bd[c], w.bb[c], w.bi[c], acc, c, gdv.z);
                            gj.w = uw_pixel_bwd(g.w, J.w, d.w, w.bd[c], w.bb[c], w.bi[c], acc, c, gdv.w);
                            if (IMG) {
                                if (GJ) gstore_stream((gptr<float4>)(GJ + c * npix + p), gj);
                                __asm__ volatile("" : "+v"(acc[c]), "+v"(acc[3 + c]), "+v"(acc[6 + c]), "+v"(gdv.x),
                                                 "+v"(gdv.y), "+v"(gdv.z), "+v"(gdv.w)::"memory");
                            } else {
                                __asm__ volatile("" : "+v"(acc[c]), "+v"(acc[3 + c]), "+v"(acc[6 + c])::"memory");
                            }
                        }
                        if (IMG && GD) gstore_stream((gptr<float4>)(GD + p), gdv);
                    }
                };
                if (img)
                    channels(std::true_type{});
                else
                    channels(std::false_type{});
            }
        } else {
            // ragged tail (or an image whose size is not a multiple of 4): per pixel
            for (int it = 0; it < n_it; ++it) {
                const long long p = p0 + ((long long)it * NT + tx) * 4;
                for (long long q = p; q < p + 4 && q < npix; ++q) {
                    const float d = Dp[q];
                    float gd = 0.0f;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float gj = uw_pixel_bwd(Gp[c * npix + q], Jp[c * npix + q], d, w.bd[c], w.bb[c],
                                                      w.bi[c], acc, c, gd);
                        if (GJ) gstore_stream(GJ + c * npix + q, gj);
                    }
                    if (GD) gstore_stream(GD + q, gd);
                }
            }
        }
    }
    double accd[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) accd[k] = (double)acc[k];
    const double tot = block_sum_n<9, NT>(accd, red9, tx);
    if (active && tx < 9) part[(long long)tx * n_slots + bid] = tot;   // column-major partials
    if (active && tx == 0) part_row[bid] = row;
}

}  // namespace osim
