// Sonar image formation kernels for gfx950 (Sec. III-A.2 of arXiv 2503.01074).
//
// Forward, per frame:
//   k_bin   one workgroup per chunk of returns: Eq. (2) intensity and bin of
//           every return, then an LDS counting sort of the chunk by polar tile
//           (a tile is a block of whole range rows).  Writes the chunk's
//           (tile-local bin, intensity) pairs grouped by tile and the chunk's
//           per-tile offsets.  No global atomics.
//   k_tile  one workgroup per polar tile: gathers the tile's pairs from every
//           chunk and sums them into an LDS histogram (binning by summation),
//           then applies the gain, the optional range-wise normalisation
//           (each row over its maximum) and the speckle of Eq. (3)-(6) per
//           bin and streams the tile out row-major.
//   k_fan   one thread per mirror pair of fan pixels: FP64 polar coordinates,
//           bilinear interpolation of the polar image.
//   k_bin_uw    (plans with camera frames) k_bin plus the camera forward.
//   k_tile_uw   (plans with camera frames and wide tiles) k_tile plus the
//               camera forward, workgroups of both kinds interleaved.
// Backward, per frame:
//   k_pair_bwd  (plans, tables of at most 64 materials) one workgroup per
//               forward tile: the tile's polar gradient read once into LDS,
//               then the adjoint of binning, gain, the multiplicative speckle
//               and Eq. (2) from the (bin, material) pairs and ranges the
//               forward left, summed in order-independent 64-bit fixed point.
//   k_fant_bwd  (plans) rows of the transposed fan operator built at plan
//               creation: each bin's fan gradient gathered through its
//               entries in FP64 (a mirrored row yields a bin and its mirror
//               bin), plus the polar gradient; adjoint of the additive
//               speckle term (sigma_phi, sigma_sa partial sums).
//   k_tile_bwd  (plain entry points) one workgroup per polar tile: transpose of the fan as a gather
//               of the fan pixels whose stencil touches the tile, accumulated
//               in LDS in 64-bit fixed point (order-independent, so the sums
//               are bit-reproducible), plus the polar gradient; adjoint of the
//               additive speckle term (sigma_phi, sigma_sa partial sums).
//   k_ret_bwd   one workgroup per chunk of returns: adjoint of binning as a
//               gather of the bin gradient at each return, then of gain,
//               multiplicative speckle and Eq. (2) (alpha, gain, sigma_sm and
//               reflectivity partial sums).
//   k_ret_uw_bwd  (plans with camera frames) k_ret_bwd plus the camera backward.
//   k_rownorm_bwd (range-normalised frames) one workgroup per range row:
//               adjoint of the row normalisation, before the return gather.
#include <type_traits>

#include "device.hpp"
#include "launch.hpp"
#include "reduce_body.hpp"
#include "uw_body.hpp"

namespace osim {

// ---------------------------------------------------------------------------
// k_bin
// ---------------------------------------------------------------------------
// Binning chunk `bid` of the launch (NT threads, R returns each).  With matp
// the pairs carry the material id and the reflectivity-free factor
// cos(gamma) exp(-kappa alpha r) (the tile multiplies by the reflectivity),
// and with pair_r the ranges of the pairs are written too, in the same order
// (a second pass through the staging memory): what the pair backward reads
// instead of the returns.
template <class Src, int NT, int R>
__device__ __forceinline__ void bin_block(const Src &src, const oceansim_sonar_params *params, const float *refl,
                                          int n_mat, int bid) {
    extern __shared__ int4 lds_raw[];
    int local;
    const int fi = src.locate(bid, KBIN, local);
    const SonarDev f = src.frame(fi);
    const int tid = threadIdx.x;
    const int n_tiles = f.n_tiles;
    int *hist = reinterpret_cast<int *>(lds_raw);                    // n_tiles + 1
    __shared__ int scan_tmp[NT];
    uint2 *stage = reinterpret_cast<uint2 *>(hist + ((n_tiles + 1 + 3) & ~3));  // R * NT
    const bool matp = f.matp != 0;

    const float alpha = params[f.param_row].alpha;
    const long long base = (long long)local * (R * NT);
    const float inv_tb = 1.0f / (float)f.tile_bins;

    for (int t = tid; t <= n_tiles; t += NT) hist[t] = 0;
    __syncthreads();

    // restrict-qualified views: the optional bin output never aliases the
    // returns, so the loads of all R returns can be in flight together
    const gptr<const float> __restrict__ X = f.x;
    const gptr<const float> __restrict__ Y = f.y;
    const gptr<const float> __restrict__ Z = f.z;
    const gptr<const float> __restrict__ NX = f.nx;
    const gptr<const float> __restrict__ NY = f.ny;
    const gptr<const float> __restrict__ NZ = f.nz;
    const gptr<const int> __restrict__ MAT = f.mat;
    const float *__restrict__ RF = refl;
    const gptr<int> __restrict__ BO = f.bin_of_return;
    const bool want_r = f.pair_r != nullptr;
    // trk: tile << 14 | rank within the tile (-1: no pair); chunks hold at most 2^14 returns
    int trk[R];
    uint32_t lbin[R];
    float inten[R], rr[R];
    // Groups of RG returns: all their loads, then their reflectivity gathers,
    // are in flight together (clamped indices: a load under the per-return
    // branches would wait for itself before the next return's); pairs for
    // small chunks, whose workgroups share the launch with camera workgroups
    constexpr int RG = (R <= 4 && NT == kBlock) ? 2 : 4;
#pragma unroll
    for (int q0 = 0; q0 < R; q0 += RG) {
        float xs[RG], ys[RG], zs[RG], nxs[RG], nys[RG], nzs[RG], rfs[RG];
        int ms[RG], bs[RG];
        double rs[RG];
#pragma unroll
        for (int u = 0; u < RG; ++u) {
            const long long k = base + (long long)(q0 + u) * NT + tid;
            const long long kc = k < f.n ? k : f.n - 1;
            xs[u] = X[kc];
            ys[u] = Y[kc];
            zs[u] = Z[kc];
            nxs[u] = NX[kc];
            nys[u] = NY[kc];
            nzs[u] = NZ[kc];
            ms[u] = MAT[kc];
        }
#pragma unroll
        for (int u = 0; u < RG; ++u) {
            const long long k = base + (long long)(q0 + u) * NT + tid;
            const int b = return_bin(f, xs[u], ys[u], zs[u], ms[u], n_mat, rs[u]);
            if (BO && k < f.n) BO[k] = b;
            bs[u] = k < f.n ? b : -1;   // a valid bin implies a valid material
        }
        if (!matp) {
#pragma unroll
            for (int u = 0; u < RG; ++u) rfs[u] = RF[bs[u] >= 0 ? ms[u] : 0];
        }
#pragma unroll
        for (int u = 0; u < RG; ++u) {
            const int q = q0 + u, b = bs[u];
            trk[q] = -1;
            if (b >= 0) {
                float cosg, att;
                inten[q] = return_intensity(f, xs[u], ys[u], zs[u], nxs[u], nys[u], nzs[u], rs[u],
                                            matp ? 1.0f : rfs[u], alpha, cosg, att);
                rr[q] = (float)rs[u];
                // tile t = b / tile_bins by a float reciprocal (b < 2^24 and
                // b / tile_bins < 2^12, so the product is within 2^-11 of the
                // quotient and one correction step makes it exact)
                int t = (int)((float)b * inv_tb);
                int lb = b - t * f.tile_bins;
                if (lb < 0) {
                    --t;
                    lb += f.tile_bins;
                } else if (lb >= f.tile_bins) {
                    ++t;
                    lb -= f.tile_bins;
                }
                lbin[q] = (uint32_t)lb | (matp ? (uint32_t)ms[u] << 16 : 0u);
                trk[q] = (t << 14) | atomicAdd(&hist[t], 1);
            }
        }
    }
    __syncthreads();
    block_exclusive_scan<NT>(hist, n_tiles, scan_tmp);

    const gptr<int> off = f.chunk_off + (long long)local * (n_tiles + 1);
    for (int t = tid; t <= n_tiles; t += NT) off[t] = hist[t];
#pragma unroll
    for (int q = 0; q < R; ++q)
        if (trk[q] >= 0)
            stage[hist[trk[q] >> 14] + (trk[q] & 16383)] = make_uint2(lbin[q], __float_as_uint(inten[q]));
    __syncthreads();
    const int total = hist[n_tiles];
    const gptr<uint2> dst = f.pairs + base;
    for (int k = tid; k < total; k += NT) gstore(dst + k, stage[k]);
    if (want_r) {
        // the ranges, in the pairs' order, through the same staging memory
        float *rstage = reinterpret_cast<float *>(stage);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (trk[q] >= 0) rstage[hist[trk[q] >> 14] + (trk[q] & 16383)] = rr[q];
        __syncthreads();
        const gptr<float> rdst = f.pair_r + base;
        for (int k = tid; k < total; k += NT) rdst[k] = rstage[k];
    }
}

template <class Src, int NT, int R>
__global__ __launch_bounds__(NT) void k_bin(Src src, const oceansim_sonar_params *params, const float *refl,
                                            int n_mat) {
    bin_block<Src, NT, R>(src, params, refl, n_mat, blockIdx.x);
}

// The binning chunks of the sonar frames and, in the same launch, the camera
// forward of a plan (workgroups n_bin_blocks and up): the chunks are few and
// latency-bound, so the camera's HBM stream fills the rest of the chip.
template <class Src, int R>
__global__ __launch_bounds__(kBlock) void k_bin_uw(Src src, const oceansim_sonar_params *params,
                                                   const float *refl, int n_mat, int n_bin_blocks,
                                                   Table<UwDev> usrc, const oceansim_water_params *wparams) {
    if ((int)blockIdx.x < n_bin_blocks)
        bin_block<Src, kBlock, R>(src, params, refl, n_mat, blockIdx.x);
    else
        uw_fwd_block<Table<UwDev>, kBlock>(usrc, wparams, blockIdx.x - n_bin_blocks, threadIdx.x);
}

// ---------------------------------------------------------------------------
// k_tile
// ---------------------------------------------------------------------------
// Additive term of Eq. (3)-(4) for the four bins b0..b0+3 (b0 % 4 == 0), which
// share one Philox call; rows/columns advance with the linear index.
struct AddCtx {
    float sigma_sa, inv_sigma_phi;
};

__device__ __forceinline__ float additive_term(const SonarDev &f, const AddCtx &c, int i, int j, uint32_t word,
                                               float &E_out, float &rho_out, float &R_out, float &phi_out) {
    const float R = range_ramp(f, i);
    const float phi = bin_azimuth(f, j);
    const float E = expf(-(phi * phi) * c.inv_sigma_phi);
    const float rho = rayleigh_of_word(word);
    E_out = E;
    rho_out = rho;
    R_out = R;
    phi_out = phi;
    return R * (1.0f + 0.5f * E * (c.sigma_sa * rho));
}

// Entry j of the fan's column table: {sin, cos} of column j's centre azimuth.
__device__ __forceinline__ void write_fan_column(const SonarDev &f, int j) {
    double sn, cs;
    sincos(((double)j + 0.5) * f.dphi - f.half_az, &sn, &cs);
    const gptr<double> cd = (gptr<double>)f.cols;
    cd[2 * j] = sn;
    cd[2 * j + 1] = cs;
}

// Consecutive polar tiles of a frame read neighbouring segments of every
// binning chunk, so the cache line at each segment boundary is shared by two
// tiles: the tile kernels give each XCD runs of this many consecutive tiles
// (read through one L2) instead of every eighth tile.
constexpr int kTileXcdRun = 8;
constexpr int kTileLoads = 8;      // pair gathers in flight per thread of a forward tile
constexpr int kPairBwdLoads = 4;   // ... of a pair backward tile (more would cost occupancy)

// Visits the pairs of polar tile `tile` of frame f: its segment in every
// binning chunk, for NT chunks at a time, flattened so that every thread
// takes pairs (independent loads) whatever the segment lengths, LOADS per
// thread per round (each pair's segment found from a coarse LDS map of the
// flat range, built with the prefix, and a short search of the prefix;
// indices past the end re-read the last pair and are not visited).
// seg_map: LDS of 2 NT entries.  fn(pair, range):
// WITH_R loads the pair's range from f.pair_r with the pair (else 0).  pre()
// runs once, after the first offset loads are issued and before they are
// used: independent arithmetic placed there overlaps their latency.
// Contains barriers.
template <int NT, int LOADS, bool WITH_R, class Fn, class Pre>
__device__ __forceinline__ void for_tile_pairs(const SonarDev &f, int tile, int *seg_end, int *seg_start, int *wtot,
                                               unsigned short *seg_map, Fn fn, Pre pre) {
    const int tid = threadIdx.x;
    const int stride = f.n_tiles + 1;
    for (int c0 = 0; c0 < f.n_chunks; c0 += NT) {
        const int c = c0 + tid;
        // the offsets of chunk c (clamped: a thread past the last chunk
        // re-reads the last one and takes an empty segment)
        const int cl = c < f.n_chunks ? c : f.n_chunks - 1;
        const gptr<const int> off = f.chunk_off + (long long)cl * stride + tile;
        const int o0 = off[0], o1 = off[1];
        if (c0 == 0) pre();
        const int s0 = o0, len = c < f.n_chunks ? o1 - o0 : 0;
        int total;
        const int incl = block_inclusive_scan1<NT>(len, wtot, total);
        seg_end[tid] = incl;
        seg_start[tid] = s0 - (incl - len);   // pair index = seg_start[c] + flat index
        // the coarse segment map of the flat range (shift: the same in every lane)
        const int shift = seg_map_shift(total, 2 * NT);
        seg_map_fill(seg_map, tid, incl - len, incl, total, shift);
        __syncthreads();
        for (int k0 = 0; k0 < total; k0 += NT * LOADS) {
            uint2 q[LOADS];
            float rv[LOADS];
#pragma unroll
            for (int u = 0; u < LOADS; ++u) {
                const int k = min(k0 + u * NT + tid, total - 1);
                const int cc = seg_find<NT>(seg_end, seg_map, shift, k);   // the segment holding k
                // below 2^31 (the frame's returns): chunk index and size are
                // below 2^24, so a 24-bit product gives the chunk's base
                const uint32_t idx = (uint32_t)__umul24((unsigned)(c0 + cc), (unsigned)f.chunk) +
                                     (uint32_t)(seg_start[cc] + k);
                q[u] = gload(f.pairs + idx);
                rv[u] = WITH_R ? f.pair_r[idx] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < LOADS; ++u)
                if (k0 + u * NT + tid < total) fn(q[u], rv[u]);
        }
        __syncthreads();
    }
    if (f.n_chunks <= 0) pre();
}

// Wave-level stream compaction: every wave walks its share of [0, n), queues
// the indices x with pred(x) in its own LDS queue (2 x 64 entries of type Q,
// which must hold n - 1) and runs work(x) 64 at a time, so the costly work of
// the sparse set keeps all lanes busy.  Call from every thread; no workgroup
// barrier inside.
template <int NT, class Q, class Pred, class Work>
__device__ __forceinline__ void wave_compact(int n, Q *queues, Pred pred, Work work) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    constexpr int NW = NT / kWave;
    const int per = ((n + NW - 1) / NW + kWave - 1) / kWave * kWave;
    const int lo = min(w * per, n), hi = min(lo + per, n);
    Q *qw = queues + w * 2 * kWave;
    int qn = 0;
    auto sync = [&]() __attribute__((always_inline)) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    for (int base = lo; base < hi; base += kWave) {
        const int x = base + lane;
        const bool p = x < hi && pred(x);
        const unsigned long long mask = __ballot(p);
        if (p) qw[qn + __popcll(mask & ((1ull << lane) - 1ull))] = x;   // qn < 64: within the queue
        qn += __popcll(mask);
        sync();
        if (qn >= kWave) {
            work(qw[lane]);
            const int t = qw[lane + kWave];   // the tail beyond the first 64 (read before it moves)
            sync();
            if (lane + kWave < qn) qw[lane] = t;
            qn -= kWave;
            sync();
        }
    }
    if (lane < qn) work(qw[lane]);
}

// Forward polar tile `bid` of the launch (NT threads).  COL_REGS: every
// frame's n_az divides 4 NT, so a thread's groups of four bins (4 NT bins
// apart) always fall on the same four columns, and their beam-pattern
// factors are kept in registers instead of an LDS column table (which the
// launch then does not reserve).
template <class Src, int NT, bool COL_REGS>
__device__ __forceinline__ void tile_fwd_block(const Src &src, const oceansim_sonar_params *params, const float *refl,
                                               int n_mat, int bid) {
    extern __shared__ int4 lds_raw[];
    constexpr int NW = NT / kWave;
    __shared__ unsigned short queues[NW * 2 * kWave];   // tile-local bins (< kMaxFwdTileBins)
    static_assert(NW * 2 * kWave >= 2 * NT, "the queues hold the pair walk's segment map");
    static_assert(kMaxFwdTileBins <= 65536, "queue entries are 16-bit");
    __shared__ float refl_s[kLaneHistMats];
    __shared__ int seg_end[NT], seg_start[NT], wtot[NW];
    int tile;
    const int fi = src.locate(bid, KTILE, tile);
    const SonarDev f = src.frame(fi);
    const int tid = threadIdx.x;
    const int nb = f.n_range * f.n_az;
    const int b_lo = tile * f.tile_bins;
    const int b_hi = min(b_lo + f.tile_bins, nb);
    const int nbins = b_hi - b_lo;
    float *acc = reinterpret_cast<float *>(lds_raw);               // [tile_bins]
    float *etab = acc + f.tile_bins;                               // [n_az]: beam pattern of Eq. 3 per column
    const bool speckle = f.speckle != SPECKLE_OFF;
    const bool matp = f.matp != 0;
    const oceansim_sonar_params pr = params[f.param_row];
    const AddCtx ctx{pr.sigma_sa, 1.0f / pr.sigma_phi};
    const int q_first = b_lo >> 2, q_last = (b_hi - 1) >> 2;
    // the column factor exp(-phi_j^2 / sigma_phi): once per column of the
    // tile's rows in LDS, or for the thread's own four columns in registers
    float ereg[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (speckle) {
        if (COL_REGS) {
            // n_az divides 4 NT, a power of two: the column of bin b is b & (n_az - 1)
            const int am = f.n_az - 1;
            const int j0 = ((q_first + tid) << 2) & am;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const float phi = bin_azimuth(f, (j0 + w) & am);
                ereg[w] = expf(-(phi * phi) * ctx.inv_sigma_phi);
            }
        } else {
            for (int j = tid; j < f.n_az; j += NT) {
                const float phi = bin_azimuth(f, j);
                etab[j] = expf(-(phi * phi) * ctx.inv_sigma_phi);
            }
        }
    }
    // material pairs carry cos x attenuation: the reflectivity is applied here
    if (matp)
        for (int k = tid; k < n_mat; k += NT) refl_s[k] = refl[k];

    // side job for the fan launch that follows: {sin, cos} of the column-centre azimuths
    if (f.cols)
        for (int j = tile * NT + tid; j < f.n_az; j += f.n_tiles * NT) write_fan_column(f, j);
    // the histogram starts 16-byte aligned: 16-byte stores while nbins is a
    // multiple of four (acc is followed by the column table)
    if ((nbins & 3) == 0)
        for (int k = 4 * tid; k < nbins; k += 4 * NT) *reinterpret_cast<float4 *>(acc + k) = make_float4(0.f, 0.f, 0.f, 0.f);
    else
        for (int k = tid; k < nbins; k += NT) acc[k] = 0.0f;
    __syncthreads();

    // additive term of Eq. (3)-(4) for the group of four consecutive
    // frame-linear bins starting at 4q (one Philox call)
    const bool row_groups = COL_REGS && f.n_az >= 4;   // a group lies in one row, whose index is b >> az_shift
    const int az_shift = __builtin_ctz((unsigned)f.n_az);
    auto additive_group = [&](int q, float (&add)[4]) __attribute__((always_inline)) {
        const int b0 = q << 2;
        const Words wd = philox((uint32_t)q, f.frame_id, 0u, 0u, f.seed_lo, f.seed_hi);
        if (row_groups) {
            const float R = range_ramp(f, b0 >> az_shift);
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const float rho = rayleigh_of_word(pick(wd, (uint32_t)w));
                add[w] = R * (1.0f + 0.5f * ereg[w] * (ctx.sigma_sa * rho));
            }
            return;
        }
        int i = b0 / f.n_az;
        int j = b0 - i * f.n_az;
        float R = range_ramp(f, i);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            // R_i (1 + 0.5 E_j sigma_sa rho)
            const float rho = rayleigh_of_word(pick(wd, (uint32_t)w));
            add[w] = R * (1.0f + 0.5f * (COL_REGS ? ereg[w] : etab[j]) * (ctx.sigma_sa * rho));
            if (++j == f.n_az) {
                j = 0;
                R = range_ramp(f, ++i);
            }
        }
    };

    // binning by summation of the tile's pairs (and, for a pair backward, the
    // largest |cos x attenuation| among them)
    float cemax = 0.0f;
    for_tile_pairs<NT, kTileLoads, false>(
        f, tile, seg_end, seg_start, wtot, queues,   // the queues serve as the segment map until the compaction
        [&](uint2 q, float) __attribute__((always_inline)) {
            const uint32_t lb = matp ? (q.x & 0xffffu) : q.x;
            if (lb >= (uint32_t)nbins) return;
            const float I = matp ? refl_s[q.x >> 16] * __uint_as_float(q.y) : __uint_as_float(q.y);
            cemax = fmaxf(cemax, __builtin_fabsf(__uint_as_float(q.y)));
            atomicAdd(&acc[lb], I);
        },
        []() {});
    if (f.tile_cemax) {
        __shared__ unsigned s_cemax;
        if (tid == 0) s_cemax = 0u;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) cemax = fmaxf(cemax, __shfl_down(cemax, off, kWave));
        __syncthreads();
        if ((tid & (kWave - 1)) == 0) atomicMax(&s_cemax, __float_as_uint(cemax));   // non-negative: ordered as bits
        __syncthreads();
        if (tid == 0) f.tile_cemax[tile] = __uint_as_float(s_cemax);
    }

    float G = pr.gain;
    if (f.saved_p)   // the binned sums P, for the backward of a range-normalised frame
        for (int k = tid; k < nbins; k += NT) f.saved_p[b_lo + k] = acc[k];
    if (f.range_norm) {
        // range-wise normalisation: each row of Q = G P over its maximum when
        // that is positive (the maximum over the positive entries: NaN and
        // non-positive values do not count), else the row as it is; acc then
        // holds the normalised Q, so the gain below is 1
        unsigned *rmax = reinterpret_cast<unsigned *>(COL_REGS ? etab : etab + f.n_az);   // [rows of the tile]
        const int rows = nbins / f.n_az;
        for (int r = tid; r < rows; r += NT) rmax[r] = 0u;
        __syncthreads();
        for (int k = tid; k < nbins; k += NT) {
            const float q = G * acc[k];
            if (q > 0.0f) atomicMax(&rmax[k / f.n_az], __float_as_uint(q));   // positive floats order as their bits
        }
        __syncthreads();
        for (int k = tid; k < nbins; k += NT) {
            const float m = __uint_as_float(rmax[k / f.n_az]);
            const float q = G * acc[k];
            acc[k] = m > 0.0f ? q / m : q;
        }
        __syncthreads();
        G = 1.0f;
    }
    if (speckle) {
        // Q m for the nonzero bins only (the others have Q m = 0 whatever m),
        // compacted per wave so that the draws keep the lanes busy
        wave_compact<NT>(
            nbins, queues, [&](int x) __attribute__((always_inline)) { return acc[x] != 0.0f; },
            [&](int x) __attribute__((always_inline)) {
                float gz;
                const float m = speckle_factor(f, (uint32_t)(b_lo + x), pr.sigma_sm, &gz);
                acc[x] = (G * acc[x]) * m;
            });
        __syncthreads();
    }

    // out = Q m + additive term (speckle) or G P, groups of four bins, float4 stores
    const bool acc_aligned = (b_lo & 3) == 0;   // a group's four bins are one 16-byte LDS load
    auto store_group = [&](int q, const float (&add)[4]) __attribute__((always_inline)) {
        const int b0 = q << 2;
        float out[4];
        bool in[4];
        const bool full = b0 >= b_lo && b0 + 3 < b_hi;
        float a[4];
        if (full && acc_aligned) {
            const float4 v = *reinterpret_cast<const float4 *>(acc + (b0 - b_lo));
            a[0] = v.x;
            a[1] = v.y;
            a[2] = v.z;
            a[3] = v.w;
        }
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            in[w] = full || (b0 + w >= b_lo && b0 + w < b_hi);
            if (!(full && acc_aligned)) a[w] = in[w] ? acc[b0 + w - b_lo] : 0.0f;
            out[w] = speckle ? a[w] + add[w] : G * a[w];
        }
        if (in[0] && in[3]) {
            gstore((gptr<float4>)(f.polar + b0), make_float4(out[0], out[1], out[2], out[3]));
        } else {
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (in[w]) f.polar[b0 + w] = out[w];
        }
    };
    for (int q = q_first + tid; q <= q_last; q += NT) {
        float add[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (speckle) additive_group(q, add);
        store_group(q, add);
    }
}

template <class Src, int NT, bool COL_REGS>
__global__ __launch_bounds__(NT) void k_tile(Src src, const oceansim_sonar_params *params, const float *refl,
                                             int n_mat) {
    tile_fwd_block<Src, NT, COL_REGS>(src, params, refl, n_mat, xcd_grouped_id<kTileXcdRun>(blockIdx.x, gridDim.x));
}

// k_tile_uw (plans with camera frames and wide tiles): the forward tiles and
// the camera forward in one launch.  The tiles are bound by their VALU work
// (speckle draws), the camera by HBM; apart, each leaves the other's unit
// idle, and two streams do not overlap them (the first launch fills the chip).
// The camera workgroups are spread evenly through the dispatch order
// (workgroup x is a camera one when floor((x+1) C / N) > floor(x C / N), C of
// N in all), so every CU holds both kinds while both last.  A camera
// workgroup runs two camera blocks of kBlock threads side by side.
template <class Src, bool COL_REGS>
__global__ __launch_bounds__(kWideThreads) void k_tile_uw(Src src, const oceansim_sonar_params *params,
                                                          const float *refl, int n_mat, int n_tile_blocks,
                                                          int n_cam_groups, Table<UwDev> usrc,
                                                          const oceansim_water_params *wparams, int n_cam_blocks) {
    static_assert(kWideThreads == 2 * kBlock, "two camera blocks per wide workgroup");
    const FusedSlot slot = fused_slot(xcd_grouped_id<kTileXcdRun>(blockIdx.x, gridDim.x), n_tile_blocks, n_cam_groups);
    if (slot.cam) {
        // the same in every lane of a wave: scalar, so the camera frame's
        // fields load into scalar registers
        const int cb = __builtin_amdgcn_readfirstlane(2 * slot.index + (int)(threadIdx.x >= kBlock));
        if (cb < n_cam_blocks) uw_fwd_block<Table<UwDev>, kBlock>(usrc, wparams, cb, threadIdx.x & (kBlock - 1));
    } else {
        tile_fwd_block<Src, kWideThreads, COL_REGS>(src, params, refl, n_mat, slot.index);
    }
}

// ---------------------------------------------------------------------------
// k_fan: pixel u (left half, x <= 0) and its mirror W-1-u share rho and |phi|.
// ---------------------------------------------------------------------------
// Load of polar-image element `idx` through a 32-bit byte offset from the
// uniform image base (a polar image has at most 2^24 bins).
__device__ __forceinline__ float polar_at(gptr<const float> base, int idx) {
    return *(gptr<const float>)((gptr<const char>)base + (uint32_t)idx * 4u);
}

// Elements idx and idx + 1 of a polar image (same row) in one load: a pair of
// floats whose address is 4-byte aligned.
typedef float f32x2_a4_t __attribute__((ext_vector_type(2), aligned(4)));
__device__ __forceinline__ float2 polar_pair_at(gptr<const float> base, int idx) {
    const f32x2_a4_t v = *(gptr<const f32x2_a4_t>)((gptr<const char>)base + (uint32_t)idx * 4u);
    return make_float2(v.x, v.y);
}

// IMAGE = false: the stencil records alone (geometry only; the polar image is
// not read and the fan is not written).
template <class Src, bool IMAGE = true>
__global__ __launch_bounds__(kBlock) void k_fan(Src src) {
    int local;
    const int fi = src.locate(xcd_grouped_id<16>(blockIdx.x, gridDim.x), KFAN, local);
    const SonarDev f = src.frame(fi);
    // a workgroup covers kFanTileU pixel pairs x kFanTileV rows; each wave an 8 x 8 patch
    // of pairs per load instruction (rows 8 apart across a thread's kFanRows),
    // so the gathers of one instruction stay within a few polar rows
    const int n_groups = (f.fan_h + kFanTileV - 1) / kFanTileV;
    const int col = local / n_groups;            // vertically adjacent tiles are consecutive
    const int g = local - col * n_groups;
    const int lane = threadIdx.x & (kWave - 1);
    const int u = col * kFanTileU + (threadIdx.x / kWave) * 8 + (lane & 7);
    if (u >= f.half_w) return;
    const int v0 = g * kFanTileV + (lane >> 3);
    const gptr<const float> __restrict__ polar = f.polar;
    const gptr<float> __restrict__ fan = f.fan;
    const int um = f.fan_w - 1 - u;
    {
        // A tile wholly outside the sector (nearest corner beyond r_max,
        // farthest within r_min, or every pixel beyond the edge azimuth, with
        // a relative margin far above rounding so that no pixel's own test
        // could pass) only writes its zeros: the same outputs, without the
        // geometry or the column-table loads.
        const int u_lo = col * kFanTileU, u_hi = min(u_lo + kFanTileU, f.half_w) - 1;
        const int v_lo = g * kFanTileV, v_hi = min(v_lo + kFanTileV, f.fan_h) - 1;
        const double ax_min = (0.5 * (double)f.fan_w - (double)u_hi - 0.5) * f.fan_s;
        const double ax_max = (0.5 * (double)f.fan_w - (double)u_lo - 0.5) * f.fan_s;
        const double yc_min = ((double)f.fan_h - (double)v_hi - 0.5) * f.fan_s;
        const double yc_max = ((double)f.fan_h - (double)v_lo - 0.5) * f.fan_s;
        const double near2 = ax_min * ax_min + yc_min * yc_min, far2 = ax_max * ax_max + yc_max * yc_max;
        const double edge_l = ax_min * f.cos_half_az, edge_r = yc_max * f.sin_half_az;
        const bool outside = near2 > f.r_max * f.r_max * (1.0 + 1e-9) || far2 < f.r_min * f.r_min * (1.0 - 1e-9) ||
                             edge_l - edge_r > 1e-9 * (edge_l + edge_r);
        if (outside) {
            gptr<float> row = fan + (long long)v0 * f.fan_w;
            gptr<int4> rec = f.stencil ? f.stencil + (long long)v0 * f.half_w + u : nullptr;
#pragma unroll
            for (int r = 0; r < kFanRows; ++r) {
                if (v0 + 8 * r < f.fan_h) {
                    if (IMAGE) {
                        row[u] = 0.0f;
                        if (um != u) row[um] = 0.0f;
                    }
                    if (rec) gstore(rec, make_int4(-1, 0, 0, 0));
                }
                row += 8LL * f.fan_w;
                if (rec) rec += 8LL * f.half_w;
            }
            return;
        }
    }
    // left-half pixel (v, u) and its mirror W-1-u: exact offsets from the apex
    const double ax = (0.5 * (double)f.fan_w - (double)u - 0.5) * f.fan_s;   // = -x_c >= 0
    const double ax2 = ax * ax;
    const int row1 = f.n_range > 1 ? f.n_az : 0;
    const int col1 = f.n_az > 1 ? 1 : 0;
    const int mirror = f.n_az > 1 ? f.n_az - 2 : 0;
    // geometry of every row first, then all gathers, then the blends: the
    // loads of the rows are in flight together.  The mirror pixel's stencil
    // is the left one's reflected: first column N_phi - 2 - j0, weights swapped.
    int i0[kFanRows], jL[kFanRows], jn[kFanRows];
    float ct[kFanRows], cL[kFanRows];
    double yc[kFanRows], rho2[kFanRows], sn[kFanRows], cn[kFanRows];
    bool in[kFanRows];
    const gptr<const double> cols = (gptr<const double>)f.cols;   // {sin, cos} per column
#pragma unroll
    for (int r = 0; r < kFanRows; ++r) {
        yc[r] = ((double)f.fan_h - (double)(v0 + 8 * r) - 0.5) * f.fan_s;
        rho2[r] = __builtin_fma(yc[r], yc[r], ax2);
        in[r] = v0 + 8 * r < f.fan_h && fan_inside(f, ax, yc[r], rho2[r]);
        // the column-table loads of all rows in flight together (the index is
        // clamped to the table, so they need no guard)
        jn[r] = f.n_az > 1 ? fan_column_guess(f, ax, yc[r]) : 0;
        sn[r] = cols[2 * jn[r]];
        cn[r] = cols[2 * jn[r] + 1];
    }
#pragma unroll
    for (int r = 0; r < kFanRows; ++r) {
        i0[r] = jL[r] = 0;
        ct[r] = cL[r] = 0.0f;
        if (in[r]) {   // waves wholly outside the sector skip the stencil
            fan_radial_fast(f, rho2[r], i0[r], ct[r]);
            const float e = f.n_az > 1 ? fan_column_offset(f, ax, yc[r], sn[r], cn[r]) : 0.0f;
            axis_from_offset(jn[r], e, f.n_az, jL[r], cL[r]);
        }
    }
    float a[kFanRows][8];
#pragma unroll
    for (int r = 0; r < kFanRows; ++r) {
        const int b0 = (int)__umul24((unsigned)i0[r], (unsigned)f.n_az), b1 = b0 + row1;   // < 2^24 bins
        const int jr = mirror - jL[r];
        if (!IMAGE || !in[r]) {
#pragma unroll
            for (int k = 0; k < 8; ++k) a[r][k] = 0.0f;
            continue;
        }
        if (col1) {
            // the two columns of each row are adjacent: one load per row and pixel
            const float2 p0 = polar_pair_at(polar, b0 + jL[r]), p1 = polar_pair_at(polar, b1 + jL[r]);
            const float2 p2 = polar_pair_at(polar, b0 + jr), p3 = polar_pair_at(polar, b1 + jr);
            a[r][0] = p0.x;
            a[r][1] = p0.y;
            a[r][2] = p1.x;
            a[r][3] = p1.y;
            a[r][4] = p2.x;
            a[r][5] = p2.y;
            a[r][6] = p3.x;
            a[r][7] = p3.y;
        } else {
            a[r][0] = a[r][1] = polar_at(polar, b0 + jL[r]);
            a[r][2] = a[r][3] = polar_at(polar, b1 + jL[r]);
            a[r][4] = a[r][5] = polar_at(polar, b0 + jr);
            a[r][6] = a[r][7] = polar_at(polar, b1 + jr);
        }
    }
    gptr<float> row = fan + (long long)v0 * f.fan_w;
    gptr<int4> rec = f.stencil ? f.stencil + (long long)v0 * f.half_w + u : nullptr;
    const long long row_step = 8LL * f.fan_w, rec_step = 8LL * f.half_w;
#pragma unroll
    for (int r = 0; r < kFanRows; ++r) {
        if (v0 + 8 * r < f.fan_h) {
            float t, t1, s, s1;
            decode_weight(ct[r], t, t1);
            decode_weight(cL[r], s, s1);
            const float left = t1 * (s1 * a[r][0] + s * a[r][1]) + t * (s1 * a[r][2] + s * a[r][3]);
            const float right = t1 * (s * a[r][4] + s1 * a[r][5]) + t * (s * a[r][6] + s1 * a[r][7]);
            if (IMAGE) {
                row[u] = in[r] ? left : 0.0f;
                if (um != u) row[um] = in[r] ? right : 0.0f;
            }
            if (rec)
                gstore(rec, in[r] ? make_int4(i0[r], jL[r], __float_as_int(ct[r]), __float_as_int(cL[r]))
                                  : make_int4(-1, 0, 0, 0));
        }
        row += row_step;
        if (rec) rec += rec_step;
    }
}

// ---------------------------------------------------------------------------
// k_tile_bwd
// ---------------------------------------------------------------------------
constexpr int kRowBatch = 1024;

// Relative margin of the candidate bounds: far above FP64 rounding (1e-16)
// and far below a pixel, so every pixel whose computed stencil can touch
// the tile is enumerated and almost no other.
constexpr double kCandEps = 1e-7;

// Left-half pixel interval [ua, ub] of fan row v whose centres lie within
// radial distance [rlo, rhi] of the apex and inside the sector; the exact
// stencil test decides membership.
__device__ __forceinline__ void row_interval(const SonarDev &f, int v, double rlo, double rhi, double inv_s,
                                             int &ua, int &ub) {
    const double s = f.fan_s;
    const double y = ((double)f.fan_h - (double)v - 0.5) * s;
    ua = 1;
    ub = 0;
    if (y > rhi) return;
    double xo = __builtin_sqrt(rhi * rhi - y * y);
    if (f.half_az < 1.5707963267948966) {
        const double xs = y * f.tan_half_az * (1.0 + kCandEps) + kCandEps * s;
        xo = xo < xs ? xo : xs;
    }
    const double xi = rlo > y ? __builtin_sqrt(rlo * rlo - y * y) : 0.0;
    if (xi > xo) return;
    // left half: x in [-xo, -xi]  ->  u = x / s + W/2 - 1/2
    const double c = 0.5 * (double)f.fan_w - 0.5;
    const double a = -xo * inv_s + c, b = -xi * inv_s + c;
    int lo = (int)__builtin_ceil(a - 1e-6), hi = (int)__builtin_floor(b + 1e-6);
    lo = lo < 0 ? 0 : lo;
    hi = hi > f.half_w - 1 ? f.half_w - 1 : hi;
    ua = lo;
    ub = hi;
}

// Candidate pixels of a tile, one batch of fan rows at a time: per-row
// intervals and their exclusive prefix in LDS (kRowBatch / NT rows per
// thread, one workgroup scan).  Returns the batch total.
template <int NT>
__device__ __forceinline__ int load_row_batch(const SonarDev &f, int vb, int nrows, double rlo, double rhi,
                                              double inv_s, int *row_u0, int *row_pre, int *wtot) {
    constexpr int RPT = kRowBatch / NT;
    __syncthreads();
    int cnt[RPT];
    int sum = 0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int rr = threadIdx.x * RPT + q;
        cnt[q] = 0;
        if (rr < nrows) {
            int ua, ub;
            row_interval(f, vb + rr, rlo, rhi, inv_s, ua, ub);
            row_u0[rr] = ua;
            cnt[q] = ub >= ua ? ub - ua + 1 : 0;
        }
        sum += cnt[q];
    }
    int total;
    int run = block_inclusive_scan1<NT>(sum, wtot, total) - sum;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int rr = threadIdx.x * RPT + q;
        if (rr < nrows) row_pre[rr] = run;
        run += cnt[q];
    }
    if (threadIdx.x == 0) row_pre[nrows] = total;
    __syncthreads();
    return total;
}

// Row of candidate k within a batch: the last r with row_pre[r] <= k.
__device__ __forceinline__ int row_of(const int *row_pre, int nrows, int k) {
    int lo = 0, hi = nrows - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_pre[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}


// Round x (|x| < 2^51) to the nearest integer, as an int64, by adding
// 1.5 * 2^52: the sum's mantissa then holds the integer offset by 2^51.
__device__ __forceinline__ long long round_to_ll(double x) {
    const double t = x + 6755399441055744.0;
    return (long long)__double_as_longlong(t) - 0x4338000000000000LL;
}

// SAVED: every frame of the launch carries the stencils saved by its forward
// pass (the geometry is not recomputed); otherwise frames may mix both kinds.
// Backward polar tile `bid` of the n_blocks tiles of the launch (kBwdThreads
// threads).
template <class Src, bool SAVED>
__device__ __forceinline__ void tile_bwd_block(const Src &src, const oceansim_sonar_params *params, double *part,
                                               int n_slots, float *grad_refl_zero, int n_mat_zero, int bid,
                                               int n_blocks) {
    constexpr int NT = kBwdThreads;
    extern __shared__ int4 lds_raw[];
    long long *acc = reinterpret_cast<long long *>(lds_raw);
    __shared__ int row_u0[kRowBatch];
    __shared__ int row_pre[kRowBatch + 1];
    __shared__ int wtot[NT / kWave];
    __shared__ unsigned poison[kMaxTileBins / 32];
    __shared__ double red[NT / kWave];
    __shared__ int sh_exp;        // fixed-point exponent: values are stored times 2^(50 - sh_exp)
    __shared__ int sh_shift;

    int local;
    const int lid = xcd_grouped_id<8>(bid, n_blocks);   // also this tile's partial-sum slot
    const int fi = src.locate(lid, KTILEB, local);
    const SonarDev f = src.frame(fi);
    const int tile = f.n_tiles_b - 1 - local;   // outer tiles (most pixels) first
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave;

    // the atomic reflectivity path (many materials) accumulates into a zeroed table
    if (grad_refl_zero)
        for (int k = bid * NT + tid; k < n_mat_zero; k += n_blocks * NT) grad_refl_zero[k] = 0.0f;

    const int nb = f.n_range * f.n_az;
    const int b_lo = tile * f.tile_bins_b;
    const int b_hi = min(b_lo + f.tile_bins_b, nb);
    const int nbins = b_hi - b_lo;
    const int ia = tile * f.rows_per_tile_b;
    const int ib = min(ia + f.rows_per_tile_b, f.n_range);

    for (int k = tid; k < nbins; k += NT) acc[k] = 0;
    for (int k = tid; k < (nbins + 31) / 32; k += NT) poison[k] = 0u;
    if (tid == 0) sh_exp = -100000;
    __syncthreads();

    const bool have_fan = f.grad_fan != nullptr && f.fan_h > 0 && f.fan_w > 0;
    if (have_fan) {
        const double s = f.fan_s;
        // pixels whose stencil touches rows [ia, ib) lie at radial distance
        // [r_min + (ia - 1/2) dr, r_min + (ib + 1/2) dr) within [r_min, r_max]
        double rlo = f.r_min + ((double)ia - 0.5) * f.dr;
        double rhi = f.r_min + ((double)ib + 0.5) * f.dr;
        rlo = (rlo < f.r_min ? f.r_min : rlo) * (1.0 - kCandEps);
        rhi = (rhi > f.r_max ? f.r_max : rhi) * (1.0 + kCandEps);
        const double rlo2 = rlo * rlo, rhi2 = rhi * rhi;
        const double cmin = cos(f.half_az < 1.5707963267948966 ? f.half_az : 1.5707963267948966);
        const double ymin = rlo * cmin - s, ymax = rhi + s;
        const double H = (double)f.fan_h;
        int v_lo = (int)__builtin_floor(H - 0.5 - ymax / s);
        int v_hi = (int)__builtin_ceil(H - 0.5 - (ymin > 0.0 ? ymin : 0.0) / s);
        v_lo = v_lo < 0 ? 0 : v_lo;
        v_hi = v_hi > f.fan_h - 1 ? f.fan_h - 1 : v_hi;
        const int W = f.fan_w;
        // Pixels that can add to one bin lie in its 2 x 2-cell neighbourhood:
        // radial extent <= 2 dr, angular <= 2 dphi at radius <= rhi.  Their
        // count bounds |bin sum| / max|g|; with a safety factor of 2 it keeps
        // every scaled sum below 2^50.
        const double wr = 2.0 * f.dr, wa = 2.0 * f.dphi * rhi;
        const double pix_bound = 2.0 * ((wr * wa + 1.5 * s * 2.0 * (wr + wa)) / (s * s) + 8.0) + 16.0;

        const double inv_s = 1.0 / s;
        for (int vb = v_lo; vb <= v_hi; vb += kRowBatch) {
            const int nrows = min(kRowBatch, v_hi - vb + 1);
            const int total = load_row_batch<NT>(f, vb, nrows, rlo, rhi, inv_s, row_u0, row_pre, wtot);
            // Rounds of U candidates per thread: the gradient pair (and the saved
            // stencil) of every candidate is loaded once, into registers; the
            // round's largest finite |gradient| sets the fixed-point scale
            // (what is accumulated is rescaled by an arithmetic shift when it
            // grows); then the contributions go to LDS from the registers.
            constexpr int U = SAVED ? 4 : 1;
            for (int k0 = 0; k0 < total; k0 += U * NT) {
                float G0[U], G1[U];
                int4 REC[U];
                int UU[U], VV[U];
                float mxf = 0.0f;
#pragma unroll
                for (int q = 0; q < U; ++q) {
                    const int k = k0 + q * NT + tid;
                    G0[q] = G1[q] = 0.0f;
                    REC[q] = make_int4(-1, 0, 0, 0);
                    UU[q] = -1;
                    VV[q] = 0;
                    if (k < total) {
                        const int r = row_of(row_pre, nrows, k);
                        const int v = vb + r;
                        const int u = row_u0[r] + (k - row_pre[r]);
                        const gptr<const float> grow = f.grad_fan + (long long)v * W;
                        UU[q] = u;
                        VV[q] = v;
                        G0[q] = grow[u];
                        G1[q] = (W - 1 - u) != u ? grow[W - 1 - u] : 0.0f;
                        if (SAVED || f.stencil) REC[q] = gload(f.stencil + ((long long)v * f.half_w + u));
                    }
                }
#pragma unroll
                for (int q = 0; q < U; ++q) {
                    const float a0 = __builtin_fabsf(G0[q]), a1 = __builtin_fabsf(G1[q]);
                    if (a0 <= 3.4028235e38f && a0 > mxf) mxf = a0;
                    if (a1 <= 3.4028235e38f && a1 > mxf) mxf = a1;
                }
                double mx = (double)mxf;
                for (int off = 32; off > 0; off >>= 1) {
                    const double o = __shfl_down(mx, off, kWave);
                    mx = o > mx ? o : mx;
                }
                if (lane == 0) red[wave] = mx;
                __syncthreads();
                if (tid == 0) {
                    double m = 0.0;
                    for (int k = 0; k < NT / kWave; ++k) m = red[k] > m ? red[k] : m;
                    int e = sh_exp;
                    int shift = 0;
                    if (m > 0.0) {
                        int en;
                        frexp(m * pix_bound, &en);   // m * bound < 2^en
                        if (en > e) {
                            shift = e == -100000 ? 0 : en - e;
                            e = en;
                        }
                    }
                    sh_shift = shift > 63 ? 63 : shift;   // 63: all accumulated so far rounds away
                    sh_exp = e;
                }
                __syncthreads();
                if (sh_shift > 0) {
                    // rescale what is accumulated to the larger exponent (an
                    // arithmetic shift: deterministic)
                    const int sh = sh_shift;
                    for (int k = tid; k < nbins; k += NT) acc[k] = sh >= 63 ? 0 : (acc[k] >> sh);
                    __syncthreads();
                }
                // no nonzero finite value yet: only non-finite ones (poison) can act
                const double scale = sh_exp == -100000 ? 0.0 : ldexp(1.0, 50 - sh_exp);
#pragma unroll
                for (int q = 0; q < U; ++q) {
                    const int u = UU[q];
                    const int um = W - 1 - u;
                    const float g0 = G0[q], g1 = G1[q];
                    if (u < 0 || (g0 == 0.0f && g1 == 0.0f)) continue;
                    if (SAVED || f.stencil) {
                        // stencil saved by the forward pass
                        const int4 rec = REC[q];
                        const int i0 = rec.x;
                        if (i0 < 0) continue;
                        const int i1 = f.n_range == 1 ? i0 : i0 + 1;
                        if (i1 < ia || i0 >= ib) continue;
                        float t, omt;
                        decode_weight(__int_as_float(rec.z), t, omt);
                        const float es = __int_as_float(rec.w);
                        for (int side = 0; side < 2; ++side) {
                            if (side == 1 && um == u) break;
                            const float g = side == 0 ? g0 : g1;
                            if (g == 0.0f) continue;
                            const bool one_col = f.n_az == 1;
                            const int j0 = side == 0 || one_col ? rec.y : f.n_az - 2 - rec.y;
                            const int j1 = one_col ? j0 : j0 + 1;
                            float sw, omsw;
                            decode_weight(side == 0 || one_col ? es : -es, sw, omsw);
                            const bool finite = __builtin_isfinite(g);
                            const double gd = (double)g * scale;
                            const double wr0 = (double)omt * gd, wr1 = (double)t * gd;
#pragma unroll
                            for (int a = 0; a < 2; ++a) {
                                const int ii = a == 0 ? i0 : i1;
                                if (ii < ia || ii >= ib || (a == 1 && i1 == i0)) continue;
                                const double wa_ = a == 0 ? wr0 : wr1;
#pragma unroll
                                for (int c = 0; c < 2; ++c) {
                                    if (c == 1 && one_col) continue;
                                    const int lb = (ii - ia) * f.n_az + (c == 0 ? j0 : j1);
                                    if (!finite) {
                                        atomicOr(&poison[lb >> 5], 1u << (lb & 31));
                                        continue;
                                    }
                                    const long long qv = round_to_ll(wa_ * (double)(c == 0 ? omsw : sw));
                                    if (qv != 0)
                                        atomicAdd(reinterpret_cast<unsigned long long *>(&acc[lb]),
                                                  (unsigned long long)qv);
                                }
                            }
                        }
                    } else if (!SAVED) {
                        // geometry recomputed in FP64
                        const int v = VV[q];
                        const double ax = (0.5 * (double)W - (double)u - 0.5) * s;
                        const double yc = (H - (double)v - 0.5) * s;
                        const double rho2 = ax * ax + yc * yc;
                        if (rho2 < rlo2 || rho2 > rhi2) continue;
                        Stencil st;
                        if (!fan_radial(f, __builtin_sqrt(rho2), st)) continue;
                        if (st.i1 < ia || st.i0 >= ib) continue;
                        const double phi = atan2(ax, yc);
                        for (int side = 0; side < 2; ++side) {
                            if (side == 1 && um == u) break;
                            const float g = side == 0 ? g0 : g1;
                            if (g == 0.0f) continue;
                            if (!fan_angular(f, side == 0 ? phi : -phi, st)) continue;
                            const bool finite = __builtin_isfinite(g);
                            const double gd = (double)g * scale;
                            const double wr0 = (1.0 - st.t) * gd, wr1 = st.t * gd;
                            const double wc0 = 1.0 - st.s, wc1 = st.s;
                            const bool two_rows = st.i1 != st.i0, two_cols = st.j1 != st.j0;
#pragma unroll
                            for (int a = 0; a < 2; ++a) {
                                const int ii = a == 0 ? st.i0 : st.i1;
                                if (ii < ia || ii >= ib || (a == 1 && !two_rows)) continue;
                                const double wa_ = a == 0 ? wr0 : wr1;
#pragma unroll
                                for (int c = 0; c < 2; ++c) {
                                    if (c == 1 && !two_cols) continue;
                                    const int lb = (ii - ia) * f.n_az + (c == 0 ? st.j0 : st.j1);
                                    if (!finite) {
                                        atomicOr(&poison[lb >> 5], 1u << (lb & 31));
                                        continue;
                                    }
                                    const long long qv = round_to_ll(wa_ * (c == 0 ? wc0 : wc1));
                                    if (qv != 0)
                                        atomicAdd(reinterpret_cast<unsigned long long *>(&acc[lb]),
                                                  (unsigned long long)qv);
                                }
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
    }

    // epilogue: fixed point -> float, plus the polar gradient; adjoint of Eq. (3)-(4)
    const oceansim_sonar_params pr = params[f.param_row];
    const double inv_scale = (have_fan && sh_exp != -100000) ? ldexp(1.0, sh_exp - 50) : 0.0;
    const AddCtx ctx{pr.sigma_sa, 1.0f / pr.sigma_phi};
    const double dsphi = 0.5 * (double)pr.sigma_sa / ((double)pr.sigma_phi * (double)pr.sigma_phi);
    double g_sphi = 0.0, g_ssa = 0.0;
    const int q_first = b_lo >> 2, q_last = (b_hi - 1) >> 2;
    for (int q = q_first + tid; q <= q_last; q += NT) {
        const int b0 = q << 2;
        Words wd{0u, 0u, 0u, 0u};
        if (f.speckle != SPECKLE_OFF) wd = philox((uint32_t)q, f.frame_id, 0u, 0u, f.seed_lo, f.seed_hi);
        int i = b0 / f.n_az;
        int j = b0 - i * f.n_az;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int b = b0 + w;
            if (b >= b_lo && b < b_hi) {
                const int lb = b - b_lo;
                double g = (double)acc[lb] * inv_scale;
                if (poison[lb >> 5] & (1u << (lb & 31))) g = __builtin_nan("");
                if (f.grad_polar) g += (double)f.grad_polar[b];
                f.grad_img[b] = (float)g;
                if (f.speckle != SPECKLE_OFF) {
                    float E, rho, R, phi;
                    additive_term(f, ctx, i, j, pick(wd, (uint32_t)w), E, rho, R, phi);
                    // d add / d sigma_sa and d add / d sigma_phi of Eq. (3)-(4)
                    const double t = g * (double)R * (double)E * (double)rho;
                    g_ssa += 0.5 * t;
                    g_sphi += t * dsphi * ((double)phi * (double)phi);
                }
            }
            if (++j == f.n_az) { j = 0; ++i; }
        }
    }
    __shared__ double red2[2 * (NT / kWave)];
    const double sums[2] = {g_sphi, g_ssa};
    const double tot = block_sum_n<2, NT>(sums, red2);   // thread 0: sigma_phi, thread 1: sigma_sa
    // partial sums column-major: part[c * n_slots + slot], then the slots' rows
    if (tid == 0) {
        reinterpret_cast<int *>(part + 5LL * n_slots)[lid] = f.param_row;
        part[0LL * n_slots + lid] = 0.0;
        part[1LL * n_slots + lid] = 0.0;
        part[2LL * n_slots + lid] = tot;
        part[4LL * n_slots + lid] = 0.0;
    }
    if (tid == 1) part[3LL * n_slots + lid] = tot;
}

// Saved stencils need fewer registers: three workgroups per CU (six waves per
// SIMD); the recomputing variant keeps four waves per SIMD.
template <class Src, bool SAVED>
__global__ __launch_bounds__(kBwdThreads, SAVED ? 6 : 4) void k_tile_bwd(Src src, const oceansim_sonar_params *params,
                                                          double *part, int n_slots, float *grad_refl_zero,
                                                          int n_mat_zero) {
    tile_bwd_block<Src, SAVED>(src, params, part, n_slots, grad_refl_zero, n_mat_zero, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// k_ret_bwd
// ---------------------------------------------------------------------------
// Return chunk `bid` of the n_blocks chunks of the launch.
//
// Small reflectivity tables (n_mat <= kLaneHistMats) are reduced per
// workgroup in LDS without thread-private columns: each material's
// contributions are added as 64-bit fixed point, scaled from that
// material's own largest magnitude in the chunk (a first pass takes the
// maxima), so the integer sums are exact, order-independent and therefore
// reproducible, and each keeps ~2^-39 of its material's largest term; a
// non-finite contribution makes its material's partial sum NaN.  The table
// needs 12 bytes per material, so the launch keeps its occupancy (and room
// for camera workgroups).
template <class Src, int R>
__device__ __forceinline__ void ret_bwd_block(const Src &src, const oceansim_sonar_params *params,
                                              const float *refl, int n_mat, double *part, int slot_base,
                                              int n_slots, double *refl_part, float *grad_refl_atomic, int bid,
                                              int n_blocks) {
    extern __shared__ int4 lds_raw[];
    // [n_mat] fixed-point sums, then [n_mat] magnitude maxima (float bits;
    // 0x7f800001 and up: a non-finite contribution); the same memory later
    // serves the workgroup reductions
    long long *racc = reinterpret_cast<long long *>(lds_raw);
    unsigned *rmax = reinterpret_cast<unsigned *>(racc + n_mat);
    double *red3 = reinterpret_cast<double *>(lds_raw);
    int local;
    const int fi = src.locate(bid, KRET, local);
    const SonarDev f = src.frame(fi);
    const int tid = threadIdx.x;
    const bool table = refl_part != nullptr;

    if (table)
        for (int k = tid; k < n_mat; k += kBlock) {
            racc[k] = 0;
            rmax[k] = 0u;
        }
    __syncthreads();

    const oceansim_sonar_params pr = params[f.param_row];
    const float G = pr.gain;
    double g_alpha = 0.0, g_gain = 0.0, g_ssm = 0.0;
    const long long base = (long long)local * (R * kBlock);
    float gr_q[R];
    int m_q[R];   // -1: no contribution (past the frame's end, a miss, or the atomic path)
#pragma unroll
    for (int q = 0; q < R; ++q) {
        m_q[q] = -1;
        gr_q[q] = 0.0f;
    }
    // Groups of RG returns: all their loads, then all their gathers, are in
    // flight together (clamped indices, no masked loads: a load under a branch
    // in the unrolled loop would wait for itself before the next return's)
    constexpr int RG = R < 4 ? R : 4;
#pragma unroll
    for (int q0 = 0; q0 < R; q0 += RG) {
    float xs[RG], ys[RG], zs[RG], nxs[RG], nys[RG], nzs[RG], gis[RG], rfs[RG];
    int ms[RG], bs[RG];
    double rs[RG];
#pragma unroll
    for (int u = 0; u < RG; ++u) {
        const long long k = base + (long long)(q0 + u) * kBlock + tid;
        const long long kc = k < f.n ? k : f.n - 1;
        xs[u] = f.x[kc];
        ys[u] = f.y[kc];
        zs[u] = f.z[kc];
        nxs[u] = f.nx[kc];
        nys[u] = f.ny[kc];
        nzs[u] = f.nz[kc];
        ms[u] = f.mat[kc];
    }
#pragma unroll
    for (int u = 0; u < RG; ++u) {
        const long long k = base + (long long)(q0 + u) * kBlock + tid;
        const int b = return_bin(f, xs[u], ys[u], zs[u], ms[u], n_mat, rs[u]);
        bs[u] = k < f.n ? b : -1;   // a valid bin implies a valid material
    }
#pragma unroll
    for (int u = 0; u < RG; ++u) {
        gis[u] = f.grad_img[bs[u] >= 0 ? bs[u] : 0];   // dL / d(polar image) at the return's bin
        rfs[u] = refl[bs[u] >= 0 ? ms[u] : 0];
    }
#pragma unroll
    for (int u = 0; u < RG; ++u) {
        const int q = q0 + u;
        const int b = bs[u], m = ms[u];
        if (b < 0) continue;
        const float xf = xs[u], yf = ys[u], zf = zs[u];
        const double r = rs[u];
        float cosg, att;
        const float I = return_intensity(f, xf, yf, zf, nxs[u], nys[u], nzs[u], r, rfs[u], pr.alpha, cosg, att);
        const float gI_t = gis[u];
        float z = 0.0f;
        const float mult = speckle_factor(f, (uint32_t)b, pr.sigma_sm, &z);
        const double gIt = (double)gI_t;
        // dL/dQ at the bin: through the multiplicative speckle, or (range-
        // normalised frames, a uniform branch) as the row-normalisation
        // adjoint left it, with the row's scale for the multiplicative draw
        double gq = (double)mult * gIt;
        if (f.range_norm) gq = (double)f.dldq[b];
        const double gI = (double)G * gq;   // dL / dI_k
        g_alpha += gI * (double)I * (-f.kappa * r);
        g_gain += gq * (double)I;
        // (for a range-normalised frame the row kernel adds the sigma_sm term)
        if (f.speckle == SPECKLE_PAPER && !f.range_norm) g_ssm += gIt * (double)G * (double)I * (double)z;
        const float gr = (float)(gI * (double)cosg * (double)att);
        if (table) {
            m_q[q] = m;
            gr_q[q] = gr;
            atomicMax(&rmax[m], __float_as_uint(__builtin_fabsf(gr)));   // ordered as the magnitudes
        } else {
            atomicAdd(&grad_refl_atomic[m], gr);
        }
    }
    // keep the next group's loads below this one (registers for one group)
    __builtin_amdgcn_sched_barrier(0);
    }
    if (table) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int m = m_q[q];
            if (m < 0) continue;
            const unsigned mb = rmax[m];
            if (mb >= 0x7f800000u || mb == 0u) continue;   // non-finite (flagged) or all zero
            int e;
            frexpf(__uint_as_float(mb), &e);                // largest magnitude < 2^e
            // |scaled| < 2^50, and at most 2^12 of them per workgroup: the sum fits
            const long long v = round_to_ll((double)gr_q[q] * ldexp(1.0, 50 - e));
            if (v != 0) atomicAdd(reinterpret_cast<unsigned long long *>(&racc[m]), (unsigned long long)v);
        }
        __syncthreads();
        // partial sums column-major: refl_part[m * n_ret_slots + slot]
        for (int m = tid; m < n_mat; m += kBlock) {
            const unsigned mb = rmax[m];
            double sum = 0.0;
            if (mb >= 0x7f800000u) {
                sum = __builtin_nan("");
            } else if (mb != 0u) {
                int e;
                frexpf(__uint_as_float(mb), &e);
                sum = (double)racc[m] * ldexp(1.0, e - 50);
            }
            refl_part[(long long)m * n_blocks + bid] = sum;
        }
    }
    __syncthreads();
    const double sums[3] = {g_alpha, g_gain, g_ssm};
    const double tot = block_sum_n<3>(sums, red3);   // thread 0: alpha, 1: gain, 2: sigma_sm
    // partial sums column-major: part[c * n_slots + slot]
    const long long slot = slot_base + bid;
    if (tid == 0) {
        reinterpret_cast<int *>(part + 5LL * n_slots)[slot] = f.param_row;
        part[0LL * n_slots + slot] = tot;
        part[2LL * n_slots + slot] = 0.0;
        part[3LL * n_slots + slot] = 0.0;
    }
    if (tid == 1) part[1LL * n_slots + slot] = tot;
    if (tid == 2) part[4LL * n_slots + slot] = tot;
}

template <class Src, int R>
__global__ __launch_bounds__(kBlock) void k_ret_bwd(Src src, const oceansim_sonar_params *params,
                                                    const float *refl, int n_mat, double *part, int slot_base,
                                                    int n_slots, double *refl_part, float *grad_refl_atomic) {
    ret_bwd_block<Src, R>(src, params, refl, n_mat, part, slot_base, n_slots, refl_part, grad_refl_atomic,
                          blockIdx.x, gridDim.x);
}

// The return chunks of the sonar frames and, in the same launch, the camera
// backward of a plan (workgroups n_ret_blocks and up): the camera's HBM
// stream runs beside the latency-bound gathers of the returns.
template <class Src, int R>
__global__ __launch_bounds__(kBlock) void k_ret_uw_bwd(Src src, const oceansim_sonar_params *params,
                                                       const float *refl, int n_mat, double *part, int slot_base,
                                                       int n_slots, double *refl_part, float *grad_refl_atomic,
                                                       int n_ret_blocks, UwBwdCompanion uw) {
    if ((int)blockIdx.x < n_ret_blocks) {
        ret_bwd_block<Src, R>(src, params, refl, n_mat, part, slot_base, n_slots, refl_part, grad_refl_atomic,
                              blockIdx.x, n_ret_blocks);
    } else {
        __shared__ double red9[9 * (kBlock / kWave)];
        uw_bwd_block<Table<UwDev>, kBlock>(Table<UwDev>{uw.table, uw.n}, uw.params, uw.part, uw.part_row,
                                           blockIdx.x - n_ret_blocks, uw.blocks, red9);
    }
}

// ---------------------------------------------------------------------------
// k_pair_bwd (plans whose frames carry material pairs, tables of at most 64
// materials): the adjoint of binning, gain, the multiplicative speckle and
// Eq. (2), one workgroup per forward polar tile, from the pairs and ranges the
// plan's forward pass left.  The tile's dL/d(polar image) is read once into
// LDS (coalesced) and each return looks its bin up there, instead of
// gathering it from global memory at the return's bin; the returns
// themselves are not read again.  Frames without a transposed fan operator
// also get the adjoint of the additive speckle term here (their
// dL/d(polar image) is the polar gradient itself).
//
// The pairs' order within a chunk follows the forward's LDS atomics and may
// change between runs, so the per-return sums are order-independent: each
// contribution is scaled by a power of two chosen from an a priori bound on
// its magnitude in this tile (the tile's largest finite |dL/dI~|, the largest
// value of the multiplicative factor, the largest reflectivity, the largest
// |cos x attenuation| of the tile's pairs, which the forward tile records,
// and the tile's far range edge), rounded to a 64-bit integer and
// summed in integers: the sums are exact and bit-reproducible, each term kept
// to ~2^-40 of its bound (at 2^21 returns per frame; finer for fewer).  A
// non-finite contribution makes its sum NaN.
// ---------------------------------------------------------------------------
// |m| and |z| of the multiplicative draw: -ln u <= 24 ln 2 for u >= 2^-24,
// so a gamma factor is at most 24 ln 2 and |z| at most sqrt(48 ln 2).
constexpr double kGammaMax = 16.635532333438686;
constexpr double kGaussMax = 5.7678665758658466;

// A value known to be the same in every lane of the wave, moved to scalar
// registers (the compiler cannot prove it for values read back from LDS).
__device__ __forceinline__ double uniform_f64(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ long long scale_round(double x, double scale) {
    return round_to_ll(x * scale);
}

// 2^sc with |x| * 2^sc < 2^(50 - extra) for |x| <= bound, where 2^extra
// covers the number of terms (n <= 2^(11 + extra)), so that a sum of up to n
// scaled terms stays below 2^61.  fixed_extra: extra for n terms (lg, the
// smallest with 2^lg >= n, at most 62, from the leading zeros of n - 1).
__device__ __forceinline__ int fixed_extra(long long n) {
    const int lg = n <= 1 ? 0 : min(62, 64 - __builtin_clzll((unsigned long long)(n - 1)));
    return lg > 11 ? lg - 11 : 0;
}
__device__ __forceinline__ int fixed_exponent(double bound, int extra) {
    int e = 0;
    if (bound > 0.0) frexp(bound, &e);   // bound < 2^e
    return 50 - e - extra;
}

// COL_REGS: every frame's n_az divides 4 kWideThreads, so each thread's groups
// of four bins fall on the same four columns: their beam-pattern factors are
// computed once, and the additive adjoint sums g R rho per column, weighted by
// the column's factors at the end.
template <class Src, bool COL_REGS>
__device__ __forceinline__ void pair_bwd_block(const Src &src, const oceansim_sonar_params *params,
                                               const float *refl, int n_mat, double *part, int slot_base,
                                               int n_slots, double *refl_part, int n_refl_slots, int bid) {
    constexpr int NT = kWideThreads;
    constexpr int NW = NT / kWave;
    extern __shared__ int4 lds_raw[];
    __shared__ int seg_end[NT], seg_start[NT], wtot[NW];
    __shared__ unsigned short seg_map[2 * NT];
    __shared__ float refl_s[kLaneHistMats];
    __shared__ unsigned long long racc[kLaneHistMats];
    __shared__ unsigned long long rbad;
    __shared__ float wmax[NW], wrmax[NW];
    __shared__ long long lred[3 * NW];
    __shared__ double dred[2 * NW];
    __shared__ unsigned bad_any;
    int tile;
    const int fi = src.locate(bid, KTILE, tile);
    const SonarDev f = src.frame(fi);
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int nb = f.n_range * f.n_az;
    const int b_lo = tile * f.tile_bins;
    const int b_hi = min(b_lo + f.tile_bins, nb);
    float *gt = reinterpret_cast<float *>(lds_raw);   // [tile_bins]: dL/d(polar image) of the tile's bins
    const oceansim_sonar_params pr = params[f.param_row];
    const float G = pr.gain;
    float rl = 0.0f;   // the largest finite |reflectivity| among the thread's materials
    for (int k = tid; k < n_mat; k += NT) {
        const float r = refl[k];
        refl_s[k] = r;
        racc[k] = 0ull;
        const float a = __builtin_fabsf(r);
        if (a <= 3.4028235e38f && a > rl) rl = a;
    }
    if (tid == 0) {
        rbad = 0ull;
        bad_any = 0u;
    }

    // 1. the tile's gradient into LDS; without an operator this kernel also
    // owns the adjoint of the additive term of Eq. (3)-(4)
    const bool own_add = f.ft_ptr == nullptr;
    const gptr<const float> gsrc = own_add ? f.grad_polar : (gptr<const float>)f.grad_img;
    const bool add_adj = own_add && f.speckle != SPECKLE_OFF;
    const AddCtx ctx{pr.sigma_sa, 1.0f / pr.sigma_phi};
    const double dsphi = 0.5 * (double)pr.sigma_sa / ((double)pr.sigma_phi * (double)pr.sigma_phi);
    double g_sphi = 0.0, g_ssa = 0.0;
    float gmax = 0.0f;
    const int q_first = b_lo >> 2, q_last = (b_hi - 1) >> 2;
    const bool row_groups = f.n_az >= 4;   // with COL_REGS: a group of four bins lies in row b >> az_shift
    const int az_shift = __builtin_ctz((unsigned)f.n_az);
    // COL_REGS: the thread's four columns' E_j and phi_j^2 E_j, and per column
    // the sum of dL/dI~ R_i rho over the thread's rows (a few groups per
    // thread: summed in FP32, then combined in FP64)
    double ecol[4] = {0.0, 0.0, 0.0, 0.0}, pecol[4] = {0.0, 0.0, 0.0, 0.0};
    float scol[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (COL_REGS && add_adj) {
        // n_az divides 4 kWideThreads, a power of two: the column of bin b is b & (n_az - 1)
        const int am = f.n_az - 1;
        const int j0 = ((q_first + tid) << 2) & am;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const float phi = bin_azimuth(f, (j0 + w) & am);
            const float E = expf(-(phi * phi) * ctx.inv_sigma_phi);
            ecol[w] = (double)E;
            pecol[w] = (double)E * ((double)phi * (double)phi);
        }
    }
    for (int q = q_first + tid; q <= q_last; q += NT) {
        const int b0 = q << 2;
        bool in[4];
        float g[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) in[w] = b0 + w >= b_lo && b0 + w < b_hi;
        if (!gsrc) {
#pragma unroll
            for (int w = 0; w < 4; ++w) g[w] = 0.0f;
        } else if (in[0] && in[3]) {
            const float4 v = gload((gptr<const float4>)(gsrc + b0));
            g[0] = v.x;
            g[1] = v.y;
            g[2] = v.z;
            g[3] = v.w;
        } else {
#pragma unroll
            for (int w = 0; w < 4; ++w) g[w] = in[w] ? gsrc[b0 + w] : 0.0f;
        }
        if (in[0] && in[3] && (b_lo & 3) == 0) {
            // one 16-byte LDS store (gt starts 16-byte aligned)
            *reinterpret_cast<float4 *>(gt + (b0 - b_lo)) = make_float4(g[0], g[1], g[2], g[3]);
        } else {
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (in[w]) gt[b0 + w - b_lo] = g[w];
        }
        {
            // the largest finite |dL/dI~| (bins outside the tile read as 0)
            float a[4];
#pragma unroll
            for (int w = 0; w < 4; ++w) a[w] = __builtin_fabsf(g[w]) <= 3.4028235e38f ? __builtin_fabsf(g[w]) : 0.0f;
            gmax = fmaxf(gmax, fmaxf(fmaxf(a[0], a[1]), fmaxf(a[2], a[3])));
        }
        if (add_adj && COL_REGS && row_groups) {
            // the group lies in one row
            const Words wd = philox((uint32_t)q, f.frame_id, 0u, 0u, f.seed_lo, f.seed_hi);
            const float R = range_ramp(f, b0 >> az_shift);
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (in[w]) {
                    const float rho = rayleigh_of_word(pick(wd, (uint32_t)w));
                    scol[w] = __builtin_fmaf(g[w] * rho, R, scol[w]);
                }
        } else if (add_adj && COL_REGS) {
            const Words wd = philox((uint32_t)q, f.frame_id, 0u, 0u, f.seed_lo, f.seed_hi);
            int i = b0 / f.n_az;
            int j = b0 - i * f.n_az;
            float R = range_ramp(f, i);
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                if (in[w]) {
                    const float rho = rayleigh_of_word(pick(wd, (uint32_t)w));
                    scol[w] = __builtin_fmaf(g[w] * rho, R, scol[w]);
                }
                if (++j == f.n_az) {
                    j = 0;
                    R = range_ramp(f, ++i);
                }
            }
        } else if (add_adj) {
            const Words wd = philox((uint32_t)q, f.frame_id, 0u, 0u, f.seed_lo, f.seed_hi);
            int i = b0 / f.n_az;
            int j = b0 - i * f.n_az;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                if (in[w]) {
                    float E, rho, R, phi;
                    additive_term(f, ctx, i, j, pick(wd, (uint32_t)w), E, rho, R, phi);
                    // d add / d sigma_sa and d add / d sigma_phi of Eq. (3)-(4)
                    const double t = (double)g[w] * (double)R * (double)E * (double)rho;
                    g_ssa += 0.5 * t;
                    g_sphi += t * dsphi * ((double)phi * (double)phi);
                }
                if (++j == f.n_az) {
                    j = 0;
                    ++i;
                }
            }
        }
    }
    if (COL_REGS && add_adj) {
        // d add / d sigma_sa = sum 0.5 g R E rho, d add / d sigma_phi = sum g R E rho dsphi phi^2
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            g_ssa += 0.5 * ecol[w] * (double)scol[w];
            g_sphi += dsphi * pecol[w] * (double)scol[w];
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        gmax = fmaxf(gmax, __shfl_down(gmax, off, kWave));
        rl = fmaxf(rl, __shfl_down(rl, off, kWave));
    }
    if (lane == 0) {
        wmax[wave] = gmax;
        wrmax[wave] = rl;
    }
    __syncthreads();
    float Mg = 0.0f, Rmax = 0.0f;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        Mg = fmaxf(Mg, wmax[k]);
        Rmax = fmaxf(Rmax, wrmax[k]);
    }

    // 2. bounds of one return's contributions in this tile, and their scales
    // (the largest |cos x attenuation| of the tile's pairs is the forward's)
    const int ia = tile * f.rows_per_tile;
    const int ib = min(ia + f.rows_per_tile, f.n_range);
    const double r_hi = f.r_min + (double)ib * f.dr;
    const double Emax = (double)f.tile_cemax[tile];
    const double Mm = f.speckle == SPECKLE_GAMMA   ? kGammaMax
                      : f.speckle == SPECKLE_PAPER ? 0.5 + __builtin_fabs((double)pr.sigma_sm) * kGaussMax
                                                   : 1.0;
    const double safety = 1.01;
    const double absG = __builtin_fabs((double)G);
    const double B_refl = safety * absG * Mm * (double)Mg * Emax;                  // |dL/dI cos att|
    const double B_alpha = B_refl * (double)Rmax * f.kappa * r_hi * 1.001;        // |dL/dI I kappa r|
    const double B_gain = safety * Mm * (double)Mg * (double)Rmax * Emax;          // |dL/dQ I|
    const double B_ssm = safety * (double)Mg * absG * (double)Rmax * Emax * kGaussMax;   // |g G I z|
    const int extra = fixed_extra(f.n > 0 ? f.n : 1);
    const int e_refl = fixed_exponent(B_refl, extra), e_alpha = fixed_exponent(B_alpha, extra);
    const int e_gain = fixed_exponent(B_gain, extra), e_ssm = fixed_exponent(B_ssm, extra);
    // the scales are the same in every lane: held in scalar registers
    const double s_refl = uniform_f64(ldexp(1.0, min(e_refl, 1000)));
    const double s_alpha = uniform_f64(ldexp(1.0, min(e_alpha, 1000)));
    const double s_gain = uniform_f64(ldexp(1.0, min(e_gain, 1000)));
    const double s_ssm = uniform_f64(ldexp(1.0, min(e_ssm, 1000)));
    const bool refl_ok = __builtin_isfinite(B_refl);
    const bool paper = f.speckle == SPECKLE_PAPER;

    // 3. the tile's returns: dL/dI = G m dL/dI~ at the return's bin
    long long a_alpha = 0, a_gain = 0, a_ssm = 0;
    // non-finite contributions per sum (alpha, gain, sigma_sm)
    bool bad_a = !__builtin_isfinite(B_alpha), bad_g = !__builtin_isfinite(B_gain);
    bool bad_s = paper && !__builtin_isfinite(B_ssm);
    const double neg_kappa = -f.kappa;
    for_tile_pairs<NT, kPairBwdLoads, true>(f, tile, seg_end, seg_start, wtot, seg_map, [&](uint2 pq, float r) __attribute__((always_inline)) {
        const uint32_t lb = pq.x & 0xffffu;
        const int m = (int)(pq.x >> 16);
        if (lb >= (uint32_t)(b_hi - b_lo) || m >= n_mat) return;
        const float ce = __uint_as_float(pq.y);   // cos(gamma) exp(-kappa alpha r)
        float z = 0.0f;
        const float mult = speckle_factor(f, (uint32_t)(b_lo + (int)lb), pr.sigma_sm, &z);
        const float g = gt[lb];
        const double gq = (double)mult * (double)g;   // dL/dQ at the bin
        const double gI = (double)G * gq;             // dL/dI_k
        const float I = refl_s[m] * ce;
        const double xr = gI * (double)ce;
        const double xa = gI * (double)I * (neg_kappa * (double)r);
        const double xg = gq * (double)I;
        if (paper) {
            // the speckle mode is a frame's, the same across the wave: the
            // empty asm statement keeps this a branch (not computed and
            // discarded for the other modes)
            __asm__ volatile("");
            const double xs = (double)g * (double)G * (double)I * (double)z;
            if (__builtin_isfinite(xs)) a_ssm += scale_round(xs, s_ssm); else bad_s = true;
        }
        if (__builtin_isfinite(xr)) {
            const long long v = scale_round(xr, s_refl);
            if (v != 0) atomicAdd(&racc[m], (unsigned long long)v);
        } else {
            atomicOr(&rbad, 1ull << m);
        }
        if (__builtin_isfinite(xa)) a_alpha += scale_round(xa, s_alpha); else bad_a = true;
        if (__builtin_isfinite(xg)) a_gain += scale_round(xg, s_gain); else bad_g = true;
    }, []() {});

    // 4. workgroup sums (integers: any order; doubles: a fixed order)
    long long lv[3] = {a_alpha, a_gain, a_ssm};
    double dv[2] = {g_sphi, g_ssa};
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) lv[k] += __shfl_down(lv[k], off, kWave);
#pragma unroll
        for (int k = 0; k < 2; ++k) dv[k] += __shfl_down(dv[k], off, kWave);
    }
    const unsigned bad_bits = (bad_a ? 1u : 0u) | (bad_g ? 2u : 0u) | (bad_s ? 4u : 0u);
    if (bad_bits) atomicOr(&bad_any, bad_bits);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) lred[k * NW + wave] = lv[k];
#pragma unroll
        for (int k = 0; k < 2; ++k) dred[k * NW + wave] = dv[k];
    }
    __syncthreads();
    const long long slot = slot_base + bid;
    if (tid < 5) {
        double v;
        if (tid < 3) {
            long long t = 0;
            for (int k = 0; k < NW; ++k) t += lred[tid * NW + k];
            const double sc = tid == 0 ? s_alpha : tid == 1 ? s_gain : s_ssm;
            v = ((bad_any >> tid) & 1u) ? __builtin_nan("") : (double)t / sc;
        } else {
            double t = 0.0;
            for (int k = 0; k < NW; ++k) t += dred[(tid - 3) * NW + k];
            v = t;
        }
        // columns: 0 alpha, 1 gain, 2 sigma_phi, 3 sigma_sa, 4 sigma_sm
        const int col = tid == 0 ? 0 : tid == 1 ? 1 : tid == 2 ? 4 : tid == 3 ? 2 : 3;
        part[(long long)col * n_slots + slot] = v;
        if (tid == 0) reinterpret_cast<int *>(part + 5LL * n_slots)[slot] = f.param_row;
    }
    for (int m = tid; m < n_mat; m += NT) {
        const bool pm = !refl_ok || ((rbad >> m) & 1ull);
        refl_part[(long long)m * n_refl_slots + bid] = pm ? __builtin_nan("") : (double)(long long)racc[m] / s_refl;
    }
}

// Held to six waves per SIMD (80 VGPRs) so that three workgroups fit per CU.
template <class Src, bool COL_REGS>
__global__ __launch_bounds__(kWideThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_pair_bwd(
    Src src, const oceansim_sonar_params *params, const float *refl, int n_mat, double *part, int slot_base,
    int n_slots, double *refl_part, int n_refl_slots) {
    pair_bwd_block<Src, COL_REGS>(src, params, refl, n_mat, part, slot_base, n_slots, refl_part, n_refl_slots,
                                  xcd_grouped_id<kTileXcdRun>(blockIdx.x, gridDim.x));
}

// k_pair_uw_bwd (plans with camera frames): the pair backward tiles and the
// camera backward in one launch, interleaved through the dispatch order as in
// k_tile_uw (workgroup x is a camera one when floor((x+1) C / N) >
// floor(x C / N)), so the VALU-bound tiles and the HBM-bound camera share
// every CU.  A camera workgroup runs two camera blocks of kBlock threads side
// by side, one channel's loads in flight at a time (within the tiles'
// register budget).
template <class Src, bool COL_REGS>
__global__ __launch_bounds__(kWideThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_pair_uw_bwd(
    Src src, const oceansim_sonar_params *params, const float *refl, int n_mat, double *part, int slot_base,
    int n_slots, double *refl_part, int n_tile_blocks, int n_cam_groups, UwBwdCompanion uw) {
    static_assert(kWideThreads == 2 * kBlock, "two camera blocks per wide workgroup");
    const FusedSlot slot = fused_slot(xcd_grouped_id<kTileXcdRun>(blockIdx.x, gridDim.x), n_tile_blocks, n_cam_groups);
    if (slot.cam) {
        __shared__ double red9[2 * 9 * (kBlock / kWave)];
        // the same in every lane of a wave: scalar, so the camera frame's
        // fields load into scalar registers
        const int half = __builtin_amdgcn_readfirstlane(threadIdx.x >= kBlock ? 1 : 0);
        const int cb = __builtin_amdgcn_readfirstlane(2 * slot.index + half);
        uw_bwd_block<Table<UwDev>, kBlock, true>(Table<UwDev>{uw.table, uw.n}, uw.params, uw.part, uw.part_row, cb,
                                                 uw.blocks, red9 + half * 9 * (kBlock / kWave),
                                                 (int)(threadIdx.x & (kBlock - 1)), cb < uw.blocks);
    } else {
        pair_bwd_block<Src, COL_REGS>(src, params, refl, n_mat, part, slot_base, n_slots, refl_part, n_tile_blocks,
                                      slot.index);
    }
}

// ---------------------------------------------------------------------------
// k_fant_bwd: the polar gradient through the frames' transposed fan operators
// (plans), BPT consecutive bins per thread: dL/dI[b] is the sum of weight *
// dL/dF over the bin's entries, in FP64 and in the entries' fixed order
// (each product of two floats is exact in FP64), plus the direct polar
// gradient; then the adjoint of Eq. (3)-(4) as in the tile epilogue.  No
// candidate search, no fixed-point scale, no workgroup barrier before the
// partial sums.
//
// The entries of a wave's 64 * BPT consecutive bins are contiguous: the wave
// reads them in coalesced 64-entry chunks (lane k takes entry k of a chunk),
// so the loads of one instruction are one span of 512 bytes and its fan
// gathers are the neighbouring pixels of neighbouring bins; the products go
// to the wave's slice of LDS, and each lane then sums its own bins' runs.
// More bins per thread amortise the workgroup's fixed costs (frame lookup,
// pointer loads, partial sums) where there are many bins to share the chip.
// With a mirrored operator (even fan width) a thread's rows are bins of the
// left half of the azimuth columns: each entry is gathered at its pixel and
// at the mirrored pixel, giving the row's bin and its mirror bin at once from
// half the operator bytes.
// ---------------------------------------------------------------------------
constexpr int kFantChunks = 8;   // 64-entry chunks staged per round (512 entries per wave; mirrored: 256)
constexpr size_t kFuseLdsBytes = 16384;   // LDS of a return-gather workgroup that camera workgroups may share

// MIRROR: the batch has mirrored operators (their rows produce two bins;
// without any, the kernel keeps one output per row and fewer registers).
template <class Src, int BPT, bool MIRROR>
__global__ __launch_bounds__(kBlock) void k_fant_bwd(Src src, const oceansim_sonar_params *params, double *part,
                                                     int n_slots, float *grad_refl_zero, int n_mat_zero) {
    __shared__ double prod[kBlock / kWave][kFantChunks * kWave];
    int local;
    const int bid = blockIdx.x;
    const int fi = src.locate(bid, KFANT, local);
    const SonarDev f = src.frame(fi);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    // operator rows: the bins, or (mirrored layout) the bins of the first
    // ceil(N_phi / 2) columns, each also standing for its mirror bin
    constexpr int NO = MIRROR ? 2 * BPT : BPT;   // outputs per thread
    const bool mir = MIRROR && f.ft_mirror != 0 && f.ft_ptr;
    const int ncol = mir ? (f.n_az + 1) >> 1 : f.n_az;
    const int nrow = f.n_range * ncol;
    const int h0 = (local * kBlock + tid) * BPT;   // this thread's first row
    // Loads first, without branches (indices clamped), so that they are in
    // flight together while the speckle factors are computed: the parameter
    // row (before any store, so it may come through the scalar cache), this
    // lane's rows' operator pointers and the direct polar gradient.
    const oceansim_sonar_params pr = params[f.param_row];
    // the wave's span of entries [w_lo, w_hi): uniform addresses, so scalar
    // loads, and the only ones the entry loads wait for
    const int wb = (local * kBlock + __builtin_amdgcn_readfirstlane(wave) * kWave) * BPT;
    int w_lo = 0, w_hi = 0;
    if (f.ft_ptr) {
        w_lo = f.ft_ptr[wb < nrow ? wb : nrow];
        w_hi = f.ft_ptr[wb + kWave * BPT < nrow ? wb + kWave * BPT : nrow];
    }
    int p[BPT + 1];   // this lane's rows' entries start at p[0..BPT-1] and end at p[BPT]
#pragma unroll
    for (int m = 0; m <= BPT; ++m) p[m] = f.ft_ptr ? f.ft_ptr[h0 + m < nrow ? h0 + m : nrow] : 0;
    // output bins: ob[m] is row m's own bin, ob[BPT + m] (MIRROR) its mirror bin (-1:
    // none, plain layout or a middle column that is its own mirror); -1 past
    // the end
    int ob[MIRROR ? NO : 1];
    if constexpr (MIRROR) {
        int i = h0 / ncol, j = h0 - i * ncol;
#pragma unroll
        for (int m = 0; m < BPT; ++m) {
            const bool in = h0 + m < nrow;
            const int jm = f.n_az - 1 - j;
            ob[m] = in ? i * f.n_az + j : -1;
            ob[BPT + m] = in && mir && jm != j ? i * f.n_az + jm : -1;
            if (++j == ncol) {
                j = 0;
                ++i;
            }
        }
    }
    // output bin k (plain rows are the bins themselves)
    auto out_bin = [&](int k) __attribute__((always_inline)) -> int {
        if constexpr (MIRROR) return ob[k];
        else return h0 + k < nrow ? h0 + k : -1;
    };
    // (without a polar gradient the load reads this frame's own gradient
    // buffer, a valid address, and the value is discarded: a select, not a
    // branch that would wait for the load)
    float gpol[NO];
    {
        const bool has = f.grad_polar != nullptr;
        const gptr<const float> src_pol = has ? f.grad_polar : (gptr<const float>)f.grad_img;
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            const int bk = out_bin(k);
            const float v = src_pol[bk >= 0 ? bk : 0];
            gpol[k] = has ? v : 0.0f;
        }
    }
    // the atomic reflectivity path (many materials) accumulates into a zeroed table
    if (grad_refl_zero)
        for (int k = bid * kBlock + tid; k < n_mat_zero; k += (int)gridDim.x * kBlock) grad_refl_zero[k] = 0.0f;
    // per output bin, the factors of the adjoint of Eq. (3)-(4): R E rho and
    // phi^2; computed once, while the first round's gathers are in flight
    float fac[NO], phi2[NO];
    auto speckle_factors = [&]() __attribute__((always_inline)) {
        const AddCtx ctx{pr.sigma_sa, 1.0f / pr.sigma_phi};
        Words wd{0u, 0u, 0u, 0u};
        int wq = -1;
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            const int b = out_bin(k);
            fac[k] = phi2[k] = 0.0f;
            if (f.speckle != SPECKLE_OFF && b >= 0) {
                // the bin's Philox word is the one its forward tile drew
                if ((b >> 2) != wq) {
                    wq = b >> 2;
                    wd = philox((uint32_t)wq, f.frame_id, 0u, 0u, f.seed_lo, f.seed_hi);
                }
                const int i = b / f.n_az, j = b - i * f.n_az;
                float E, rho, R, phi;
                additive_term(f, ctx, i, j, pick(wd, (uint32_t)(b & 3)), E, rho, R, phi);
                fac[k] = R * E * rho;
                phi2[k] = phi * phi;
            }
        }
    };
    bool have_factors = false;
    double gs[NO];
#pragma unroll
    for (int k = 0; k < NO; ++k) gs[k] = 0.0;
    // Rounds of NC coalesced 64-entry chunks; MIR: each entry also gathers
    // the mirrored pixel, whose products fill the slice's second half.
    auto rounds = [&](auto nc, auto mirror) __attribute__((always_inline)) {
        constexpr int NC = decltype(nc)::value;
        constexpr bool MIR = decltype(mirror)::value;
        double *slice = prod[wave];
        for (int r0 = w_lo; r0 < w_hi; r0 += NC * kWave) {
            // Every lane loads (past the end it re-reads the wave's last entry,
            // whose product no row sums): no branch in the unrolled loads, so
            // all the chunk's loads, then all its gathers, are in flight together.
            uint2 en[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int e = r0 + c * kWave + lane;
                en[c] = gload(f.ft_ent + (e < w_hi ? e : w_hi - 1));
            }
            if (!have_factors) {   // uniform: under the first round's entry loads
                speckle_factors();
                have_factors = true;
            }
            float gv[NC], gm[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if constexpr (MIR) {
                    const unsigned u = en[c].x & 0xffffu;
                    const unsigned row = __umul24(en[c].x >> 16, (unsigned)f.fan_w);   // < 2^31
                    gv[c] = f.grad_fan[row + u];
                    gm[c] = f.grad_fan[row + ((unsigned)f.fan_w - 1u - u)];
                } else {
                    gv[c] = f.grad_fan[(long long)en[c].x];
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double w = (double)__uint_as_float(en[c].y);
                slice[c * kWave + lane] = w * (double)gv[c];
                if constexpr (MIR) slice[(NC + c) * kWave + lane] = w * (double)gm[c];
            }
            // the wave's own LDS writes, then its reads (no other wave touches the slice)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int a = p[0] > r0 ? p[0] : r0;
            const int z = p[BPT] < r0 + NC * kWave ? p[BPT] : r0 + NC * kWave;
            for (int e = a; e < z; ++e) {
                const double v = slice[e - r0];
                int m = 0;
#pragma unroll
                for (int k = 1; k < BPT; ++k) m += e >= p[k] ? 1 : 0;
#pragma unroll
                for (int k = 0; k < BPT; ++k) gs[k] += m == k ? v : 0.0;
                if constexpr (MIR && MIRROR) {
                    const double vm = slice[NC * kWave + e - r0];
#pragma unroll
                    for (int k = 0; k < BPT; ++k) gs[BPT + k] += m == k ? vm : 0.0;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    };
    if (f.ft_ptr) {
        if (mir)
            rounds(std::integral_constant<int, kFantChunks / 2>{}, std::integral_constant<bool, MIRROR>{});
        else
            rounds(std::integral_constant<int, kFantChunks>{}, std::false_type{});
    }
    if (!have_factors) speckle_factors();
    double g_sphi = 0.0, g_ssa = 0.0;
    const double dsphi = 0.5 * (double)pr.sigma_sa / ((double)pr.sigma_phi * (double)pr.sigma_phi);
#pragma unroll
    for (int k = 0; k < NO; ++k) {
        const int b = out_bin(k);
        if (b < 0) {
            if constexpr (MIRROR) continue;   // a missing mirror bin; later rows may follow
            else break;                       // past the end
        }
        const double g = gs[k] + (double)gpol[k];
        f.grad_img[b] = (float)g;
        // d add / d sigma_sa and d add / d sigma_phi of Eq. (3)-(4) (zero
        // factors without speckle)
        const double t = g * (double)fac[k];
        g_ssa += 0.5 * t;
        g_sphi += t * dsphi * (double)phi2[k];
    }
    __shared__ double red2[2 * (kBlock / kWave)];
    const double sums[2] = {g_sphi, g_ssa};
    const double tot = block_sum_n<2, kBlock>(sums, red2);   // thread 0: sigma_phi, thread 1: sigma_sa
    if (tid == 0) {
        reinterpret_cast<int *>(part + 5LL * n_slots)[bid] = f.param_row;
        part[0LL * n_slots + bid] = 0.0;
        part[1LL * n_slots + bid] = 0.0;
        part[2LL * n_slots + bid] = tot;
        part[4LL * n_slots + bid] = 0.0;
    }
    if (tid == 1) part[3LL * n_slots + bid] = tot;
}

// ---------------------------------------------------------------------------
// k_rownorm_bwd: adjoint of the range-wise normalisation, one workgroup per
// range row of each range-normalised frame.  With gN = dL/d(normalised Q)
// (the polar gradient times the multiplicative speckle factor, or alone
// without speckle), a row normalised by its maximum m = Q_j* gives
// dL/dQ_j = gN_j / m - [j = j*] (sum_k gN_k Q_k) / m^2; other rows pass gN.
// The maximum is the forward's (over the positive entries of G P, from the
// saved sums), j* the first column attaining it; the sum is FP64 in a fixed
// order.  Writes dL/dQ per bin, and the row's partial sum of dL/d sigma_sm
// (the paper's multiplicative draw acts on the normalised row) to its slot.
// ---------------------------------------------------------------------------
template <class Src>
__global__ __launch_bounds__(kBlock) void k_rownorm_bwd(Src src, const oceansim_sonar_params *params, double *part,
                                                        int slot_base, int n_slots) {
    __shared__ unsigned s_max;
    __shared__ int s_arg;
    __shared__ double s_sum;
    int i;
    const int fi = src.locate(blockIdx.x, KROW, i);
    const SonarDev f = src.frame(fi);
    const oceansim_sonar_params pr = params[f.param_row];
    const float G = pr.gain;
    const int tid = threadIdx.x;
    const int r0 = i * f.n_az;
    if (tid == 0) {
        s_max = 0u;
        s_arg = f.n_az;
    }
    __syncthreads();
    for (int j = tid; j < f.n_az; j += kBlock) {
        const float q = G * f.saved_p[r0 + j];
        if (q > 0.0f) atomicMax(&s_max, __float_as_uint(q));   // positive floats order as their bits
    }
    __syncthreads();
    const float m = __uint_as_float(s_max);
    const bool norm = m > 0.0f;
    const double scale = norm ? 1.0 / (double)m : 1.0;
    auto g_norm = [&](int b, double &gssm) -> double {   // dL/d(normalised Q) at bin b
        double g = (double)f.grad_img[b];
        gssm = 0.0;
        if (f.speckle != SPECKLE_OFF) {
            float z = 0.0f;
            const double gt = g;
            g *= (double)speckle_factor(f, (uint32_t)b, pr.sigma_sm, &z);
            if (f.speckle == SPECKLE_PAPER)   // d/d sigma_sm of (normalised Q) m
                gssm = gt * ((double)(G * f.saved_p[b]) * scale) * (double)z;
        }
        return g;
    };
    extern __shared__ int4 lds_raw[];
    double *gnr = reinterpret_cast<double *>(lds_raw);   // [n_az]: dL/d(normalised Q) of the row
    double ps = 0.0, pssm = 0.0;
    for (int j = tid; j < f.n_az; j += kBlock) {
        const float q = G * f.saved_p[r0 + j];
        if (norm && q == m) atomicMin(&s_arg, j);
        double gs;
        const double gn = g_norm(r0 + j, gs);
        gnr[j] = gn;
        ps += gn * (double)q;
        pssm += gs;
    }
    const double sums[2] = {ps, pssm};
    __shared__ double red2[2 * (kBlock / kWave)];
    const double tot = block_sum_n<2, kBlock>(sums, red2);   // thread 0: the row sum, 1: sigma_sm
    if (tid == 0) s_sum = tot;
    // the row's partial sums: column 4 (sigma_sm), zeros elsewhere
    const long long slot = slot_base + blockIdx.x;
    if (tid == 0) {
        reinterpret_cast<int *>(part + 5LL * n_slots)[slot] = f.param_row;
        part[0LL * n_slots + slot] = 0.0;
        part[1LL * n_slots + slot] = 0.0;
        part[2LL * n_slots + slot] = 0.0;
        part[3LL * n_slots + slot] = 0.0;
    }
    if (tid == 1) part[4LL * n_slots + slot] = tot;
    __syncthreads();
    const int js = s_arg;
    const double S = s_sum, md = (double)m;
    for (int j = tid; j < f.n_az; j += kBlock) {
        const int b = r0 + j;
        double d = gnr[j];   // this thread's own entry
        if (norm) {
            d /= md;
            if (j == js) d -= S / (md * md);
        }
        f.dldq[b] = (float)d;
    }
}

// Column table of the fan frames (workgroup = frame), the input the fan
// kernel's stencils need besides the geometry.
template <class Src>
__global__ __launch_bounds__(kBlock) void k_fan_cols(Src src) {
    const SonarDev f = src.frame((int)blockIdx.x);
    if (f.cols)
        for (int j = threadIdx.x; j < f.n_az; j += kBlock) write_fan_column(f, j);
}

// ---------------------------------------------------------------------------
// k_reduce_sonar: fixed-order sums of the partials.  Blocks [0, n_rows * 8)
// produce grad_params[row][col] from the slots of the frames using that row;
// the following n_mat blocks (small tables) produce grad_refl.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_reduce_sonar(SonarReduce a) {
    __shared__ double red[kBlock / kWave];
    sonar_reduce_block(a, blockIdx.x, red);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define OSIM_DISPATCH_R(R_, ...)                       \
    switch (R_) {                                      \
        case 2: { constexpr int RR = 2; __VA_ARGS__; } break;   \
        case 4: { constexpr int RR = 4; __VA_ARGS__; } break;   \
        case 8: { constexpr int RR = 8; __VA_ARGS__; } break;   \
        case 16: { constexpr int RR = 16; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;          \
    }

template <class Src>
static hipError_t launch_fwd(const Src &src, const SonarGrid &g, const oceansim_sonar_params *params,
                             const float *refl, int n_mat, hipStream_t st, const UwCompanion *uw) {
    // a plan's camera forward rides along in the binning launch (few,
    // latency-bound workgroups with little LDS); wide binning workgroups
    // (chunks above 4096 returns) take 64 KB of LDS each, so the camera
    // frames then run in a launch of their own
    const bool wide = g.chunk > 4096;
    const bool with_uw = uw && uw->blocks > 0;
    if (g.bin_blocks > 0 || (with_uw && !wide)) {
        const size_t lds = (size_t)((g.max_tiles + 1 + 3) & ~3) * 4 + (size_t)g.chunk * 8;
        if (wide) {
            if (g.chunk != kWideThreads * 16) return hipErrorInvalidValue;
            OSIM_LAUNCH("k_bin", (k_bin<Src, kWideThreads, 16>), dim3(g.bin_blocks), dim3(kWideThreads), lds, st,
                        src, params, refl, n_mat);
        } else if (with_uw) {
            OSIM_DISPATCH_R(g.chunk / kBlock,
                            OSIM_LAUNCH("k_bin_uw", (k_bin_uw<Src, RR>), dim3(g.bin_blocks + uw->blocks),
                                        dim3(kBlock), lds, st, src, params, refl, n_mat, g.bin_blocks,
                                        Table<UwDev>{uw->table, uw->n}, uw->params));
        } else {
            OSIM_DISPATCH_R(g.chunk / kBlock,
                            OSIM_LAUNCH("k_bin", (k_bin<Src, kBlock, RR>), dim3(g.bin_blocks), dim3(kBlock), lds,
                                        st, src, params, refl, n_mat));
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // LDS of a tile: the histogram, the column table (unless the columns'
    // factors live in registers), the row maxima
    const bool wide_tiles = g.max_tile_bins > kMaxTileBins;
    const bool col_regs = wide_tiles && g.wide_col_regs;
    const size_t tile_lds = (size_t)g.max_tile_bins * 4 + (col_regs ? 0 : (size_t)g.max_n_az * 4) +
                            (size_t)g.max_rows_per_tile * 4;
    if (with_uw && wide && wide_tiles) {
        // wide tiles and the camera forward side by side in one launch
        const int groups = (uw->blocks + 1) / 2;
        if (col_regs)
            OSIM_LAUNCH("k_tile_uw", (k_tile_uw<Src, true>), dim3(g.tile_blocks + groups), dim3(kWideThreads),
                        tile_lds, st, src, params, refl, n_mat, g.tile_blocks, groups, Table<UwDev>{uw->table, uw->n},
                        uw->params, uw->blocks);
        else
            OSIM_LAUNCH("k_tile_uw", (k_tile_uw<Src, false>), dim3(g.tile_blocks + groups), dim3(kWideThreads),
                        tile_lds, st, src, params, refl, n_mat, g.tile_blocks, groups, Table<UwDev>{uw->table, uw->n},
                        uw->params, uw->blocks);
    } else {
        if (with_uw && wide) {
            hipError_t e = uw_forward_table(uw->table, uw->n, uw->blocks, uw->params, st);
            if (e != hipSuccess) return e;
        }
        if (col_regs)
            OSIM_LAUNCH("k_tile", (k_tile<Src, kWideThreads, true>), dim3(g.tile_blocks), dim3(kWideThreads),
                        tile_lds, st, src, params, refl, n_mat);
        else if (wide_tiles)
            OSIM_LAUNCH("k_tile", (k_tile<Src, kWideThreads, false>), dim3(g.tile_blocks), dim3(kWideThreads),
                        tile_lds, st, src, params, refl, n_mat);
        else
            OSIM_LAUNCH("k_tile", (k_tile<Src, kBlock, false>), dim3(g.tile_blocks), dim3(kBlock), tile_lds, st, src,
                        params, refl, n_mat);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g.fan_blocks > 0) {
        OSIM_LAUNCH("k_fan", (k_fan<Src>), dim3(g.fan_blocks), dim3(kBlock), 0, st, src);
        e = hipGetLastError();
    }
    return e;
}

template <class Src>
static hipError_t launch_bwd(const Src &src, int n_frames, const SonarGrid &g,
                             const oceansim_sonar_params *params, int n_rows, const float *refl, int n_mat,
                             double *part, double *refl_part, float *grad_params, float *grad_refl,
                             hipStream_t st, SonarReduce *defer, const UwBwdCompanion *uwb) {
    const bool lane_hist = n_mat <= kLaneHistMats;
    if (g.pair_bwd) {
        // operator rows of the frames with a fan gradient, then one pair
        // workgroup per forward tile; the camera backward in its own launch
        const int n_slots = g.fant_blocks + g.tile_blocks;
        hipError_t e = hipSuccess;
        if (g.fant_blocks > 0) {
#define OSIM_FANT(B, M)                                                                                     \
    OSIM_LAUNCH("k_fant_bwd", (k_fant_bwd<Src, B, M>), dim3(g.fant_blocks), dim3(kBlock), 0, st, src, params, \
                part, n_slots, (float *)nullptr, n_mat)
            switch (g.fant_bpt * 2 + (g.fant_mirror ? 1 : 0)) {
                case 2: OSIM_FANT(1, false); break;
                case 3: OSIM_FANT(1, true); break;
                case 4: OSIM_FANT(2, false); break;
                case 5: OSIM_FANT(2, true); break;
                case 8: OSIM_FANT(4, false); break;
                case 9: OSIM_FANT(4, true); break;
                default: return hipErrorInvalidValue;
            }
#undef OSIM_FANT
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        const bool with_uw = uwb && uwb->blocks > 0;
        const int groups = with_uw ? (uwb->blocks + 1) / 2 : 0;
        if (g.tile_blocks > 0 && with_uw && g.tile_blocks >= groups) {
            // the camera backward interleaved with the pair workgroups, where
            // these are enough to hide it (the camera part keeps one
            // channel's loads in flight, slower on its own)
            if (g.wide_col_regs)
                OSIM_LAUNCH("k_pair_uw_bwd", (k_pair_uw_bwd<Src, true>), dim3(g.tile_blocks + groups),
                            dim3(kWideThreads), (size_t)g.max_tile_bins * 4, st, src, params, refl, n_mat, part,
                            g.fant_blocks, n_slots, refl_part, g.tile_blocks, groups, *uwb);
            else
                OSIM_LAUNCH("k_pair_uw_bwd", (k_pair_uw_bwd<Src, false>), dim3(g.tile_blocks + groups),
                            dim3(kWideThreads), (size_t)g.max_tile_bins * 4, st, src, params, refl, n_mat, part,
                            g.fant_blocks, n_slots, refl_part, g.tile_blocks, groups, *uwb);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        } else {
            if (g.tile_blocks > 0) {
                if (g.wide_col_regs)
                    OSIM_LAUNCH("k_pair_bwd", (k_pair_bwd<Src, true>), dim3(g.tile_blocks), dim3(kWideThreads),
                                (size_t)g.max_tile_bins * 4, st, src, params, refl, n_mat, part, g.fant_blocks,
                                n_slots, refl_part, g.tile_blocks);
                else
                    OSIM_LAUNCH("k_pair_bwd", (k_pair_bwd<Src, false>), dim3(g.tile_blocks), dim3(kWideThreads),
                                (size_t)g.max_tile_bins * 4, st, src, params, refl, n_mat, part, g.fant_blocks,
                                n_slots, refl_part, g.tile_blocks);
                e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
            if (with_uw) {
                e = uw_backward_table(uwb->table, uwb->n, uwb->blocks, uwb->params, uwb->part, uwb->part_row, st);
                if (e != hipSuccess) return e;
            }
        }
        SonarReduce a;
        a.part = part;
        a.n_slots = n_slots;
        a.n_rows = n_rows;
        a.grad_params = grad_params;
        a.refl_part = refl_part;
        a.ret_slots = g.tile_blocks;
        a.n_mat = n_mat;
        a.grad_refl = grad_refl;
        a.blocks = n_rows * OCEANSIM_SONAR_GRAD_WIDTH + n_mat;
        if (defer) {
            *defer = a;
            return hipSuccess;
        }
        OSIM_LAUNCH("k_reduce_sonar", k_reduce_sonar, dim3(a.blocks), dim3(kBlock), 0, st, a);
        return hipGetLastError();
    }
    // partial-sum slots: polar workgroups (tiles, or bin blocks through the
    // transposed fan operators), then return chunks
    const int polar_blocks = g.use_fant ? g.fant_blocks : g.tile_b_blocks;
    const int n_slots = polar_blocks + g.ret_blocks + g.row_blocks;
    hipError_t e = hipSuccess;
    if (g.use_fant && g.fant_blocks > 0) {
        float *gz = lane_hist ? (float *)nullptr : grad_refl;
#define OSIM_FANT(B, M)                                                                                     \
    OSIM_LAUNCH("k_fant_bwd", (k_fant_bwd<Src, B, M>), dim3(g.fant_blocks), dim3(kBlock), 0, st, src, params, \
                part, n_slots, gz, n_mat)
        switch (g.fant_bpt * 2 + (g.fant_mirror ? 1 : 0)) {
            case 2: OSIM_FANT(1, false); break;
            case 3: OSIM_FANT(1, true); break;
            case 4: OSIM_FANT(2, false); break;
            case 5: OSIM_FANT(2, true); break;
            case 8: OSIM_FANT(4, false); break;
            case 9: OSIM_FANT(4, true); break;
            default: return hipErrorInvalidValue;
        }
#undef OSIM_FANT
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    } else if (!g.use_fant && g.tile_b_blocks > 0) {
        if (g.all_saved)
            OSIM_LAUNCH("k_tile_bwd", (k_tile_bwd<Src, true>), dim3(g.tile_b_blocks), dim3(kBwdThreads),
                        (size_t)g.max_tile_bins_b * 8, st, src, params, part, n_slots,
                        lane_hist ? (float *)nullptr : grad_refl, n_mat);
        else
            OSIM_LAUNCH("k_tile_bwd", (k_tile_bwd<Src, false>), dim3(g.tile_b_blocks), dim3(kBwdThreads),
                        (size_t)g.max_tile_bins_b * 8, st, src, params, part, n_slots,
                        lane_hist ? (float *)nullptr : grad_refl, n_mat);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (g.row_blocks > 0) {   // range-normalised frames: dL/dQ per bin before the return gather
        OSIM_LAUNCH("k_rownorm_bwd", (k_rownorm_bwd<Src>), dim3(g.row_blocks), dim3(kBlock),
                    (size_t)g.max_n_az * sizeof(double), st, src, params, part, polar_blocks + g.ret_blocks, n_slots);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int uw_blocks = uwb ? uwb->blocks : 0;
    size_t lds = lane_hist ? (size_t)n_mat * 12 : 0;
    if (lds < (size_t)3 * (kBlock / kWave) * 8) lds = (size_t)3 * (kBlock / kWave) * 8;
    // the camera workgroups would reserve the same LDS: fused only while it
    // still leaves room for eight of them per CU
    const bool fuse = uw_blocks > 0 && lds <= kFuseLdsBytes;
    double *rp = lane_hist ? refl_part : nullptr;
    float *ga = lane_hist ? nullptr : grad_refl;
    if (fuse) {
        OSIM_DISPATCH_R(g.ret_chunk / kBlock,
                        OSIM_LAUNCH("k_ret_uw_bwd", (k_ret_uw_bwd<Src, RR>), dim3(g.ret_blocks + uw_blocks),
                                    dim3(kBlock), lds, st, src, params, refl, n_mat, part, polar_blocks, n_slots, rp,
                                    ga, g.ret_blocks, *uwb));
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    } else {
        if (g.ret_blocks > 0) {
            OSIM_DISPATCH_R(g.ret_chunk / kBlock,
                            OSIM_LAUNCH("k_ret_bwd", (k_ret_bwd<Src, RR>), dim3(g.ret_blocks), dim3(kBlock), lds, st,
                                        src, params, refl, n_mat, part, polar_blocks, n_slots, rp, ga));
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (uw_blocks > 0) {
            e = uw_backward_table(uwb->table, uwb->n, uwb->blocks, uwb->params, uwb->part, uwb->part_row, st);
            if (e != hipSuccess) return e;
        }
    }
    // small tables are reduced here; the atomic path was zeroed by the polar
    // kernel, unless there was none (then the reduction writes zeros)
    const bool refl_blocks = lane_hist || polar_blocks == 0;
    SonarReduce a;
    a.part = part;
    a.n_slots = n_slots;
    a.n_rows = n_rows;
    a.grad_params = grad_params;
    a.refl_part = lane_hist ? refl_part : nullptr;
    a.ret_slots = g.ret_blocks;
    a.n_mat = n_mat;
    a.grad_refl = grad_refl;
    a.blocks = n_rows * OCEANSIM_SONAR_GRAD_WIDTH + (refl_blocks ? n_mat : 0);
    if (defer) {
        *defer = a;
        return hipSuccess;
    }
    OSIM_LAUNCH("k_reduce_sonar", k_reduce_sonar, dim3(a.blocks), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t sonar_forward_one(const SonarDev &f, const SonarGrid &g, const oceansim_sonar_params *params,
                             const float *refl, int n_mat, hipStream_t st) {
    return launch_fwd(One<SonarDev>{f}, g, params, refl, n_mat, st, nullptr);
}
hipError_t sonar_forward_table(const SonarDev *t, int n, const SonarGrid &g,
                               const oceansim_sonar_params *params, const float *refl, int n_mat,
                               hipStream_t st, const UwCompanion *uw) {
    return launch_fwd(Table<SonarDev>{t, n}, g, params, refl, n_mat, st, uw);
}
hipError_t sonar_fan_stencils_table(const SonarDev *t, int n, const SonarGrid &g, hipStream_t st) {
    if (n <= 0 || g.fan_blocks == 0) return hipSuccess;
    const Table<SonarDev> src{t, n};
    OSIM_LAUNCH("k_fan_cols", k_fan_cols<Table<SonarDev>>, dim3(n), dim3(kBlock), 0, st, src);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    OSIM_LAUNCH("k_fan", (k_fan<Table<SonarDev>, false>), dim3(g.fan_blocks), dim3(kBlock), 0, st, src);
    return hipGetLastError();
}

hipError_t sonar_backward_one(const SonarDev &f, const SonarGrid &g, const oceansim_sonar_params *params,
                              int n_rows, const float *refl, int n_mat, double *part, double *refl_part,
                              float *grad_params, float *grad_refl, hipStream_t st) {
    return launch_bwd(One<SonarDev>{f}, 1, g, params, n_rows, refl, n_mat, part, refl_part, grad_params,
                      grad_refl, st, nullptr, nullptr);
}
hipError_t sonar_backward_table(const SonarDev *t, int n, const SonarGrid &g,
                                const oceansim_sonar_params *params, int n_rows, const float *refl,
                                int n_mat, double *part, double *refl_part, float *grad_params,
                                float *grad_refl, hipStream_t st, SonarReduce *defer,
                                const UwBwdCompanion *uwb) {
    return launch_bwd(Table<SonarDev>{t, n}, n, g, params, n_rows, refl, n_mat, part, refl_part, grad_params,
                      grad_refl, st, defer, uwb);
}

}  // namespace osim
