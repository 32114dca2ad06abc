/*
 * OceanSim sensor image formation -- FP64 CPU ORACLE.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU library computes.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * path never does.  It shares no code, header, table or constant with the HIP
 * library: the Philox generator, the geometry and every formula below are
 * written independently of it.
 *
 * Every quantity is evaluated in IEEE double precision (g++/gcc -O2, no
 * -ffast-math).  Inputs that the GPU receives as float are promoted exactly.
 *
 * Paper: "OceanSim: A GPU-Accelerated Underwater Robot Perception Simulation
 * Framework" (arXiv 2503.01074).
 *   - Camera model: Sec. III-A.1, Eq. (1).
 *   - Sonar return intensity: Sec. III-A.2, Eq. (2).
 *   - Range/azimuth binning by summation: Sec. III-A.2 (text after Eq. 2).
 *   - Additive speckle: Eq. (3)-(4); multiplicative speckle: Eq. (5)-(6).
 *   - 130 deg / 20 deg field of view defaults: Sec. III-A.2, last paragraph.
 * Readings where the paper is silent (gain, two-way path factor, gamma
 * speckle, RNG counter layout, fan geometry, range-wise normalisation) are listed in the design notes
 * and restated at each function below.
 *
 * Parity status per function:
 *   orc_philox4x32_10   pinned (published known-answer vectors)
 *   orc_sonar_forward   pinned (closed forms, brute-force bins, moments;
 *                       range-wise normalisation: row peaks, empty and
 *                       negative rows, gain and scale invariance)
 *   orc_sonar_backward  pinned (FP64 central differences of the forward,
 *                       with and without the range-wise normalisation)
 *   orc_fan_forward     pinned (constant / linear fields, symmetry)
 *   orc_fan_adjoint     pinned (adjoint identity against orc_fan_forward)
 *   orc_uw_forward      pinned (Eq. 1 special cases)
 *   orc_uw_backward     pinned (FP64 central differences)
 *   orc_barometer       pinned (hydrostatic closed forms, noise law)
 *   orc_raycast         pinned (closed forms: planes, boxes, a sphere's
 *                       tessellation; rays that miss; hit ordering)
 *   orc_dvl             pinned (Janus geometry, exact recovery without
 *                       noise, least squares against a library solver,
 *                       dropout counts, the measurement schedule in closed
 *                       form for constant ranges)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Four 32-bit counter words, two 32-bit key      */
/* words, ten rounds.  Each round multiplies counter words 0 and 2 by fixed  */
/* 32-bit constants, keeps both halves of the 64-bit products, and permutes  */
/* and xors them with the other counter words and the round key; the key is  */
/* bumped by two Weyl constants between rounds.                              */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = M0 * (uint64_t)c0;
        uint64_t p1 = M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_philox_many(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i)
        orc_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

/* A 32-bit word to a uniform in (0, 1]: keep the top 24 bits, add one, scale
 * by 2^-24.  Exact in both float and double, never zero (so log is finite). */
static double orc_uniform(uint32_t w)
{
    return ((double)(w >> 8) + 1.0) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------------- */
/* Sonar configuration.                                                      */
/* ------------------------------------------------------------------------- */
enum { ORC_SPECKLE_OFF = 0, ORC_SPECKLE_PAPER = 1, ORC_SPECKLE_GAMMA = 2 };

typedef struct {
    /* polar grid and field of view (Sec. III-A.2: 130 deg x 20 deg) */
    double r_min, r_max;   /* metres, grid spans [r_min, r_max)            */
    double fov_az, fov_el; /* radians, full angles centred on boresight    */
    double kappa;          /* path factor: exp(-kappa*alpha*r), 2 = two-way */
    /* physical parameters */
    double alpha;          /* Eq. 2 attenuation coefficient [1/m]           */
    double gain;           /* scalar gain applied after binning             */
    double sigma_phi;      /* Eq. 3 beam-pattern parameter [rad^2]          */
    double sigma_sa;       /* Eq. 4 Rayleigh parameter                      */
    double sigma_sm;       /* Eq. 6 Gaussian standard deviation             */
    int32_t n_range, n_azimuth;
    int32_t fan_h, fan_w;
    int32_t speckle_mode;  /* ORC_SPECKLE_*                                 */
    int32_t gamma_k;       /* shape of the gamma speckle (integer 1..8)     */
    uint32_t seed_lo, seed_hi, frame_id;
    double fan_band;       /* ambiguity band, in units of the pixel size    */
    int32_t range_norm;    /* 1: range-wise normalisation after the gain    */
} orc_sonar_cfg;

/* ------------------------------------------------------------------------- */
/* Per-return geometry and intensity, Eq. (2), plus the bin it falls in.     */
/* Sensor frame: x forward, y left, z up.  Azimuth phi = atan2(y, x).  A     */
/* return counts only if it is a hit (mat >= 0), lies in [r_min, r_max),     */
/* in [-fov_az/2, fov_az/2) and within the elevation cone                    */
/* |z| <= r sin(fov_el/2).  Returns the bin (i*N_phi + j) or -1.             */
/* ------------------------------------------------------------------------- */
static int64_t orc_return_bin(const orc_sonar_cfg *c, double x, double y, double z,
                              int32_t mat, double *r_out)
{
    if (mat < 0) return -1;
    double r = sqrt(x * x + y * y + z * z);
    *r_out = r;
    if (!(r > 0.0)) return -1;
    double phi = atan2(y, x);
    if (!(r >= c->r_min && r < c->r_max)) return -1;
    if (!(phi >= -0.5 * c->fov_az && phi < 0.5 * c->fov_az)) return -1;
    if (!(fabs(z) <= r * sin(0.5 * c->fov_el))) return -1;
    int64_t i = (int64_t)floor((r - c->r_min) * c->n_range / (c->r_max - c->r_min));
    int64_t j = (int64_t)floor((phi + 0.5 * c->fov_az) * c->n_azimuth / c->fov_az);
    /* r < r_max and phi < fov_az/2 were tested above; an index equal to N can
     * only come from rounding in the last place, and belongs to the last bin */
    if (i > c->n_range - 1) i = c->n_range - 1;
    if (j > c->n_azimuth - 1) j = c->n_azimuth - 1;
    return i * c->n_azimuth + j;
}

/* Eq. (2): I = A_r * ( -v_in/|v_in| . v_n/|v_n| ) * exp(-kappa * alpha * r).
 * v_in points from the sensor to the return, i.e. v_in = (x, y, z).  A
 * back-facing normal (negative cosine) returns nothing; a zero normal gives 0.
 * cos_out receives the clamped cosine and att_out the exponential factor.   */
static double orc_return_intensity(const orc_sonar_cfg *c, double x, double y, double z,
                                   double nx, double ny, double nz, double r, double refl,
                                   double *cos_out, double *att_out)
{
    double nn = sqrt(nx * nx + ny * ny + nz * nz);
    double cosg = 0.0;
    if (nn > 0.0) cosg = -(x * nx + y * ny + z * nz) / (r * nn);
    if (cosg < 0.0) cosg = 0.0;
    double att = exp(-c->kappa * c->alpha * r);
    *cos_out = cosg;
    *att_out = att;
    return refl * cosg * att;
}

/* Bin centres: r_i = r_min + (i + 1/2) dr, phi_j = -fov/2 + (j + 1/2) dphi.  */
static double orc_bin_range(const orc_sonar_cfg *c, int i)
{
    double dr = (c->r_max - c->r_min) / c->n_range;
    return c->r_min + (i + 0.5) * dr;
}
static double orc_bin_azimuth(const orc_sonar_cfg *c, int j)
{
    double dphi = c->fov_az / c->n_azimuth;
    return -0.5 * c->fov_az + (j + 0.5) * dphi;
}

/* ------------------------------------------------------------------------- */
/* Speckle draws for bin b (linear index i*N_phi + j) of one frame.          */
/*   rayleigh: unit-scale Rayleigh variate sqrt(-2 ln u_A); Eq. (4) then     */
/*             reads w_sa = sigma_sa * rayleigh.                             */
/*   gauss   : standard normal (Box-Muller, cosine branch); Eq. (6) reads    */
/*             w_sm = sigma_sm * gauss.                                      */
/*   gamma_m : Gamma(k, 1/k) variate -(1/k) ln(u_1 ... u_k) (mean 1).        */
/* Counter layout (key = (seed_lo, seed_hi)):                                */
/*   additive      ctr = (b / 4, frame_id, 0, 0), word b % 4                  */
/*   gaussian      ctr = (b / 2, frame_id, 1, 0), words 2(b%2), 2(b%2)+1      */
/*   gamma group g ctr = (b, frame_id, 2, g), words 0..3 -> u_{4g+1..4g+4}    */
/* ------------------------------------------------------------------------- */
static void orc_speckle_draws(const orc_sonar_cfg *c, uint32_t b,
                              double *rayleigh, double *gauss, double *gamma_m)
{
    uint32_t key[2] = { c->seed_lo, c->seed_hi };
    uint32_t out[4];

    uint32_t ca[4] = { b / 4u, c->frame_id, 0u, 0u };
    orc_philox4x32_10(ca, key, out);
    double ua = orc_uniform(out[b % 4u]);
    *rayleigh = sqrt(-2.0 * log(ua));

    uint32_t cg[4] = { b / 2u, c->frame_id, 1u, 0u };
    orc_philox4x32_10(cg, key, out);
    double u0 = orc_uniform(out[2u * (b % 2u)]);
    double u1 = orc_uniform(out[2u * (b % 2u) + 1u]);
    *gauss = sqrt(-2.0 * log(u0)) * cos(2.0 * ORC_PI * u1);

    double prod = 1.0;
    int k = c->gamma_k;
    for (int g = 0; 4 * g < k; ++g) {
        uint32_t cm[4] = { b, c->frame_id, 2u, (uint32_t)g };
        orc_philox4x32_10(cm, key, out);
        for (int w = 0; w < 4 && 4 * g + w < k; ++w) prod *= orc_uniform(out[w]);
    }
    *gamma_m = (k > 0) ? -log(prod) / k : 1.0;
}

/* Additive term of Eq. (3) and the multiplicative factor of Eq. (5) for one
 * bin.  OFF mode: additive 0, factor 1 (the speckle stage is skipped).
 * PAPER: factor 0.5 + w_sm (Eq. 5-6).  GAMMA: factor ~ Gamma(k, 1/k).       */
static void orc_speckle_terms(const orc_sonar_cfg *c, int i, int j, double *add, double *mul,
                              double *rayleigh_out, double *gauss_out)
{
    if (c->speckle_mode == ORC_SPECKLE_OFF) {
        *add = 0.0; *mul = 1.0;
        if (rayleigh_out) *rayleigh_out = 0.0;
        if (gauss_out) *gauss_out = 0.0;
        return;
    }
    uint32_t b = (uint32_t)((int64_t)i * c->n_azimuth + j);
    double rayleigh, gauss, gamma_m;
    orc_speckle_draws(c, b, &rayleigh, &gauss, &gamma_m);
    double ri = orc_bin_range(c, i);
    double pj = orc_bin_azimuth(c, j);
    double w_sa = c->sigma_sa * rayleigh;                                /* Eq. 4 */
    *add = (ri * ri) / (c->r_max * c->r_max) *
           (1.0 + 0.5 * exp(-(pj * pj) / c->sigma_phi) * w_sa);           /* Eq. 3 */
    if (c->speckle_mode == ORC_SPECKLE_PAPER)
        *mul = 0.5 + c->sigma_sm * gauss;                                /* Eq. 5-6 */
    else
        *mul = gamma_m;
    if (rayleigh_out) *rayleigh_out = rayleigh;
    if (gauss_out) *gauss_out = gauss;
}

/* Exposed for the distribution tests: additive and multiplicative speckle
 * factors of every bin of one frame, row-major [n_range][n_azimuth].        */
void orc_speckle_fields(const orc_sonar_cfg *c, double *add, double *mul)
{
    int64_t nb = (int64_t)c->n_range * c->n_azimuth;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        int i = (int)(b / c->n_azimuth), j = (int)(b % c->n_azimuth);
        orc_speckle_terms(c, i, j, add + b, mul + b, NULL, NULL);
    }
}

/* ------------------------------------------------------------------------- */
/* Polar -> Cartesian fan.                                                   */
/* Apex at the bottom centre of an H x W image, boresight pointing up, the   */
/* sensor's left on the image's left.  Square pixels of side                 */
/*   s = max(r_max / H, 2 r_max sin(fov/2) / W)      (fov <= pi),            */
/* pixel centres at half-integers.  Pixel (v, u) sits at                     */
/*   x_c = (u + 1/2 - W/2) s,  y_c = (H - v - 1/2) s,                        */
/*   rho = hypot(x_c, y_c),    phi = atan2(-x_c, y_c).                       */
/* Outside r_min <= rho <= r_max, |phi| <= fov/2 the pixel is 0.  Inside, it */
/* is the bilinear interpolation of the polar image on its bin centres, with */
/* the fractional coordinates clamped to the grid (clamp to edge).           */
/* ------------------------------------------------------------------------- */
typedef struct {
    int inside;
    int i0, i1, j0, j1;
    double t, s;          /* range and azimuth weights of i1 and j1 */
    int ambiguous;
} orc_fan_px;

static void orc_fan_pixel(const orc_sonar_cfg *c, int v, int u, orc_fan_px *p)
{
    int H = c->fan_h, W = c->fan_w;
    double half = 0.5 * c->fov_az;
    double s1 = c->r_max / H;
    double s2 = 2.0 * c->r_max * sin(half) / W;
    double s = s1 > s2 ? s1 : s2;
    double xc = (u + 0.5 - 0.5 * W) * s;
    double yc = (H - v - 0.5) * s;
    double rho = hypot(xc, yc);
    double phi = atan2(-xc, yc);

    double band = c->fan_band * s;
    p->ambiguous = (fabs(rho - c->r_min) < band) || (fabs(rho - c->r_max) < band) ||
                   (fabs(fabs(phi) - half) * rho < band);
    p->inside = (rho >= c->r_min && rho <= c->r_max && phi >= -half && phi <= half);
    p->i0 = p->i1 = p->j0 = p->j1 = 0;
    p->t = p->s = 0.0;
    if (!p->inside) return;

    int Nr = c->n_range, Np = c->n_azimuth;
    double dr = (c->r_max - c->r_min) / Nr;
    double dphi = c->fov_az / Np;
    double fr = (rho - c->r_min) / dr - 0.5;
    double fp = (phi + half) / dphi - 0.5;
    if (fr < 0.0) fr = 0.0;
    if (fr > Nr - 1) fr = Nr - 1;
    if (fp < 0.0) fp = 0.0;
    if (fp > Np - 1) fp = Np - 1;
    if (Nr == 1) { p->i0 = p->i1 = 0; p->t = 0.0; }
    else {
        int i0 = (int)floor(fr);
        if (i0 > Nr - 2) i0 = Nr - 2;
        p->i0 = i0; p->i1 = i0 + 1; p->t = fr - i0;
    }
    if (Np == 1) { p->j0 = p->j1 = 0; p->s = 0.0; }
    else {
        int j0 = (int)floor(fp);
        if (j0 > Np - 2) j0 = Np - 2;
        p->j0 = j0; p->j1 = j0 + 1; p->s = fp - j0;
    }
}

void orc_fan_forward(const orc_sonar_cfg *c, const double *img, double *fan, uint8_t *ambiguous)
{
    int H = c->fan_h, W = c->fan_w, Np = c->n_azimuth;
#pragma omp parallel for schedule(static)
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            orc_fan_px p;
            orc_fan_pixel(c, v, u, &p);
            double val = 0.0;
            if (p.inside) {
                double a = img[(int64_t)p.i0 * Np + p.j0], b = img[(int64_t)p.i0 * Np + p.j1];
                double d = img[(int64_t)p.i1 * Np + p.j0], e = img[(int64_t)p.i1 * Np + p.j1];
                val = (1 - p.t) * (1 - p.s) * a + (1 - p.t) * p.s * b +
                      p.t * (1 - p.s) * d + p.t * p.s * e;
            }
            fan[(int64_t)v * W + u] = val;
            if (ambiguous) ambiguous[(int64_t)v * W + u] = (uint8_t)p.ambiguous;
        }
    }
}

/* Transpose of orc_fan_forward: every pixel's gradient is scattered, with its
 * four bilinear weights, onto the bins it was interpolated from.  Plain
 * sequential scatter in pixel order. */
void orc_fan_adjoint(const orc_sonar_cfg *c, const double *g_fan, double *g_img)
{
    int H = c->fan_h, W = c->fan_w, Np = c->n_azimuth;
    memset(g_img, 0, sizeof(double) * (size_t)c->n_range * Np);
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            orc_fan_px p;
            orc_fan_pixel(c, v, u, &p);
            if (!p.inside) continue;
            double g = g_fan[(int64_t)v * W + u];
            g_img[(int64_t)p.i0 * Np + p.j0] += (1 - p.t) * (1 - p.s) * g;
            g_img[(int64_t)p.i0 * Np + p.j1] += (1 - p.t) * p.s * g;
            g_img[(int64_t)p.i1 * Np + p.j0] += p.t * (1 - p.s) * g;
            g_img[(int64_t)p.i1 * Np + p.j1] += p.t * p.s * g;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Sonar forward for one frame.                                              */
/*   1. per return: Eq. (2) intensity and its bin;                           */
/*   2. binning: P[b] = sum of the intensities that fall in bin b;           */
/*   3. gain: Q = G P;                                                       */
/*   4. speckle, Eq. (3)-(6): out = Q m + a (OFF: out = Q);                  */
/*   5. optional fan of out.                                                 */
/* Any output pointer may be NULL.  refl has n_mat entries; a material id at */
/* or beyond n_mat is treated as a miss.  Returns 0.                         */
/* ------------------------------------------------------------------------- */
/* ------------------------------------------------------------------------- */
/* Range-wise normalisation (Sec. III-A.2 mentions normalising the binned    */
/* image range by range and gives no formula).  Reading: after the gain and  */
/* before the speckle, each range row i of Q = G P is divided by its maximum */
/* over azimuth, m_i = max_j Q_ij, when m_i > 0; a row whose maximum is 0 or */
/* negative (an empty row in particular) is left as it is.  NaN entries are  */
/* skipped by the maximum.  j*_i is the first column attaining m_i: the      */
/* subgradient of the maximum is taken there.                                */
/* ------------------------------------------------------------------------- */
static void orc_row_max(const double *Q, int n, double *m, int *jstar)
{
    double best = -INFINITY;
    int at = -1;
    for (int j = 0; j < n; ++j)
        if (Q[j] > best) {
            best = Q[j];
            at = j;
        }
    *m = best;
    *jstar = at;
}

int orc_sonar_forward(const orc_sonar_cfg *c, int64_t n,
                      const float *x, const float *y, const float *z,
                      const float *nx, const float *ny, const float *nz,
                      const int32_t *mat, const float *refl, int32_t n_mat,
                      double *intensity, int32_t *bins, double *P, double *out,
                      double *fan, uint8_t *fan_ambiguous)
{
    int64_t nb = (int64_t)c->n_range * c->n_azimuth;
    double *Pw = P ? P : (double *)malloc(sizeof(double) * nb);
    double *Ow = out ? out : (double *)malloc(sizeof(double) * nb);
    int64_t *bk = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    double *Ik = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));

    /* step 1 */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        int32_t m = mat[k];
        if (m >= n_mat) m = -1;
        double r = 0.0, cosg, att;
        int64_t b = orc_return_bin(c, x[k], y[k], z[k], m, &r);
        double I = 0.0;
        if (b >= 0)
            I = orc_return_intensity(c, x[k], y[k], z[k], nx[k], ny[k], nz[k], r, refl[m],
                                     &cosg, &att);
        bk[k] = b;
        Ik[k] = I;
    }
    /* step 2: sum in return order */
    for (int64_t b = 0; b < nb; ++b) Pw[b] = 0.0;
    for (int64_t k = 0; k < n; ++k)
        if (bk[k] >= 0) Pw[bk[k]] += Ik[k];
    /* step 3: gain, then (optionally) the range-wise normalisation; the
       normalised image goes through Ow */
    for (int64_t b = 0; b < nb; ++b) Ow[b] = c->gain * Pw[b];
    if (c->range_norm)
        for (int i = 0; i < c->n_range; ++i) {
            double *row = Ow + (int64_t)i * c->n_azimuth;
            double m;
            int js;
            orc_row_max(row, c->n_azimuth, &m, &js);
            if (m > 0.0)
                for (int j = 0; j < c->n_azimuth; ++j) row[j] /= m;
        }
    /* step 4 */
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        int i = (int)(b / c->n_azimuth), j = (int)(b % c->n_azimuth);
        double add, mul;
        orc_speckle_terms(c, i, j, &add, &mul, NULL, NULL);
        double Q = Ow[b];
        Ow[b] = (c->speckle_mode == ORC_SPECKLE_OFF) ? Q : Q * mul + add;
    }
    /* step 5 */
    if (fan && c->fan_h > 0 && c->fan_w > 0) orc_fan_forward(c, Ow, fan, fan_ambiguous);

    for (int64_t k = 0; k < n; ++k) {
        if (bins) bins[k] = (int32_t)bk[k];
        if (intensity) intensity[k] = Ik[k];
    }
    free(bk);
    free(Ik);
    if (!P) free(Pw);
    if (!out) free(Ow);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Sonar backward for one frame: gradient of                                 */
/*   L = <g_polar, out> + <g_fan, fan>                                       */
/* with respect to refl[n_mat] (accumulated into g_refl) and the parameters  */
/*   g_par[0] alpha, [1] gain, [2] sigma_phi, [3] sigma_sa, [4] sigma_sm     */
/* (accumulated).  The forward is recomputed; nothing is saved between calls.*/
/* Either gradient input may be NULL (zero).  g_out (optional) receives the  */
/* gradient of L with respect to the polar output, [n_range][n_azimuth].     */
/* g_refl_abs / g_par_abs (optional) accumulate the sums of the magnitudes   */
/* of the terms each gradient component adds up: the condition of that sum, */
/* against which a float32 evaluation's rounding error is measured.  The    */
/* terms are taken fully expanded: the polar-output gradient of a bin is    */
/* itself a sum (the fan's pixels that read the bin, weighted, plus the     */
/* direct polar gradient), so the magnitudes use that sum's own magnitude   */
/* sum, the fan adjoint of |g_fan| plus |g_polar|, in its place.            */
/* ------------------------------------------------------------------------- */
int orc_sonar_backward(const orc_sonar_cfg *c, int64_t n,
                       const float *x, const float *y, const float *z,
                       const float *nx, const float *ny, const float *nz,
                       const int32_t *mat, const float *refl, int32_t n_mat,
                       const double *g_polar, const double *g_fan,
                       double *g_refl, double *g_par, double *g_out,
                       double *g_refl_abs, double *g_par_abs)
{
    int64_t nb = (int64_t)c->n_range * c->n_azimuth;
    double *P = (double *)malloc(sizeof(double) * nb);
    double *gO = (double *)malloc(sizeof(double) * nb);
    double *gP = (double *)malloc(sizeof(double) * nb);
    orc_sonar_forward(c, n, x, y, z, nx, ny, nz, mat, refl, n_mat, NULL, NULL, P, NULL, NULL,
                      NULL);

    /* adjoint of step 5 (fan) plus the direct polar gradient */
    if (g_fan && c->fan_h > 0 && c->fan_w > 0) orc_fan_adjoint(c, g_fan, gO);
    else memset(gO, 0, sizeof(double) * nb);
    if (g_polar)
        for (int64_t b = 0; b < nb; ++b) gO[b] += g_polar[b];
    if (g_out) memcpy(g_out, gO, sizeof(double) * nb);
    /* magnitude sum of each bin's output gradient (for the conditions) */
    double *gOa = NULL;
    if (g_refl_abs || g_par_abs) {
        gOa = (double *)malloc(sizeof(double) * nb);
        if (g_fan && c->fan_h > 0 && c->fan_w > 0) {
            int64_t npx = (int64_t)c->fan_h * c->fan_w;
            double *af = (double *)malloc(sizeof(double) * npx);
            for (int64_t q = 0; q < npx; ++q) af[q] = fabs(g_fan[q]);
            orc_fan_adjoint(c, af, gOa);
            free(af);
        } else {
            memset(gOa, 0, sizeof(double) * nb);
        }
        if (g_polar)
            for (int64_t b = 0; b < nb; ++b) gOa[b] += fabs(g_polar[b]);
    }

    /* the normalisation of step 3: per row, the maximum and where it is
       (scale[i] = 1 / m_i for a normalised row, else 1) */
    double *scale = (double *)malloc(sizeof(double) * c->n_range);
    int *jst = (int *)malloc(sizeof(int) * c->n_range);
    {
        double *row = (double *)malloc(sizeof(double) * c->n_azimuth);
        for (int i = 0; i < c->n_range; ++i) {
            for (int j = 0; j < c->n_azimuth; ++j) row[j] = c->gain * P[(int64_t)i * c->n_azimuth + j];
            double m;
            orc_row_max(row, c->n_azimuth, &m, &jst[i]);
            scale[i] = (c->range_norm && m > 0.0) ? 1.0 / m : 1.0;
            if (!(c->range_norm && m > 0.0)) jst[i] = -1;
        }
        free(row);
    }

    /* adjoint of step 4: gN[b] = dL/d(normalised image) (gNa: magnitude sums) */
    double *gN = (double *)malloc(sizeof(double) * nb);
    double *gNa = gOa ? (double *)malloc(sizeof(double) * nb) : NULL;
    double *gPa = gOa ? (double *)malloc(sizeof(double) * nb) : NULL;
    double gG = 0.0, gsphi = 0.0, gssa = 0.0, gssm = 0.0;
    double aG = 0.0, asphi = 0.0, assa = 0.0, assm = 0.0, aalpha = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
        int i = (int)(b / c->n_azimuth), j = (int)(b % c->n_azimuth);
        double Q = c->gain * P[b] * scale[i];   /* the (normalised) image the speckle acts on */
        double ga = gOa ? gOa[b] : 0.0;   /* magnitude sum of gO[b] */
        double gQ, mulv = 1.0;
        if (c->speckle_mode == ORC_SPECKLE_OFF) {
            gQ = gO[b];
        } else {
            double add, mul, rayleigh, gauss;
            orc_speckle_terms(c, i, j, &add, &mul, &rayleigh, &gauss);
            gQ = gO[b] * mul;
            mulv = mul;
            double ri = orc_bin_range(c, i), pj = orc_bin_azimuth(c, j);
            double R = ri * ri / (c->r_max * c->r_max);
            double E = exp(-(pj * pj) / c->sigma_phi);
            /* d add / d sigma_sa and d add / d sigma_phi, from Eq. (3)-(4) */
            double fsa = R * 0.5 * E * rayleigh;
            double fphi = R * 0.5 * c->sigma_sa * rayleigh * E * (pj * pj) / (c->sigma_phi * c->sigma_phi);
            gssa += gO[b] * fsa;
            gsphi += gO[b] * fphi;
            assa += ga * fabs(fsa);
            asphi += ga * fabs(fphi);
            if (c->speckle_mode == ORC_SPECKLE_PAPER) {
                gssm += gO[b] * Q * gauss;
                assm += ga * fabs(Q * gauss);
            }
        }
        gN[b] = gQ;
        if (gNa) gNa[b] = ga * fabs(mulv);
    }
    /* adjoint of step 3: a normalised row N_j = Q_j / Q_j* gives
       dL/dQ_k = gN_k / m - [k = j*] sum_j gN_j Q_j / m^2; then Q = G P */
    for (int i = 0; i < c->n_range; ++i) {
        const int64_t r0 = (int64_t)i * c->n_azimuth;
        double S = 0.0, Sa = 0.0;
        if (jst[i] >= 0)
            for (int j = 0; j < c->n_azimuth; ++j) {
                S += gN[r0 + j] * (c->gain * P[r0 + j]);
                if (gNa) Sa += gNa[r0 + j] * fabs(c->gain * P[r0 + j]);
            }
        for (int j = 0; j < c->n_azimuth; ++j) {
            const int64_t b = r0 + j;
            double gQ = gN[b] * scale[i], gQa = gNa ? gNa[b] * fabs(scale[i]) : 0.0;
            if (j == jst[i]) {
                gQ -= S * scale[i] * scale[i];
                gQa += Sa * scale[i] * scale[i];
            }
            gG += gQ * P[b];
            aG += gQa * fabs(P[b]);
            gP[b] = c->gain * gQ;
            if (gPa) gPa[b] = gQa * fabs(c->gain);
        }
    }
    free(gN);
    free(gNa);
    free(scale);
    free(jst);

    /* adjoint of steps 1-2: each return reads the gradient of its bin */
    double galpha = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        int32_t m = mat[k];
        if (m >= n_mat) m = -1;
        double r = 0.0, cosg, att;
        int64_t b = orc_return_bin(c, x[k], y[k], z[k], m, &r);
        if (b < 0) continue;
        double I = orc_return_intensity(c, x[k], y[k], z[k], nx[k], ny[k], nz[k], r, refl[m],
                                        &cosg, &att);
        double gI = gP[b];
        double gIa = gPa ? gPa[b] : 0.0;
        g_refl[m] += gI * cosg * att;
        galpha += gI * I * (-c->kappa * r);
        if (g_refl_abs) g_refl_abs[m] += gIa * fabs(cosg * att);
        aalpha += gIa * fabs(I * c->kappa * r);
    }
    g_par[0] += galpha;
    g_par[1] += gG;
    g_par[2] += gsphi;
    g_par[3] += gssa;
    g_par[4] += gssm;
    if (g_par_abs) {
        g_par_abs[0] += aalpha;
        g_par_abs[1] += aG;
        g_par_abs[2] += asphi;
        g_par_abs[3] += assa;
        g_par_abs[4] += assm;
    }
    free(P);
    free(gO);
    free(gP);
    free(gOa);
    free(gPa);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Underwater image formation, Eq. (1), per pixel and colour channel c:      */
/*   I_c = J_c exp(-beta_D,c d) + B_inf,c (1 - exp(-beta_B,c d)).            */
/* (beta_D is the paper's beta_attn, beta_B its beta_bs.)  The product       */
/* beta*d is taken as 0 when beta = 0, so an infinite depth with a zero      */
/* coefficient leaves the term untouched.  1 - exp(-x) is evaluated as       */
/* -expm1(-x).  Images are planar [3][npix]; depth is [npix].                */
/* ------------------------------------------------------------------------- */
static double orc_beta_d(double beta, double d)
{
    return beta == 0.0 ? 0.0 : beta * d;
}

void orc_uw_forward(int64_t npix, const float *J, const float *depth, const double *beta_d,
                    const double *beta_b, const double *b_inf, double *out)
{
    for (int ch = 0; ch < 3; ++ch) {
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < npix; ++p) {
            double d = depth[p];
            double xd = orc_beta_d(beta_d[ch], d);
            double xb = orc_beta_d(beta_b[ch], d);
            out[ch * npix + p] = (double)J[ch * npix + p] * exp(-xd) + b_inf[ch] * (-expm1(-xb));
        }
    }
}

/* Gradient of L = <g_out, I> with respect to beta_D[3], beta_B[3], B_inf[3]
 * (accumulated into g_par[0..2], [3..5], [6..8]) and optionally to J and d
 * (overwritten).  Differentiating Eq. (1) with T = exp(-beta_D d) and
 * S = exp(-beta_B d):
 *   dI/dbeta_D = -J T d,  dI/dbeta_B = B_inf S d,  dI/dB_inf = 1 - S,
 *   dI/dJ = T,            dI/dd = -beta_D J T + B_inf beta_B S.              */
void orc_uw_backward(int64_t npix, const float *J, const float *depth, const double *beta_d,
                     const double *beta_b, const double *b_inf, const double *g_out,
                     double *g_par, double *g_J, double *g_d, double *g_par_abs)
{
    if (g_d)
        for (int64_t p = 0; p < npix; ++p) g_d[p] = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
        double s_bd = 0.0, s_bb = 0.0, s_binf = 0.0;
        double a_bd = 0.0, a_bb = 0.0, a_binf = 0.0;
        for (int64_t p = 0; p < npix; ++p) {
            double d = depth[p];
            double T = exp(-orc_beta_d(beta_d[ch], d));
            double S = exp(-orc_beta_d(beta_b[ch], d));
            double one_minus_S = -expm1(-orc_beta_d(beta_b[ch], d));
            double g = g_out[ch * npix + p];
            double Jv = J[ch * npix + p];
            /* the d-weighted terms vanish where T or S does (0 * inf := 0) */
            if (T != 0.0) {
                s_bd += g * (-Jv * T * d);
                a_bd += fabs(g * Jv * T * d);
            }
            if (S != 0.0) {
                s_bb += g * (b_inf[ch] * S * d);
                a_bb += fabs(g * b_inf[ch] * S * d);
            }
            s_binf += g * one_minus_S;
            a_binf += fabs(g * one_minus_S);
            if (g_J) g_J[ch * npix + p] = g * T;
            if (g_d) g_d[p] += g * (-beta_d[ch] * Jv * T + b_inf[ch] * beta_b[ch] * S);
        }
        g_par[ch] += s_bd;
        g_par[3 + ch] += s_bb;
        g_par[6 + ch] += s_binf;
        if (g_par_abs) {
            g_par_abs[ch] += a_bd;
            g_par_abs[3 + ch] += a_bb;
            g_par_abs[6 + ch] += a_binf;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Navigation sensors of Sec. III-A (no equations are printed; the readings  */
/* are stated here and in the design notes).                                 */
/* ------------------------------------------------------------------------- */

/* A standard normal from two counter words: Box-Muller, cosine branch. */
static double orc_gauss(uint32_t w0, uint32_t w1)
{
    return sqrt(-2.0 * log(orc_uniform(w0))) * cos(2.0 * ORC_PI * orc_uniform(w1));
}

/* Barometer: the pressure at depth d below the free surface is the
 * atmospheric pressure plus the weight of the water column,
 *   P = p_atm + rho g max(d, 0) + sigma z,
 * with optional Gaussian noise z ~ N(0, 1) (sigma = 0: none).  Sample k
 * draws z from Philox4x32-10 counter (k mod 2^32, k / 2^32, 3, 0), words 0
 * and 1, under key (seed_lo, seed_hi). */
void orc_barometer(int64_t n, const float *depth, double p_atm, double rho, double g, double sigma,
                   uint32_t seed_lo, uint32_t seed_hi, double *pressure)
{
    const uint32_t key[2] = {seed_lo, seed_hi};
    for (int64_t k = 0; k < n; ++k) {
        double d = depth[k];
        double col = d > 0.0 ? rho * g * d : 0.0;
        double z = 0.0;
        if (sigma != 0.0) {
            uint32_t ctr[4] = {(uint32_t)k, (uint32_t)((uint64_t)k >> 32), 3u, 0u}, w[4];
            orc_philox4x32_10(ctr, key, w);
            z = orc_gauss(w[0], w[1]);
        }
        pressure[k] = p_atm + col + sigma * z;
    }
}

/* Beam i of a four-beam convex Janus array, in the sensor frame (x forward,
 * y left, z up): tilted by `janus` from the downward vertical, at azimuth
 * 45 + 90 i degrees. */
void orc_dvl_beam(int i, double janus, double b[3])
{
    double psi = ORC_PI / 4.0 + (ORC_PI / 2.0) * (double)i;
    b[0] = sin(janus) * cos(psi);
    b[1] = sin(janus) * sin(psi);
    b[2] = -cos(janus);
}

/* DVL over n_ticks ticks (times t[k], seconds, increasing) for n_inst
 * independent instances.  Inputs per (tick k, instance n): the slant ranges
 * of the four beams to the bottom, ranges[(k n_inst + n) 4 + i] (metres; not
 * finite or outside [range_min, range_max]: no return on that beam), and the
 * true velocity vel[(k n_inst + n) 3 + c] (sensor frame, m/s).
 *
 *  - Adaptive rate: the DVL measures when the time since its last
 *    measurement reaches the ping period of the current altitude,
 *      T = max(period_min, pings_per_output * 2 r_ref / sound_speed),
 *    r_ref the largest valid beam range (range_max when no beam is valid),
 *    i.e. the two-way travel time of the farthest beam times the pings
 *    averaged into one output; the first tick always measures.
 *  - Measurement: each valid beam reports the along-beam velocity
 *    u_i = b_i . v + sigma_v z_i, z_i ~ N(0, 1) from Philox4x32-10 counter
 *    (k, n, 4, i / 2), words 2 (i mod 2) and 2 (i mod 2) + 1 (Box-Muller,
 *    cosine branch), key (seed_lo, seed_hi); the velocity is the least-
 *    squares solution of b_i . x = u_i over the valid beams.
 *  - Dropout: with fewer than min_beams valid beams the measurement is
 *    invalid.
 * Output status[k n_inst + n]: 0 no measurement at this tick, 1 a velocity,
 * 2 dropout; vout[(k n_inst + n) 3 + c] the velocity (status 1) or NaN. */
void orc_dvl(int32_t n_ticks, int32_t n_inst, const double *t, const float *ranges, const float *vel,
             double janus, double range_min, double range_max, int32_t min_beams, double sigma_v,
             double sound_speed, double pings_per_output, double period_min, uint32_t seed_lo,
             uint32_t seed_hi, double *vout, int32_t *status)
{
    const uint32_t key[2] = {seed_lo, seed_hi};
    double beams[4][3];
    for (int i = 0; i < 4; ++i) orc_dvl_beam(i, janus, beams[i]);
#pragma omp parallel for schedule(static)
    for (int32_t n = 0; n < n_inst; ++n) {
        double t_last = 0.0;
        int have_last = 0;
        for (int32_t k = 0; k < n_ticks; ++k) {
            const int64_t row = (int64_t)k * n_inst + n;
            const float *r = ranges + 4 * row;
            int valid[4], nv = 0;
            double r_ref = 0.0;
            for (int i = 0; i < 4; ++i) {
                double ri = r[i];
                valid[i] = isfinite(ri) && ri >= range_min && ri <= range_max;
                if (valid[i]) {
                    ++nv;
                    if (ri > r_ref) r_ref = ri;
                }
            }
            if (nv == 0) r_ref = range_max;
            double period = pings_per_output * 2.0 * r_ref / sound_speed;
            if (period < period_min) period = period_min;
            int due = !have_last || (t[k] - t_last >= period);
            double *vo = vout + 3 * row;
            vo[0] = vo[1] = vo[2] = NAN;
            if (!due) {
                status[row] = 0;
                continue;
            }
            have_last = 1;
            t_last = t[k];
            if (nv < min_beams) {
                status[row] = 2;
                continue;
            }
            /* normal equations (B^T B) x = B^T u over the valid beams */
            double A[3][3] = {{0}}, rhs[3] = {0};
            const float *v = vel + 3 * row;
            for (int i = 0; i < 4; ++i) {
                if (!valid[i]) continue;
                double z = 0.0;
                if (sigma_v != 0.0) {
                    uint32_t ctr[4] = {(uint32_t)k, (uint32_t)n, 4u, (uint32_t)(i / 2)}, w[4];
                    orc_philox4x32_10(ctr, key, w);
                    z = orc_gauss(w[2 * (i % 2)], w[2 * (i % 2) + 1]);
                }
                double u = beams[i][0] * v[0] + beams[i][1] * v[1] + beams[i][2] * v[2] + sigma_v * z;
                for (int a = 0; a < 3; ++a) {
                    rhs[a] += beams[i][a] * u;
                    for (int c = 0; c < 3; ++c) A[a][c] += beams[i][a] * beams[i][c];
                }
            }
            /* Cramer's rule on the symmetric 3 x 3 system */
            double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                         A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                         A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
            double x[3];
            for (int c = 0; c < 3; ++c) {
                double M[3][3];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) M[a][b] = b == c ? rhs[a] : A[a][b];
                x[c] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                        M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                        M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) / det;
            }
            vo[0] = x[0];
            vo[1] = x[1];
            vo[2] = x[2];
            status[row] = 1;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Ray casting of the sonar's returns (Sec. III-A.2 obtains the returns from */
/* the renderer's ray tracing): the rays of a beam x elevation pattern from  */
/* a sensor pose against a triangle mesh, closest hit by brute force over    */
/* every triangle, in double precision.                                      */
/*                                                                           */
/* Pattern: beam b (of n_beams) at azimuth -fov_az/2 + (b + 1/2) fov_az /    */
/* n_beams, ray r (of n_rays) at elevation -fov_el/2 + (r + 1/2) fov_el /    */
/* n_rays; direction (cos el cos az, cos el sin az, sin el) in the sensor    */
/* frame (x forward, y left, z up); return k = b n_rays + r.  Pose: world =  */
/* R sensor + p (R row-major).  A hit is the nearest point with 0 < t <=     */
/* t_max on a triangle (edges included); its position is written in the     */
/* sensor frame (t d), its normal is the triangle's (v1 - v0) x (v2 - v0),   */
/* normalised and rotated into the sensor frame, and its material that of    */
/* the triangle; a miss has material -1 and zero coordinates.                */
/*                                                                           */
/* Inside test: the signed volumes s_i = d . ((v_j - o) x (v_k - o)) over    */
/* the edges (j, k) opposite each vertex i; the ray meets the triangle when  */
/* all three share the sign of their sum (which is d . n), and s_i / sum are */
/* the barycentric coordinates of the crossing point.  Unlike a solve in the */
/* triangle's own plane this stays decisive on slivers.                      */
/*                                                                           */
/* ambiguous[k] flags rays whose nearest hit lies within `band` (barycentric */
/* units) of a triangle edge, whose two nearest hits on different triangles */
/* are closer than band * t, whose nearest triangle is a sliver             */
/* (|n| < band L^2, L its longest edge) or is met at grazing incidence       */
/* (|d . n| < band |n|), whose hit lies within band * t_max of the casting   */
/* distance, or that pass within `band` of the edge of a triangle they miss  */
/* no farther than their hit (any such triangle, for a ray that misses):     */
/* there the nearest triangle, or its point and normal, is not decided by    */
/* the geometry alone at single precision.                                   */
/* ------------------------------------------------------------------------- */
void orc_raycast(int64_t n_vert, const float *vert, int64_t n_tri, const int32_t *tri, const int32_t *tri_mat,
                 const float *pos, const float *rot, int32_t n_beams, int32_t n_rays, double fov_az,
                 double fov_el, double t_max, double band, int64_t n_sel, const int64_t *sel, double *x,
                 double *y, double *z, double *nx, double *ny, double *nz, int32_t *mat, uint8_t *ambiguous)
{
    (void)n_vert;
    /* the returns k = sel[s] (s < n_sel), or all of them (sel NULL); output s */
    const int64_t n_out = sel ? n_sel : (int64_t)n_beams * n_rays;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < n_out; ++s) {
        const int64_t kk = sel ? sel[s] : s;
        const int64_t k = s;
        const int32_t b = (int32_t)(kk / n_rays), r = (int32_t)(kk % n_rays);
        const double az = -0.5 * fov_az + ((double)b + 0.5) * fov_az / n_beams;
        const double el = -0.5 * fov_el + ((double)r + 0.5) * fov_el / n_rays;
        const double ds[3] = {cos(el) * cos(az), cos(el) * sin(az), sin(el)};
        double dw[3], o[3];
        for (int i = 0; i < 3; ++i) {
            dw[i] = rot[3 * i] * ds[0] + rot[3 * i + 1] * ds[1] + rot[3 * i + 2] * ds[2];
            o[i] = pos[i];
        }
        double best = INFINITY, second = INFINITY, near = INFINITY;
        int best_amb = 0;
        int64_t best_tri = -1;
        double best_n[3] = {0, 0, 0};
        for (int64_t f = 0; f < n_tri; ++f) {
            double v[3][3];   /* vertices relative to the ray origin */
            for (int j = 0; j < 3; ++j) {
                const float *V = vert + 3 * (int64_t)tri[3 * f + j];
                for (int i = 0; i < 3; ++i) v[j][i] = (double)V[i] - o[i];
            }
            double sv[3];
            for (int j = 0; j < 3; ++j) {
                const double *P = v[(j + 1) % 3], *Q = v[(j + 2) % 3];
                const double c0 = P[1] * Q[2] - P[2] * Q[1];
                const double c1 = P[2] * Q[0] - P[0] * Q[2];
                const double c2 = P[0] * Q[1] - P[1] * Q[0];
                sv[j] = dw[0] * c0 + dw[1] * c1 + dw[2] * c2;
            }
            const double tot = sv[0] + sv[1] + sv[2];
            if (tot == 0.0) continue;   /* degenerate, or the ray runs in the plane */
            const double u0 = sv[0] / tot, u1 = sv[1] / tot, u2 = sv[2] / tot;
            const double umin = fmin(u0, fmin(u1, u2));
            if (umin < -band) continue;
            double t = 0.0;
            for (int i = 0; i < 3; ++i) t += (u0 * v[0][i] + u1 * v[1][i] + u2 * v[2][i]) * dw[i];
            if (umin < 0.0 || t > t_max) {
                /* a near miss (within band of an edge) or a hit just beyond
                 * the casting distance */
                if (t > 0.0 && t <= t_max * (1.0 + band)) near = fmin(near, t);
                continue;
            }
            if (!(t > 0.0)) continue;
            if (t < best) {
                second = best;
                best = t;
                best_tri = f;
                double e1[3], e2[3], e3[3], n[3];
                for (int i = 0; i < 3; ++i) {
                    e1[i] = v[1][i] - v[0][i];
                    e2[i] = v[2][i] - v[0][i];
                    e3[i] = v[2][i] - v[1][i];
                }
                n[0] = e1[1] * e2[2] - e1[2] * e2[1];
                n[1] = e1[2] * e2[0] - e1[0] * e2[2];
                n[2] = e1[0] * e2[1] - e1[1] * e2[0];
                const double nl = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
                const double l2 = fmax(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2],
                                       fmax(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2],
                                            e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2]));
                const double dn = n[0] * dw[0] + n[1] * dw[1] + n[2] * dw[2];
                const double margin = fmin(u0, fmin(u1, u2));
                best_amb = margin < band || nl < band * l2 || fabs(dn) < band * nl;
                for (int i = 0; i < 3; ++i) best_n[i] = nl > 0.0 ? n[i] / nl : 0.0;
            } else if (t < second) {
                second = t;
            }
        }
        if (best_tri < 0) {
            x[k] = y[k] = z[k] = nx[k] = ny[k] = nz[k] = 0.0;
            mat[k] = -1;
            ambiguous[k] = near < INFINITY;
            continue;
        }
        x[k] = best * ds[0];
        y[k] = best * ds[1];
        z[k] = best * ds[2];
        /* world normal into the sensor frame: R^T n */
        nx[k] = rot[0] * best_n[0] + rot[3] * best_n[1] + rot[6] * best_n[2];
        ny[k] = rot[1] * best_n[0] + rot[4] * best_n[1] + rot[7] * best_n[2];
        nz[k] = rot[2] * best_n[0] + rot[5] * best_n[1] + rot[8] * best_n[2];
        mat[k] = tri_mat[best_tri];
        ambiguous[k] = (best_amb || second - best < band * best || near <= best * (1.0 + band) ||
                        best > t_max * (1.0 - band)) ? 1 : 0;
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
