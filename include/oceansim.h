/*
 * oceansim.h -- C ABI of the MI355X (gfx950) OceanSim image-formation library.
 *
 * Computes, on the GPU, the data-parallel part of the sensor models of
 * "OceanSim: A GPU-Accelerated Underwater Robot Perception Simulation
 * Framework" (arXiv 2503.01074):
 *
 *   - imaging-sonar image formation from ray-cast returns (Sec. III-A.2):
 *     per-return intensity (Eq. 2), range x azimuth binning by summation,
 *     a scalar gain, speckle noise (Eq. 3-6, or a gamma-distributed
 *     multiplicative speckle), and a polar-to-Cartesian fan image;
 *   - the underwater colour image-formation model (Sec. III-A.1, Eq. 1).
 *
 * plus the adjoints of both with respect to their physical parameters.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every pointer named *_dev or held in a frame descriptor is DEVICE memory
 *    of the current HIP device.  Descriptors and sizes are host memory and are
 *    not retained after the call returns (plans excepted, see below).
 *  - The caller owns and frees every buffer.  Plain calls allocate nothing:
 *    scratch memory is the caller's workspace, sized by the matching
 *    *_workspace_size query; it must be 256-byte aligned.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream) and never synchronise it.
 *  - Arguments are validated before anything is enqueued.  On error nothing
 *    is enqueued, a negative oceansim_status is returned and
 *    oceansim_last_error() (per thread) describes it.  No call aborts or
 *    throws.  Faults of enqueued kernels surface as OCEANSIM_E_HIP from a
 *    later call or from the caller's own synchronisation.
 *  - Image and polar buffers, J, depth and gradient images must be 16-byte
 *    aligned (float4 access); misalignment is OCEANSIM_E_INVALID_ARG.
 *  - Gradient outputs are overwritten, never accumulated.
 *  - Physical parameters live in device-resident rows so that an optimiser
 *    can update them in place between calls; the library reads them on the
 *    device and does not check their values (a non-finite value gives
 *    non-finite outputs, never an out-of-bounds access).
 */
#ifndef OCEANSIM_H
#define OCEANSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OCEANSIM_ABI_VERSION 5

typedef enum {
    OCEANSIM_OK = 0,
    OCEANSIM_E_INVALID_ARG = -1,  /* NULL / misaligned pointer, bad enum, bad value */
    OCEANSIM_E_SHAPE = -2,        /* sizes out of range or inconsistent            */
    OCEANSIM_E_WORKSPACE = -3,    /* workspace too small or misaligned            */
    OCEANSIM_E_UNSUPPORTED = -4,  /* valid request beyond this build's limits     */
    OCEANSIM_E_HIP = -5           /* a HIP runtime call failed                     */
} oceansim_status;

/* Text for the last non-OK status returned on the calling thread. */
const char *oceansim_last_error(void);

/* OCEANSIM_ABI_VERSION of the loaded library. */
int oceansim_abi_version(void);

/* ======================================================================== */
/* Imaging sonar (Sec. III-A.2)                                             */
/* ======================================================================== */

/* Speckle model applied after binning and gain.
 *  OFF   : out = Q                                (no noise)
 *  PAPER : out = Q (0.5 + w_sm) + w~_sa           Eq. (3)-(6)
 *  GAMMA : out = Q m + w~_sa,  m ~ Gamma(k, 1/k)  (unit-mean multiplicative
 *          speckle of integer shape k in 1..8, additive term of Eq. 3-4)
 * where Q = G P is the gained bin sum and
 *   w~_sa = (r_i^2 / r_max^2) (1 + 0.5 exp(-phi_j^2 / sigma_phi) w_sa),
 *   w_sa ~ Rayleigh(sigma_sa),  w_sm ~ N(0, sigma_sm^2),
 * at the bin centre (r_i, phi_j).  Random numbers come from Philox4x32-10
 * (Salmon et al., SC'11) keyed by (seed_lo, seed_hi); bin b = i N_phi + j of
 * frame frame_id draws
 *   additive  : counter (b/4, frame_id, 0, 0), word b%4
 *   gaussian  : counter (b/2, frame_id, 1, 0), words 2(b%2), 2(b%2)+1
 *               (Box-Muller, cosine branch)
 *   gamma     : counter (b, frame_id, 2, g), words 0..3, g = 0, 1
 * each word w mapping to the uniform ((w >> 8) + 1) 2^-24 in (0, 1].      */
enum {
    OCEANSIM_SPECKLE_OFF = 0,
    OCEANSIM_SPECKLE_PAPER = 1,
    OCEANSIM_SPECKLE_GAMMA = 2
};

/* One DEVICE-resident row of differentiable sonar parameters (32 bytes).
 * Frames select a row with oceansim_sonar_frame.param_row.               */
typedef struct {
    float alpha;      /* Eq. 2 attenuation coefficient [1/m]             */
    float gain;       /* G, applied to the bin sums                      */
    float sigma_phi;  /* Eq. 3 beam-pattern parameter [rad^2]            */
    float sigma_sa;   /* Eq. 4 Rayleigh parameter of the additive speckle */
    float sigma_sm;   /* Eq. 6 std. dev. of the multiplicative speckle   */
    float reserved[3];
} oceansim_sonar_params;

/* Columns of a sonar gradient row (one row per parameter row). */
enum {
    OCEANSIM_SONAR_GRAD_ALPHA = 0,
    OCEANSIM_SONAR_GRAD_GAIN = 1,
    OCEANSIM_SONAR_GRAD_SIGMA_PHI = 2,
    OCEANSIM_SONAR_GRAD_SIGMA_SA = 3,
    OCEANSIM_SONAR_GRAD_SIGMA_SM = 4,
    OCEANSIM_SONAR_GRAD_WIDTH = 8
};

/* One sonar frame: its returns, sensor geometry, RNG key and outputs.
 *
 * Returns (the paper's point set Q of in-view, unoccluded ray hits) are a
 * structure of arrays in the sensor frame: x forward, y left, z up, metres.
 * (nx, ny, nz) is the surface normal (any length; normalised internally).
 * mat[k] indexes the reflectivity table (A_r of Eq. 2, one entry per
 * material or semantic class); mat < 0 or mat >= n_materials is a miss.
 *
 * A hit counts if r = |x| lies in [r_min, r_max), the azimuth
 * phi = atan2(y, x) in [-fov_az/2, fov_az/2) and |z| <= r sin(fov_el/2).
 * Its intensity is refl[mat] * max(0, -x.n / (|x||n|)) * exp(-path_factor
 * alpha r) (Eq. 2; path_factor 2 = two-way travel, 1 = Eq. 2 literally).
 * It is summed into bin (i, j), i = floor((r - r_min) N_r / (r_max - r_min)),
 * j = floor((phi + fov_az/2) N_phi / fov_az); bins are row-major [N_r][N_phi].
 *
 * Fan (fan_h x fan_w > 0): apex at the bottom centre, boresight up, the
 * sensor's left on the image's left, square pixels of side
 * s = max(r_max / fan_h, 2 r_max sin(fov_az/2) / fan_w) (needs fov_az <= pi);
 * pixel (v, u) at x_c = (u + 1/2 - fan_w/2) s, y_c = (fan_h - v - 1/2) s,
 * rho = hypot(x_c, y_c), phi = atan2(-x_c, y_c).  Pixels with rho outside
 * [r_min, r_max] or |phi| > fov_az/2 are 0; others are the bilinear
 * interpolation of the polar image at bin centres, clamped to the grid.
 */
typedef struct {
    const float *x, *y, *z;          /* [n_returns] device                   */
    const float *nx, *ny, *nz;       /* [n_returns] device                   */
    const int32_t *mat;              /* [n_returns] device                   */
    int64_t n_returns;               /* >= 0 (0 = an empty scene)            */
    float r_min, r_max;              /* metres, 0 <= r_min < r_max           */
    float fov_az, fov_el;            /* radians, full angles (0, 2pi], (0, pi] */
    float path_factor;               /* kappa >= 0                           */
    int32_t n_range, n_azimuth;      /* polar bins, N_r x N_phi              */
    int32_t fan_h, fan_w;            /* fan pixels, 0 x 0 = no fan           */
    int32_t speckle_mode;            /* OCEANSIM_SPECKLE_*                   */
    int32_t gamma_k;                 /* GAMMA shape, 1..8                    */
    int32_t param_row;               /* row of the parameter table           */
    uint32_t seed_lo, seed_hi;       /* Philox key                           */
    uint32_t frame_id;               /* Philox counter word 1                */
    float *polar;                    /* out [N_r][N_phi] or NULL             */
    float *fan;                      /* out [fan_h][fan_w] or NULL           */
    int32_t *bin_of_return;          /* out [n_returns] bin or -1, or NULL   */
    const float *grad_polar;         /* backward in [N_r][N_phi] or NULL (0) */
    const float *grad_fan;           /* backward in [fan_h][fan_w] or NULL   */
    void *fan_stencil;               /* optional saved fan stencils, see
                                        oceansim_fan_stencil_size: written by
                                        the forward when non-NULL (and a fan
                                        is rendered), read by the backward
                                        instead of recomputing the fan
                                        geometry.  Same geometry in both. */
    int32_t range_norm;              /* 1: range-wise normalisation: after the
                                        gain each range row is divided by its
                                        maximum over azimuth when that is
                                        positive (rows with a maximum <= 0
                                        are left as they are); 0: none.  The
                                        paper (Sec. III-A.2) names the step
                                        without a formula: this is a reading. */
    float *saved_p;                  /* [N_r][N_phi] binned sums P (before the
                                        gain): written by the forward when
                                        non-NULL; the backward of a frame with
                                        range_norm = 1 reads it (required
                                        there: the adjoint of a row maximum
                                        needs the row).  Plans keep their own. */
} oceansim_sonar_frame;

/* Bytes of the fan_stencil buffer of a fan_h x fan_w fan (16 per pair of
 * mirror-image pixels: the bilinear rows, columns and weights of the pair). */
size_t oceansim_fan_stencil_size(int32_t fan_h, int32_t fan_w);

/* Workspace bytes for oceansim_sonar_render (with_backward = 0) or for
 * oceansim_sonar_render_backward (with_backward = 1) on these frames. */
int oceansim_sonar_workspace_size(const oceansim_sonar_frame *frames, int32_t n_frames,
                                  int32_t n_materials, int32_t with_backward, size_t *bytes);

/* Forward sonar rendering of n_frames frames (uneven sizes allowed) in one
 * set of launches.  params_dev: [n_param_rows] device rows; refl_dev:
 * [n_materials] device reflectivities.  For every frame, polar and/or fan
 * must be non-NULL.  Bin sums are accumulated in float32 in an order that
 * may change between runs (results may differ in the last bits). */
int oceansim_sonar_render(const oceansim_sonar_frame *frames, int32_t n_frames,
                          const oceansim_sonar_params *params_dev, int32_t n_param_rows,
                          const float *refl_dev, int32_t n_materials,
                          void *workspace, size_t workspace_bytes, void *stream);

/* oceansim_sonar_render without allocation and without a workspace argument,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * scratch memory the kernels need (the binning pass's pairs and per-chunk
 * offsets, the frame table of a batch, column tables and an internal polar
 * image where a frame asks for the fan only) is a static device array of
 * 64 MiB per GPU, held until the process ends; frames that need more (about
 * 7 M returns in all) are rejected with OCEANSIM_E_UNSUPPORTED before
 * anything is enqueued.  Nothing in the scratch has to start at zero.  The
 * array is shared by every call on a GPU: calls that overlap in time on one
 * GPU (on different streams, or from different threads) race and must be
 * ordered by the caller.  Otherwise identical to oceansim_sonar_render,
 * outputs included. */
int oceansim_sonar_render_noalloc(const oceansim_sonar_frame *frames, int32_t n_frames,
                                  const oceansim_sonar_params *params_dev, int32_t n_param_rows,
                                  const float *refl_dev, int32_t n_materials, void *stream);

/* Gradient of L = sum_f <grad_polar_f, polar_f> + <grad_fan_f, fan_f> with
 * respect to the reflectivity table (grad_refl_dev [n_materials]) and every
 * parameter row (grad_params_dev [n_param_rows][OCEANSIM_SONAR_GRAD_WIDTH],
 * columns OCEANSIM_SONAR_GRAD_*; unused columns are written 0).  The forward
 * pass is recomputed from the returns and the RNG counters; nothing is saved
 * between the calls.  Reductions use a fixed order: repeated calls on the
 * same inputs give bit-identical gradients when n_materials <= 64. */
int oceansim_sonar_render_backward(const oceansim_sonar_frame *frames, int32_t n_frames,
                                   const oceansim_sonar_params *params_dev, int32_t n_param_rows,
                                   const float *refl_dev, int32_t n_materials,
                                   float *grad_refl_dev, float *grad_params_dev,
                                   void *workspace, size_t workspace_bytes, void *stream);

/* ======================================================================== */
/* Underwater colour image formation (Sec. III-A.1, Eq. 1)                  */
/*   I_c = J_c exp(-beta_D,c d) + B_inf,c (1 - exp(-beta_B,c d))            */
/* beta_D is the paper's beta_attn and beta_B its beta_bs; beta*d is taken  */
/* as 0 when beta = 0.                                                      */
/* ======================================================================== */

/* One DEVICE-resident row of water parameters (48 bytes), channels R, G, B. */
typedef struct {
    float beta_d[3];
    float beta_b[3];
    float b_inf[3];
    float reserved[3];
} oceansim_water_params;

/* Columns of a water gradient row: beta_d[0..2], beta_b[0..2], b_inf[0..2]. */
#define OCEANSIM_WATER_GRAD_WIDTH 9

/* One camera frame.  J and out are planar [3][H][W] float32; depth [H][W]. */
typedef struct {
    const float *J;            /* in-air image                            */
    const float *depth;        /* metres                                  */
    float *out;                /* forward output (may alias nothing)      */
    int32_t H, W;
    int32_t param_row;         /* row of the water table                  */
    const float *grad_out;     /* backward input [3][H][W]                */
    float *grad_J;             /* backward output [3][H][W] or NULL       */
    float *grad_depth;         /* backward output [H][W] or NULL          */
} oceansim_uw_frame;

/* Eq. (1) on n_frames images (uneven sizes allowed) in one launch. */
int oceansim_uw_form(const oceansim_uw_frame *frames, int32_t n_frames,
                     const oceansim_water_params *params_dev, int32_t n_param_rows,
                     void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes for oceansim_uw_form (with_backward = 0) or
 * oceansim_uw_form_backward (with_backward = 1). */
int oceansim_uw_workspace_size(const oceansim_uw_frame *frames, int32_t n_frames,
                               int32_t with_backward, size_t *bytes);

/* Gradient of L = sum_f <grad_out_f, out_f> with respect to every water row
 * (grad_params_dev [n_param_rows][OCEANSIM_WATER_GRAD_WIDTH]) and, where
 * requested, to J and depth.  Fixed-order reductions: bit-reproducible. */
int oceansim_uw_form_backward(const oceansim_uw_frame *frames, int32_t n_frames,
                              const oceansim_water_params *params_dev, int32_t n_param_rows,
                              float *grad_params_dev, void *workspace, size_t workspace_bytes,
                              void *stream);

/* ======================================================================== */
/* Camera input conditioning and output encoding (Sec. III-A.1)            */
/*                                                                          */
/* Eq. (1) attenuates with the distance d travelled along the line of      */
/* sight, which the paper calls depth or range.  A renderer's depth buffer  */
/* holds z-depth (distance along the optical axis); with pinhole            */
/* intrinsics (fx, fy, cx, cy in pixels, pixel (u, v) centred at            */
/* (u + 1/2, v + 1/2)) the range of pixel (u, v) is                         */
/*   r = z * sqrt(1 + ((u + 1/2 - cx) / fx)^2 + ((v + 1/2 - cy) / fy)^2).   */
/* Colour enters and leaves as 8-bit sRGB (IEC 61966-2-1 transfer function) */
/* while Eq. (1) acts on linear intensities: decoding maps code c to        */
/* srgb_to_linear(c / 255) rounded to the nearest float; encoding maps a    */
/* linear value x to floor(255 * linear_to_srgb(min(max(x, 0), 1)) + 1/2),  */
/* computed exactly (NaN encodes as 0).                                     */
/* ======================================================================== */

/* One camera frame to condition.  Either input may be NULL, which skips   */
/* that half.  srgb_in is interleaved [H][W][channels_in] bytes (3: RGB,     */
/* 4: RGBA, alpha ignored); J is planar [3][H][W]; zdepth, range,           */
/* grad_range and grad_zdepth are [H][W].  Buffers 16-byte aligned.  An     */
/* empty frame (H or W 0) is skipped and needs no buffers.                  */
typedef struct {
    const uint8_t *srgb_in;    /* forward input, or NULL                   */
    const float *zdepth;       /* forward input (metres), or NULL          */
    float *J;                  /* forward output, needed with srgb_in      */
    float *range;              /* forward output, needed with zdepth       */
    const float *grad_range;   /* backward input                           */
    float *grad_zdepth;        /* backward output                          */
    int32_t H, W;              /* 0 <= H, W <= 65535                        */
    int32_t channels_in;       /* 3 or 4 (read only with srgb_in)          */
    float fx, fy, cx, cy;      /* fx, fy finite and nonzero; cx, cy finite */
} oceansim_cam_frame;

/* Decode srgb_in into J and convert zdepth into range on n_frames frames   */
/* (uneven sizes allowed; no workspace).  Non-finite or non-positive depths */
/* pass through the scale unchanged in kind (0 -> 0, inf -> inf, NaN ->     */
/* NaN).                                                                    */
int oceansim_cam_condition(const oceansim_cam_frame *frames, int32_t n_frames, void *stream);

/* Adjoint of the range conversion: grad_zdepth = grad_range * r / z, the   */
/* per-pixel scale above.  Decoding has no adjoint (its input is integer).  */
int oceansim_cam_condition_backward(const oceansim_cam_frame *frames, int32_t n_frames, void *stream);

/* One image to encode: I planar [3][H][W] linear float in, srgb_out         */
/* interleaved [H][W][channels_out] bytes out (4: alpha written as 255).    */
typedef struct {
    const float *I;
    uint8_t *srgb_out;
    int32_t H, W;              /* 0 <= H, W <= 65535                        */
    int32_t channels_out;      /* 3 or 4                                   */
} oceansim_cam_out_frame;

int oceansim_cam_encode(const oceansim_cam_out_frame *frames, int32_t n_frames, void *stream);

/* ======================================================================== */
/* Navigation sensors (Sec. III-A): barometer and DVL                       */
/*                                                                          */
/* The paper describes both without equations; these are the readings.      */
/* Random numbers come from Philox4x32-10 as for the sonar speckle, normals */
/* by Box-Muller (cosine branch) from two words.                            */
/* ======================================================================== */

/* Barometer: the pressure at depth d (metres below the free surface) is the
 * atmospheric pressure plus the weight of the water column, with optional
 * Gaussian noise:  P = p_atm + rho g max(d, 0) + sigma z,  z ~ N(0, 1) from
 * counter (k mod 2^32, k / 2^32, 3, 0), words 0 and 1, for sample k. */
typedef struct {
    double p_atm;        /* Pa, user-defined atmospheric pressure          */
    double rho;          /* kg / m^3, user-defined water density (>= 0)    */
    double g;            /* m / s^2 (>= 0)                                  */
    double sigma;        /* Pa, noise standard deviation (0: none)          */
    uint32_t seed_lo, seed_hi;
} oceansim_baro_params;

/* pressure_dev[k] (float32, Pa) for depth_dev[k] (float32, m), k < n;
 * device buffers, 4-byte aligned; params is host memory.  Asynchronous. */
int oceansim_barometer(const float *depth_dev, int64_t n, const oceansim_baro_params *params,
                       float *pressure_dev, void *stream);

/* DVL: a four-beam convex Janus array in the sensor frame (x forward, y
 * left, z up); beam i is tilted by janus_angle from the downward vertical at
 * azimuth 45 + 90 i degrees.  Per instance (a vehicle or a Monte Carlo run)
 * and tick k (times t[k], seconds, increasing, shared by the instances):
 *  - beam i is valid when its slant range to the bottom is finite and in
 *    [range_min, range_max];
 *  - adaptive rate: a measurement is due when t[k] minus the time of the
 *    instance's last measurement reaches the ping period of the current
 *    altitude, max(period_min, pings_per_output * 2 r_ref / sound_speed),
 *    r_ref the largest valid range (range_max without a valid beam),
 *    evaluated in double precision in that order; the first tick measures;
 *  - a due measurement with at least min_beams valid beams is the least-
 *    squares velocity from the valid beams' along-beam velocities
 *    b_i . v + sigma_v z_i, z_i ~ N(0, 1) from counter (k, n, 4, i / 2),
 *    words 2 (i mod 2), 2 (i mod 2) + 1 (status 1); with fewer it is a
 *    dropout (status 2, velocity NaN); no measurement: status 0, NaN.
 * Layouts (device, tick-major): t [n_ticks] double (8-byte aligned); ranges
 * [n_ticks][n_inst][4] float (16-byte aligned); velocity and velocity_out
 * [n_ticks][n_inst][3] float; status [n_ticks][n_inst] int32.  params is
 * host memory (janus_angle in (0, pi/2), min_beams 3 or 4). */
typedef struct {
    double janus_angle;        /* rad                                       */
    double range_min, range_max;   /* m, operational range of a beam       */
    int32_t min_beams;         /* valid beams needed for a velocity: 3 or 4 */
    double sigma_v;            /* m / s, along-beam velocity noise (0: none) */
    double sound_speed;        /* m / s                                      */
    double pings_per_output;   /* pings averaged into one output            */
    double period_min;         /* s, shortest measurement period            */
    uint32_t seed_lo, seed_hi;
} oceansim_dvl_params;

int oceansim_dvl(const double *t_dev, const float *ranges_dev, const float *velocity_dev, int32_t n_ticks,
                 int32_t n_inst, const oceansim_dvl_params *params, float *velocity_out_dev, int32_t *status_dev,
                 void *stream);

/* ======================================================================== */
/* Ray casting of the sonar's returns (Sec. III-A.2 takes the returns from  */
/* the renderer's ray tracing against the scene): a triangle mesh held on   */
/* the device in a bounding-volume hierarchy, and the closest hits of a     */
/* sonar's beam x elevation ray pattern, written as the return buffers of   */
/* an oceansim_sonar_frame.                                                 */
/* ======================================================================== */

typedef struct oceansim_scene oceansim_scene;

/* Builds the hierarchy of a mesh on the host and uploads it to the current
 * device (synchronously; the scene owns that device memory until
 * oceansim_scene_destroy).  vertices [n_vertices][3] float32 (world frame,
 * metres), triangles [n_triangles][3] int32 vertex indices, tri_mat
 * [n_triangles] int32 material ids: all HOST memory, not retained.  The
 * normal of a triangle (v0, v1, v2) is (v1 - v0) x (v2 - v0).  Triangles
 * whose area is negligible at single precision, |(v1 - v0) x (v2 - v0)| <
 * 2^-20 L^2 with L the longest edge (needles and points), are dropped: no ray
 * can hit them decidedly.  A mesh of no (kept) triangles is valid: every ray
 * misses.  Errors: OCEANSIM_E_INVALID_ARG for NULL arrays, an index outside
 * [0, n_vertices) or a non-finite vertex; OCEANSIM_E_UNSUPPORTED beyond 2^28
 * triangles or for a coordinate beyond 2^40 in magnitude; OCEANSIM_E_HIP when
 * the upload fails.  On error *scene is NULL
 * and nothing stays allocated. */
int oceansim_scene_create(const float *vertices, int64_t n_vertices, const int32_t *triangles,
                          const int32_t *tri_mat, int64_t n_triangles, oceansim_scene **scene);

typedef struct {
    int64_t n_triangles;   /* triangles kept                                  */
    int64_t n_dropped;     /* degenerate triangles dropped                    */
    int64_t n_nodes;       /* two-child nodes (each holds both child boxes)   */
    int64_t n_leaves;
    int32_t depth;         /* deepest leaf (the root is at depth 0), <= 32    */
    int32_t max_leaf;      /* most triangles in one leaf (<= 8)               */
    double sah_cost;       /* surface-area cost of the tree (node visit = 1,  */
                           /* triangle test = 1), per ray through the root box */
    uint64_t device_bytes; /* device memory the scene holds                  */
} oceansim_scene_info;

int oceansim_scene_get_info(const oceansim_scene *scene, oceansim_scene_info *info);

/* The figures oceansim_scene_create would report for this mesh, from a build
 * on the host alone (no device is touched, nothing stays allocated): sizes
 * the device memory of a scene before creating it.  Same arguments and
 * errors as oceansim_scene_create (upload errors aside). */
int oceansim_scene_measure(const float *vertices, int64_t n_vertices, const int32_t *triangles,
                           const int32_t *tri_mat, int64_t n_triangles, oceansim_scene_info *info);

/* Frees the scene's device memory (after synchronising the device).  NULL is
 * accepted. */
int oceansim_scene_destroy(oceansim_scene *scene);

/* One sensor pose and its ray pattern.  Beam b (of n_beams) points at
 * azimuth -fov_az/2 + (b + 1/2) fov_az / n_beams, ray r (of n_rays) of a beam
 * at elevation -fov_el/2 + (r + 1/2) fov_el / n_rays; the direction in the
 * sensor frame (x forward, y left, z up) is (cos el cos az, cos el sin az,
 * sin el), and return k = b n_rays + r.  The pose maps the sensor frame into
 * the world: world = R sensor + pos, R row-major.  The closest hit with
 * 0 < t <= t_max along the ray (triangle edges included) is written to
 * return k in the sensor frame: the point t d, the unit normal of the hit
 * triangle (R^T n), and its material id.  A miss writes material -1 and
 * zeros.  Output buffers: DEVICE memory, float32 / int32 [n_beams * n_rays],
 * 4-byte aligned; NULL skips a coordinate or normal output (mat is
 * required). */
typedef struct {
    float pos[3];
    float rot[9];
    int32_t n_beams, n_rays;
    float fov_az, fov_el;   /* rad: fov_az in (0, 2 pi], fov_el in [0, pi)  */
    float t_max;            /* casting distance, m, > 0                     */
    float *x, *y, *z, *nx, *ny, *nz;
    int32_t *mat;
} oceansim_ray_frame;

/* Casts the ray patterns of n_frames poses (host array, not retained)
 * against the scene, on `stream` (asynchronous; the scene must outlive the
 * enqueued work).  Allocates nothing.  Rays of one beam are cast by
 * neighbouring threads, so the returns come out in beam order.  Errors:
 * OCEANSIM_E_INVALID_ARG (NULL scene or mat, bad pattern, non-finite pose,
 * a scene of another device), OCEANSIM_E_UNSUPPORTED beyond 2^31 - 1 rays in a
 * frame or for a position beyond 2^40 in magnitude. */
int oceansim_raycast(const oceansim_scene *scene, const oceansim_ray_frame *frames, int32_t n_frames,
                     void *stream);

/* ======================================================================== */
/* Plans: a batch of sonar and camera frames prepared once and launched     */
/* many times, optionally replayed from HIP graphs.                         */
/* ======================================================================== */

typedef struct oceansim_plan oceansim_plan;

enum {
    OCEANSIM_PLAN_BACKWARD = 1,   /* also prepare the adjoint launch           */
    OCEANSIM_PLAN_GRAPH = 2,      /* capture each launch sequence in a graph   */
    OCEANSIM_PLAN_AUTOTUNE = 4    /* time launch-shape candidates at creation  */
};

/* Validates every frame, chooses launch shapes, allocates the plan's own
 * device memory (workspaces, frame tables, transposed fan operators), uploads the
 * frame tables and, with OCEANSIM_PLAN_GRAPH, captures the forward (and
 * backward) launch sequences into HIP graphs.  A plan holding both sonar and
 * camera frames runs the camera forward inside the sonar binning launch and
 * the camera backward inside the sonar return-gather launch (one dispatch
 * for both, when the return gather's LDS leaves room), so the camera's HBM
 * traffic overlaps latency-bound sonar work.  The plan keeps every pointer
 * of the descriptors, parameter tables and gradient outputs until
 * oceansim_plan_destroy: the caller keeps them alive, and may change their
 * CONTENTS (new returns, images, parameters) between launches, not the
 * shapes.  Sonar frames are rendered (forward) into their polar/fan outputs;
 * with OCEANSIM_PLAN_BACKWARD their grad_polar/grad_fan inputs and the
 * camera frames' grad_out are read by oceansim_plan_backward, which writes
 * grad_refl_dev [n_materials], grad_sonar_params_dev [n_sonar_rows][8] and
 * grad_water_params_dev [n_water_rows][9] (each may be NULL when there are no
 * frames of that kind).  The fan of a frame is a fixed linear map of its
 * polar image; for frames with a fan and a fan gradient a backward plan
 * builds the transpose of that map once, at creation (for each polar bin,
 * the fan pixels that read it and their bilinear weights, from the same
 * stencils the fan kernel computes: one int per bin plus 8 bytes per
 * pixel-bin pair, on the order of 40 bytes per fan pixel), and its backward
 * gathers each bin's fan gradient through it.  With an even fan width (at
 * most 65535 x 65535 pixels) the two halves of the fan are exact mirror
 * images, and the operator holds the bins of the first ceil(n_azimuth / 2)
 * columns only: each also yields its mirror bin from the mirrored pixels
 * (about 20 bytes per fan pixel).  The plan's forward saves no
 * stencils (a caller's own fan_stencil buffer is still written).  The
 * forward is the image formation of oceansim_sonar_render (Sec. III-A.2,
 * Eq. 2-6, and the fan) and oceansim_uw_form (Sec. III-A.1, Eq. 1); the
 * backward is their adjoint and reads what the plan's latest forward left
 * (bins), so order the two on one stream.  In a backward plan a frame's
 * grad_fan needs its fan output (OCEANSIM_E_INVALID_ARG otherwise).
 *
 * OCEANSIM_PLAN_AUTOTUNE times the forward launch (with the plan's camera
 * frames carried along, and, when the backward runs from the forward's
 * material pairs, together with that backward) for a small set of tile and
 * chunk sizes, then, with a fan backward, 1, 2 and 4 operator rows per
 * thread, and keeps the fastest whose outputs agree with the default shape's
 * (1e-5 relative); results are cached per process and,
 * when the environment variable OCEANSIM_TUNE_CACHE names a file, in that
 * JSON file, keyed by GPU architecture, CU count and a size class of the
 * batch.  Tuning runs the launches, so it reads the inputs (which must hold
 * representative returns) and writes the outputs and gradients.  When the
 * environment variable OCEANSIM_PLAN_SHAPE is set to "tile_bins,chunk"
 * (tile_bins 1..16384, chunk 512, 1024, 2048, 4096 or 8192 returns), plans
 * take that forward tile target and binning chunk instead of the heuristic or
 * the autotuner (OCEANSIM_E_INVALID_ARG for any other value): it replays a
 * shape a tuned plan picked, e.g. for tests at the tuned configuration.  All work of
 * creation is done on `stream`, which is synchronised.  Errors: the status
 * codes above; on error *plan is NULL and nothing stays allocated.        */
int oceansim_plan_create(const oceansim_sonar_frame *sonar, int32_t n_sonar,
                         const oceansim_uw_frame *camera, int32_t n_camera,
                         const oceansim_sonar_params *sonar_params_dev, int32_t n_sonar_rows,
                         const float *refl_dev, int32_t n_materials,
                         const oceansim_water_params *water_params_dev, int32_t n_water_rows,
                         float *grad_refl_dev, float *grad_sonar_params_dev,
                         float *grad_water_params_dev, int32_t flags, void *stream,
                         oceansim_plan **plan);

/* Enqueue the plan's forward / backward launches on `stream`. */
int oceansim_plan_forward(oceansim_plan *plan, void *stream);
int oceansim_plan_backward(oceansim_plan *plan, void *stream);

/* Launch shapes in use: {forward tile bins, returns per chunk, operator rows
 * per backward workgroup (a row is a polar bin, or a bin and its mirror bin;
 * 0 without a sonar backward), graphs in use (0/1)}. */
int oceansim_plan_shape(const oceansim_plan *plan, int32_t shape[4]);

/* Frees the plan's device memory and graphs (after synchronising the
 * device).  NULL is accepted. */
int oceansim_plan_destroy(oceansim_plan *plan);

/* ======================================================================== */
/* Tracing                                                                  */
/* ======================================================================== */

/* enable = 1 starts a new trace: from then on every kernel the library
 * launches is bracketed by HIP events recorded on its launch stream.
 * enable = 0 stops recording (the collected records are kept).            */
int oceansim_trace_enable(int32_t enable);

/* Waits for the recorded events and writes one line per kernel name,
 * "name calls total_us\n", into buf (truncated to len bytes, NUL-ended).
 * *needed receives the full length (may be NULL).                         */
int oceansim_trace_summary(char *buf, size_t len, size_t *needed);

#ifdef __cplusplus
}
#endif

#endif /* OCEANSIM_H */
