/*
 * satsplat.h — C ABI of the MI355X (gfx950) hot path of SatSplat (arXiv 2606.28581):
 * the differentiable 2D-Gaussian-surfel rasterizer under affine satellite cameras
 * (forward and backward) and the geometric sun-view shadow-map pass.
 *
 * Paper passages implemented (section / equation of the paper):
 *   surfels                 Sec. 3.1 "2D Gaussian Splatting", Eqs. (2dgs_splat_param), (2dgs_splat_H)
 *   affine camera           Sec. 3.1 Eq. (affine_camera); Sec. 3.2 Eq. (decompose_affine_camera)
 *   ray-splat intersection  Sec. 3.2 Eqs. (affine2dgs_uv2screen), (affine2dgs_screen2uv), (affine2dgs_Qq)
 *   depth / sort key        Sec. 3.2 Eq. (depth_affine_camera), "Rasterization"
 *   low-pass floor          Sec. 3.2 "Degenerate Solutions"
 *   normal                  Sec. 3.2 "Normal Definition"
 *   compositing             Sec. 3.2 Eq. (rasterization), 16x16 tiles by default
 *   image formation         Sec. 3.1 Eq. (image_formation)
 *   camera delta            Sec. 3.3: F'_xy = F_xy + dF_xy, dF_xy a 2x4 matrix
 *   sun camera              Sec. 3.3 Eq. (sun_camera_Bxy); Supp. A
 *   soft shadow test        Sec. 3.1 (exponential-shadow-map filtering of the sun test)
 *
 * Conventions
 *   - Every call returns ss_status: SS_OK (0) or a negative error code.  No call aborts,
 *     no C++ exception crosses the ABI.  ss_last_error() gives a thread-local message.
 *   - Tensors are caller-owned DEVICE memory unless marked "host".  The library never
 *     frees caller memory.  Scratch memory is one caller-provided workspace per plan
 *     (size from ss_plan_workspace_size); the library itself allocates no device memory.
 *   - Compute calls are asynchronous on the caller's HIP stream.  Only ss_plan_check
 *     and ss_count_pairs block (they read device counters back).
 *   - Gradient outputs are overwritten, not accumulated into.
 *   - Pixel (i, j) of a view (column i, row j) samples the image-plane point
 *     (i + 0.5, j + 0.5).  Per-pixel outputs of all views are concatenated: view v
 *     owns pixels [pix_off[v], pix_off[v+1]) with pix_off the running sum of W*H; a
 *     C-channel output stores view v as planar [C][H][W] starting at C*pix_off[v].
 *   - World coordinates are metres (scene centred near the origin for FP32
 *     conditioning); F_xy maps world metres to pixels.
 */
#ifndef SATSPLAT_H
#define SATSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ss_status;
#define SS_OK               0
#define SS_ERR_INVALID_ARG (-1)   /* bad pointer, size, setting or state                 */
#define SS_ERR_CAPACITY    (-2)   /* workspace too small for the pairs this input needs   */
#define SS_ERR_HIP         (-3)   /* a HIP runtime call failed                            */
#define SS_ERR_UNSUPPORTED (-4)   /* device is not gfx950, or a setting outside the range */
#define SS_ERR_STATE       (-5)   /* call order violated (e.g. backward before forward)   */

typedef struct ss_context ss_context;
typedef struct ss_plan ss_plan;
typedef struct ihipStream_t *ss_stream;   /* hipStream_t; NULL = default stream */

/* Rasterizer constants.  alpha_min and T_min are the stated workload values; the rest
 * are readings where the paper gives no number (documented with the design). */
typedef struct ss_raster_settings {
    uint32_t struct_size;   /* sizeof(ss_raster_settings)                              */
    int32_t  tile_size;     /* 8, 16 (paper default, Sec. 3.2) or 32                    */
    int32_t  batch_depth;   /* surfel records staged in LDS per batch (1..256; capped at
                               tile_size^2, one record per thread)                      */
    float    alpha_min;     /* skip a surfel at a pixel when alpha < alpha_min (1/255)  */
    float    alpha_max;     /* alpha = min(alpha_max, o * G) (0.99)                     */
    float    T_min;         /* stop before transmittance would drop below T_min (1e-4) */
    float    lowpass_sigma; /* sigma of the screen-space low-pass floor, px (sqrt(2)/2) */
    int32_t  lowpass_mode;  /* 0: floor applied to every surfel; 1: degenerate only     */
    float    det_rel_eps;   /* degenerate iff |det T| <= eps * |T|_F^2 (1e-6)            */
    float    esm_c;         /* exponential-shadow-map sharpness, 1/m (2.0)              */
    float    esm_bias;      /* shadow depth bias, m (0.5)                               */
    int32_t  sun_map_size;  /* S: sun-view depth map is S x S (1024)                    */
    int32_t  tile_order;    /* raster dispatch order: 0 = static (tiles dealt to the 8
                               XCDs in chunks of neighbouring tiles; default); 1 = the
                               same assignment with each XCD's tiles of at least twice
                               the mean list length dispatched first                   */
} ss_raster_settings;

/* Surfels, structure of arrays, FP32 device memory (Sec. 3.1 2DGS parameterisation).
 * Activations (exp of log-scales, sigmoid of opacity, quaternion -> axes) are applied
 * by the caller before the call. */
typedef struct ss_surfels {
    int64_t      n;
    const float *mean;      /* [n,3] centre p_k, metres                                 */
    const float *t_u;       /* [n,3] tangent axis (unit)                                */
    const float *t_v;       /* [n,3] tangent axis (unit)                                */
    const float *scale;     /* [n,2] s_u, s_v, metres (linear)                          */
    const float *opacity;   /* [n]   in (0,1)                                           */
    const float *albedo;    /* [n,3] linear RGB                                         */
} ss_surfels;

/* Views: affine cameras and per-image radiometry (Sec. 3.1, 3.3).  width/height are
 * HOST arrays fixed at plan creation; the rest are device pointers read at call time. */
typedef struct ss_views {
    int32_t      n;
    const int32_t *width;   /* host [n] */
    const int32_t *height;  /* host [n] */
    const float *Fxy;       /* [n,2,4] initial camera rows [B_xy | b_xy], world m -> px */
    const float *dF;        /* [n,2,4] learnable delta, or NULL (= 0)                    */
    const float *colC;      /* [n,3,3] per-image colour gain C, or NULL (= I)            */
    const float *colc;      /* [n,3]   per-image colour bias c, or NULL (= 0)            */
    const float *ambient;   /* [n,3]   ambient light L_a, or NULL (= 0)                  */
    const float *sun;       /* [n,2]   sun (azimuth phi, elevation theta), radians, phi
                                       from world +x towards +y; NULL if no shadow pass */
    float        b_z;       /* max altitude: depth is b_z - z (Eq. depth_affine_camera)  */
} ss_views;

/* ---------------------------------------------------------------- lifecycle */
const char *ss_last_error(void);
void        ss_default_settings(ss_raster_settings *out);

/* Create a context on HIP device `device`; fails with SS_ERR_UNSUPPORTED unless the
 * device is gfx950. */
ss_status ss_context_create(int32_t device, ss_context **out);
ss_status ss_context_destroy(ss_context *ctx);

/* A plan fixes the surfel count, the view sizes and the settings.  Views must be
 * 1..32767 pixels on each side.  Nothing is allocated on the device. */
ss_status ss_plan_create(ss_context *ctx, int64_t n_surfels, int32_t n_views,
                         const int32_t *width, const int32_t *height,
                         const ss_raster_settings *settings, ss_plan **out);
ss_status ss_plan_destroy(ss_plan *plan);

/* Change tile size / batch depth / thresholds of an existing plan (same workspace;
 * the workspace is always sized for the smallest tile size). */
ss_status ss_plan_set_settings(ss_plan *plan, const ss_raster_settings *settings);

/* Workspace bytes for capacities of `main_pairs` (tile, surfel) pairs over all main
 * views and `sun_pairs` over all sun views.  Capacities may be 0 (then only
 * ss_count_pairs may run). */
ss_status ss_plan_workspace_size(ss_plan *plan, int64_t main_pairs, int64_t sun_pairs,
                                 size_t *bytes);

/* Bind caller-owned device memory (256-byte aligned, >= the queried size) as the
 * plan's workspace.  The plan keeps the binning of the last forward in it for the
 * backward, so the workspace must stay alive and untouched between the two. */
ss_status ss_plan_bind_workspace(ss_plan *plan, void *workspace, size_t bytes,
                                 int64_t main_pairs, int64_t sun_pairs);

/* Count the (tile, surfel) pairs the given surfels and cameras need (main views, and
 * sun views when views->sun != NULL; else *sun_pairs = 0).  Blocks on `stream`. */
ss_status ss_count_pairs(ss_plan *plan, const ss_surfels *s, const ss_views *v,
                         int64_t *main_pairs, int64_t *sun_pairs, ss_stream stream);

/* Read the capacity-overflow state of the last calls (blocks on `stream`).
 * *overflowed = 1 if a forward or shadow pass needed more pairs than bound; its
 * outputs are then incomplete (memory-safe) and must be recomputed after rebinding
 * a larger workspace.  *main_pairs / *sun_pairs: pairs needed by the last calls. */
ss_status ss_plan_check(ss_plan *plan, int32_t *overflowed, int64_t *main_pairs,
                        int64_t *sun_pairs, ss_stream stream);

/* ------------------------------------------------------------------ forward
 * Rasterize all views (Sec. 3.2): per-surfel projection (Eqs. affine2dgs_Qq,
 * depth_affine_camera) with F' = F + dF (Sec. 3.3), centre-depth order, 16x16 (or
 * tile_size) binning, front-to-back compositing (Eq. rasterization) of albedo, sun
 * visibility, depth and normal, then the image formation (Eq. image_formation).
 *   vis      [n_views, n] per-view per-surfel sun visibility in [0,1] composited as the
 *            V channel, or NULL: then V == 1 everywhere (no shadows, I = C A + c).
 * Outputs (all required):
 *   image    [3 * P] I,   albedo_out [3 * P] A,   vis_out [P] V (1.0 if vis == NULL),
 *   depth    [P] D = sum w z (unnormalised; background contributes 0),
 *   normal   [3 * P] world-space N = sum w n,  T_final [P],
 *   last     [P] int32: 1 + position, in the pixel's tile list, of its last contributor.
 * P = sum of width*height.  albedo_out, vis_out, T_final and last are the saved state
 * the backward needs. */
ss_status ss_forward(ss_plan *plan, const ss_surfels *s, const ss_views *v,
                     const float *vis, float *image, float *albedo_out, float *vis_out,
                     float *depth, float *normal, float *T_final, int32_t *last,
                     ss_stream stream);

/* ----------------------------------------------------------------- backward
 * Adjoint of ss_forward for the same surfels/views/vis (the plan must hold that
 * forward's binning).  Upstream gradients d_image [3P], d_depth [P], d_normal [3P];
 * each may be NULL (= 0).  Transmittance is recomputed back to front from T_final,
 * no per-pixel lists are stored.  Outputs (overwritten; all required):
 *   d_mean [n,3], d_t_u [n,3], d_t_v [n,3], d_scale [n,2], d_opacity [n],
 *   d_albedo [n,3]  (summed over views),
 *   d_dF [n_views,2,4], d_colC [n_views,3,3], d_colc [n_views,3], d_ambient [n_views,3].
 * vis is a stop-gradient input (no gradient is returned for it). */
ss_status ss_backward(ss_plan *plan, const ss_surfels *s, const ss_views *v,
                      const float *vis, const float *albedo_out, const float *vis_out,
                      const float *T_final, const int32_t *last, const float *d_image,
                      const float *d_depth, const float *d_normal, float *d_mean,
                      float *d_t_u, float *d_t_v, float *d_scale, float *d_opacity,
                      float *d_albedo, float *d_dF, float *d_colC, float *d_colc,
                      float *d_ambient, ss_stream stream);

/* ------------------------------------------------ geometric regularisers
 * Depth distortion (the distortion term of the paper's training loss, Supp. B, in the
 * squared 2DGS form): per pixel
 *     dist = sum over pairs i > j of its contributors of w_i w_j (m_i - m_j)^2,
 * m = z * depth_scale the normalised depth of each (pixel, surfel) pair.  The forward
 * variant composites it as an extra channel; the backward variant adds its adjoint for an
 * upstream gradient d_dist.  aux is state the forward saves for the backward (the depth of
 * the pixel's first contributor and two moments of the depths relative to it, which keep
 * the moments from cancelling in FP32).  P = sum of width*height. */
typedef struct ss_geom_io {
    uint32_t struct_size;   /* sizeof(ss_geom_io)                                      */
    float    depth_scale;   /* m = z * depth_scale, > 0 (e.g. 1 / scene half extent)   */
    float   *dist;          /* [P] forward output; unused by the backward              */
    float   *aux;           /* [3, P] written by the forward, read by the backward     */
    const float *d_dist;    /* [P] upstream gradient for the backward, or NULL (= 0)   */
} ss_geom_io;

/* ss_forward with the distortion channel (same arguments and outputs, plus geom). */
ss_status ss_forward_geom(ss_plan *plan, const ss_surfels *s, const ss_views *v,
                          const float *vis, float *image, float *albedo_out, float *vis_out,
                          float *depth, float *normal, float *T_final, int32_t *last,
                          const ss_geom_io *geom, ss_stream stream);
/* ss_backward plus the adjoint of the distortion for geom->d_dist; geom->aux must hold
 * what ss_forward_geom saved for the same inputs. */
ss_status ss_backward_geom(ss_plan *plan, const ss_surfels *s, const ss_views *v,
                           const float *vis, const float *albedo_out, const float *vis_out,
                           const float *T_final, const int32_t *last, const float *d_image,
                           const float *d_depth, const float *d_normal, const ss_geom_io *geom,
                           float *d_mean, float *d_t_u, float *d_t_v, float *d_scale,
                           float *d_opacity, float *d_albedo, float *d_dF, float *d_colC,
                           float *d_colc, float *d_ambient, ss_stream stream);

/* Depth-gradient normals and the normal-consistency loss (Sec. 3.2 "Normal Definition",
 * Eq. surface_normal) on the rendered maps of all views.  Per view v with P_v pixels:
 * the expected depth zbar = D / (1 - T) (the accumulated opacity is a constant: no
 * gradient flows into T) is back-projected through F' = F + dF with the fixed depth row
 * (world point p with B'_xy p + b'_xy = pixel centre, b_z - p_z = zbar); N_d is the
 * normalised cross product of the central differences of that point map along x and y,
 * oriented like the rendered normals (against B'_x x B'_y taken with negative z);
 *     loss[v] = weight / P_v * sum over valid pixels of (1 - N . N_d),
 * N the composited normal map.  A pixel is valid when it is not on the view's border
 * and 1 - T >= tau at it and at its four neighbours.
 *   depth [P], T_final [P], normal [3P]: the forward's outputs (planar per view).
 *   loss [n_views] (written), normal_d [3P] (written, 0 where invalid) or NULL.
 *   d_depth [P], d_normal [3P], d_dF [n_views,2,4] or NULL: gradients of sum_v loss[v],
 *   ADDED to what they hold, so that the image loss's upstream gradients can be
 *   accumulated in the same buffers before ss_backward(_geom).
 * Uses the plan's workspace (bound) and its views; sizes are those of the plan. */
ss_status ss_normal_loss(ss_plan *plan, const ss_views *v, const float *depth,
                         const float *T_final, const float *normal, float weight, float tau,
                         float *loss, float *normal_d, float *d_depth, float *d_normal,
                         float *d_dF, ss_stream stream);

/* ------------------------------------------------------------ training step
 * The optimiser around the rasterizer (Supp. B "Experimental Settings": Adam with per-group
 * learning rates, L1 image loss, camera-delta optimisation from a start step).
 * Raw surfel parameters, SS_RAW_FLOATS per surfel, row-major [n, 13]: mean (3, metres),
 * log s_u, log s_v, opacity logit, rotation quaternion (w, x, y, z) of any non-zero norm,
 * albedo (3).  Activated (the ss_surfels arrays): scale = exp(log scale), opacity =
 * sigmoid(logit), t_u and t_v = the first two columns of the rotation of q / |q| (the
 * third is the normal, Sec. 3.1). */
#define SS_RAW_FLOATS 13
typedef struct ss_adam_config {
    uint32_t struct_size;   /* sizeof(ss_adam_config)                                   */
    float lr_mean, lr_scale, lr_opacity, lr_quat, lr_albedo;   /* surfel groups           */
    float lr_dF;            /* camera delta                                             */
    float lr_colour;        /* colour gain C and bias c (the ambient term is not trained) */
    float beta1, beta2, eps;
    int32_t camera_start;   /* the camera-delta group is updated from this step on; its
                               bias correction counts its own steps, t - camera_start + 1 */
} ss_adam_config;

/* Activated surfel arrays ([n,3] mean, t_u, t_v, albedo, [n,2] scale, [n] opacity) from
 * the raw parameters. */
ss_status ss_surfel_activate(int64_t n, const float *raw, float *mean, float *t_u, float *t_v,
                             float *scale, float *opacity, float *albedo, ss_stream stream);
/* Raw parameters [n, 13] from activated arrays (t_u, t_v orthonormal; scale > 0;
 * opacity in (0, 1)): log scale, logit opacity, and a quaternion of the frame
 * [t_u, t_v, t_u x t_v] (its sign is arbitrary: q and -q give the same frame). */
ss_status ss_surfel_raw(int64_t n, const float *mean, const float *t_u, const float *t_v,
                        const float *scale, const float *opacity, const float *albedo, float *raw,
                        ss_stream stream);
/* One Adam step (t = step >= 1, bias-corrected: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)) on the raw parameters, with
 * their gradient obtained from the gradients of the activated arrays (d_*, as written by
 * ss_backward); then the activated arrays are rewritten from the new raw parameters.
 * raw, m, v: [n, 13] (m, v start at zero). */
ss_status ss_adam_surfels(int64_t n, float *raw, float *m, float *v, const float *d_mean,
                          const float *d_t_u, const float *d_t_v, const float *d_scale,
                          const float *d_opacity, const float *d_albedo,
                          const ss_adam_config *cfg, int32_t step, float *mean, float *t_u,
                          float *t_v, float *scale, float *opacity, float *albedo,
                          ss_stream stream);
/* Adam on the per-view terms: dF [nv,2,4] (from cfg->camera_start on), colC [nv,3,3] and
 * colc [nv,3]; any group may be NULL (not trained); m_*, v_* have the group's shape.  The
 * camera-delta gradient is d_dF + d_dF_extra (d_dF_extra may be NULL; e.g. the normal-
 * consistency term's, which ss_normal_loss adds to its own buffer). */
ss_status ss_adam_views(int32_t nv, float *dF, float *m_dF, float *v_dF, const float *d_dF,
                        const float *d_dF_extra, float *colC, float *m_colC, float *v_colC, const float *d_colC,
                        float *colc, float *m_colc, float *v_colc, const float *d_colc,
                        const ss_adam_config *cfg, int32_t step, ss_stream stream);
/* L1 image loss of every view of the plan: loss[v] = weight / (3 P_v) * sum over its pixels
 * and channels of |image - target| (planar layout as ss_forward's image), and
 * d_image = weight sign(image - target) / (3 P_v) (written; sign(0) = 0). */
ss_status ss_image_loss_l1(ss_plan *plan, const float *image, const float *target, float weight,
                           float *loss, float *d_image, ss_stream stream);

/* ------------------------------------------------- geometry-aware initialisation
 * Initial surfels on a DSM (Sec. 3.4 "Area-Weighted Sampling", "Splat Orientation").
 * z: device [ny, nx] FP32 node heights at (x0 + i gsd, y0 + j gsd); cell (j, i) spans
 * nodes j..j+1, i..i+1.  Each cell's tangents are (g, 0, dzx) and (0, g, dzy) (dzx, dzy
 * the means of its two edge differences), its area a = |dx x dy| and its normal
 * (-dzx, -dzy, g) / |.|; its sampling weight is the integer floor(65536 a / g^2 + 1/2).
 * Sample k (0 <= k < n) draws Philox4x32-10 with key (seed & 0xffffffff, seed >> 32) at
 * counters (k, 0, 0, 0) = r0..r3 and (k, 1, 0, 0) = r4..r7: the cell is the first whose
 * cumulative weight (row-major) exceeds (r1 2^32 + r0) mod W (W the total weight); the
 * centre is at fractional position (r2, r3) / 2^32 in the cell with bilinear height;
 * t_u = normalise(r - (r . n) n) for r = (r4, r5, r6) / 2^31 - 1 (the x axis if that is
 * shorter than 1e-6), t_v = n x t_u; s_u = s_v = sqrt(W g^2 / 65536 / n) (the spacing of
 * n samples over the surface area); opacity and albedo take the given values.
 * Outputs: the ss_surfels arrays of the n surfels, and cell [n] (or NULL) the chosen
 * cell index.  Workspace: device memory of ss_dsm_init_workspace_size bytes, 256-byte
 * aligned. */
ss_status ss_dsm_init_workspace_size(int32_t nx, int32_t ny, size_t *bytes);
ss_status ss_dsm_init(int32_t nx, int32_t ny, const float *z, float x0, float y0, float gsd,
                      int64_t n, uint64_t seed, float opacity, float albedo, void *workspace,
                      size_t bytes, float *mean, float *t_u, float *t_v, float *scale,
                      float *opacity_out, float *albedo_out, int64_t *cell, ss_stream stream);

/* -------------------------------------------------------------- shadow pass
 * Geometric sun-view shadow map (Sec. 3.3 Eq. sun_camera_Bxy, Supp. A; Sec. 3.1 soft
 * shadow test).  Per view: sun camera B_sun = lam * B'_xy (I - [0 0 s]) with
 * s = (cos phi / tan theta, sin phi / tan theta, 1) and a viewport (lam, offset) that
 * maps the flattened surfel-centre bounding box onto the central 98 % of an S x S map;
 * depth-only compositing of the same surfels in the same depth order over a background
 * at z_far = b_z - min z + 10 m; then per surfel k the 3x3 exponential-shadow-map test
 *   vis[v,k] = min(1, mean_t exp(esm_c (D_t - (b_z - p_k,z) + esm_bias))).
 * Requires views->sun.  Outputs: vis [n_views, n]; sun_depth [n_views, S, S] or NULL.
 * The main-view binning held for the backward is not touched. */
ss_status ss_shadow_plain(ss_plan *plan, const ss_surfels *s, const ss_views *v,
                          float *sun_depth, float *vis, ss_stream stream);

/* ---------------------------------------------------------- debug / testing
 * Copy out the binning of the last forward (which = 0) or shadow pass (which = 1):
 *   order       [n]           uint32 surfel indices in centre-depth order
 *   surf_tiles  [n_views,n,4] int32 tile range tx_lo,tx_hi,ty_lo,ty_hi (lo>hi: none)
 *   tile_ranges [n_tiles,2]   uint32 [start,end) into tile_lists, n_tiles over all
 *                             views in view order, row-major tiles inside a view
 *   tile_lists  [pairs]       uint32 surfel indices (pairs = *n_pairs)
 *   records     [n_views,n,24] float projected-surfel records, or NULL (the shadow
 *                             pass keeps only floats 0..15; 16..23 read as zero)
 * *n_tiles and *n_pairs (host) receive the sizes; any output pointer may be NULL. */
ss_status ss_debug_binning(ss_plan *plan, int32_t which, uint32_t *order,
                           int32_t *surf_tiles, uint32_t *tile_ranges,
                           uint32_t *tile_lists, float *records, int64_t *n_tiles,
                           int64_t *n_pairs, ss_stream stream);

/* Sun cameras of the last shadow pass: [n_views, 9] doubles B_sun (2x3 row-major),
 * b_sun (2), z_far (host memory; blocks on stream). */
ss_status ss_debug_sun_cameras(ss_plan *plan, double *out, ss_stream stream);

/* ------------------------------------------------------- batched step / graph
 * One training-step pass over all views: the shadow pass (when views->sun != NULL; it
 * writes io->vis) then the forward with io->vis as the visibility channel, then the
 * backward with the given upstream gradients.  All buffers as in ss_forward,
 * ss_backward and ss_shadow_plain; vis may be NULL only when views->sun is NULL. */
typedef struct ss_step_io {
    uint32_t struct_size;       /* sizeof(ss_step_io)                                    */
    float   *vis;               /* [n_views, n]                                          */
    float   *sun_depth;         /* [n_views, S, S] or NULL (then kept in the workspace)  */
    float   *image, *albedo_out, *vis_out, *depth, *normal, *T_final;
    int32_t *last;
    const float *d_image, *d_depth, *d_normal;          /* each may be NULL              */
    float   *d_mean, *d_t_u, *d_t_v, *d_scale, *d_opacity, *d_albedo;
    float   *d_dF, *d_colC, *d_colc, *d_ambient;
} ss_step_io;

typedef struct ss_graph ss_graph;

ss_status ss_step(ss_plan *plan, const ss_surfels *s, const ss_views *v, const ss_step_io *io,
                  ss_stream stream);

/* Capture ss_step with these exact pointers into a HIP graph (no host synchronisation
 * and no memset nodes inside; grids are sized by the bound pair capacities, counts stay
 * on the device).  Replays read the current contents of all input buffers.  A replay
 * does not check capacity: after a replay the caller must call ss_plan_check, which
 * reports whether the data needed more pairs than bound (the outputs are then incomplete);
 * then rebind a larger workspace and rebuild the graph.  Binding a workspace or changing
 * the settings invalidates every graph captured from the plan: ss_graph_launch then
 * returns SS_ERR_STATE and launches nothing.  The plan must outlive its graphs. */
ss_status ss_graph_build(ss_plan *plan, const ss_surfels *s, const ss_views *v,
                         const ss_step_io *io, ss_graph **out);
ss_status ss_graph_launch(ss_graph *graph, ss_stream stream);
ss_status ss_graph_destroy(ss_graph *graph);

/* Autotuner: times ss_step (median of `reps` runs after one warm run, HIP events) for
 * tile_size in {8, 16, 32} x batch_depth in {32, 64, 128, 256} and leaves the plan on
 * the fastest; *best receives those settings, best_ms its step time.  Candidates whose
 * pairs exceed the bound capacities are skipped (bind capacities counted with
 * tile_size 8, the largest pair count, to try all); so are batch depths above the tile's
 * thread count (tile_size^2: one staged record per thread).  table (host, may be NULL)
 * receives 12 x 3 doubles: tile, batch, ms (ms < 0: skipped). */
ss_status ss_autotune(ss_plan *plan, const ss_surfels *s, const ss_views *v,
                      const ss_step_io *io, int32_t reps, ss_raster_settings *best,
                      double *best_ms, double *table, ss_stream stream);

/* ------------------------------------------------- learned shadow surrogate
 * Not in the paper: a small MLP that stands in for the geometric shadow pass, trained
 * on that pass's labels; the geometric pass stays its fallback.  Network: features of
 * the normalised centre p_hat = fl32(fl32(p - centre) * inv_half), sin and cos of
 * pi 2^k p_hat_c for k = 0..15 and c = 0..2 (interleaved per frequency, coordinate
 * major), then cos phi, sin phi, sin theta, cos theta, zero padded to 128;
 * 128 -> 64 -> 64 -> 64 (ReLU) -> 1.  BF16 weights and activations, FP32 accumulation
 * on MFMA.  Parameters: one FP32 vector [W1 (64x128, row = output), b1, W2 (64x64),
 * b2, W3 (64x64), b3, w4 (64), b4] of 16641 floats (caller-owned device memory). */
typedef struct ss_mlp ss_mlp;
typedef struct ss_mlp_config {
    uint32_t struct_size;   /* sizeof(ss_mlp_config)             */
    float    centre[3];     /* normalisation centre, metres      */
    float    inv_half;      /* 1 / normalisation half extent, 1/m */
} ss_mlp_config;
#define SS_MLP_PARAMS 16641

ss_status ss_mlp_create(ss_context *ctx, const ss_mlp_config *cfg, ss_mlp **out);
ss_status ss_mlp_destroy(ss_mlp *mlp);
/* Workspace for training batches of up to max_points (inference needs only the
 * weight copies, max_points may be 0). */
ss_status ss_mlp_workspace_size(ss_mlp *mlp, int64_t max_points, size_t *bytes);
ss_status ss_mlp_bind_workspace(ss_mlp *mlp, void *workspace, size_t bytes, int64_t max_points);
/* out[i] = logit (or sigmoid(logit) when prob != 0).  all_pairs = 0: point i has
 * position pts[i] and sun sun[i], M = n_pts = n_sun.  all_pairs = 1: M = n_sun * n_pts,
 * point i has position pts[i % n_pts] and sun sun[i / n_pts].  pts [n_pts,3],
 * sun [n_sun,2] (phi, theta) radians. */
ss_status ss_mlp_forward(ss_mlp *mlp, const float *w, const float *pts, int64_t n_pts,
                         const float *sun, int64_t n_sun, int32_t all_pairs, int32_t prob,
                         float *out, ss_stream stream);
/* Gradient (overwritten, [16641]) of  scale * sum_i L_i  for M <= max_points paired
 * points, with L_i = BCE-with-logits(logit_i, labels[i]) when labels != NULL, else
 * L_i = d_logits[i] * logit_i.  loss (device float[1] or NULL) receives
 * scale * sum_i BCE_i.  Backward rounding: each pre-activation gradient is rounded to
 * BF16 before it enters a product (same points as the forward's BF16 operands). */
ss_status ss_mlp_backward(ss_mlp *mlp, const float *w, const float *pts, const float *sun,
                          int64_t M, const float *labels, const float *d_logits, float scale,
                          float *d_w, float *loss, ss_stream stream);
/* Allocation-free variant of ss_mlp_backward, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight training or serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, outputs and rounding as ss_mlp_backward (the same
 * kernels run), but the MLP needs no bound workspace: the buffers live in a fixed device
 * array inside the library of 15.1 MiB per device (held from library load until the
 * process ends), laid out for M <= SS_NOALLOC_MAX_POINTS points; a larger M returns
 * SS_ERR_CAPACITY and launches nothing.  The call allocates nothing, device or host
 * memory.  All calls on one device share that array: calls that overlap on one device
 * (two streams, two threads) race and must be ordered by the caller.  The device address
 * of the array is taken when the context is created (ss_context_create). */
#define SS_NOALLOC_MAX_POINTS 16384
ss_status ss_mlp_backward_noalloc(ss_mlp *mlp, const float *w, const float *pts, const float *sun,
                                  int64_t M, const float *labels, const float *d_logits,
                                  float scale, float *d_w, float *loss, ss_stream stream);
/* Adam on FP32 master weights (step counts from 1). */
ss_status ss_mlp_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr,
                      float beta1, float beta2, float eps, int32_t step, ss_stream stream);
/* Surrogate shadow pass: vis[v,k] = sigmoid(MLP(p_k, sun_v)) for every view and surfel;
 * points with |vis - 0.5| < band fall back to the geometric pass (ss_shadow_plain's
 * definition), rasterizing only the sun-map tiles their 3x3 windows touch.  Requires
 * views->sun.  The number of fallback points is reported by ss_plan_stats ([6]).  With
 * band == 0 only the network runs: no sun camera, binning or raster, and sun_depth is
 * not written. */
ss_status ss_shadow_surrogate(ss_plan *plan, ss_mlp *mlp, const float *w, const ss_surfels *s,
                              const ss_views *v, float band, float *vis, float *sun_depth,
                              ss_stream stream);

/* ------------------------------------------------------------ measurement
 * Stage timing: when enabled, the library records a HIP event pair on the call's
 * stream around each stage below; ss_plan_read_timing blocks until the recorded
 * events completed, adds their elapsed times to ms[stage] / launches[stage] (host
 * arrays of SS_NUM_STAGES) and forgets them.  Stages that are a single kernel:
 * RASTER_FWD, RASTER_BWD, PROJECT, PROJECT_BWD, SUN_RASTER, SHADOW_QUERY. */
#define SS_STAGE_DEPTH_SORT   0   /* depth keys, 4-pass radix sort, gather into rank order */
#define SS_STAGE_PROJECT      1   /* main-view projection + tile ranges                    */
#define SS_STAGE_BIN          2   /* pair-count scan, emission, tile sort, tile ranges     */
#define SS_STAGE_RASTER_FWD   3
#define SS_STAGE_RASTER_BWD   4
#define SS_STAGE_PROJECT_BWD  5
#define SS_STAGE_REDUCE       6   /* gradient zeroing, colour and camera-delta reductions  */
#define SS_STAGE_SUN_CAMERA   7   /* scene bounds + sun cameras                            */
#define SS_STAGE_SUN_PROJECT  8
#define SS_STAGE_SUN_BIN      9
#define SS_STAGE_SUN_RASTER  10   /* depth-only compositing of the sun maps                */
#define SS_STAGE_SHADOW_QUERY 11
#define SS_STAGE_MLP         12   /* surrogate MLP inference (weight copy + fused forward)  */
#define SS_STAGE_FALLBACK_FLAG 13 /* surrogate fallback: flag points and their sun tiles    */
#define SS_STAGE_NORMAL_LOSS 14   /* depth-gradient normals and the normal-consistency loss */
#define SS_STAGE_IMAGE_LOSS  15   /* L1 image loss and its gradient                         */
#define SS_NUM_STAGES        16
ss_status ss_plan_set_timing(ss_plan *plan, int32_t enable);
ss_status ss_plan_read_timing(ss_plan *plan, double *ms, int64_t *launches);
const char *ss_stage_name(int32_t stage);

/* Work counters of the last forward / shadow pass (blocks on stream), host int64[7]:
 *   [0] pairs bound (tile, surfel) main views   [1] contributing (pixel, surfel) pairs
 *   [2] evaluated (pixel, surfel) pairs after per-wave culling (main views)
 *   [3] pairs bound, sun views   [4] contributing pairs, sun   [5] evaluated pairs, sun
 *   [6] fallback points of the last surrogate shadow pass */
ss_status ss_plan_stats(ss_plan *plan, int64_t *out, ss_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* SATSPLAT_H */
