// Internal declarations of the gfx950 SatSplat hot path: data layouts shared by the
// kernels and the C-ABI layer.  Nothing here is part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace ss {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------------
// Projected-surfel record: one per (view, depth rank), 24 floats = 96 B = 6 x float4,
// array-of-structures so an LDS batch load is 6 contiguous float4 per record.  The raster
// kernels gather records at random, so each sits in a slot that is one aligned piece of an
// L2 line (at a 96-byte stride half of them would straddle two lines): view records in
// 128-byte slots (the last 32 B zero), sun-view records, of which only vec4 0..3 exist, in
// 64-byte slots.
//   vec4 0: box_x, box_y, c_hi.x, c_hi.y
//   vec4 1: c_lo.x, c_lo.y, off_u, off_f
//   vec4 2: Q00, Q01, Q10, Q11
//   vec4 3: o, z0, k_u, k_v
//   vec4 4: albedo r, g, b, v
//   vec4 5: n_x, n_y, n_z, nsign
//   c      : projected centre B'_xy p + b'_xy as FP32 hi + lo (hi + lo = the FP64 value
//            to ~1e-14 relative), so x - c keeps full FP32 precision far from the origin.
//   Q      : (B'_xy [s_u t_u, s_v t_v])^-1, screen -> uv (Eq. affine2dgs_Qq)
//   z0, k  : depth plane z(u,v) = z0 - k_u u - k_v v, z0 = b_z - p_z,
//            k = (s_u t_u.z, s_v t_v.z) (Eq. depth_affine_camera on Eq. affine2dgs_uv2screen)
//   off_u  : 0, or +inf for a degenerate surfel (no uv branch)
//   off_f  : 0, or +inf when the low-pass floor is off for this surfel
//   box    : inclusive pixel box as int16 pairs (lo | hi << 16) for per-wave culling
//   v      : sun visibility composited into the V channel (1 when none is given)
//   nsign  : +-1, normal orientation (n = nsign * m / |m|, m = t_u x t_v)
// The depth-only (sun-view) raster reads only vec4 0..3, the only ones sun records hold.
// Raster work counters (contributing, evaluated pairs): every wave adds to the slot of its
// tile modulo kStatSlots, each slot on its own 128-byte line, so the adds of 10^6 waves
// do not queue on one address; readers sum the slots.
constexpr int kStatSlots = 256;
constexpr int kStatStride = 16;   // 64-bit words per slot
constexpr int kRecFloats = 24;
constexpr int kRecVec4 = 6;
constexpr int kRecStride4 = 8;      // float4 per view record slot
constexpr int kSunRecStride4 = 4;   // float4 per sun-view record slot

// Per-(view, surfel) record gradient, 16 floats (written with one 16-lane atomic
// instruction per wave after a transpose reduction).
enum GradField {
    G_CX = 0, G_CY, G_Q00, G_Q01, G_Q10, G_Q11, G_Z0, G_KU, G_KV, G_O,
    G_AR, G_AG, G_AB, G_NX, G_NY, G_NZ, G_COUNT
};
constexpr int kGradFloats = 16;

struct ViewDesc {
    int32_t W, H, tiles_x, tiles_y;
    int64_t pix_off;
    int32_t tile_off;
    int32_t pad;
};

// FP64 sun camera of one view: B_sun (2x3), b_sun (2), z_far.
struct SunCam {
    double B[6];
    double b[2];
    double zfar;
    double pad[7];
};

// Per-view back-projection of the depth-normal loss: Minv = [B_x; B_y; (0,0,-1)]^-1
// (row-major) and the view direction d = B_x x B_y with d_z < 0.
struct GeomCam {
    double Minv[9];
    double d[3];
    double pad[4];
};

struct RasterConsts {
    float alpha_min, alpha_max, T_min, inv_s2;
    int32_t lowpass_mode;
    int32_t batch;
    float esm_c, esm_bias;
    float two_inv_s2;   // 2 inv_s2, a kernel argument so that loops read it from an SGPR
    double alpha_min_d, sigma_d, det_rel_eps_d;
    // dispatch order of the raster kernels: block b rasterizes tile torder[b] (a
    // permutation from launch_tile_order), or xcd_tile(b) when null
    const uint32_t *torder;
};

// Depth-distortion channel of the view raster (the 2DGS squared form of the distortion
// loss): per pixel the forward writes dist = sum over contributor pairs of
// w_i w_j (m_i - m_j)^2, m = z * ds, and saves aux = (z_ref, M1, M2): the depth of the
// pixel's first contributor and sum w m', sum w m'^2 of m' = (z - z_ref) * ds (shifted
// so the moments do not cancel); the backward reads aux and the upstream d_dist.
// Planar over all pixels of all views: aux[k * P + g].
struct DistArgs {
    float ds;
    float *dist;
    float *aux;
    const float *d_dist;
    int64_t P;
};

struct SurfelPtrs {
    const float *mean, *t_u, *t_v, *scale, *opacity, *albedo;
    int64_t n;
};

// Workgroups go round-robin to the 8 XCDs, each with its own L2, and an XCD never takes
// another's.  XCD x gets chunks x, x + 8, x + 16, ... of kXcdChunk consecutive ids: the
// tiles of a few tile rows (or the views of a few blocks of surfels) share one L2, and
// every XCD samples the whole id range, so work that varies along it (views of different
// size and density) is spread evenly; one contiguous run per XCD left the busiest XCD
// 8 % above the mean.  With CHUNKED false every XCD gets one contiguous run instead, for
// id ranges whose work is even along them (sun maps: equal sizes, similar content), where
// it keeps more neighbours under one L2.  Bijective on [0, nblocks): the last
// nblocks % (8 kXcdChunk) ids map to themselves.
constexpr int kXcdChunk = 512;
template <bool CHUNKED = true>
__device__ __forceinline__ int xcd_tile(int bid, int nblocks)
{
    constexpr int kXcd = 8;
    if (!CHUNKED) {
        const int q = nblocks / kXcd, r = nblocks % kXcd;
        const int x = bid % kXcd, i = bid / kXcd;
        return x * q + min(x, r) + i;
    }
    const int full = nblocks - nblocks % (kXcd * kXcdChunk);
    if (bid >= full) return bid;
    const int x = bid % kXcd, i = bid / kXcd;
    return ((i / kXcdChunk) * kXcd + x) * kXcdChunk + i % kXcdChunk;
}

// Heavy tiles first (longest-processing-time-first, in two classes): keeps every tile on
// the XCD that xcd_tile<CHUNKED> gives it, and reorders each XCD's blocks so that its
// tiles with at least twice the mean list length (total_pairs / ntiles) run first, each
// class in its original order.  order[b] = tile for block b; parts holds
// 8 * tile_order_blocks(ntiles) + 8 words.
int tile_order_blocks(int32_t ntiles);
hipError_t launch_tile_order(const uint32_t *ranges, int32_t ntiles,
                             const unsigned long long *total_pairs, bool chunked,
                             uint32_t *order, uint32_t *parts, hipStream_t st);

// ------------------------------------------------------------------- launchers
// sort.hip
// Temp bytes of radix_sort_pairs for up to max_items items in up to max_segs segments.
size_t radix_temp_bytes(int64_t max_items, int32_t max_segs);
hipError_t fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t st);
hipError_t fill_f32(float *p, float value, int64_t count, hipStream_t st);
// Exclusive scan of per-(view, rank) tile counts (contiguous, depth-rank order):
// out[v*n + r] = sum of counts before (v, r); out[V*n] = total; flags[0] |= 1 if the
// total exceeds 2^32-1 or `cap`; counters[which] = total (uint64).
hipError_t scan_pair_counts(const uint32_t *counts, int64_t n,
                            int32_t nv, uint32_t *out, uint32_t *partials,
                            unsigned long long *counters, int which, uint32_t *flags,
                            uint64_t cap, hipStream_t st);
size_t scan_temp_elems(int64_t len);
// Items that arrive grouped in segments, each sorted on its own keys minus a base:
// segment v holds items [offs[v * stride], offs[(v + 1) * stride]) (clamped to the live
// count) with keys in [views[v].tile_off, views[v].tile_off + 2^bits).  The result equals
// a stable sort of the whole array on the key.  With `ranges` (nkeys entries of
// (begin, end), interleaved), the sort also writes each key's output run; keys with no
// item get (0, 0).
struct SortSegments {
    const uint32_t *offs;
    int64_t stride;
    int32_t nseg;
    const ViewDesc *views;
    uint32_t *ranges;
    int64_t nkeys;
};
// Stable LSD radix sort of (key, value) uint32 pairs on the low `bits` bits of key
// (of key minus its segment base with `seg`).  Item count is n_dev ? min(*n_dev, cap) :
// n_host.  Returns (via *result_in_b) whether the sorted data ended in the b buffers.
// KT = uint16_t sorts keys local to their segment (tile ids within a view, at most
// 2^16 per view); the tile ranges are then written at the segment's base plus the key.
template <typename KT>
hipError_t radix_sort_pairs(KT *keys_a, uint32_t *vals_a, KT *keys_b,
                            uint32_t *vals_b, int64_t cap, const unsigned long long *n_dev,
                            int64_t n_host, int bits, void *temp, bool *result_in_b,
                            hipStream_t st, const SortSegments *seg = nullptr);

// raster.hip
hipError_t launch_depth_keys(const float *mean, int64_t n, float bz, uint32_t *keys,
                             uint32_t *vals, hipStream_t st);
hipError_t launch_gather_params(const uint32_t *order, const SurfelPtrs &s, float *out,
                                hipStream_t st);
// vis_rank: visibility per (rank, view), [n][nv] (see launch_vis_to_rank), or NULL.
hipError_t launch_project(const float *sorted, int64_t n, int32_t nv, const ViewDesc *views,
                          const float *Fxy, const float *dF, const SunCam *sun,
                          const float *vis_rank, float bz, int ts, const RasterConsts &rc,
                          float *rec, short4 *tiles, uint32_t *counts, const uint32_t *tmask,
                          hipStream_t st);
// out[rank * nv + v] = vis[v * n + order[rank]]; rank (n entries) is scratch that ends up
// holding the inverse of order.
hipError_t launch_vis_to_rank(const float *vis, int64_t n, int32_t nv, const uint32_t *order,
                              uint32_t *rank, float *out, hipStream_t st);
// keys16: tile ids local to the view as uint16 (views of at most 2^16 tiles), else the
// global tile id as uint32; `keys` points at the chosen width.
hipError_t launch_emit(const uint32_t *order, int64_t n, int32_t nv, const ViewDesc *views,
                       const short4 *tiles, const uint32_t *counts, const uint32_t *offsets,
                       uint64_t cap, void *keys, bool keys16, uint32_t *vals,
                       const uint32_t *tmask, hipStream_t st);
hipError_t launch_raster_fwd(int ts, bool depth_only, bool has_vis, int32_t total_tiles,
                             int32_t nv, const ViewDesc *views, const uint32_t *ranges,
                             const uint32_t *lists, const float *rec, int64_t n,
                             const RasterConsts &rc, const float *colC, const float *colc,
                             const float *amb, const SunCam *sun, float *image, float *A,
                             float *V, float *D, float *N, float *T, int32_t *last,
                             unsigned long long *stats, unsigned long long *cmask, hipStream_t st,
                             const DistArgs *dist = nullptr);
hipError_t launch_raster_bwd(int ts, bool has_vis, int32_t total_tiles, int32_t nv,
                             const ViewDesc *views, const uint32_t *ranges,
                             const uint32_t *lists, const float *rec, int64_t n,
                             const RasterConsts &rc, const float *colC, const float *colc,
                             const float *amb, const float *A, const float *V,
                             const float *T, const int32_t *last, const float *dI,
                             const float *dD, const float *dN, float *recgrad,
                             float *colour_partials, const unsigned long long *cmask,
                             hipStream_t st, const DistArgs *dist = nullptr);
// Contributor masks (8x8 tiles): for tile t with list start s, word w of pixel (lane) l is
// cmask[(s / 64 + t + w) * 64 + l], bit b set iff list position 64 w + b was composited;
// the ranges of different tiles are disjoint, so (pairs / 64 + tiles + 1) * 64 words suffice.
size_t cmask_words(int64_t pair_cap, int32_t tiles);
hipError_t launch_colour_reduce(const float *partials, int32_t nv, const ViewDesc *views,
                                float *d_colC, float *d_colc, float *d_amb, hipStream_t st);
int project_bwd_blocks(int64_t n);
hipError_t launch_project_bwd(const float *sorted, int64_t n, const uint32_t *order,
                              int32_t nv, const float *Fxy, const float *dF, double det_rel_eps,
                              const float *recgrad, float *d_mean, float *d_tu, float *d_tv,
                              float *d_scale, float *d_opac, float *d_alb, float *dF_partials,
                              hipStream_t st);
hipError_t launch_dF_reduce(const float *partials, int nblocks, int32_t nv, float *d_dF,
                            hipStream_t st);
// out row (v, order[r]) = the first row_words words of in row (v, r), in rows in_stride
// words apart (words past in_stride read as zero)
hipError_t launch_unpermute_rows(const uint32_t *order, int64_t n, int32_t nv,
                                 const uint32_t *in, int in_stride, int row_words,
                                 uint32_t *out, hipStream_t st);
hipError_t launch_unpermute_tiles(const uint32_t *order, int64_t n, int32_t nv, const short4 *t,
                                  int32_t *out, hipStream_t st);
hipError_t launch_map_through(const uint32_t *order, int64_t n_order,
                              const unsigned long long *n_dev, int64_t cap, const uint32_t *in,
                              uint32_t *out, hipStream_t st);

// geom.hip: depth-gradient normals and the normal-consistency loss over all views.
// seeds: one float2 per pixel; partials: normal_loss_blocks(host views) * nv * 10 doubles;
// cams: nv entries.  loss [nv] is written; d_depth, d_normal and d_dF are added to.
int normal_loss_blocks(const ViewDesc *host_views, int32_t nv);
hipError_t launch_normal_loss(const ViewDesc *views, const ViewDesc *host_views, int32_t nv,
                              int64_t max_view_pixels,
                              const float *Fxy, const float *dF, const float *D, const float *T,
                              const float *Nr, float weight, float tau, GeomCam *cams,
                              float2 *seeds, double *partials, float *loss, float *Nd_out,
                              float *d_depth, float *d_normal, float *d_dF, hipStream_t st);

// train.hip: surfel activations, fused activation adjoint + Adam, per-view Adam, L1 loss.
// lr: mean, scale, opacity, quaternion, albedo, camera delta, colour.
struct AdamArgs {
    float lr[7];
    float beta1, beta2, eps;
    int32_t camera_start;
};
hipError_t launch_surfel_activate(int64_t n, const float *raw, float *mean, float *tu, float *tv,
                                  float *scale, float *opacity, float *albedo, hipStream_t st);
hipError_t launch_surfel_raw(int64_t n, const float *mean, const float *tu, const float *tv,
                             const float *scale, const float *opacity, const float *albedo,
                             float *raw, hipStream_t st);
hipError_t launch_adam_surfels(int64_t n, float *raw, float *m, float *v, const float *g_mean,
                               const float *g_tu, const float *g_tv, const float *g_scale,
                               const float *g_opacity, const float *g_albedo, const AdamArgs &a,
                               int32_t step, float *mean, float *tu, float *tv, float *scale,
                               float *opacity, float *albedo, hipStream_t st);
hipError_t launch_adam_views(int32_t nv, float *dF, float *m_dF, float *v_dF, const float *g_dF,
                             const float *g_dF2, float *colC, float *m_C, float *v_C, const float *g_C, float *colc,
                             float *m_c, float *v_c, const float *g_c, const AdamArgs &a,
                             int32_t step, hipStream_t st);
int l1_blocks(int64_t max_view_pixels);
hipError_t launch_l1_loss(const ViewDesc *views, int32_t nv, int64_t max_view_pixels,
                          const float *img, const float *tgt, float weight, float *d_img,
                          double *partials, float *loss, hipStream_t st);

// init.hip: geometry-aware initialisation on a DSM (area-weighted sampling, frames).
size_t dsm_init_workspace_bytes(int nx, int ny);
hipError_t launch_dsm_init(int nx, int ny, const float *z, double x0, double y0, double g, int64_t n,
                           uint64_t seed, float opacity, float albedo, void *ws, float *mean,
                           float *tu, float *tv, float *scale, float *opac, float *alb,
                           int64_t *cell, hipStream_t st);

// shadow.hip
int bounds_blocks(int64_t n);
hipError_t launch_sun_cameras(const float *mean, int64_t n, int32_t nv, const float *Fxy,
                              const float *dF, const float *sun, float bz, int32_t S,
                              double *bounds_partials, SunCam *out, hipStream_t st);
hipError_t launch_shadow_query(const float *mean, int64_t n, int32_t nv, const SunCam *sun,
                               const float *sun_depth, int32_t S, float bz, float esm_c,
                               float esm_bias, float *vis, float band, hipStream_t st);
hipError_t launch_flag_tiles(const float *mean, int64_t n, int32_t nv, const SunCam *sun,
                             const ViewDesc *views, int32_t S, int ts, const float *vis,
                             float band, uint32_t *tmask, unsigned long long *count, hipStream_t st);

}  // namespace ss
