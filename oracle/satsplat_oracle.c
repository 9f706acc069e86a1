/*
 * FP64 CPU oracle for the affine-camera 2D-Gaussian-surfel rasterizer and the
 * sun-view shadow pass.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke entry point and the CPU
 * baseline leg of the benchmark may load this library.  The product path never calls
 * it, and it shares no code with the HIP kernels.
 *
 * It is deliberately plain: every pixel walks ALL surfels in centre-depth order
 * (no tiles, no culling, no early batching), in double precision, with the inputs
 * (FP32 arrays) widened exactly.  Paper references are to SatSplat (arXiv 2606.28581):
 *   image formation           Sec. 3.1, Eq. (image_formation)
 *   affine camera             Sec. 3.1, Eq. (affine_camera); Sec. 3.2 Eq. (decompose_affine_camera)
 *   surfel                    Sec. 3.1, Eqs. (2dgs_splat_param), (2dgs_splat_H)
 *   ray-splat intersection    Sec. 3.2, Eqs. (affine2dgs_uv2screen), (affine2dgs_screen2uv),
 *                             (affine2dgs_Qq)
 *   depth function            Sec. 3.2, Eq. (depth_affine_camera)
 *   degenerate / low-pass     Sec. 3.2, "Degenerate Solutions"
 *   normal                    Sec. 3.2, "Normal Definition"
 *   tiles, centre-depth sort,
 *   alpha blending            Sec. 3.2, "Rasterization", Eq. (rasterization)
 *   camera delta              Sec. 3.3, F'_xy = F_xy + dF_xy
 *   sun camera                Sec. 3.3, Eq. (sun_camera_Bxy); Supp. A, Eqs. (S1)-(S4)
 *   ESM-softened shadow test  Sec. 3.1 (shadow-mapping note after the image formation)
 *
 * Readings where the paper is silent (shared with the GPU path, listed in the design
 * notes): alpha = min(alpha_max, o*G) with alpha_max = 0.99; skip alpha < alpha_min;
 * stop before the surfel that would take T below T_min; low-pass sigma = sqrt(2)/2 px
 * applied to every surfel (mode 0) or only to degenerate ones (mode 1); degenerate iff
 * |det T| <= eps*|T|_F^2; normals flipped to face the camera; V == 1 when no
 * visibility is given; sun-map background at z_far; 3x3 ESM window.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double alpha_min, alpha_max, T_min, sigma, det_rel_eps;
    int32_t lowpass_mode;   /* 0: low-pass floor for every surfel; 1: degenerate only */
    double esm_c, esm_bias;
    double depth_scale;     /* normalised depth m = z * depth_scale (distortion term)  */
} or_settings;

/* One surfel as seen by one affine camera, everything in FP64. */
typedef struct {
    double p[3], tu[3], tv[3], su, sv;
    double M[3][2];         /* [s_u t_u, s_v t_v]                                   */
    double T[2][2];         /* B_xy * M  (uv -> screen)                             */
    double Q[2][2];         /* T^-1      (screen -> uv)                             */
    double c[2];            /* B_xy p + b_xy                                        */
    int    degenerate;
    int    filter_on;
    double z0;              /* b_z - p_z : centre depth                             */
    double k[2];            /* (s_u t_u.z, s_v t_v.z): z(u,v) = z0 - k.(u,v)        */
    double m[3], mnorm, nsign, n[3];
    double o, a[3], v;
} or_proj;

typedef struct {
    double B[2][3], b[2];
} or_cam;

static void cam_from(const float *F, const float *dF, or_cam *cam)
{
    /* F' = F + dF (Sec. 3.3); F is [2,4] row-major: [B_xy | b_xy] */
    for (int r = 0; r < 2; ++r) {
        for (int j = 0; j < 3; ++j)
            cam->B[r][j] = (double)F[r * 4 + j] + (dF ? (double)dF[r * 4 + j] : 0.0);
        cam->b[r] = (double)F[r * 4 + 3] + (dF ? (double)dF[r * 4 + 3] : 0.0);
    }
}

static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static void project_one(const or_cam *cam, double bz, const float *mean, const float *tu,
                        const float *tv, const float *scale, float opac, const float *alb,
                        double vis, const or_settings *st, or_proj *pr)
{
    for (int i = 0; i < 3; ++i) {
        pr->p[i] = mean[i]; pr->tu[i] = tu[i]; pr->tv[i] = tv[i]; pr->a[i] = alb[i];
    }
    pr->su = scale[0]; pr->sv = scale[1];
    pr->o = opac; pr->v = vis;
    for (int i = 0; i < 3; ++i) {
        pr->M[i][0] = pr->su * pr->tu[i];
        pr->M[i][1] = pr->sv * pr->tv[i];
    }
    for (int r = 0; r < 2; ++r) {
        for (int q = 0; q < 2; ++q) {
            double s = 0.0;
            for (int i = 0; i < 3; ++i) s += cam->B[r][i] * pr->M[i][q];
            pr->T[r][q] = s;
        }
        double s = cam->b[r];
        for (int i = 0; i < 3; ++i) s += cam->B[r][i] * pr->p[i];
        pr->c[r] = s;
    }
    double det = pr->T[0][0] * pr->T[1][1] - pr->T[0][1] * pr->T[1][0];
    double fro2 = pr->T[0][0] * pr->T[0][0] + pr->T[0][1] * pr->T[0][1] +
                  pr->T[1][0] * pr->T[1][0] + pr->T[1][1] * pr->T[1][1];
    pr->degenerate = !(fabs(det) > st->det_rel_eps * fro2);
    if (!pr->degenerate) {
        pr->Q[0][0] = pr->T[1][1] / det;  pr->Q[0][1] = -pr->T[0][1] / det;
        pr->Q[1][0] = -pr->T[1][0] / det; pr->Q[1][1] = pr->T[0][0] / det;
    } else {
        memset(pr->Q, 0, sizeof pr->Q);
    }
    pr->filter_on = (st->lowpass_mode == 0) || pr->degenerate;
    /* depth function B_z = [0,0,-1], b_z = max altitude: z = b_z - P_z(u,v) */
    pr->z0 = bz - pr->p[2];
    pr->k[0] = pr->M[2][0];
    pr->k[1] = pr->M[2][1];
    /* normal = t_u x t_v (normalised), oriented against the main view direction
     * d = B_x x B_y chosen with d_z < 0 (looking down). */
    cross3(pr->tu, pr->tv, pr->m);
    pr->mnorm = sqrt(pr->m[0] * pr->m[0] + pr->m[1] * pr->m[1] + pr->m[2] * pr->m[2]);
    double d[3];
    cross3(cam->B[0], cam->B[1], d);
    if (d[2] > 0) { d[0] = -d[0]; d[1] = -d[1]; d[2] = -d[2]; }
    double nd = pr->m[0] * d[0] + pr->m[1] * d[1] + pr->m[2] * d[2];
    pr->nsign = (nd > 0) ? -1.0 : 1.0;
    for (int i = 0; i < 3; ++i) pr->n[i] = pr->nsign * pr->m[i] / pr->mnorm;
}

/* ------------------------------------------------------------------ depth order */
typedef struct { float kap; int64_t idx; } key_t_;

static int cmp_key(const void *A, const void *B)
{
    const key_t_ *a = (const key_t_ *)A, *b = (const key_t_ *)B;
    if (a->kap < b->kap) return -1;
    if (a->kap > b->kap) return 1;
    /* equal values: -0 before +0, then ascending index */
    int sa = signbit(a->kap) ? 0 : 1, sb = signbit(b->kap) ? 0 : 1;
    if (sa != sb) return sa - sb;
    return (a->idx < b->idx) ? -1 : (a->idx > b->idx);
}

/* Centre-depth order (Sec. 3.2, Rasterization + Eq. depth_affine_camera): the key is the
 * FP32 difference kappa = b_z - p_z, ascending, ties by ascending surfel index. */
void or_depth_order(int64_t n, const float *mean, float bz, int64_t *order)
{
    key_t_ *k = (key_t_ *)malloc(sizeof(key_t_) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        volatile float d = bz - mean[3 * i + 2];
        k[i].kap = d;
        k[i].idx = i;
    }
    qsort(k, (size_t)n, sizeof(key_t_), cmp_key);
    for (int64_t i = 0; i < n; ++i) order[i] = k[i].idx;
    free(k);
}

/* ------------------------------------------------------------- per pixel kernel */
typedef struct {
    int64_t sidx;           /* surfel index */
    double alpha, G, oG, rho, u[2], d[2], z, Tb;
    int ubranch;
} or_hit;

typedef struct {
    double A[3], V, D, N[3], T;
    int64_t count;
    int ambiguous;
    uint64_t sig;           /* digest of the pixel's discrete decisions (test support) */
} or_px;

/* Folds one decision into a pixel's signature (FNV-1a over 64-bit words).  The
 * signature changes whenever the set of contributing surfels, a branch, a clamp, a
 * degenerate flag or a normal orientation changes; finite-difference tests use it to discard steps that cross
 * a discontinuity. */
static uint64_t sig_mix(uint64_t h, uint64_t word)
{
    for (int b = 0; b < 8; ++b) {
        h ^= (word >> (8 * b)) & 0xFFu;
        h *= 1099511628211ull;
    }
    return h;
}

/* Front-to-back compositing (Eq. rasterization) at pixel centre x over all surfels in
 * the global depth order.  If hits != NULL the contributing pairs are recorded. */
static void render_pixel(const or_proj *pj, const int64_t *order, int64_t n, double x,
                         double y, const or_settings *st, int has_vis, or_px *out,
                         or_hit *hits, int64_t max_hits)
{
    double T = 1.0;
    memset(out, 0, sizeof *out);
    out->sig = 1469598103934665603ull;
    const double inv_s2 = 1.0 / (st->sigma * st->sigma);
    for (int64_t r = 0; r < n; ++r) {
        const or_proj *p = &pj[order[r]];
        double dx = x - p->c[0], dy = y - p->c[1];
        double u0 = 0, u1 = 0, rho_u = INFINITY, rho_f = INFINITY;
        if (!p->degenerate) {
            u0 = p->Q[0][0] * dx + p->Q[0][1] * dy;
            u1 = p->Q[1][0] * dx + p->Q[1][1] * dy;
            rho_u = u0 * u0 + u1 * u1;
        }
        if (p->filter_on) rho_f = (dx * dx + dy * dy) * inv_s2;
        int ub = rho_u <= rho_f;
        double rho = ub ? rho_u : rho_f;
        if (isinf(rho)) continue;
        double G = exp(-0.5 * rho);
        double oG = p->o * G;
        double alpha = oG < st->alpha_max ? oG : st->alpha_max;
        if (fabs(oG - st->alpha_min) <= 1e-5 * st->alpha_min) out->ambiguous = 1;
        if (alpha < st->alpha_min) continue;
        double Tn = T * (1.0 - alpha);
        if (fabs(Tn - st->T_min) <= 1e-5 * st->T_min) out->ambiguous = 1;
        if (Tn < st->T_min) {
            out->sig = sig_mix(out->sig, ~(uint64_t)order[r]);
            break;
        }
        out->sig = sig_mix(out->sig, (uint64_t)order[r] << 4 | (uint64_t)(p->nsign < 0) << 3 |
                                     (uint64_t)ub << 2 | (uint64_t)(oG >= st->alpha_max) << 1 |
                                     (uint64_t)p->degenerate);
        if (fabs(oG - st->alpha_max) <= 1e-5) out->ambiguous = 1;
        if (!p->degenerate && p->filter_on && fabs(rho_u - rho_f) <= 1e-5 * rho)
            out->ambiguous = 1;
        double w = alpha * T;
        double z = ub ? p->z0 - p->k[0] * u0 - p->k[1] * u1 : p->z0;
        for (int i = 0; i < 3; ++i) {
            out->A[i] += w * p->a[i];
            out->N[i] += w * p->n[i];
        }
        if (has_vis) out->V += w * p->v;
        out->D += w * z;
        if (hits && out->count < max_hits) {
            or_hit *h = &hits[out->count];
            h->sidx = order[r]; h->alpha = alpha; h->G = G; h->oG = oG; h->rho = rho;
            h->u[0] = u0; h->u[1] = u1; h->d[0] = dx; h->d[1] = dy; h->z = z; h->Tb = T;
            h->ubranch = ub;
        }
        out->count++;
        T = Tn;
    }
    out->T = T;
}

static void colour_terms(const float *colC, const float *colc, const float *amb, int v,
                         double C[3][3], double c[3], double La[3])
{
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) C[i][j] = colC ? colC[v * 9 + i * 3 + j] : (i == j);
        c[i] = colc ? colc[v * 3 + i] : 0.0;
        La[i] = amb ? amb[v * 3 + i] : 0.0;
    }
}

static or_proj *project_view(int64_t n, const float *mean, const float *tu, const float *tv,
                             const float *scale, const float *opac, const float *alb,
                             const float *vis_v, const or_cam *cam, double bz,
                             const or_settings *st)
{
    or_proj *pj = (or_proj *)malloc(sizeof(or_proj) * (size_t)(n > 0 ? n : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        project_one(cam, bz, mean + 3 * i, tu + 3 * i, tv + 3 * i, scale + 2 * i, opac[i],
                    alb + 3 * i, vis_v ? (double)vis_v[i] : 1.0, st, &pj[i]);
    return pj;
}

static int view_of(const int64_t *poff, int nv, int64_t g)
{
    int v = 0;
    while (v + 1 < nv && g >= poff[v + 1]) ++v;
    return v;
}

/* Depth distortion of one pixel (the 2DGS form of the Mip-NeRF 360 distortion the paper
 * weights in its loss, Supp. B): the sum over ordered pairs of contributors of
 * w_i w_j (m_i - m_j)^2, m = z * depth_scale, written as the plain double sum. */
static double pixel_distortion(const or_hit *hits, int64_t count, double ds)
{
    double d = 0.0;
    for (int64_t i = 0; i < count; ++i) {
        const double wi = hits[i].alpha * hits[i].Tb, mi = hits[i].z * ds;
        for (int64_t j = 0; j < i; ++j) {
            const double wj = hits[j].alpha * hits[j].Tb, mj = hits[j].z * ds;
            d += wi * wj * (mi - mj) * (mi - mj);
        }
    }
    return d;
}

/*
 * Forward render.  Pixels are addressed by a global index g over the concatenation of
 * all views (view v covers [poff[v], poff[v+1]), row-major inside the view).  If sel is
 * NULL all pixels are rendered and outputs are laid out per view planar CHW exactly
 * like the GPU outputs; otherwise outputs are compact, one entry per selected pixel
 * (image/A/N as [nsel,3]).
 */
void or_forward(int64_t n, const float *mean, const float *tu, const float *tv,
                const float *scale, const float *opac, const float *alb,
                int32_t nv, const int32_t *W, const int32_t *H, const float *Fxy,
                const float *dF, const float *colC, const float *colc, const float *amb,
                const float *vis, float bz, const or_settings *st,
                int64_t nsel, const int64_t *sel,
                double *img, double *Aout, double *Vout, double *Dout, double *Nout,
                double *Tout, int64_t *count, uint8_t *ambig, uint64_t *sig, double *dist)
{
    int64_t *poff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv + 1));
    poff[0] = 0;
    for (int v = 0; v < nv; ++v) poff[v + 1] = poff[v] + (int64_t)W[v] * H[v];
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    or_depth_order(n, mean, bz, order);
    int64_t total = sel ? nsel : poff[nv];
    for (int v = 0; v < nv; ++v) {
        or_cam cam;
        cam_from(Fxy + 8 * v, dF ? dF + 8 * v : NULL, &cam);
        or_proj *pj = project_view(n, mean, tu, tv, scale, opac, alb,
                                   vis ? vis + (int64_t)v * n : NULL, &cam, bz, st);
        double C[3][3], c[3], La[3];
        colour_terms(colC, colc, amb, v, C, c, La);
        #pragma omp parallel
        {
        /* the distortion needs every contributor of the pixel */
        const int64_t max_hits = dist ? (n > 0 ? n : 1) : 0;
        or_hit *hits = dist ? (or_hit *)malloc(sizeof(or_hit) * (size_t)max_hits) : NULL;
        #pragma omp for schedule(dynamic, 16)
        for (int64_t s = 0; s < total; ++s) {
            int64_t g = sel ? sel[s] : s;
            if (g < poff[v] || g >= poff[v + 1]) continue;
            int64_t local = g - poff[v];
            int64_t P = poff[v + 1] - poff[v];
            int i = (int)(local % W[v]), j = (int)(local / W[v]);
            or_px px;
            render_pixel(pj, order, n, i + 0.5, j + 0.5, st, vis != NULL, &px, hits, max_hits);
            if (dist) dist[sel ? s : g] = pixel_distortion(hits, px.count, st->depth_scale);
            double Vp = vis ? px.V : 1.0;
            double I[3];
            for (int ch = 0; ch < 3; ++ch) {
                double ca = c[ch];
                for (int q = 0; q < 3; ++q) ca += C[ch][q] * px.A[q];
                I[ch] = ca * (Vp + (1.0 - Vp) * La[ch]);
            }
            if (sel) {
                for (int ch = 0; ch < 3; ++ch) {
                    img[3 * s + ch] = I[ch]; Aout[3 * s + ch] = px.A[ch];
                    Nout[3 * s + ch] = px.N[ch];
                }
                Vout[s] = Vp; Dout[s] = px.D; Tout[s] = px.T; count[s] = px.count;
                ambig[s] = (uint8_t)px.ambiguous;
                if (sig) sig[s] = px.sig;
            } else {
                int64_t b3 = 3 * poff[v];
                for (int ch = 0; ch < 3; ++ch) {
                    img[b3 + ch * P + local] = I[ch]; Aout[b3 + ch * P + local] = px.A[ch];
                    Nout[b3 + ch * P + local] = px.N[ch];
                }
                Vout[g] = Vp; Dout[g] = px.D; Tout[g] = px.T; count[g] = px.count;
                ambig[g] = (uint8_t)px.ambiguous;
                if (sig) sig[g] = px.sig;
            }
        }
        free(hits);
        }
        free(pj);
    }
    free(order);
    free(poff);
}

static void atomic_add(double *a, double v)
{
    #pragma omp atomic
    *a += v;
}

/*
 * Analytic adjoint of or_forward (reverse sweep of Eq. rasterization per pixel, then
 * the chain rule through the affine intersection, the projection, the normal and the
 * camera delta).  Upstream gradients dI [.,3], dD [.], dN [.,3] are given per pixel in
 * the same layout as the forward outputs (full planar per view, or compact for sel);
 * any of them may be NULL.  All gradient outputs are overwritten.
 */
void or_backward(int64_t n, const float *mean, const float *tu, const float *tv,
                 const float *scale, const float *opac, const float *alb,
                 int32_t nv, const int32_t *W, const int32_t *H, const float *Fxy,
                 const float *dF, const float *colC, const float *colc, const float *amb,
                 const float *vis, float bz, const or_settings *st,
                 int64_t nsel, const int64_t *sel,
                 const float *dI, const float *dD, const float *dN, const float *dDist,
                 double *g_mean, double *g_tu, double *g_tv, double *g_scale,
                 double *g_opac, double *g_alb, double *g_dF, double *g_colC,
                 double *g_colc, double *g_amb)
{
    memset(g_mean, 0, sizeof(double) * 3 * n); memset(g_tu, 0, sizeof(double) * 3 * n);
    memset(g_tv, 0, sizeof(double) * 3 * n);   memset(g_scale, 0, sizeof(double) * 2 * n);
    memset(g_opac, 0, sizeof(double) * n);     memset(g_alb, 0, sizeof(double) * 3 * n);
    memset(g_dF, 0, sizeof(double) * 8 * nv);  memset(g_colC, 0, sizeof(double) * 9 * nv);
    memset(g_colc, 0, sizeof(double) * 3 * nv); memset(g_amb, 0, sizeof(double) * 3 * nv);
    int64_t *poff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv + 1));
    poff[0] = 0;
    for (int v = 0; v < nv; ++v) poff[v + 1] = poff[v] + (int64_t)W[v] * H[v];
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    or_depth_order(n, mean, bz, order);
    int64_t total = sel ? nsel : poff[nv];
    const double inv_s2 = 1.0 / (st->sigma * st->sigma);
    const int64_t max_hits = n > 0 ? n : 1;
    for (int v = 0; v < nv; ++v) {
        or_cam cam;
        cam_from(Fxy + 8 * v, dF ? dF + 8 * v : NULL, &cam);
        or_proj *pj = project_view(n, mean, tu, tv, scale, opac, alb,
                                   vis ? vis + (int64_t)v * n : NULL, &cam, bz, st);
        double C[3][3], c[3], La[3];
        colour_terms(colC, colc, amb, v, C, c, La);
        #pragma omp parallel
        {
            or_hit *hits = (or_hit *)malloc(sizeof(or_hit) * (size_t)max_hits);
            double lB[2][3] = {{0}}, lb[2] = {0}, lC[3][3] = {{0}}, lc[3] = {0}, lLa[3] = {0};
            #pragma omp for schedule(dynamic, 16)
            for (int64_t s = 0; s < total; ++s) {
                int64_t g = sel ? sel[s] : s;
                if (g < poff[v] || g >= poff[v + 1]) continue;
                int64_t local = g - poff[v];
                int64_t P = poff[v + 1] - poff[v];
                int i = (int)(local % W[v]), j = (int)(local / W[v]);
                double gI[3] = {0, 0, 0}, gD = 0, gN[3] = {0, 0, 0};
                for (int ch = 0; ch < 3; ++ch) {
                    int64_t at = sel ? 3 * s + ch : 3 * poff[v] + ch * P + local;
                    if (dI) gI[ch] = dI[at];
                    if (dN) gN[ch] = dN[at];
                }
                if (dD) gD = dD[sel ? s : g];
                const double gDist = dDist ? (double)dDist[sel ? s : g] : 0.0;
                const double ds = st->depth_scale;
                or_px px;
                render_pixel(pj, order, n, i + 0.5, j + 0.5, st, vis != NULL, &px, hits,
                             max_hits);
                /* image formation adjoint (Eq. image_formation) */
                double Vp = vis ? px.V : 1.0, gA[3] = {0, 0, 0}, gV = 0;
                for (int ch = 0; ch < 3; ++ch) {
                    double ca = c[ch];
                    for (int q = 0; q < 3; ++q) ca += C[ch][q] * px.A[q];
                    double shade = Vp + (1.0 - Vp) * La[ch];
                    double gs = gI[ch] * shade;
                    for (int q = 0; q < 3; ++q) { gA[q] += C[ch][q] * gs; lC[ch][q] += gs * px.A[q]; }
                    lc[ch] += gs;
                    if (vis) {
                        gV += gI[ch] * ca * (1.0 - La[ch]);
                        lLa[ch] += gI[ch] * ca * (1.0 - Vp);
                    }
                }
                /* reverse sweep over the contributing surfels */
                double gS = 0.0;
                for (int64_t h = px.count - 1; h >= 0; --h) {
                    const or_hit *hh = &hits[h];
                    const or_proj *p = &pj[hh->sidx];
                    double a = hh->alpha, Tb = hh->Tb, w = a * Tb;
                    double gf = gA[0] * p->a[0] + gA[1] * p->a[1] + gA[2] * p->a[2] +
                                gD * hh->z + gN[0] * p->n[0] + gN[1] * p->n[1] +
                                gN[2] * p->n[2] + (vis ? gV * p->v : 0.0);
                    double dz = w * gD;
                    if (gDist != 0.0) {
                        /* distortion: d/dw_h and d/dm_h of sum_{i<j} w_i w_j (m_i - m_j)^2 */
                        const double mh = hh->z * ds;
                        double cw = 0.0, cm = 0.0;
                        for (int64_t q = 0; q < px.count; ++q) {
                            if (q == h) continue;
                            const double wq = hits[q].alpha * hits[q].Tb, dm = mh - hits[q].z * ds;
                            cw += wq * dm * dm;
                            cm += wq * dm;
                        }
                        gf += gDist * cw;
                        dz += gDist * 2.0 * w * cm * ds;
                    }
                    double dalpha = Tb * gf - gS / (1.0 - a);
                    gS += w * gf;
                    double dn[3] = {w * gN[0], w * gN[1], w * gN[2]};
                    double dO = 0, dG = 0;
                    if (hh->oG < st->alpha_max) { dO = hh->G * dalpha; dG = p->o * dalpha; }
                    double drho = -0.5 * hh->G * dG;
                    double dQ[2][2] = {{0, 0}, {0, 0}}, dd[2], dk[2] = {0, 0};
                    if (hh->ubranch) {
                        double du0 = 2 * hh->u[0] * drho - p->k[0] * dz;
                        double du1 = 2 * hh->u[1] * drho - p->k[1] * dz;
                        dk[0] = -hh->u[0] * dz; dk[1] = -hh->u[1] * dz;
                        dQ[0][0] = du0 * hh->d[0]; dQ[0][1] = du0 * hh->d[1];
                        dQ[1][0] = du1 * hh->d[0]; dQ[1][1] = du1 * hh->d[1];
                        dd[0] = p->Q[0][0] * du0 + p->Q[1][0] * du1;
                        dd[1] = p->Q[0][1] * du0 + p->Q[1][1] * du1;
                    } else {
                        dd[0] = 2 * inv_s2 * hh->d[0] * drho;
                        dd[1] = 2 * inv_s2 * hh->d[1] * drho;
                    }
                    double dc[2] = {-dd[0], -dd[1]};
                    double dz0 = dz;
                    /* Q = T^-1  ->  dT = -Q^T dQ Q^T */
                    double dT[2][2] = {{0, 0}, {0, 0}};
                    if (!p->degenerate) {
                        double t1[2][2];
                        for (int r = 0; r < 2; ++r)
                            for (int q = 0; q < 2; ++q)
                                t1[r][q] = p->Q[0][r] * dQ[0][q] + p->Q[1][r] * dQ[1][q];
                        for (int r = 0; r < 2; ++r)
                            for (int q = 0; q < 2; ++q)
                                dT[r][q] = -(t1[r][0] * p->Q[q][0] + t1[r][1] * p->Q[q][1]);
                    }
                    /* T = B M, c = B p + b */
                    double dM[3][2], dp[3];
                    for (int r = 0; r < 2; ++r) {
                        for (int q = 0; q < 3; ++q)
                            lB[r][q] += dT[r][0] * p->M[q][0] + dT[r][1] * p->M[q][1] +
                                        dc[r] * p->p[q];
                        lb[r] += dc[r];
                    }
                    for (int q = 0; q < 3; ++q) {
                        dM[q][0] = cam.B[0][q] * dT[0][0] + cam.B[1][q] * dT[1][0];
                        dM[q][1] = cam.B[0][q] * dT[0][1] + cam.B[1][q] * dT[1][1];
                        dp[q] = cam.B[0][q] * dc[0] + cam.B[1][q] * dc[1];
                    }
                    dp[2] -= dz0;                       /* z0 = b_z - p_z */
                    dM[2][0] += dk[0]; dM[2][1] += dk[1]; /* k = M[2][:] */
                    /* M = [s_u t_u, s_v t_v] */
                    double dsu = 0, dsv = 0, dtu[3], dtv[3];
                    for (int q = 0; q < 3; ++q) {
                        dsu += p->tu[q] * dM[q][0];
                        dsv += p->tv[q] * dM[q][1];
                        dtu[q] = p->su * dM[q][0];
                        dtv[q] = p->sv * dM[q][1];
                    }
                    /* n = sign * m / |m|, m = t_u x t_v */
                    double ndn = p->n[0] * dn[0] + p->n[1] * dn[1] + p->n[2] * dn[2];
                    double dm[3], cr[3];
                    for (int q = 0; q < 3; ++q)
                        dm[q] = p->nsign * (dn[q] - p->n[q] * ndn) / p->mnorm;
                    cross3(p->tv, dm, cr);
                    for (int q = 0; q < 3; ++q) dtu[q] += cr[q];
                    cross3(dm, p->tu, cr);
                    for (int q = 0; q < 3; ++q) dtv[q] += cr[q];
                    int64_t k = hh->sidx;
                    for (int q = 0; q < 3; ++q) {
                        atomic_add(&g_mean[3 * k + q], dp[q]);
                        atomic_add(&g_tu[3 * k + q], dtu[q]);
                        atomic_add(&g_tv[3 * k + q], dtv[q]);
                        atomic_add(&g_alb[3 * k + q], w * gA[q]);
                    }
                    atomic_add(&g_scale[2 * k + 0], dsu);
                    atomic_add(&g_scale[2 * k + 1], dsv);
                    atomic_add(&g_opac[k], dO);
                }
            }
            #pragma omp critical
            {
                for (int r = 0; r < 2; ++r) {
                    for (int q = 0; q < 3; ++q) g_dF[8 * v + 4 * r + q] += lB[r][q];
                    g_dF[8 * v + 4 * r + 3] += lb[r];
                }
                for (int r = 0; r < 3; ++r) {
                    for (int q = 0; q < 3; ++q) g_colC[9 * v + 3 * r + q] += lC[r][q];
                    g_colc[3 * v + r] += lc[r];
                    g_amb[3 * v + r] += lLa[r];
                }
            }
            free(hits);
        }
        free(pj);
    }
    free(order);
    free(poff);
}

/*
 * Tile-binning reference for one camera: for every surfel the FP64 support box of all
 * pixels where alpha >= alpha_min can hold (ellipse of the u-branch and disk of the
 * low-pass branch), its pixel range and tile range.  Empty ranges are lo > hi.
 * out_c [n,2], out_h [n,2] (half extents in px), pix [n,4] = i_lo,i_hi,j_lo,j_hi,
 * tiles [n,4] = tx_lo,tx_hi,ty_lo,ty_hi.
 */
void or_binning(int64_t n, const float *mean, const float *tu, const float *tv,
                const float *scale, const float *opac, const double *B6, const double *b2,
                float bz, int32_t W, int32_t H, int32_t ts, const or_settings *st,
                double *out_c, double *out_h, int32_t *pix, int32_t *tiles)
{
    or_cam cam;
    for (int r = 0; r < 2; ++r) {
        for (int q = 0; q < 3; ++q) cam.B[r][q] = B6[3 * r + q];
        cam.b[r] = b2[r];
    }
    static const float zero3[3] = {0, 0, 0};
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        or_proj p;
        project_one(&cam, bz, mean + 3 * i, tu + 3 * i, tv + 3 * i, scale + 2 * i, opac[i],
                    zero3, 1.0, st, &p);
        out_c[2 * i] = p.c[0]; out_c[2 * i + 1] = p.c[1];
        int32_t *px = pix + 4 * i, *tl = tiles + 4 * i;
        px[0] = 0; px[1] = -1; px[2] = 0; px[3] = -1;
        tl[0] = 0; tl[1] = -1; tl[2] = 0; tl[3] = -1;
        out_h[2 * i] = out_h[2 * i + 1] = 0.0;
        if (!(p.o >= st->alpha_min)) continue;
        double r = sqrt(2.0 * log(p.o / st->alpha_min));
        double hx = 0.0, hy = 0.0;
        if (!p.degenerate) {
            hx = r * sqrt(p.T[0][0] * p.T[0][0] + p.T[0][1] * p.T[0][1]);
            hy = r * sqrt(p.T[1][0] * p.T[1][0] + p.T[1][1] * p.T[1][1]);
        }
        if (p.filter_on) {
            double f = st->sigma * r;
            if (f > hx) hx = f;
            if (f > hy) hy = f;
        }
        out_h[2 * i] = hx; out_h[2 * i + 1] = hy;
        double ilo = ceil(p.c[0] - hx - 0.5), ihi = floor(p.c[0] + hx - 0.5);
        double jlo = ceil(p.c[1] - hy - 0.5), jhi = floor(p.c[1] + hy - 0.5);
        if (ilo < 0) ilo = 0;
        if (jlo < 0) jlo = 0;
        if (ihi > W - 1) ihi = W - 1;
        if (jhi > H - 1) jhi = H - 1;
        if (ilo > ihi || jlo > jhi) continue;
        px[0] = (int32_t)ilo; px[1] = (int32_t)ihi; px[2] = (int32_t)jlo; px[3] = (int32_t)jhi;
        tl[0] = px[0] / ts; tl[1] = px[1] / ts; tl[2] = px[2] / ts; tl[3] = px[3] / ts;
    }
}

/* Camera B (2x3) and b (2) of view v in FP64 (F' = F + dF). */
void or_view_camera(const float *Fxy, const float *dF, int32_t v, double *B6, double *b2)
{
    or_cam cam;
    cam_from(Fxy + 8 * v, dF ? dF + 8 * v : NULL, &cam);
    for (int r = 0; r < 2; ++r) {
        for (int q = 0; q < 3; ++q) B6[3 * r + q] = cam.B[r][q];
        b2[r] = cam.b[r];
    }
}

/*
 * Sun camera of view v (Sec. 3.3 Eq. sun_camera_Bxy; Supp. A): flatten along
 * s = (cos(phi)/tan(theta), sin(phi)/tan(theta), 1) onto z = 0, then project with the
 * main camera's B_xy, then a viewport (scale lam, offset o) that maps the flattened
 * bounding box of the 8 corners of the surfel-centre AABB onto the central 98 % of the
 * S x S map:  B_sun = lam * B_xy (I - [0 0 s]),  b_sun = o.
 * Also returns z_far = b_z - min(p_z) + 10 m (sun-map background depth).
 */
void or_sun_camera(int64_t n, const float *mean, const float *Fxy, const float *dF,
                   const float *sun, int32_t v, float bz, int32_t S, double *Bs6,
                   double *bs2, double *zfar)
{
    or_cam cam;
    cam_from(Fxy + 8 * v, dF ? dF + 8 * v : NULL, &cam);
    double phi = sun[2 * v], theta = sun[2 * v + 1];
    double s[3] = {cos(phi) / tan(theta), sin(phi) / tan(theta), 1.0};
    double Bf[2][3];
    for (int r = 0; r < 2; ++r) {
        Bf[r][0] = cam.B[r][0];
        Bf[r][1] = cam.B[r][1];
        Bf[r][2] = cam.B[r][2] - (cam.B[r][0] * s[0] + cam.B[r][1] * s[1] + cam.B[r][2] * s[2]);
    }
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i)
        for (int q = 0; q < 3; ++q) {
            double x = mean[3 * i + q];
            if (x < lo[q]) lo[q] = x;
            if (x > hi[q]) hi[q] = x;
        }
    if (n == 0) { lo[0] = lo[1] = lo[2] = hi[0] = hi[1] = hi[2] = 0.0; }
    double plo[2] = {INFINITY, INFINITY}, phi2[2] = {-INFINITY, -INFINITY};
    for (int cidx = 0; cidx < 8; ++cidx) {
        double P[3] = {(cidx & 1) ? hi[0] : lo[0], (cidx & 2) ? hi[1] : lo[1],
                       (cidx & 4) ? hi[2] : lo[2]};
        for (int r = 0; r < 2; ++r) {
            double x = Bf[r][0] * P[0] + Bf[r][1] * P[1] + Bf[r][2] * P[2];
            if (x < plo[r]) plo[r] = x;
            if (x > phi2[r]) phi2[r] = x;
        }
    }
    double ext = phi2[0] - plo[0];
    if (phi2[1] - plo[1] > ext) ext = phi2[1] - plo[1];
    double lam = ext > 0 ? 0.98 * S / ext : 1.0;
    for (int r = 0; r < 2; ++r) {
        for (int q = 0; q < 3; ++q) Bs6[3 * r + q] = lam * Bf[r][q];
        bs2[r] = 0.5 * S - lam * 0.5 * (plo[r] + phi2[r]);
    }
    *zfar = (double)bz - lo[2] + 10.0;
}

/*
 * Sun-view depth at a list of texels (tx, ty) of an S x S map rendered with camera
 * (Bs, bs): the same compositing as the main view, depth channel only, over an opaque
 * background at z_far:  D_sun = sum_i w_i z_i + T_final * z_far.
 */
void or_sun_depth(int64_t n, const float *mean, const float *tu, const float *tv,
                  const float *scale, const float *opac, const double *Bs6,
                  const double *bs2, float bz, double zfar, const or_settings *st,
                  int64_t ntex, const int32_t *tex, double *out, uint8_t *ambig)
{
    or_cam cam;
    for (int r = 0; r < 2; ++r) {
        for (int q = 0; q < 3; ++q) cam.B[r][q] = Bs6[3 * r + q];
        cam.b[r] = bs2[r];
    }
    static const float zero3[3] = {0, 0, 0};
    or_proj *pj = (or_proj *)malloc(sizeof(or_proj) * (size_t)(n > 0 ? n : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        project_one(&cam, bz, mean + 3 * i, tu + 3 * i, tv + 3 * i, scale + 2 * i, opac[i],
                    zero3, 1.0, st, &pj[i]);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    or_depth_order(n, mean, bz, order);
    #pragma omp parallel for schedule(dynamic, 8)
    for (int64_t t = 0; t < ntex; ++t) {
        or_px px;
        render_pixel(pj, order, n, tex[2 * t] + 0.5, tex[2 * t + 1] + 0.5, st, 0, &px, NULL, 0);
        out[t] = px.D + px.T * zfar;
        if (ambig) ambig[t] = (uint8_t)px.ambiguous;
    }
    free(order);
    free(pj);
}

/*
 * Per-surfel sun visibility for one view: the surfel centre p_k is projected into the
 * sun map, and the 3x3 texels around floor(x_s) give an exponential-shadow-map test
 *   v_k = min(1, (1/9) sum_t exp(c_e (D_t - d_k + beta))),  d_k = b_z - p_k,z,
 * with texels outside the map reading the background z_far.  `sel` lists the surfels
 * (NULL = all n); D_sun is rendered only at the texels those surfels need.
 */
void or_shadow(int64_t n, const float *mean, const float *tu, const float *tv,
               const float *scale, const float *opac, const float *Fxy, const float *dF,
               const float *sun, int32_t v, float bz, int32_t S, const or_settings *st,
               int64_t nsel, const int64_t *sel, double *vis_out, uint8_t *ambig_out)
{
    double Bs[6], bs[2], zfar;
    or_sun_camera(n, mean, Fxy, dF, sun, v, bz, S, Bs, bs, &zfar);
    int64_t m = sel ? nsel : n;
    int32_t *tex = (int32_t *)malloc(sizeof(int32_t) * 18 * (size_t)(m > 0 ? m : 1));
    uint8_t *inside = (uint8_t *)malloc(9 * (size_t)(m > 0 ? m : 1));
    for (int64_t s = 0; s < m; ++s) {
        int64_t k = sel ? sel[s] : s;
        double x = bs[0], y = bs[1];
        for (int q = 0; q < 3; ++q) {
            x += Bs[q] * mean[3 * k + q];
            y += Bs[3 + q] * mean[3 * k + q];
        }
        double fx = floor(x), fy = floor(y);
        for (int t = 0; t < 9; ++t) {
            double tx = fx + (t % 3) - 1, ty = fy + (t / 3) - 1;
            int in = tx >= 0 && ty >= 0 && tx < S && ty < S;
            inside[9 * s + t] = (uint8_t)in;
            tex[18 * s + 2 * t] = in ? (int32_t)tx : 0;
            tex[18 * s + 2 * t + 1] = in ? (int32_t)ty : 0;
        }
    }
    double *D = (double *)malloc(sizeof(double) * 9 * (size_t)(m > 0 ? m : 1));
    uint8_t *tamb = (uint8_t *)malloc(9 * (size_t)(m > 0 ? m : 1));
    or_sun_depth(n, mean, tu, tv, scale, opac, Bs, bs, bz, zfar, st, 9 * m, tex, D, tamb);
    for (int64_t s = 0; s < m; ++s) {
        int64_t k = sel ? sel[s] : s;
        double dk = (double)bz - mean[3 * k + 2];
        double acc = 0.0;
        for (int t = 0; t < 9; ++t) {
            double Dt = inside[9 * s + t] ? D[9 * s + t] : zfar;
            acc += exp(st->esm_c * (Dt - dk + st->esm_bias));
        }
        acc /= 9.0;
        vis_out[s] = acc < 1.0 ? acc : 1.0;
        if (ambig_out) {
            uint8_t a = 0;
            for (int t = 0; t < 9; ++t) a |= inside[9 * s + t] ? tamb[9 * s + t] : 0;
            ambig_out[s] = a;
        }
    }
    free(tamb);
    free(D);
    free(inside);
    free(tex);
}

int32_t or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count for the parallel loops over pixels (timing only; results do not depend on it). */
void or_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
