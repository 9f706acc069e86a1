// Training step around the rasterizer (SatSplat, arXiv 2606.28581, Supp. B "Experimental
// Settings": Adam with per-group learning rates, L1 image loss, camera optimisation from a
// start step): surfel activations, one fused pass per surfel for the activation adjoint +
// Adam + re-activation, Adam over the per-view camera delta and colour terms, and the L1
// image loss with its gradient.
//
// Raw surfel parameters, 13 floats per surfel: mean (3), log scale (2), opacity logit (1),
// quaternion (w, x, y, z) (4), albedo (3).  Activated: scale = exp, opacity = sigmoid,
// (t_u, t_v) = first two columns of the rotation of q / |q|.  The fused Adam pass reads
// the raw parameters, both moments and the six activated-gradient arrays and writes the
// raw parameters, both moments and the activated arrays: HBM-bound, ~0.5 KB per surfel.
#include "ss_internal.h"

namespace ss {

constexpr int kRaw = 13;
constexpr int kTrainThreads = 256;

__device__ __forceinline__ void frame_of(const float (&q)[4], float (&tu)[3], float (&tv)[3])
{
    const float inv = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, z = q[3] * inv;
    tu[0] = 1.f - 2.f * (y * y + z * z); tu[1] = 2.f * (x * y + w * z); tu[2] = 2.f * (x * z - w * y);
    tv[0] = 2.f * (x * y - w * z); tv[1] = 1.f - 2.f * (x * x + z * z); tv[2] = 2.f * (y * z + w * x);
}

__device__ __forceinline__ void write_activated(int64_t i, const float (&r)[kRaw], float *mean,
                                                float *tu, float *tv, float *scale,
                                                float *opacity, float *albedo)
{
    float q[4] = {r[6], r[7], r[8], r[9]}, u[3], v[3];
    frame_of(q, u, v);
    for (int k = 0; k < 3; ++k) {
        mean[3 * i + k] = r[k];
        tu[3 * i + k] = u[k];
        tv[3 * i + k] = v[k];
        albedo[3 * i + k] = r[10 + k];
    }
    scale[2 * i] = expf(r[3]);
    scale[2 * i + 1] = expf(r[4]);
    opacity[i] = 1.f / (1.f + expf(-r[5]));
}

__global__ __launch_bounds__(kTrainThreads) void k_surfel_activate(
    int64_t n, const float *__restrict__ raw, float *__restrict__ mean, float *__restrict__ tu,
    float *__restrict__ tv, float *__restrict__ scale, float *__restrict__ opacity,
    float *__restrict__ albedo)
{
    const int64_t i = (int64_t)blockIdx.x * kTrainThreads + threadIdx.x;
    if (i >= n) return;
    float r[kRaw];
    for (int k = 0; k < kRaw; ++k) r[k] = raw[kRaw * i + k];
    write_activated(i, r, mean, tu, tv, scale, opacity, albedo);
}

// Raw parameters from activated arrays: log scale, logit opacity, and the quaternion of
// the frame [t_u, t_v, t_u x t_v] by Shepperd's method (largest of w, x, y, z first).
__global__ __launch_bounds__(kTrainThreads) void k_surfel_raw(
    int64_t n, const float *__restrict__ mean, const float *__restrict__ tu,
    const float *__restrict__ tv, const float *__restrict__ scale,
    const float *__restrict__ opacity, const float *__restrict__ albedo, float *__restrict__ raw)
{
    const int64_t i = (int64_t)blockIdx.x * kTrainThreads + threadIdx.x;
    if (i >= n) return;
    const float u[3] = {tu[3 * i], tu[3 * i + 1], tu[3 * i + 2]};
    const float v[3] = {tv[3 * i], tv[3 * i + 1], tv[3 * i + 2]};
    const float nn[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    // R[row][col], columns u, v, n
    const float R00 = u[0], R10 = u[1], R20 = u[2], R01 = v[0], R11 = v[1], R21 = v[2];
    const float R02 = nn[0], R12 = nn[1], R22 = nn[2];
    const float tr = R00 + R11 + R22;
    float w, x, y, z;
    if (tr > 0.f) {
        const float s = 2.f * sqrtf(tr + 1.f);
        w = 0.25f * s; x = (R21 - R12) / s; y = (R02 - R20) / s; z = (R10 - R01) / s;
    } else if (R00 > R11 && R00 > R22) {
        const float s = 2.f * sqrtf(1.f + R00 - R11 - R22);
        w = (R21 - R12) / s; x = 0.25f * s; y = (R01 + R10) / s; z = (R02 + R20) / s;
    } else if (R11 > R22) {
        const float s = 2.f * sqrtf(1.f + R11 - R00 - R22);
        w = (R02 - R20) / s; x = (R01 + R10) / s; y = 0.25f * s; z = (R12 + R21) / s;
    } else {
        const float s = 2.f * sqrtf(1.f + R22 - R00 - R11);
        w = (R10 - R01) / s; x = (R02 + R20) / s; y = (R12 + R21) / s; z = 0.25f * s;
    }
    float *r = raw + kRaw * i;
    for (int k = 0; k < 3; ++k) {
        r[k] = mean[3 * i + k];
        r[10 + k] = albedo[3 * i + k];
    }
    r[3] = logf(scale[2 * i]);
    r[4] = logf(scale[2 * i + 1]);
    const float o = opacity[i];
    r[5] = logf(o / (1.f - o));
    r[6] = w; r[7] = x; r[8] = y; r[9] = z;
}

__device__ __forceinline__ void adam_one(float &theta, float &m, float &v, float g, float lr,
                                         const AdamArgs &a, float bc1, float bc2)
{
    m = a.beta1 * m + (1.f - a.beta1) * g;
    v = a.beta2 * v + (1.f - a.beta2) * g * g;
    const float mh = m / bc1, vh = v / bc2;
    theta -= lr * mh / (sqrtf(vh) + a.eps);
}

// activation adjoint + Adam + re-activation, one thread per surfel
__global__ __launch_bounds__(kTrainThreads) void k_adam_surfels(
    int64_t n, float *__restrict__ raw, float *__restrict__ m, float *__restrict__ v,
    const float *__restrict__ g_mean, const float *__restrict__ g_tu,
    const float *__restrict__ g_tv, const float *__restrict__ g_scale,
    const float *__restrict__ g_opacity, const float *__restrict__ g_albedo, AdamArgs a,
    float bc1, float bc2, float *__restrict__ mean, float *__restrict__ tu,
    float *__restrict__ tv, float *__restrict__ scale, float *__restrict__ opacity,
    float *__restrict__ albedo)
{
    const int64_t i = (int64_t)blockIdx.x * kTrainThreads + threadIdx.x;
    if (i >= n) return;
    float r[kRaw], g[kRaw];
    for (int k = 0; k < kRaw; ++k) r[k] = raw[kRaw * i + k];
    for (int k = 0; k < 3; ++k) {
        g[k] = g_mean[3 * i + k];
        g[10 + k] = g_albedo[3 * i + k];
    }
    g[3] = g_scale[2 * i] * expf(r[3]);
    g[4] = g_scale[2 * i + 1] * expf(r[4]);
    const float o = 1.f / (1.f + expf(-r[5]));
    g[5] = g_opacity[i] * o * (1.f - o);
    {
        // d(t_u, t_v)/d(q / |q|), then the projection of the normalisation
        const float nq = sqrtf(r[6] * r[6] + r[7] * r[7] + r[8] * r[8] + r[9] * r[9]);
        const float w = r[6] / nq, x = r[7] / nq, y = r[8] / nq, z = r[9] / nq;
        const float gu0 = g_tu[3 * i], gu1 = g_tu[3 * i + 1], gu2 = g_tu[3 * i + 2];
        const float gv0 = g_tv[3 * i], gv1 = g_tv[3 * i + 1], gv2 = g_tv[3 * i + 2];
        float gq[4];
        gq[0] = 2.f * (z * gu1 - y * gu2) + 2.f * (-z * gv0 + x * gv2);
        gq[1] = 2.f * (y * gu1 + z * gu2) + (2.f * y * gv0 - 4.f * x * gv1 + 2.f * w * gv2);
        gq[2] = (-4.f * y * gu0 + 2.f * x * gu1 - 2.f * w * gu2) + 2.f * (x * gv0 + z * gv2);
        gq[3] = (-4.f * z * gu0 + 2.f * w * gu1 + 2.f * x * gu2) + (-2.f * w * gv0 - 4.f * z * gv1 + 2.f * y * gv2);
        const float pr = w * gq[0] + x * gq[1] + y * gq[2] + z * gq[3];
        g[6] = (gq[0] - w * pr) / nq;
        g[7] = (gq[1] - x * pr) / nq;
        g[8] = (gq[2] - y * pr) / nq;
        g[9] = (gq[3] - z * pr) / nq;
    }
    for (int k = 0; k < kRaw; ++k) {
        const float lr = k < 3 ? a.lr[0] : k < 5 ? a.lr[1] : k < 6 ? a.lr[2] : k < 10 ? a.lr[3] : a.lr[4];
        float mm = m[kRaw * i + k], vv = v[kRaw * i + k];
        adam_one(r[k], mm, vv, g[k], lr, a, bc1, bc2);
        m[kRaw * i + k] = mm;
        v[kRaw * i + k] = vv;
        raw[kRaw * i + k] = r[k];
    }
    write_activated(i, r, mean, tu, tv, scale, opacity, albedo);
}

// per-view camera delta (8 floats, from camera_start on) and colour gain / bias (9 + 3)
__global__ void k_adam_views(int32_t nv, float *__restrict__ dF, float *__restrict__ m_dF,
                             float *__restrict__ v_dF, const float *__restrict__ g_dF,
                             const float *__restrict__ g_dF2,
                             float *__restrict__ colC, float *__restrict__ m_C,
                             float *__restrict__ v_C, const float *__restrict__ g_C,
                             float *__restrict__ colc, float *__restrict__ m_c,
                             float *__restrict__ v_c, const float *__restrict__ g_c, AdamArgs a,
                             int camera_on, float cbc1, float cbc2, float bc1, float bc2)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < 8 * nv) {
        if (camera_on && dF)
            adam_one(dF[k], m_dF[k], v_dF[k], g_dF[k] + (g_dF2 ? g_dF2[k] : 0.f), a.lr[5], a, cbc1, cbc2);
    } else if (k < 17 * nv) {
        const int j = k - 8 * nv;
        if (colC) adam_one(colC[j], m_C[j], v_C[j], g_C[j], a.lr[6], a, bc1, bc2);
    } else if (k < 20 * nv) {
        const int j = k - 17 * nv;
        if (colc) adam_one(colc[j], m_c[j], v_c[j], g_c[j], a.lr[6], a, bc1, bc2);
    }
}

// L1 image loss: per view weight / (3 P) sum |I - I*|; d_image = weight sign(I - I*) / (3 P).
// Grid (blocks per view, views); each thread takes kL1PerThread elements at a stride of the
// block size (coalesced), sums |d| in FP32, and the block's sum goes to one FP64 partial.
constexpr int kL1PerThread = 8;

__global__ __launch_bounds__(kTrainThreads) void k_l1_loss(
    const ViewDesc *__restrict__ views, const float *__restrict__ img,
    const float *__restrict__ tgt, float weight, float *__restrict__ d_img,
    double *__restrict__ partials, int blocks_per_view)
{
    __shared__ float red[kTrainThreads / 64];
    const int v = blockIdx.y;
    const ViewDesc vd = views[v];
    const int64_t n = 3 * (int64_t)vd.W * vd.H;
    const float step = (float)((double)weight / (double)n);
    const int64_t k0 = (int64_t)blockIdx.x * (kTrainThreads * kL1PerThread) + threadIdx.x;
    const int64_t base = 3 * vd.pix_off;
    float s = 0.f;
#pragma unroll
    for (int r = 0; r < kL1PerThread; ++r) {
        const int64_t k = k0 + (int64_t)r * kTrainThreads;
        if (k < n) {
            const float d = img[base + k] - tgt[base + k];
            s += fabsf(d);
            d_img[base + k] = d > 0.f ? step : (d < 0.f ? -step : 0.f);
        }
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kTrainThreads / 64; ++w) t += (double)red[w];
        partials[(size_t)v * blocks_per_view + blockIdx.x] = t;
    }
}

__global__ void k_l1_reduce(const ViewDesc *__restrict__ views, const double *__restrict__ partials,
                            int blocks_per_view, int32_t nv, float weight, float *__restrict__ loss)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    double s = 0.0;
    for (int b = 0; b < blocks_per_view; ++b) s += partials[(size_t)v * blocks_per_view + b];
    loss[v] = (float)((double)weight * s / (3.0 * views[v].W * (double)views[v].H));
}

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kTrainThreads - 1) / kTrainThreads); }

hipError_t launch_surfel_activate(int64_t n, const float *raw, float *mean, float *tu, float *tv,
                                  float *scale, float *opacity, float *albedo, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_surfel_activate, dim3(blocks_for(n)), dim3(kTrainThreads), 0, st, n, raw,
                       mean, tu, tv, scale, opacity, albedo);
    return hipGetLastError();
}

hipError_t launch_surfel_raw(int64_t n, const float *mean, const float *tu, const float *tv,
                             const float *scale, const float *opacity, const float *albedo,
                             float *raw, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_surfel_raw, dim3(blocks_for(n)), dim3(kTrainThreads), 0, st, n, mean, tu, tv,
                       scale, opacity, albedo, raw);
    return hipGetLastError();
}

hipError_t launch_adam_surfels(int64_t n, float *raw, float *m, float *v, const float *g_mean,
                               const float *g_tu, const float *g_tv, const float *g_scale,
                               const float *g_opacity, const float *g_albedo, const AdamArgs &a,
                               int32_t step, float *mean, float *tu, float *tv, float *scale,
                               float *opacity, float *albedo, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const float bc1 = (float)(1.0 - pow((double)a.beta1, (double)step));
    const float bc2 = (float)(1.0 - pow((double)a.beta2, (double)step));
    hipLaunchKernelGGL(k_adam_surfels, dim3(blocks_for(n)), dim3(kTrainThreads), 0, st, n, raw, m, v,
                       g_mean, g_tu, g_tv, g_scale, g_opacity, g_albedo, a, bc1, bc2, mean, tu, tv,
                       scale, opacity, albedo);
    return hipGetLastError();
}

hipError_t launch_adam_views(int32_t nv, float *dF, float *m_dF, float *v_dF, const float *g_dF,
                             const float *g_dF2, float *colC, float *m_C, float *v_C, const float *g_C, float *colc,
                             float *m_c, float *v_c, const float *g_c, const AdamArgs &a,
                             int32_t step, hipStream_t st)
{
    if (nv <= 0) return hipSuccess;
    const int cam_t = step - a.camera_start + 1;        // the camera group's own step count
    const float bc1 = (float)(1.0 - pow((double)a.beta1, (double)step));
    const float bc2 = (float)(1.0 - pow((double)a.beta2, (double)step));
    const float cbc1 = cam_t > 0 ? (float)(1.0 - pow((double)a.beta1, (double)cam_t)) : 1.f;
    const float cbc2 = cam_t > 0 ? (float)(1.0 - pow((double)a.beta2, (double)cam_t)) : 1.f;
    hipLaunchKernelGGL(k_adam_views, dim3((unsigned)((20 * nv + 255) / 256)), dim3(256), 0, st, nv, dF,
                       m_dF, v_dF, g_dF, g_dF2, colC, m_C, v_C, g_C, colc, m_c, v_c, g_c, a, cam_t > 0 ? 1 : 0,
                       cbc1, cbc2, bc1, bc2);
    return hipGetLastError();
}

int l1_blocks(int64_t max_view_pixels)
{
    return (int)((3 * max_view_pixels + kTrainThreads * kL1PerThread - 1) / (kTrainThreads * kL1PerThread));
}

hipError_t launch_l1_loss(const ViewDesc *views, int32_t nv, int64_t max_view_pixels,
                          const float *img, const float *tgt, float weight, float *d_img,
                          double *partials, float *loss, hipStream_t st)
{
    if (nv <= 0) return hipSuccess;
    const int bpv = l1_blocks(max_view_pixels);
    if (bpv > 0)
        hipLaunchKernelGGL(k_l1_loss, dim3((unsigned)bpv, (unsigned)nv), dim3(kTrainThreads), 0, st,
                           views, img, tgt, weight, d_img, partials, bpv);
    hipLaunchKernelGGL(k_l1_reduce, dim3((unsigned)((nv + 63) / 64)), dim3(64), 0, st, views, partials,
                       bpv, nv, weight, loss);
    return hipGetLastError();
}

}  // namespace ss
