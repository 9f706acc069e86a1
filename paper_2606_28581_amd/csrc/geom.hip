// Depth-gradient normals and the normal-consistency loss on the rendered maps (SatSplat,
// arXiv 2606.28581, Sec. 3.2 "Normal Definition", Eq. surface_normal): the expected depth
// zbar = D / (1 - T) of every pixel is back-projected through the view's affine camera
// F' = F + dF with the fixed depth row (B_z = (0, 0, -1), b_z), the point map is
// differentiated with central differences, N = normalise(grad_x p x grad_y p) oriented
// like the rendered normals, and per view L = weight / P * sum over valid pixels of
// (1 - N_r . N).  The accumulated opacity 1 - T is a constant (no gradient into T).  A
// pixel is valid when it is not on the border and 1 - T >= tau at it and its four
// neighbours.
//
// The back-projection p = Minv (x - b_xy, zbar - b_z) is affine with one 3x3 matrix per
// view, so the central differences are grad_x p = Minv (2, 0, dzx), grad_y p = Minv (0, 2,
// dzy) with dzx, dzy the differences of zbar: each pixel needs only its neighbours' depth.
// Image-size work with ~150 flops per pixel: the arithmetic is FP64 (the inputs and the
// stored adjoints are FP32), and the kernels are bound by their ~40 bytes per pixel.
#include "ss_internal.h"

namespace ss {

constexpr int kGeomThreads = 256;

// Per view: Minv (row-major 3x3) of M = [B_x; B_y; (0, 0, -1)] and the view direction
// d = B_x x B_y with d_z < 0 that orients the normals.
__global__ void k_geom_cameras(const float *__restrict__ Fxy, const float *__restrict__ dF,
                               int32_t nv, GeomCam *__restrict__ out)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    double B[2][3];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            B[r][c] = (double)Fxy[8 * v + 4 * r + c] + (dF ? (double)dF[8 * v + 4 * r + c] : 0.0);
    // M = [[B00 B01 B02], [B10 B11 B12], [0 0 -1]]: inverse by the block structure
    // p_z = -r_2, B_xy[:, :2] p_xy = r_01 - B_xy[:, 2] p_z
    const double det = B[0][0] * B[1][1] - B[0][1] * B[1][0];
    const double i00 = B[1][1] / det, i01 = -B[0][1] / det, i10 = -B[1][0] / det, i11 = B[0][0] / det;
    GeomCam g;
    g.Minv[0] = i00; g.Minv[1] = i01; g.Minv[2] = i00 * B[0][2] + i01 * B[1][2];
    g.Minv[3] = i10; g.Minv[4] = i11; g.Minv[5] = i10 * B[0][2] + i11 * B[1][2];
    g.Minv[6] = 0.0; g.Minv[7] = 0.0; g.Minv[8] = -1.0;
    double d0 = B[0][1] * B[1][2] - B[0][2] * B[1][1];
    double d1 = B[0][2] * B[1][0] - B[0][0] * B[1][2];
    double d2 = B[0][0] * B[1][1] - B[0][1] * B[1][0];
    if (d2 > 0) { d0 = -d0; d1 = -d1; d2 = -d2; }
    g.d[0] = d0; g.d[1] = d1; g.d[2] = d2;
    for (int k = 0; k < 4; ++k) g.pad[k] = 0.0;
    out[v] = g;
}

__device__ __forceinline__ bool covered(const float *T, int64_t g, double tau)
{
    return 1.0 - (double)T[g] >= tau;
}

__device__ __forceinline__ double zbar_at(const float *D, const float *T, int64_t g)
{
    return (double)D[g] / (1.0 - (double)T[g]);
}

// Pixels of view blockIdx.y, kGeomPx per thread at a stride of the block size: depth
// normal, loss term, d_normal (added), the z-adjoint seeds s = Minv[:, 2] . dL/dgrad p
// stored per pixel, and per block the sums of the loss terms and of dL/dMinv (10 doubles),
// reduced once per thread after its pixels.
constexpr int kGeomPx = 8;

__device__ __forceinline__ void normal_loss_pixel(
    const ViewDesc &vd, int64_t local, const GeomCam &c, const float *__restrict__ D,
    const float *__restrict__ T, const float *__restrict__ Nr, double wv, double tau,
    float *__restrict__ Nd_out, float *__restrict__ d_normal, float2 *__restrict__ seeds,
    double (&acc)[10])
{
    const int64_t P = (int64_t)vd.W * vd.H;
    const int i = (int)(local % vd.W), j = (int)(local / vd.W);
    const int64_t g = vd.pix_off + local;
    const int64_t b3 = 3 * vd.pix_off + local;
    bool valid = i > 0 && j > 0 && i < vd.W - 1 && j < vd.H - 1;
    valid = valid && covered(T, g, tau) && covered(T, g - 1, tau) && covered(T, g + 1, tau) &&
            covered(T, g - vd.W, tau) && covered(T, g + vd.W, tau);
    float2 s = make_float2(0.f, 0.f);
    float nd[3] = {0.f, 0.f, 0.f};
    if (valid) {
        const double *Mi = c.Minv;
        const double dzx = zbar_at(D, T, g + 1) - zbar_at(D, T, g - 1);
        const double dzy = zbar_at(D, T, g + vd.W) - zbar_at(D, T, g - vd.W);
        double gx[3], gy[3], n[3];
        for (int r = 0; r < 3; ++r) {
            gx[r] = 2.0 * Mi[3 * r] + dzx * Mi[3 * r + 2];
            gy[r] = 2.0 * Mi[3 * r + 1] + dzy * Mi[3 * r + 2];
        }
        n[0] = gx[1] * gy[2] - gx[2] * gy[1];
        n[1] = gx[2] * gy[0] - gx[0] * gy[2];
        n[2] = gx[0] * gy[1] - gx[1] * gy[0];
        const double inn = 1.0 / sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        const double sgn = (n[0] * c.d[0] + n[1] * c.d[1] + n[2] * c.d[2] > 0.0) ? -1.0 : 1.0;
        double N[3], R[3];
        for (int r = 0; r < 3; ++r) {
            N[r] = sgn * n[r] * inn;
            R[r] = (double)Nr[b3 + r * P];
        }
        acc[9] += 1.0 - (R[0] * N[0] + R[1] * N[1] + R[2] * N[2]);
        for (int r = 0; r < 3; ++r) {
            d_normal[b3 + r * P] += (float)(-wv * N[r]);
            nd[r] = (float)N[r];
        }
        // dL/dN = -wv N_r -> dL/dn = sgn (gN - N (N . gN)) / |n|
        double gN[3], gn[3];
        for (int r = 0; r < 3; ++r) gN[r] = -wv * R[r];
        const double pr = N[0] * gN[0] + N[1] * gN[1] + N[2] * gN[2];
        for (int r = 0; r < 3; ++r) gn[r] = sgn * (gN[r] - N[r] * pr) * inn;
        // n = gx x gy: dL/dgx = gy x gn, dL/dgy = gn x gx
        const double ggx[3] = {gy[1] * gn[2] - gy[2] * gn[1], gy[2] * gn[0] - gy[0] * gn[2],
                               gy[0] * gn[1] - gy[1] * gn[0]};
        const double ggy[3] = {gn[1] * gx[2] - gn[2] * gx[1], gn[2] * gx[0] - gn[0] * gx[2],
                               gn[0] * gx[1] - gn[1] * gx[0]};
        s.x = (float)(Mi[2] * ggx[0] + Mi[5] * ggx[1] + Mi[8] * ggx[2]);
        s.y = (float)(Mi[2] * ggy[0] + Mi[5] * ggy[1] + Mi[8] * ggy[2]);
        // dL/dMinv = ggx (2, 0, dzx)^T + ggy (0, 2, dzy)^T
        for (int r = 0; r < 3; ++r) {
            acc[3 * r] += 2.0 * ggx[r];
            acc[3 * r + 1] += 2.0 * ggy[r];
            acc[3 * r + 2] += dzx * ggx[r] + dzy * ggy[r];
        }
    }
    seeds[g] = s;
    if (Nd_out) {
        for (int r = 0; r < 3; ++r) Nd_out[b3 + r * P] = nd[r];
    }
}

__global__ __launch_bounds__(kGeomThreads) void k_normal_loss(
    const ViewDesc *__restrict__ views, const GeomCam *__restrict__ cams,
    const float *__restrict__ D, const float *__restrict__ T, const float *__restrict__ Nr,
    double weight, double tau, float *__restrict__ Nd_out, float *__restrict__ d_normal,
    float2 *__restrict__ seeds, double *__restrict__ partials, int blocks_per_view)
{
    __shared__ double red[kGeomThreads / 64][10];
    const int v = blockIdx.y;
    const ViewDesc vd = views[v];
    const int64_t P = (int64_t)vd.W * vd.H;
    const GeomCam c = cams[v];
    const double wv = weight / (double)P;
    double acc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = 0.0;
    const int64_t l0 = (int64_t)blockIdx.x * (kGeomThreads * kGeomPx) + threadIdx.x;
    for (int r = 0; r < kGeomPx; ++r) {
        const int64_t local = l0 + (int64_t)r * kGeomThreads;
        if (local < P) normal_loss_pixel(vd, local, c, D, T, Nr, wv, tau, Nd_out, d_normal, seeds, acc);
    }
    // block sums: wave shuffles, then the waves' sums through LDS
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        double x = acc[k];
        for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
        if (lane == 0) red[wave][k] = x;
    }
    __syncthreads();
    if (threadIdx.x < 10) {
        double x = 0.0;
        for (int w = 0; w < kGeomThreads / 64; ++w) x += red[w][threadIdx.x];
        partials[((size_t)v * blocks_per_view + blockIdx.x) * 10 + threadIdx.x] = x;
    }
}

// d_depth(y) += dL/dzbar(y) / (1 - T(y)) with dL/dzbar(y) = s_x(y - 1) - s_x(y + 1)
// + s_y(y - W) - s_y(y + W) (seeds of pixels outside the view count as zero).
__global__ __launch_bounds__(kGeomThreads) void k_normal_loss_depth(
    const ViewDesc *__restrict__ views, const float *__restrict__ T, double tau,
    const float2 *__restrict__ seeds, float *__restrict__ d_depth)
{
    const int v = blockIdx.y;
    const ViewDesc vd = views[v];
    const int64_t P = (int64_t)vd.W * vd.H;
    const int64_t local = (int64_t)blockIdx.x * kGeomThreads + threadIdx.x;
    if (local >= P) return;
    const int64_t g = vd.pix_off + local;
    if (!covered(T, g, tau)) return;
    const int i = (int)(local % vd.W), j = (int)(local / vd.W);
    double gz = 0.0;
    if (i > 0) gz += (double)seeds[g - 1].x;
    if (i < vd.W - 1) gz -= (double)seeds[g + 1].x;
    if (j > 0) gz += (double)seeds[g - vd.W].y;
    if (j < vd.H - 1) gz -= (double)seeds[g + vd.W].y;
    d_depth[g] += (float)(gz / (1.0 - (double)T[g]));
}

// Per view: loss[v] = weight / P * sum of the block terms; d_dF[v][:, :3] += the first two
// rows of dL/dM = -Minv^T dL/dMinv Minv^T (the translation column drops out of the
// central differences).
__global__ void k_normal_loss_reduce(const ViewDesc *__restrict__ views,
                                     const GeomCam *__restrict__ cams,
                                     const double *__restrict__ partials, int blocks_per_view,
                                     int32_t nv, double weight, float *__restrict__ loss,
                                     float *__restrict__ d_dF)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    double s[10];
    for (int k = 0; k < 10; ++k) s[k] = 0.0;
    for (int b = 0; b < blocks_per_view; ++b)
        for (int k = 0; k < 10; ++k) s[k] += partials[((size_t)v * blocks_per_view + b) * 10 + k];
    const double P = (double)views[v].W * (double)views[v].H;
    loss[v] = (float)(weight / P * s[9]);
    if (!d_dF) return;
    const double *Mi = cams[v].Minv;
    // t = Minv^T G, gM = -t Minv^T
    double t[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            t[3 * r + c] = Mi[r] * s[c] + Mi[3 + r] * s[3 + c] + Mi[6 + r] * s[6 + c];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            const double gm = -(t[3 * r] * Mi[3 * c] + t[3 * r + 1] * Mi[3 * c + 1] +
                                t[3 * r + 2] * Mi[3 * c + 2]);
            d_dF[8 * v + 4 * r + c] += (float)gm;
        }
}

int normal_loss_blocks(int64_t max_view_pixels)
{
    return (int)((max_view_pixels + kGeomThreads * kGeomPx - 1) / (kGeomThreads * kGeomPx));
}

hipError_t launch_normal_loss(const ViewDesc *views, int32_t nv, int64_t max_view_pixels,
                              const float *Fxy, const float *dF, const float *D, const float *T,
                              const float *Nr, float weight, float tau, GeomCam *cams,
                              float2 *seeds, double *partials, float *loss, float *Nd_out,
                              float *d_depth, float *d_normal, float *d_dF, hipStream_t st)
{
    if (nv <= 0) return hipSuccess;
    const int bpv = normal_loss_blocks(max_view_pixels);
    hipLaunchKernelGGL(k_geom_cameras, dim3((unsigned)((nv + 63) / 64)), dim3(64), 0, st, Fxy, dF, nv,
                       cams);
    if (bpv > 0) {
        hipLaunchKernelGGL(k_normal_loss, dim3((unsigned)bpv, (unsigned)nv), dim3(kGeomThreads), 0, st,
                           views, cams, D, T, Nr, (double)weight, (double)tau, Nd_out, d_normal,
                           seeds, partials, bpv);
        const int dbl = (int)((max_view_pixels + kGeomThreads - 1) / kGeomThreads);
        hipLaunchKernelGGL(k_normal_loss_depth, dim3((unsigned)dbl, (unsigned)nv), dim3(kGeomThreads),
                           0, st, views, T, (double)tau, seeds, d_depth);
    }
    hipLaunchKernelGGL(k_normal_loss_reduce, dim3((unsigned)((nv + 63) / 64)), dim3(64), 0, st, views,
                       cams, partials, bpv, nv, (double)weight, loss, d_dF);
    return hipGetLastError();
}

}  // namespace ss
