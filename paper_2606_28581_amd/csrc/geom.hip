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

// zbar = D / (1 - T) of pixel g and whether 1 - T >= tau there (zbar is only used where
// it holds)
__device__ __forceinline__ double zbar_cov(const float *D, const float *T, int64_t g, double tau,
                                           bool &cov)
{
    const double a = 1.0 - (double)T[g];
    cov = a >= tau;
    return cov ? (double)D[g] / a : 0.0;
}

// Blocks of kNlCols x kNlRows pixels of view blockIdx.y, one column per thread, walked
// row by row: each thread keeps zbar of rows y - 1, y, y + 1 of its column in registers
// and the block shares row y (with one halo column on each side) through LDS, so every
// pixel's zbar is computed once (plus two halo rows per block).  Per pixel: depth normal,
// loss term, d_normal (added), the z-adjoint seeds s = Minv[:, 2] . dL/dgrad p stored per
// pixel, and per block the sums of the loss terms and of dL/dMinv (10 doubles).
constexpr int kNlCols = 256;
constexpr int kNlRows = 16;

__device__ __forceinline__ void normal_loss_pixel(
    int64_t P, int64_t g, int64_t b3, bool valid, double dzx, double dzy, const GeomCam &c,
    const float (&nr)[3], const float (&dn)[3], double wv, float *__restrict__ Nd_out,
    float *__restrict__ d_normal, float2 *__restrict__ seeds, double (&acc)[10])
{
    float2 s = make_float2(0.f, 0.f);
    float nd[3] = {0.f, 0.f, 0.f};
    if (valid) {
        const double *Mi = c.Minv;
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
            R[r] = (double)nr[r];
        }
        acc[9] += 1.0 - (R[0] * N[0] + R[1] * N[1] + R[2] * N[2]);
        for (int r = 0; r < 3; ++r) {
            d_normal[b3 + r * P] = dn[r] + (float)(-wv * N[r]);
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

__global__ __launch_bounds__(kNlCols) void k_normal_loss(
    const ViewDesc *__restrict__ views, const GeomCam *__restrict__ cams,
    const float *__restrict__ D, const float *__restrict__ T, const float *__restrict__ Nr,
    double weight, double tau, float *__restrict__ Nd_out, float *__restrict__ d_normal,
    float2 *__restrict__ seeds, double *__restrict__ partials, int blocks_per_view)
{
    __shared__ double zrow[2][kNlCols + 2];
    __shared__ int crow[2][kNlCols + 2];
    __shared__ double red[kNlCols / 64][10];
    const int v = blockIdx.y;
    const ViewDesc vd = views[v];
    const int64_t P = (int64_t)vd.W * vd.H;
    const GeomCam c = cams[v];
    const double wv = weight / (double)P;
    double acc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = 0.0;
    const int nbx = (vd.W + kNlCols - 1) / kNlCols, nby = (vd.H + kNlRows - 1) / kNlRows;
    if ((int)blockIdx.x < nbx * nby) {   // uniform over the block
        const int tid = threadIdx.x;
        const int x0 = ((int)blockIdx.x % nbx) * kNlCols, y0 = ((int)blockIdx.x / nbx) * kNlRows;
        const int y1 = min(y0 + kNlRows, vd.H);
        const int x = x0 + tid;
        const bool incol = x < vd.W;
        // threads 0 and 1 also fill the halo columns x0 - 1 and x0 + kNlCols
        const int hx = tid == 0 ? x0 - 1 : x0 + kNlCols;
        const bool halo = tid < 2 && hx >= 0 && hx < vd.W;
        const int hslot = tid == 0 ? 0 : kNlCols + 1;
        const int64_t base = vd.pix_off;
        const double one = 1.0;
        auto zbar = [&](float d, float t, bool &cov) {
            const double a = one - (double)t;
            cov = a >= tau;
            return cov ? (double)d / a : 0.0;
        };
        bool cm = false, cc = false;   // 1 - T >= tau at (x, y - 1), (x, y)
        double zm = 0.0, zc = 0.0;
        if (incol && y0 > 0) zm = zbar_cov(D, T, base + (int64_t)(y0 - 1) * vd.W + x, tau, cm);
        if (incol) zc = zbar_cov(D, T, base + (int64_t)y0 * vd.W + x, tau, cc);
        // D and T of the next row (of the column, and of the halo column) are loaded one
        // row ahead, so no row waits for its own loads behind the barrier
        float Dn = 0.f, Tn = 1.f, Dh = 0.f, Th = 1.f;
        if (incol && y0 + 1 < vd.H) {
            Dn = D[base + (int64_t)(y0 + 1) * vd.W + x];
            Tn = T[base + (int64_t)(y0 + 1) * vd.W + x];
        }
        if (halo) {
            Dh = D[base + (int64_t)y0 * vd.W + hx];
            Th = T[base + (int64_t)y0 * vd.W + hx];
        }
        for (int y = y0; y < y1; ++y) {
            bool cp = false;
            double zp = 0.0;
            if (incol && y + 1 < vd.H) zp = zbar(Dn, Tn, cp);
            const int64_t local = (int64_t)y * vd.W + x;
            float nr[3] = {0.f, 0.f, 0.f}, dn[3] = {0.f, 0.f, 0.f};
            if (incol) {
                for (int r = 0; r < 3; ++r) {
                    nr[r] = Nr[3 * base + local + r * P];
                    dn[r] = d_normal[3 * base + local + r * P];
                }
            }
            const int buf = y & 1;
            zrow[buf][tid + 1] = zc;
            crow[buf][tid + 1] = incol && cc;
            if (tid < 2) {
                bool ch = false;
                const double zh = halo ? zbar(Dh, Th, ch) : 0.0;
                zrow[buf][hslot] = zh;
                crow[buf][hslot] = ch;
            }
            if (incol && y + 2 < vd.H) {
                Dn = D[base + (int64_t)(y + 2) * vd.W + x];
                Tn = T[base + (int64_t)(y + 2) * vd.W + x];
            }
            if (halo && y + 1 < vd.H) {
                Dh = D[base + (int64_t)(y + 1) * vd.W + hx];
                Th = T[base + (int64_t)(y + 1) * vd.W + hx];
            }
            // one barrier per row: row y + 1 goes to the other buffer, whose readers (row
            // y - 1) have all passed this barrier
            __syncthreads();
            if (incol) {
                const bool valid = x > 0 && y > 0 && x < vd.W - 1 && y < vd.H - 1 && cc && cm && cp &&
                                   crow[buf][tid] && crow[buf][tid + 2];
                const double dzx = zrow[buf][tid + 2] - zrow[buf][tid];
                const double dzy = zp - zm;
                normal_loss_pixel(P, base + local, 3 * base + local, valid, dzx, dzy, c, nr, dn, wv,
                                  Nd_out, d_normal, seeds, acc);
            }
            zm = zc; cm = cc;
            zc = zp; cc = cp;
        }
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
        for (int w = 0; w < kNlCols / 64; ++w) x += red[w][threadIdx.x];
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

int normal_loss_blocks(const ViewDesc *host_views, int32_t nv)
{
    int64_t m = 0;
    for (int32_t v = 0; v < nv; ++v) {
        const int64_t nbx = ((int64_t)host_views[v].W + kNlCols - 1) / kNlCols;
        const int64_t nby = ((int64_t)host_views[v].H + kNlRows - 1) / kNlRows;
        m = std::max(m, nbx * nby);
    }
    return (int)m;
}

hipError_t launch_normal_loss(const ViewDesc *views, const ViewDesc *host_views, int32_t nv,
                              int64_t max_view_pixels,
                              const float *Fxy, const float *dF, const float *D, const float *T,
                              const float *Nr, float weight, float tau, GeomCam *cams,
                              float2 *seeds, double *partials, float *loss, float *Nd_out,
                              float *d_depth, float *d_normal, float *d_dF, hipStream_t st)
{
    if (nv <= 0) return hipSuccess;
    const int bpv = normal_loss_blocks(host_views, nv);
    hipLaunchKernelGGL(k_geom_cameras, dim3((unsigned)((nv + 63) / 64)), dim3(64), 0, st, Fxy, dF, nv,
                       cams);
    if (bpv > 0) {
        hipLaunchKernelGGL(k_normal_loss, dim3((unsigned)bpv, (unsigned)nv), dim3(kNlCols), 0, st,
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
