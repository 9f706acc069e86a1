// Geometric sun-view shadow pass (SatSplat Sec. 3.3 Eq. sun_camera_Bxy, Supp. A; the
// soft shadow test of Sec. 3.1).  The sun-view depth map itself is rendered by the
// depth-only variant of the rasterizer; this file builds the sun cameras and runs the
// per-surfel exponential-shadow-map query.
#include "ss_internal.h"
#include <cmath>

namespace ss {

constexpr int kBoundsThreads = 256;
constexpr int kBoundsItems = 8;

int bounds_blocks(int64_t n)
{
    const int64_t per = (int64_t)kBoundsThreads * kBoundsItems;
    int64_t b = (n + per - 1) / per;
    return (int)(b < 1 ? 1 : b);
}

// Per-block min/max of the surfel centres (exact: min/max are exact in any order).
__global__ void k_bounds(const float *__restrict__ mean, int64_t n, double *__restrict__ partials)
{
    __shared__ float red[6][kBoundsThreads];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t base = (int64_t)blockIdx.x * kBoundsThreads * kBoundsItems;
    for (int k = 0; k < kBoundsItems; ++k) {
        const int64_t i = base + (int64_t)k * kBoundsThreads + threadIdx.x;
        if (i < n)
            for (int q = 0; q < 3; ++q) {
                const float x = mean[3 * i + q];
                lo[q] = fminf(lo[q], x);
                hi[q] = fmaxf(hi[q], x);
            }
    }
    for (int q = 0; q < 3; ++q) { red[q][threadIdx.x] = lo[q]; red[3 + q][threadIdx.x] = hi[q]; }
    __syncthreads();
    for (int s = kBoundsThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int q = 0; q < 3; ++q) {
                red[q][threadIdx.x] = fminf(red[q][threadIdx.x], red[q][threadIdx.x + s]);
                red[3 + q][threadIdx.x] = fmaxf(red[3 + q][threadIdx.x], red[3 + q][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) partials[6 * (int64_t)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// One block: finish the bounds, then one thread per view builds its sun camera in FP64:
//   s = (cos phi / tan theta, sin phi / tan theta, 1)
//   B_flat = B'_xy (I - [0 0 s])          (flatten along s onto z = 0, then project)
//   lam, o: the flattened AABB corners fill the central 98 % of the S x S map
//   B_sun = lam B_flat, b_sun = o, z_far = b_z - min z + 10 m
__global__ void k_sun_cameras(const double *__restrict__ partials, int nparts, int64_t n,
                              int32_t nv, const float *__restrict__ Fxy,
                              const float *__restrict__ dF, const float *__restrict__ sun,
                              float bz, int32_t S, SunCam *__restrict__ out)
{
    __shared__ double lo[3], hi[3];
    if (threadIdx.x == 0) {
        double l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int b = 0; b < nparts; ++b)
            for (int q = 0; q < 3; ++q) {
                l[q] = fmin(l[q], partials[6 * b + q]);
                h[q] = fmax(h[q], partials[6 * b + 3 + q]);
            }
        if (n == 0) for (int q = 0; q < 3; ++q) l[q] = h[q] = 0.0;
        for (int q = 0; q < 3; ++q) { lo[q] = l[q]; hi[q] = h[q]; }
    }
    __syncthreads();
    for (int v = threadIdx.x; v < nv; v += blockDim.x) {
        double B[2][3];
        for (int r = 0; r < 2; ++r)
            for (int q = 0; q < 3; ++q)
                B[r][q] = (double)Fxy[8 * v + 4 * r + q] + (dF ? (double)dF[8 * v + 4 * r + q] : 0.0);
        const double phi = sun[2 * v], theta = sun[2 * v + 1];
        const double s[3] = {cos(phi) / tan(theta), sin(phi) / tan(theta), 1.0};
        double Bf[2][3];
        for (int r = 0; r < 2; ++r) {
            Bf[r][0] = B[r][0];
            Bf[r][1] = B[r][1];
            Bf[r][2] = B[r][2] - (B[r][0] * s[0] + B[r][1] * s[1] + B[r][2] * s[2]);
        }
        double plo[2] = {INFINITY, INFINITY}, phi2[2] = {-INFINITY, -INFINITY};
        for (int ci = 0; ci < 8; ++ci) {
            const double P[3] = {(ci & 1) ? hi[0] : lo[0], (ci & 2) ? hi[1] : lo[1],
                                 (ci & 4) ? hi[2] : lo[2]};
            for (int r = 0; r < 2; ++r) {
                const double x = Bf[r][0] * P[0] + Bf[r][1] * P[1] + Bf[r][2] * P[2];
                if (x < plo[r]) plo[r] = x;
                if (x > phi2[r]) phi2[r] = x;
            }
        }
        double ext = phi2[0] - plo[0];
        if (phi2[1] - plo[1] > ext) ext = phi2[1] - plo[1];
        const double lam = ext > 0 ? 0.98 * S / ext : 1.0;
        SunCam c;
        for (int r = 0; r < 2; ++r) {
            for (int q = 0; q < 3; ++q) c.B[3 * r + q] = lam * Bf[r][q];
            c.b[r] = 0.5 * S - lam * 0.5 * (plo[r] + phi2[r]);
        }
        c.zfar = (double)bz - lo[2] + 10.0;
        for (int k = 0; k < 7; ++k) c.pad[k] = 0.0;
        out[v] = c;
    }
}

hipError_t launch_sun_cameras(const float *mean, int64_t n, int32_t nv, const float *Fxy,
                              const float *dF, const float *sun, float bz, int32_t S,
                              double *bounds_partials, SunCam *out, hipStream_t st)
{
    const int nb = bounds_blocks(n);
    hipLaunchKernelGGL(k_bounds, dim3((unsigned)nb), dim3(kBoundsThreads), 0, st, mean, n,
                       bounds_partials);
    hipLaunchKernelGGL(k_sun_cameras, dim3(1), dim3(64), 0, st, bounds_partials, nb, n, nv, Fxy,
                       dF, sun, bz, S, out);
    return hipGetLastError();
}

// Per (view, surfel): project the centre into the sun map (FP64, the texel choice is a
// floor), read the 3x3 texels around it (outside the map: background z_far), and
//   vis = min(1, (1/9) sum_t exp(c_e (D_t - d_k + beta))),  d_k = b_z - p_k,z.
__global__ void k_shadow_query(const float *__restrict__ mean, int64_t n,
                               const SunCam *__restrict__ sun, const float *__restrict__ D,
                               int32_t S, float bz, float esm_c, float esm_bias,
                               float *__restrict__ vis, float band, bool rows16)
{
    // view-outermost grid: the blocks in flight read one view's sun map, which stays in L2
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (k >= n) return;
    // band > 0: only points whose current (surrogate) value lies within the band
    if (band > 0.f && !(fabsf(vis[(int64_t)v * n + k] - 0.5f) < band)) return;
    const SunCam &c = sun[v];
    const double p0 = mean[3 * k], p1 = mean[3 * k + 1], p2 = mean[3 * k + 2];
    double x = c.b[0], y = c.b[1];
    x += c.B[0] * p0; x += c.B[1] * p1; x += c.B[2] * p2;
    y += c.B[3] * p0; y += c.B[4] * p1; y += c.B[5] * p2;
    const double fx = floor(x), fy = floor(y);
    const float dk = __fsub_rn(bz, (float)p2);
    const float zfar = (float)c.zfar;
    const float *Dv = D + (int64_t)v * S * S;
    // texels in row-major window order, each row's three read together: with rows16 (S a
    // multiple of 4 and D 16-byte aligned) every map row is 16-byte aligned, and a window
    // row inside the map lies in the aligned float4 at its first texel or in that one and
    // the next
    const double tx0 = fx - 1;
    const bool cols_in = tx0 >= 0 && tx0 + 2 < S;
    float acc = 0.f;
    for (int r = 0; r < 3; ++r) {
        const double ty = fy + r - 1;
        float d[3] = {zfar, zfar, zfar};
        if (ty >= 0 && ty < S) {
            const float *row = Dv + (int64_t)ty * S;
            if (rows16 && cols_in) {
                const int64_t x0 = (int64_t)tx0, a = x0 & ~(int64_t)3;
                const int o = (int)(x0 - a);
                const float4 A = *reinterpret_cast<const float4 *>(row + a);
                float4 B = A;
                if (o >= 2) B = *reinterpret_cast<const float4 *>(row + a + 4);
                d[0] = o == 0 ? A.x : o == 1 ? A.y : o == 2 ? A.z : A.w;
                d[1] = o == 0 ? A.y : o == 1 ? A.z : o == 2 ? A.w : B.x;
                d[2] = o == 0 ? A.z : o == 1 ? A.w : o == 2 ? B.x : B.y;
            } else {
                for (int i = 0; i < 3; ++i) {
                    const double tx = tx0 + i;
                    if (tx >= 0 && tx < S) d[i] = row[(int64_t)tx];
                }
            }
        }
        for (int i = 0; i < 3; ++i) acc += expf(esm_c * (d[i] - dk + esm_bias));
    }
    acc *= (1.f / 9.f);
    vis[(int64_t)v * n + k] = fminf(1.f, acc);
}

hipError_t launch_shadow_query(const float *mean, int64_t n, int32_t nv, const SunCam *sun,
                               const float *sun_depth, int32_t S, float bz, float esm_c,
                               float esm_bias, float *vis, float band, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const bool rows16 = S % 4 == 0 && reinterpret_cast<uintptr_t>(sun_depth) % 16 == 0;
    hipLaunchKernelGGL(k_shadow_query, dim3((unsigned)((n + 255) / 256), (unsigned)nv), dim3(256),
                       0, st, mean, n, sun, sun_depth, S, bz, esm_c, esm_bias, vis, band, rows16);
    return hipGetLastError();
}

// Surrogate fallback: every point whose surrogate visibility lies within `band` of 0.5
// marks the sun-map tiles of its 3x3 texel window (same FP64 texel choice as the query)
// and is counted.  A block covers a contiguous chunk of one view's points and collects
// the view's tile set as a bitmask in LDS (the window spans at most 2 x 2 tiles); at the
// end it stores its set tiles with coalesced writes and adds its count with one atomic.
constexpr int kFlagThreads = 256;
constexpr int kFlagChunk = 8192;         // points per block

__global__ __launch_bounds__(kFlagThreads) void k_flag_tiles(
    const float *__restrict__ mean, int64_t n, const SunCam *__restrict__ sun,
    const ViewDesc *__restrict__ views, int32_t S, int ts, const float *__restrict__ vis,
    float band, uint32_t *__restrict__ tmask, unsigned long long *__restrict__ count)
{
    extern __shared__ uint32_t bits[];
    __shared__ uint32_t nflag;
    const int v = blockIdx.y;
    const ViewDesc vd = views[v];
    const int ntiles = vd.tiles_x * vd.tiles_y;
    const int nwords = (ntiles + 31) >> 5;
    for (int i = threadIdx.x; i < nwords; i += kFlagThreads) bits[i] = 0u;
    if (threadIdx.x == 0) nflag = 0u;
    __syncthreads();
    const SunCam &c = sun[v];
    const int64_t k0 = (int64_t)blockIdx.x * kFlagChunk;
    const int64_t k1 = min(n, k0 + (int64_t)kFlagChunk);
    uint32_t mine = 0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += kFlagThreads) {
        if (!(fabsf(vis[(int64_t)v * n + k] - 0.5f) < band)) continue;
        ++mine;
        const double p0 = mean[3 * k], p1 = mean[3 * k + 1], p2 = mean[3 * k + 2];
        double x = c.b[0], y = c.b[1];
        x += c.B[0] * p0; x += c.B[1] * p1; x += c.B[2] * p2;
        y += c.B[3] * p0; y += c.B[4] * p1; y += c.B[5] * p2;
        const double fx = floor(x), fy = floor(y);
        // texel window [fx - 1, fx + 1] x [fy - 1, fy + 1] clipped to the map
        const double xl = fmax(fx - 1.0, 0.0), xh = fmin(fx + 1.0, (double)(S - 1));
        const double yl = fmax(fy - 1.0, 0.0), yh = fmin(fy + 1.0, (double)(S - 1));
        if (!(xl <= xh && yl <= yh)) continue;
        const int cx0 = (int)xl / ts, cx1 = (int)xh / ts, cy0 = (int)yl / ts, cy1 = (int)yh / ts;
        for (int ty = cy0; ty <= cy1; ++ty)
            for (int tx = cx0; tx <= cx1; ++tx) {
                const int t = ty * vd.tiles_x + tx;
                atomicOr(&bits[t >> 5], 1u << (t & 31));
            }
    }
    if (mine) atomicAdd(&nflag, mine);
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += kFlagThreads)
        if ((bits[t >> 5] >> (t & 31)) & 1u) tmask[vd.tile_off + t] = 1u;
    if (threadIdx.x == 0 && nflag) atomicAdd(count, (unsigned long long)nflag);
}

// Same marking without the LDS bitmask, one point per thread, for sun maps whose tile
// set does not fit in LDS.
__global__ void k_flag_tiles_direct(const float *__restrict__ mean, int64_t n,
                                    const SunCam *__restrict__ sun,
                                    const ViewDesc *__restrict__ views, int32_t S, int ts,
                                    const float *__restrict__ vis, float band,
                                    uint32_t *__restrict__ tmask,
                                    unsigned long long *__restrict__ count)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    const bool flag = k < n && fabsf(vis[(int64_t)v * n + k] - 0.5f) < band;
    const unsigned long long wb = __ballot(flag);
    if ((threadIdx.x & 63) == 0 && wb != 0ull) atomicAdd(count, (unsigned long long)__popcll(wb));
    if (!flag) return;
    const SunCam &c = sun[v];
    const double p0 = mean[3 * k], p1 = mean[3 * k + 1], p2 = mean[3 * k + 2];
    double x = c.b[0], y = c.b[1];
    x += c.B[0] * p0; x += c.B[1] * p1; x += c.B[2] * p2;
    y += c.B[3] * p0; y += c.B[4] * p1; y += c.B[5] * p2;
    const double fx = floor(x), fy = floor(y);
    const double xl = fmax(fx - 1.0, 0.0), xh = fmin(fx + 1.0, (double)(S - 1));
    const double yl = fmax(fy - 1.0, 0.0), yh = fmin(fy + 1.0, (double)(S - 1));
    if (!(xl <= xh && yl <= yh)) return;
    const ViewDesc vd = views[v];
    const int cx0 = (int)xl / ts, cx1 = (int)xh / ts, cy0 = (int)yl / ts, cy1 = (int)yh / ts;
    for (int ty = cy0; ty <= cy1; ++ty)
        for (int tx = cx0; tx <= cx1; ++tx) tmask[vd.tile_off + ty * vd.tiles_x + tx] = 1u;
}

hipError_t launch_flag_tiles(const float *mean, int64_t n, int32_t nv, const SunCam *sun,
                             const ViewDesc *views, int32_t S, int ts, const float *vis,
                             float band, uint32_t *tmask, unsigned long long *count, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (int64_t)((S + ts - 1) / ts) * ((S + ts - 1) / ts);
    const size_t lds = (size_t)((tiles + 31) / 32) * sizeof(uint32_t);
    if (lds > 48 * 1024) {                               // sun maps above 4096^2 at 8x8 tiles
        hipLaunchKernelGGL(k_flag_tiles_direct, dim3((unsigned)((n + 255) / 256), (unsigned)nv),
                           dim3(256), 0, st, mean, n, sun, views, S, ts, vis, band, tmask, count);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_flag_tiles, dim3((unsigned)((n + kFlagChunk - 1) / kFlagChunk), (unsigned)nv),
                       dim3(kFlagThreads), lds, st, mean, n, sun, views, S, ts, vis, band, tmask,
                       count);
    return hipGetLastError();
}

}  // namespace ss
