// Geometry-aware initialisation of the surfels on a DSM (SatSplat, arXiv 2606.28581, Sec.
// 3.4): each DSM cell gets an area weight a = |dx x dy| from its finite differences,
// surfel centres are drawn with probability proportional to a, and each surfel's frame is
// built by Gram-Schmidt against the local surface normal.
//
// DSM: node heights z[j][i] at (x0 + i g, y0 + j g); cell (j, i) spans nodes j..j+1,
// i..i+1, its tangents are (g, 0, dzx) and (0, g, dzy) with dzx, dzy the means of its two
// edge differences, a = g sqrt(dzx^2 + dzy^2 + g^2), normal (-dzx, -dzy, g) / sqrt(...).
// The weights are integers (65536 per flat cell: floor(65536 a / g^2 + 1/2)) and their
// prefix sum is uint64, so every sampling decision is exact; the geometry is FP64 from
// the FP32 heights.  Sample k draws Philox4x32-10 (Salmon et al., SC 2011; key = seed,
// counters (k, 0, 0, 0) and (k, 1, 0, 0)): the first two words pick the cell, the next
// two the position inside it (bilinear height), three more a random vector that
// Gram-Schmidt turns into t_u (t_v = n x t_u).  Scales are the surface-area spacing
// sqrt(area / N); opacity and albedo are given constants.
#include "ss_internal.h"

namespace ss {

constexpr int kInitThreads = 256;
constexpr int kScanPer = 8;                                  // cells per thread in the scan
constexpr int kScanBlock = kInitThreads * kScanPer;          // cells per scan block
constexpr double kWeightOne = 65536.0;

struct Philox4 {
    uint32_t v[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
        const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    return Philox4{{c0, c1, c2, c3}};
}

struct CellSlopes {
    double dzx, dzy, s;   // s = sqrt(dzx^2 + dzy^2 + g^2)
};

__device__ __forceinline__ CellSlopes cell_slopes(const float *__restrict__ z, int nx, int cj, int ci,
                                                  double g)
{
    const double z00 = z[(size_t)cj * nx + ci], z10 = z[(size_t)cj * nx + ci + 1];
    const double z01 = z[(size_t)(cj + 1) * nx + ci], z11 = z[(size_t)(cj + 1) * nx + ci + 1];
    CellSlopes c;
    c.dzx = 0.5 * ((z10 - z00) + (z11 - z01));
    c.dzy = 0.5 * ((z01 - z00) + (z11 - z10));
    c.s = sqrt(c.dzx * c.dzx + c.dzy * c.dzy + g * g);
    return c;
}

// integer area weight per cell
__global__ __launch_bounds__(kInitThreads) void k_dsm_weights(int nx, int ny, const float *__restrict__ z,
                                                              double g, uint32_t *__restrict__ w)
{
    const int64_t ncx = nx - 1, nc = ncx * (ny - 1);
    const int64_t c = (int64_t)blockIdx.x * kInitThreads + threadIdx.x;
    if (c >= nc) return;
    const CellSlopes s = cell_slopes(z, nx, (int)(c / ncx), (int)(c % ncx), g);
    const double area = g * s.s;
    w[c] = (uint32_t)floor(area / (g * g) * kWeightOne + 0.5);
}

// inclusive uint64 prefix sum of the weights: block totals, a scan of the totals by one
// block, then each block's local scan plus its offset
__global__ __launch_bounds__(kInitThreads) void k_scan_totals(const uint32_t *__restrict__ w, int64_t nc,
                                                              unsigned long long *__restrict__ totals)
{
    __shared__ unsigned long long red[kInitThreads / 64];
    const int64_t c0 = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    unsigned long long s = 0;
    for (int k = 0; k < kScanPer; ++k)
        if (c0 + k < nc) s += w[c0 + k];
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < kInitThreads / 64; ++k) t += red[k];
        totals[blockIdx.x] = t;
    }
}

// exclusive scan of the block totals in place (one block, chunks of kInitThreads)
__global__ __launch_bounds__(kInitThreads) void k_scan_offsets(unsigned long long *__restrict__ totals,
                                                               int nblocks)
{
    __shared__ unsigned long long buf[kInitThreads];
    unsigned long long carry = 0;
    for (int b0 = 0; b0 < nblocks; b0 += kInitThreads) {
        const int b = b0 + threadIdx.x;
        const unsigned long long x = b < nblocks ? totals[b] : 0ull;
        buf[threadIdx.x] = x;
        __syncthreads();
        for (int d = 1; d < kInitThreads; d <<= 1) {
            const unsigned long long y = threadIdx.x >= d ? buf[threadIdx.x - d] : 0ull;
            __syncthreads();
            buf[threadIdx.x] += y;
            __syncthreads();
        }
        if (b < nblocks) totals[b] = carry + buf[threadIdx.x] - x;
        carry += buf[kInitThreads - 1];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kInitThreads) void k_scan_final(const uint32_t *__restrict__ w, int64_t nc,
                                                             const unsigned long long *__restrict__ offsets,
                                                             unsigned long long *__restrict__ cdf)
{
    __shared__ unsigned long long buf[kInitThreads];
    const int64_t c0 = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    unsigned long long local[kScanPer], s = 0;
    for (int k = 0; k < kScanPer; ++k) {
        s += (c0 + k < nc) ? w[c0 + k] : 0u;
        local[k] = s;
    }
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int d = 1; d < kInitThreads; d <<= 1) {
        const unsigned long long y = threadIdx.x >= d ? buf[threadIdx.x - d] : 0ull;
        __syncthreads();
        buf[threadIdx.x] += y;
        __syncthreads();
    }
    const unsigned long long before = offsets[blockIdx.x] + buf[threadIdx.x] - s;
    for (int k = 0; k < kScanPer; ++k)
        if (c0 + k < nc) cdf[c0 + k] = before + local[k];
}

__global__ __launch_bounds__(kInitThreads) void k_dsm_sample(
    int nx, int ny, const float *__restrict__ z, double x0, double y0, double g,
    const unsigned long long *__restrict__ cdf, int64_t nc, int64_t n, uint32_t key0, uint32_t key1,
    float opacity, float albedo, float *__restrict__ mean, float *__restrict__ tu,
    float *__restrict__ tv, float *__restrict__ scale, float *__restrict__ opac,
    float *__restrict__ alb, int64_t *__restrict__ cell_out)
{
    const int64_t k = (int64_t)blockIdx.x * kInitThreads + threadIdx.x;
    if (k >= n) return;
    const unsigned long long total = cdf[nc - 1];
    const Philox4 a = philox4x32_10((uint32_t)k, 0u, 0u, 0u, key0, key1);
    const Philox4 b = philox4x32_10((uint32_t)k, 1u, 0u, 0u, key0, key1);
    const unsigned long long t = (((unsigned long long)a.v[1] << 32) | a.v[0]) % total;
    // first cell whose cumulative weight exceeds t
    int64_t lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cdf[mid] > t) hi = mid; else lo = mid + 1;
    }
    const int64_t ncx = nx - 1;
    const int cj = (int)(lo / ncx), ci = (int)(lo % ncx);
    const double fx = (double)a.v[2] / 4294967296.0, fy = (double)a.v[3] / 4294967296.0;
    const double z00 = z[(size_t)cj * nx + ci], z10 = z[(size_t)cj * nx + ci + 1];
    const double z01 = z[(size_t)(cj + 1) * nx + ci], z11 = z[(size_t)(cj + 1) * nx + ci + 1];
    const double zz = (z00 * (1.0 - fx) + z10 * fx) * (1.0 - fy) + (z01 * (1.0 - fx) + z11 * fx) * fy;
    mean[3 * k] = (float)(x0 + ((double)ci + fx) * g);
    mean[3 * k + 1] = (float)(y0 + ((double)cj + fy) * g);
    mean[3 * k + 2] = (float)zz;
    const CellSlopes s = cell_slopes(z, nx, cj, ci, g);
    const double nn[3] = {-s.dzx / s.s, -s.dzy / s.s, g / s.s};
    double r[3] = {(double)b.v[0] / 2147483648.0 - 1.0, (double)b.v[1] / 2147483648.0 - 1.0,
                   (double)b.v[2] / 2147483648.0 - 1.0};
    double rn = r[0] * nn[0] + r[1] * nn[1] + r[2] * nn[2];
    double u[3] = {r[0] - rn * nn[0], r[1] - rn * nn[1], r[2] - rn * nn[2]};
    double ul = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (ul < 1e-6) {   // the random vector lies along the normal: use the x axis
        u[0] = 1.0 - nn[0] * nn[0];
        u[1] = -nn[1] * nn[0];
        u[2] = -nn[2] * nn[0];
        ul = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    }
    for (int c = 0; c < 3; ++c) u[c] /= ul;
    const double v[3] = {nn[1] * u[2] - nn[2] * u[1], nn[2] * u[0] - nn[0] * u[2], nn[0] * u[1] - nn[1] * u[0]};
    for (int c = 0; c < 3; ++c) {
        tu[3 * k + c] = (float)u[c];
        tv[3 * k + c] = (float)v[c];
        alb[3 * k + c] = albedo;
    }
    const float sp = (float)sqrt((double)total * g * g / kWeightOne / (double)n);
    scale[2 * k] = sp;
    scale[2 * k + 1] = sp;
    opac[k] = opacity;
    if (cell_out) cell_out[k] = lo;
}

static inline int64_t dsm_cells(int nx, int ny) { return (int64_t)(nx - 1) * (ny - 1); }
static inline int64_t scan_blocks(int64_t nc) { return (nc + kScanBlock - 1) / kScanBlock; }

size_t dsm_init_workspace_bytes(int nx, int ny)
{
    const int64_t nc = dsm_cells(nx, ny);
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    return al((size_t)nc * 4) + al((size_t)nc * 8) + al((size_t)scan_blocks(nc) * 8);
}

hipError_t launch_dsm_init(int nx, int ny, const float *z, double x0, double y0, double g, int64_t n,
                           uint64_t seed, float opacity, float albedo, void *ws, float *mean,
                           float *tu, float *tv, float *scale, float *opac, float *alb,
                           int64_t *cell, hipStream_t st)
{
    const int64_t nc = dsm_cells(nx, ny);
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    char *p = static_cast<char *>(ws);
    uint32_t *w = reinterpret_cast<uint32_t *>(p);
    unsigned long long *cdf = reinterpret_cast<unsigned long long *>(p + al((size_t)nc * 4));
    unsigned long long *tot = reinterpret_cast<unsigned long long *>(p + al((size_t)nc * 4) + al((size_t)nc * 8));
    const int64_t nb = scan_blocks(nc);
    hipLaunchKernelGGL(k_dsm_weights, dim3((unsigned)((nc + kInitThreads - 1) / kInitThreads)),
                       dim3(kInitThreads), 0, st, nx, ny, z, g, w);
    hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)nb), dim3(kInitThreads), 0, st, w, nc, tot);
    hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(kInitThreads), 0, st, tot, (int)nb);
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kInitThreads), 0, st, w, nc, tot, cdf);
    if (n > 0)
        hipLaunchKernelGGL(k_dsm_sample, dim3((unsigned)((n + kInitThreads - 1) / kInitThreads)),
                           dim3(kInitThreads), 0, st, nx, ny, z, x0, y0, g, cdf, nc, n,
                           (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), opacity, albedo, mean,
                           tu, tv, scale, opac, alb, cell);
    return hipGetLastError();
}

}  // namespace ss
