// Affine-camera 2D Gaussian surfel rasterizer for gfx950 (SatSplat, arXiv 2606.28581,
// Sec. 3.2-3.3): projection, binning, forward compositing, backward adjoint.
//
// Work is organised in depth-rank space: after the global centre-depth sort the
// surfel parameters are gathered once into rank order, so projection, the pair-count
// scan and the (view, rank) records are contiguous, and tile lists hold ranks.
#include "ss_internal.h"
#include <cmath>

namespace ss {

constexpr float kNegHalfLog2e = -0.72134752044448170f;   // -0.5 * log2(e)
constexpr int kParamFloats = 16;                          // gathered surfel: 4 x float4

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ int find_view(const ViewDesc *views, int nv, int tile)
{
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------------ depth keys
// kappa = fl32(b_z - p_z) (Eq. depth_affine_camera on the centre), mapped to an
// order-preserving uint32: total order over all finite floats, no altitude limit.
__global__ void k_depth_keys(const float *__restrict__ mean, int64_t n, float bz,
                             uint32_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float kap = __fsub_rn(bz, mean[3 * i + 2]);
    uint32_t b = __float_as_uint(kap);
    keys[i] = b ^ ((b >> 31) ? 0xFFFFFFFFu : 0x80000000u);
    vals[i] = (uint32_t)i;
}

hipError_t launch_depth_keys(const float *mean, int64_t n, float bz, uint32_t *keys,
                             uint32_t *vals, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_depth_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, mean,
                       n, bz, keys, vals);
    return hipGetLastError();
}

// ------------------------------------------------------- gather into rank order
// sorted[r] = (p, t_u, t_v, s_u, s_v, o, albedo) of surfel order[r], 16 floats.
__global__ void k_gather_params(const uint32_t *__restrict__ order, SurfelPtrs s,
                                float4 *__restrict__ out)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= s.n) return;
    int64_t i = order[r];
    if (i >= s.n) i = 0;   // only reachable through a sort defect; keeps the gather in bounds
    float4 a, b, c, d;
    a.x = s.mean[3 * i]; a.y = s.mean[3 * i + 1]; a.z = s.mean[3 * i + 2]; a.w = s.t_u[3 * i];
    b.x = s.t_u[3 * i + 1]; b.y = s.t_u[3 * i + 2]; b.z = s.t_v[3 * i]; b.w = s.t_v[3 * i + 1];
    c.x = s.t_v[3 * i + 2]; c.y = s.scale[2 * i]; c.z = s.scale[2 * i + 1]; c.w = s.opacity[i];
    d.x = s.albedo[3 * i]; d.y = s.albedo[3 * i + 1]; d.z = s.albedo[3 * i + 2]; d.w = 0.f;
    out[4 * r] = a; out[4 * r + 1] = b; out[4 * r + 2] = c; out[4 * r + 3] = d;
}

hipError_t launch_gather_params(const uint32_t *order, const SurfelPtrs &s, float *out,
                                hipStream_t st)
{
    if (s.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_params, dim3((unsigned)((s.n + 255) / 256)), dim3(256), 0, st,
                       order, s, reinterpret_cast<float4 *>(out));
    return hipGetLastError();
}

// Affine projection of one surfel's tangent frame (Sec. 3.2, Eqs. affine2dgs_uv2screen,
// affine2dgs_Qq): M = [s_u t_u, s_v t_v], T = B M, Q = T^-1 (zero when T is degenerate),
// and the sign that orients the normal m = t_u x t_v against the viewing direction
// d = B_x x B_y taken looking down (d_z < 0).  FP64; the projection and its backward both
// call it, so the backward sees the very Q and sign the forward used.
struct SurfelAffine {
    double M[3][2], T[2][2], Q[2][2], m[3];
    double nsign;
    bool deg;
};

__device__ __forceinline__ SurfelAffine surfel_affine(const double (&B)[2][3], const double (&tu)[3],
                                                      const double (&tv)[3], double su, double sv,
                                                      double det_rel_eps)
{
    SurfelAffine a;
    for (int i = 0; i < 3; ++i) { a.M[i][0] = su * tu[i]; a.M[i][1] = sv * tv[i]; }
    for (int row = 0; row < 2; ++row)
        for (int q = 0; q < 2; ++q) {
            double acc = 0.0;
            for (int i = 0; i < 3; ++i) acc += B[row][i] * a.M[i][q];
            a.T[row][q] = acc;
        }
    const double(&T)[2][2] = a.T;
    const double det = T[0][0] * T[1][1] - T[0][1] * T[1][0];
    const double fro2 = T[0][0] * T[0][0] + T[0][1] * T[0][1] + T[1][0] * T[1][0] + T[1][1] * T[1][1];
    a.deg = !(fabs(det) > det_rel_eps * fro2);
    a.Q[0][0] = a.Q[0][1] = a.Q[1][0] = a.Q[1][1] = 0.0;
    if (!a.deg) {
        a.Q[0][0] = T[1][1] / det; a.Q[0][1] = -T[0][1] / det;
        a.Q[1][0] = -T[1][0] / det; a.Q[1][1] = T[0][0] / det;
    }
    a.m[0] = tu[1] * tv[2] - tu[2] * tv[1];
    a.m[1] = tu[2] * tv[0] - tu[0] * tv[2];
    a.m[2] = tu[0] * tv[1] - tu[1] * tv[0];
    double dvec[3] = {B[0][1] * B[1][2] - B[0][2] * B[1][1], B[0][2] * B[1][0] - B[0][0] * B[1][2],
                      B[0][0] * B[1][1] - B[0][1] * B[1][0]};
    if (dvec[2] > 0) { dvec[0] = -dvec[0]; dvec[1] = -dvec[1]; dvec[2] = -dvec[2]; }
    const double nd = a.m[0] * dvec[0] + a.m[1] * dvec[1] + a.m[2] * dvec[2];
    a.nsign = nd > 0 ? -1.0 : 1.0;
    return a;
}

// ------------------------------------------------------------------- projection
// One thread per (rank r, view v).  Geometry in FP64 (the binning contract: tile
// ranges must be bit-identical to an FP64 reference), records rounded to FP32.
//   T = B'_xy [s_u t_u, s_v t_v]   c = B'_xy p + b'_xy   Q = T^-1   (Eq. affine2dgs_Qq)
//   degenerate iff |det T| <= eps |T|_F^2 ("Degenerate Solutions")
//   support: alpha >= alpha_min needs rho <= 2 ln(o / alpha_min); the uv-ellipse
//   {T w : |w|^2 <= rho_max} has x half-extent r |T row 0|, the low-pass disk radius
//   sigma r; pixel i is in the box iff i + 0.5 lies within the half-extent of c.
__global__ __launch_bounds__(256) void k_project(
    const float4 *__restrict__ sp, int64_t n, int32_t nv,
    const ViewDesc *__restrict__ views, const float *__restrict__ Fxy,
    const float *__restrict__ dF, const SunCam *__restrict__ sun,
    const float *__restrict__ vis_rank, float bz, int ts, RasterConsts rc,
    float4 *__restrict__ rec, short4 *__restrict__ tiles, uint32_t *__restrict__ counts,
    const uint32_t *__restrict__ tmask)
{
    // the block's 256 records are staged in LDS and written back as one contiguous run.
    // Blocks run view-innermost (block = rank block x views + view), in xcd_tile's chunked
    // order, so the views of one rank block share the surfel parameters in one L2.
    __shared__ float4 srec[256 * kRecVec4];
    const int64_t L = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int v = (int)(L % nv);
    const int64_t r0 = (L / nv) * blockDim.x;
    const bool valid = r0 + threadIdx.x < n;
    const int64_t r = valid ? r0 + threadIdx.x : n - 1;   // lanes past the end repeat the last
    const ViewDesc vd = views[v];
    double B[2][3], b[2];
    if (sun) {
        for (int q = 0; q < 3; ++q) { B[0][q] = sun[v].B[q]; B[1][q] = sun[v].B[3 + q]; }
        b[0] = sun[v].b[0]; b[1] = sun[v].b[1];
    } else {
        for (int row = 0; row < 2; ++row) {
            for (int q = 0; q < 3; ++q)
                B[row][q] = (double)Fxy[8 * v + 4 * row + q] +
                            (dF ? (double)dF[8 * v + 4 * row + q] : 0.0);
            b[row] = (double)Fxy[8 * v + 4 * row + 3] + (dF ? (double)dF[8 * v + 4 * row + 3] : 0.0);
        }
    }
    const float4 pa = sp[4 * r], pb = sp[4 * r + 1], pc = sp[4 * r + 2], pd = sp[4 * r + 3];
    const double p[3] = {pa.x, pa.y, pa.z};
    const double tu[3] = {pa.w, pb.x, pb.y};
    const double tv[3] = {pb.z, pb.w, pc.x};
    const double su = pc.y, sv = pc.z, o = pc.w;
    const SurfelAffine sa = surfel_affine(B, tu, tv, su, sv, rc.det_rel_eps_d);
    const double(&M)[3][2] = sa.M;
    const double(&T)[2][2] = sa.T;
    const double(&Q)[2][2] = sa.Q;
    const double(&m)[3] = sa.m;
    const bool deg = sa.deg;
    const double nsign = sa.nsign;
    double c[2];
    for (int row = 0; row < 2; ++row) {
        double acc = b[row];
        for (int i = 0; i < 3; ++i) acc += B[row][i] * p[i];
        c[row] = acc;
    }
    const bool filt = (rc.lowpass_mode == 0) || deg;
    const double mn = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    // support box -> pixel and tile ranges
    int ilo = 0, ihi = -1, jlo = 0, jhi = -1;
    if (o >= rc.alpha_min_d) {
        const double rr = sqrt(2.0 * log(o / rc.alpha_min_d));
        double hx = 0.0, hy = 0.0;
        if (!deg) {
            hx = rr * sqrt(T[0][0] * T[0][0] + T[0][1] * T[0][1]);
            hy = rr * sqrt(T[1][0] * T[1][0] + T[1][1] * T[1][1]);
        }
        if (filt) {
            const double f = rc.sigma_d * rr;
            if (f > hx) hx = f;
            if (f > hy) hy = f;
        }
        double xl = ceil(c[0] - hx - 0.5), xh = floor(c[0] + hx - 0.5);
        double yl = ceil(c[1] - hy - 0.5), yh = floor(c[1] + hy - 0.5);
        if (isfinite(xl) && isfinite(xh) && isfinite(yl) && isfinite(yh)) {
            if (xl < 0) xl = 0;
            if (yl < 0) yl = 0;
            if (xh > vd.W - 1) xh = vd.W - 1;
            if (yh > vd.H - 1) yh = vd.H - 1;
            if (xl <= xh && yl <= yh) {
                ilo = (int)xl; ihi = (int)xh; jlo = (int)yl; jhi = (int)yh;
            }
        }
    }
    const int64_t slot = (int64_t)v * n + r;
    short4 tl;
    uint32_t cnt = 0;
    if (ilo <= ihi) {
        tl.x = (short)(ilo / ts); tl.y = (short)(ihi / ts);
        tl.z = (short)(jlo / ts); tl.w = (short)(jhi / ts);
        if (tmask) {
            for (int ty = tl.z; ty <= tl.w; ++ty)
                for (int tx = tl.x; tx <= tl.y; ++tx)
                    cnt += tmask[vd.tile_off + ty * vd.tiles_x + tx] != 0u;
        } else {
            cnt = (uint32_t)(tl.y - tl.x + 1) * (uint32_t)(tl.w - tl.z + 1);
        }
    } else {
        tl.x = 0; tl.y = -1; tl.z = 0; tl.w = -1;
    }
    if (valid) {
        tiles[slot] = tl;
        counts[slot] = cnt;
    }
    // record
    const float chx = (float)c[0], chy = (float)c[1];
    const uint32_t boxx = ((uint32_t)(uint16_t)ilo) | ((uint32_t)(uint16_t)ihi << 16);
    const uint32_t boxy = ((uint32_t)(uint16_t)jlo) | ((uint32_t)(uint16_t)jhi << 16);
    const float inf = __builtin_inff();
    float4 *R = srec + kRecVec4 * threadIdx.x;
    R[0] = make_float4(__uint_as_float(boxx), __uint_as_float(boxy), chx, chy);
    R[1] = make_float4((float)(c[0] - (double)chx), (float)(c[1] - (double)chy),
                       deg ? inf : 0.f, filt ? 0.f : inf);
    R[2] = make_float4((float)Q[0][0], (float)Q[0][1], (float)Q[1][0], (float)Q[1][1]);
    R[3] = make_float4((float)o, (float)((double)bz - p[2]), (float)M[2][0], (float)M[2][1]);
    const float vv = vis_rank ? vis_rank[r * nv + v] : 1.f;
    R[4] = make_float4(pd.x, pd.y, pd.z, vv);
    const double s = nsign / mn;
    R[5] = make_float4((float)(s * m[0]), (float)(s * m[1]), (float)(s * m[2]), (float)nsign);
    __syncthreads();
    const int64_t nrec = min((int64_t)blockDim.x, n - r0);
    // whole slots, so every written line is written in full
    if (sun) {
        float4 *dst = rec + ((size_t)v * (size_t)n + (size_t)r0) * kSunRecStride4;
        for (int i = threadIdx.x; i < nrec * kSunRecStride4; i += blockDim.x)
            dst[i] = srec[(i >> 2) * kRecVec4 + (i & 3)];
    } else {
        float4 *dst = rec + ((size_t)v * (size_t)n + (size_t)r0) * kRecStride4;
        for (int i = threadIdx.x; i < nrec * kRecStride4; i += blockDim.x) {
            const int k = i & 7;
            dst[i] = k < kRecVec4 ? srec[(i >> 3) * kRecVec4 + k] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
}

hipError_t launch_project(const float *sorted, int64_t n, int32_t nv, const ViewDesc *views,
                          const float *Fxy, const float *dF, const SunCam *sun,
                          const float *vis_rank, float bz, int ts, const RasterConsts &rc,
                          float *rec, short4 *tiles, uint32_t *counts, const uint32_t *tmask,
                          hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256 * nv;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_project, dim3((unsigned)blocks), dim3(256), 0, st,
                       reinterpret_cast<const float4 *>(sorted), n, nv, views, Fxy, dF, sun,
                       vis_rank, bz, ts, rc, reinterpret_cast<float4 *>(rec), tiles, counts,
                       tmask);
    return hipGetLastError();
}

// Visibility arrives per view in surfel order; the projection reads it per rank.  The
// depth order is one permutation for all views, so one pass over surfels k (coalesced
// reads of every view's vis[v][k]) writes the nv values of surfel k contiguously at its
// rank: out[rank(k) * nv + v].
__global__ void k_inverse_order(const uint32_t *__restrict__ order, int64_t n,
                                uint32_t *__restrict__ rank)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t k = order[r];
    if (k < n) rank[k] = (uint32_t)r;
}

// A block transposes a chunk of surfels through LDS (rows padded to nv + 1 floats):
// reads run along k per view, writes along v per surfel (one contiguous run each).
__global__ __launch_bounds__(256) void k_vis_to_rank(const float *__restrict__ vis, int64_t n,
                                                     int32_t nv, int chunk,
                                                     const uint32_t *__restrict__ rank,
                                                     float *__restrict__ out)
{
    extern __shared__ float sv[];
    const int64_t k0 = (int64_t)blockIdx.x * chunk;
    const int cnt = (int)min((int64_t)chunk, n - k0);
    const int row = nv + 1;
    for (int i = threadIdx.x; i < cnt * nv; i += blockDim.x) {
        const int v = i / cnt, kk = i - v * cnt;
        sv[kk * row + v] = vis[(int64_t)v * n + k0 + kk];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt * nv; i += blockDim.x) {
        const int kk = i / nv, v = i - kk * nv;
        const uint32_t r = min(rank[k0 + kk], (uint32_t)(n - 1));
        out[(int64_t)r * nv + v] = sv[kk * row + v];
    }
}

hipError_t launch_vis_to_rank(const float *vis, int64_t n, int32_t nv, const uint32_t *order,
                              uint32_t *rank, float *out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (nv <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_inverse_order, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, order,
                       n, rank);
    // chunk x (nv + 1) floats of LDS, at most 64 KB
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(64, 16384 / (nv + 1)));
    const size_t lds = (size_t)chunk * (nv + 1) * sizeof(float);
    hipLaunchKernelGGL(k_vis_to_rank, dim3((unsigned)((n + chunk - 1) / chunk)), dim3(256), lds, st,
                       vis, n, nv, chunk, rank, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------------ emit
// One thread per (rank, view): one (global tile id, rank) pair per overlapped tile at
// the scanned offset.  A block's 256 ranks own one contiguous run of the output; runs
// of up to kEmitStage pairs are assembled in LDS and written out coalesced, longer ones
// go straight to memory.  Pairs beyond the bound capacity are dropped (the scan already
// raised the overflow flag).
constexpr int kEmitThreads = 256;
constexpr int kEmitStage = 1024;

template <typename KT>
__global__ __launch_bounds__(kEmitThreads) void k_emit(
    int64_t n, const ViewDesc *__restrict__ views, const short4 *__restrict__ tiles,
    const uint32_t *__restrict__ counts, const uint32_t *__restrict__ offsets, uint64_t cap,
    KT *__restrict__ keys, uint32_t *__restrict__ vals, const uint32_t *__restrict__ tmask)
{
    constexpr bool kLocal = sizeof(KT) == 2;   // tile id within the view, else global
    __shared__ KT sk[kEmitStage];
    __shared__ uint32_t sv[kEmitStage];
    const int v = blockIdx.y;
    const int64_t r0 = (int64_t)blockIdx.x * kEmitThreads;
    const int64_t r = r0 + threadIdx.x;
    const int64_t rend = min(n, r0 + kEmitThreads);
    const uint64_t b_lo = offsets[(int64_t)v * n + r0];
    const uint64_t b_hi = max(b_lo, (uint64_t)offsets[(int64_t)v * n + rend]);
    const bool staged = b_hi - b_lo <= (uint64_t)kEmitStage;   // uniform over the block
    if (r < n) {
        // the three loads are independent: issue them together
        const int64_t slot = (int64_t)v * n + r;
        const uint32_t cnt = counts[slot];
        const short4 t = tiles[slot];
        uint64_t pos = offsets[slot];
        if (cnt != 0) {
            const ViewDesc vd = views[v];
            for (int ty = t.z; ty <= t.w; ++ty)
                for (int tx = t.x; tx <= t.y; ++tx) {
                    const uint32_t lkey = (uint32_t)(ty * vd.tiles_x + tx);
                    const uint32_t gkey = (uint32_t)vd.tile_off + lkey;
                    if (tmask && tmask[gkey] == 0u) continue;
                    const KT key = (KT)(kLocal ? lkey : gkey);
                    if (staged) {
                        const uint64_t l = pos - b_lo;
                        if (l < (uint64_t)kEmitStage) {
                            sk[l] = key;
                            sv[l] = (uint32_t)r;
                        }
                    } else if (pos < cap) {
                        keys[pos] = key;
                        vals[pos] = (uint32_t)r;
                    }
                    ++pos;
                }
        }
    }
    if (!staged) return;
    __syncthreads();
    const int cnt = (int)(b_hi - b_lo);
    for (int i = threadIdx.x; i < cnt; i += kEmitThreads) {
        const uint64_t pos = b_lo + (uint64_t)i;
        if (pos < cap) {
            keys[pos] = sk[i];
            vals[pos] = sv[i];
        }
    }
}

hipError_t launch_emit(const uint32_t *, int64_t n, int32_t nv, const ViewDesc *views,
                       const short4 *tiles, const uint32_t *counts, const uint32_t *offsets,
                       uint64_t cap, void *keys, bool keys16, uint32_t *vals,
                       const uint32_t *tmask, hipStream_t st)
{
    if (n <= 0 || cap == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + kEmitThreads - 1) / kEmitThreads), (unsigned)nv);
    if (keys16)
        hipLaunchKernelGGL(k_emit<uint16_t>, grid, dim3(kEmitThreads), 0, st, n, views, tiles, counts,
                           offsets, cap, static_cast<uint16_t *>(keys), vals, tmask);
    else
        hipLaunchKernelGGL(k_emit<uint32_t>, grid, dim3(kEmitThreads), 0, st, n, views, tiles, counts,
                           offsets, cap, static_cast<uint32_t *>(keys), vals, tmask);
    return hipGetLastError();
}

// ------------------------------------------------------------ tile dispatch order
// Block b of a raster launch runs on XCD b % 8 as that XCD's (b / 8)-th block.  XCD x
// owns the blocks b = 8 i + x, i < n_x, and xcd_tile<CHUNKED>(b) names the tile each one
// rasterizes; the order below keeps that tile set per XCD and renumbers i so that the
// heavy tiles (list length >= 2 x mean) come first.  Three passes over (x, block of
// kOrdBlock consecutive i): count heavy tiles, scan the counts per XCD, write.
constexpr int kOrdBlock = 1024;

int tile_order_blocks(int32_t ntiles)
{
    const int per_xcd = (ntiles + 7) / 8;
    return (per_xcd + kOrdBlock - 1) / kOrdBlock;
}

template <bool CHUNKED>
__device__ __forceinline__ bool heavy_tile(const uint32_t *ranges, int32_t ntiles,
                                           unsigned long long total, int x, int i, int &tile)
{
    const int b = 8 * i + x;
    if (b >= ntiles) { tile = -1; return false; }
    tile = xcd_tile<CHUNKED>(b, ntiles);
    const uint64_t len = ranges[2 * tile + 1] - ranges[2 * tile];
    // len >= 2 total / ntiles without division
    return len * (uint64_t)ntiles >= 2ull * total && len > 0;
}

template <bool CHUNKED>
__global__ __launch_bounds__(kOrdBlock) void k_order_count(const uint32_t *__restrict__ ranges,
                                                           int32_t ntiles,
                                                           const unsigned long long *__restrict__ total,
                                                           uint32_t *__restrict__ parts)
{
    __shared__ uint32_t wsum[kOrdBlock / 64];
    const int x = blockIdx.y, i = blockIdx.x * kOrdBlock + threadIdx.x;
    int tile;
    const bool h = heavy_tile<CHUNKED>(ranges, ntiles, *total, x, i, tile);
    const uint64_t bal = __ballot(h);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kOrdBlock / 64; ++w) s += wsum[w];
        parts[x * gridDim.x + blockIdx.x] = s;
    }
}

// One block per XCD: exclusive scan of its block counts in place; parts[8 nblk + x] gets
// the XCD's heavy total.
__global__ __launch_bounds__(256) void k_order_scan(uint32_t *__restrict__ parts, int nblk)
{
    __shared__ uint32_t carry;
    __shared__ uint32_t wsum[4];
    const int x = blockIdx.x;
    uint32_t *p = parts + (size_t)x * nblk;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nblk; base += 256) {
        const int k = base + threadIdx.x;
        const uint32_t v = k < nblk ? p[k] : 0u;
        // inclusive scan within the wave, then across the 4 waves
        uint32_t inc = v;
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = __shfl_up(inc, d, 64);
            if (lane >= d) inc += t;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t before = carry;
        for (int q = 0; q < w; ++q) before += wsum[q];
        if (k < nblk) p[k] = before + inc - v;
        __syncthreads();
        if (threadIdx.x == 255) carry = before + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[(size_t)8 * nblk + x] = carry;
}

template <bool CHUNKED>
__global__ __launch_bounds__(kOrdBlock) void k_order_write(const uint32_t *__restrict__ ranges,
                                                           int32_t ntiles,
                                                           const unsigned long long *__restrict__ total,
                                                           const uint32_t *__restrict__ parts,
                                                           uint32_t *__restrict__ order)
{
    __shared__ uint32_t wsum[kOrdBlock / 64];
    const int x = blockIdx.y, i = blockIdx.x * kOrdBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int tile;
    const bool h = heavy_tile<CHUNKED>(ranges, ntiles, *total, x, i, tile);
    const uint64_t bal = __ballot(h);
    if (lane == 0) wsum[w] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t before = parts[x * gridDim.x + blockIdx.x];
    for (int q = 0; q < w; ++q) before += wsum[q];
    before += (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));   // heavy tiles before i
    if (tile < 0) return;
    const uint32_t heavy_total = parts[(size_t)8 * gridDim.x + x];
    const uint32_t ni = h ? before : heavy_total + ((uint32_t)i - before);
    order[8 * (size_t)ni + x] = (uint32_t)tile;
}

hipError_t launch_tile_order(const uint32_t *ranges, int32_t ntiles,
                             const unsigned long long *total_pairs, bool chunked,
                             uint32_t *order, uint32_t *parts, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    const int nblk = tile_order_blocks(ntiles);
    const dim3 grid((unsigned)nblk, 8);
    if (chunked)
        hipLaunchKernelGGL(k_order_count<true>, grid, dim3(kOrdBlock), 0, st, ranges, ntiles, total_pairs, parts);
    else
        hipLaunchKernelGGL(k_order_count<false>, grid, dim3(kOrdBlock), 0, st, ranges, ntiles, total_pairs, parts);
    hipLaunchKernelGGL(k_order_scan, dim3(8), dim3(256), 0, st, parts, nblk);
    if (chunked)
        hipLaunchKernelGGL(k_order_write<true>, grid, dim3(kOrdBlock), 0, st, ranges, ntiles, total_pairs,
                           parts, order);
    else
        hipLaunchKernelGGL(k_order_write<false>, grid, dim3(kOrdBlock), 0, st, ranges, ntiles, total_pairs,
                           parts, order);
    return hipGetLastError();
}

// ------------------------------------------------------------ per-pair evaluation
// The same FP32 sequence runs in the forward and the backward so both take the same
// discrete decisions (skip, stop, branch).
struct PairEval {
    float dx, dy, u0, u1, G, oG, alpha;
    bool ub;
};

__device__ __forceinline__ PairEval eval_pair(const float4 r0, const float4 r1, const float4 r2,
                                              const float4 r3, float fx, float fy,
                                              const RasterConsts rc)
{
    PairEval e;
    e.dx = __fsub_rn(__fsub_rn(fx, r0.z), r1.x);
    e.dy = __fsub_rn(__fsub_rn(fy, r0.w), r1.y);
    e.u0 = __fmaf_rn(r2.y, e.dy, __fmul_rn(r2.x, e.dx));
    e.u1 = __fmaf_rn(r2.w, e.dy, __fmul_rn(r2.z, e.dx));
    const float ru = __fmaf_rn(e.u0, e.u0, __fmaf_rn(e.u1, e.u1, r1.z));
    const float rf = __fmaf_rn(__fmaf_rn(e.dx, e.dx, __fmul_rn(e.dy, e.dy)), rc.inv_s2, r1.w);
    e.ub = ru <= rf;
    const float rho = e.ub ? ru : rf;
    e.G = ex2(__fmul_rn(rho, kNegHalfLog2e));
    e.oG = __fmul_rn(r3.x, e.G);
    // min(alpha_max, oG) for oG >= 0, in one median-of-three instruction
    e.alpha = __builtin_amdgcn_fmed3f(e.oG, 0.f, rc.alpha_max);
    return e;
}

__device__ __forceinline__ bool box_hits(float bx, float by, int wx0, int wy0)
{
    const uint32_t x = __builtin_amdgcn_readfirstlane(__float_as_uint(bx));
    const uint32_t y = __builtin_amdgcn_readfirstlane(__float_as_uint(by));
    const int xlo = (int)(int16_t)(x & 0xFFFFu), xhi = (int)(int16_t)(x >> 16);
    const int ylo = (int)(int16_t)(y & 0xFFFFu), yhi = (int)(int16_t)(y >> 16);
    return xlo <= wx0 + 7 && xhi >= wx0 && ylo <= wy0 + 7 && yhi >= wy0;
}


// ------------------------------------------------------------- per-pixel coverage
// Records of a batch sit in LDS as structure of arrays by float4 group: group g of
// record j at lds4[g * B + j] (B = batch), so lanes that read different records touch
// consecutive 16-byte slots.
//
// chunk_mask: lane t holds record c0 + t of a chunk of up to 64 (valid = t < count);
// returns, for the calling lane's pixel (wx0 + lane % 8, wy0 + lane / 8), the 64-bit
// mask of chunk records whose pixel box contains that pixel.  A box is separable into a
// column range and a row range, so 8 ballots over column bits and 8 over row bits give
// the whole 64 x 64 coverage matrix; lane p keeps column mask p % 8 AND row mask p / 8.
// Outside the box alpha < alpha_min holds exactly (the box bounds both rho branches at
// the alpha_min level), so skipping those pairs changes no result.
__device__ __forceinline__ uint64_t chunk_mask(float4 head, bool valid, int wx0, int wy0,
                                               int lane)
{
    uint32_t colbits = 0, rowbits = 0;
    if (valid) {
        const uint32_t x = __float_as_uint(head.x), y = __float_as_uint(head.y);
        const int clo = max((int)(int16_t)(x & 0xFFFFu) - wx0, 0);
        const int chi = min((int)(int16_t)(x >> 16) - wx0, 7);
        const int rlo = max((int)(int16_t)(y & 0xFFFFu) - wy0, 0);
        const int rhi = min((int)(int16_t)(y >> 16) - wy0, 7);
        if (clo <= chi) colbits = (0xFFu >> (7 - chi)) & (0xFFu << clo);
        if (rlo <= rhi) rowbits = (0xFFu >> (7 - rhi)) & (0xFFu << rlo);
    }
    const int lc = lane & 7, lr = lane >> 3;
    uint64_t cm = 0, rm = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint64_t bc = __ballot((colbits >> c) & 1u);
        const uint64_t br = __ballot((rowbits >> c) & 1u);
        cm = lc == c ? bc : cm;
        rm = lr == c ? br : rm;
    }
    return cm & rm;
}

// ---------------------------------------------------------------- raster forward
// One block per tile (TS x TS threads, one pixel each); wave w owns an 8x8 sub-block.
// Records of the tile list are staged in LDS in batches (one record per thread, the
// next batch prefetched into registers).  Per chunk of 64 staged records each lane
// builds the mask of records covering its pixel and composites only those, front to
// back, until its transmittance would drop below T_min; a wave whose 64 pixels all
// stopped skips the rest, the block stops when all waves have.
template <int TS, bool DEPTH_ONLY, bool HAS_VIS, bool DIST>
__global__ __launch_bounds__(TS *TS) void k_raster_fwd(
    int32_t nv, const ViewDesc *__restrict__ views, const uint32_t *__restrict__ ranges,
    const uint32_t *__restrict__ lists, const float4 *__restrict__ rec, int64_t n,
    RasterConsts rc, const float *__restrict__ colC, const float *__restrict__ colc,
    const float *__restrict__ amb, const SunCam *__restrict__ sun, float *__restrict__ image,
    float *__restrict__ Aout, float *__restrict__ Vout, float *__restrict__ Dout,
    float *__restrict__ Nout, float *__restrict__ Tout, int32_t *__restrict__ lastout,
    unsigned long long *__restrict__ stats, unsigned long long *__restrict__ cmask,
    DistArgs da)
{
    constexpr int NT = TS * TS;
    // 8x8 view passes record, per pixel and 64-position word of the tile list, which
    // records it composited (the backward walks only those)
    constexpr bool CM = TS == 8 && !DEPTH_ONLY;
    extern __shared__ float4 lds[];
    // sun maps are equal in size and even in work: one contiguous run of tiles per XCD
    const int tile = rc.torder ? (int)rc.torder[blockIdx.x]
                               : xcd_tile<!DEPTH_ONLY>((int)blockIdx.x, (int)gridDim.x);
    const int v = find_view(views, nv, tile);
    const ViewDesc vd = views[v];
    const int lt = tile - vd.tile_off;
    const int tx = lt % vd.tiles_x, ty = lt / vd.tiles_x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    constexpr int WPR = TS / 8;
    const int wx0 = tx * TS + (wave % WPR) * 8, wy0 = ty * TS + (wave / WPR) * 8;
    const int px = wx0 + (lane & 7), py = wy0 + (lane >> 3);
    const bool inside = px < vd.W && py < vd.H;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    constexpr int RS = DEPTH_ONLY ? kSunRecStride4 : kRecStride4;   // record slot
    const float4 *recv = rec + (size_t)v * (size_t)n * RS;
    float Tr = 1.f, aD = 0.f, a0 = 0.f, a1 = 0.f, a2 = 0.f, aV = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f;
    // distortion: accumulated value, reference depth, shifted first and second moments
    float dacc = 0.f, zref = 0.f, M1 = 0.f, M2 = 0.f;
    bool has_ref = false;
    int lastpos = 0, ncontrib = 0, neval = 0;
    bool done = !inside;
    const int B = min(rc.batch, NT);
    // LDS stride between a record's float4 groups: a compile-time constant (>= every
    // batch) so that the group reads are immediate offsets from one address
    constexpr int BS = NT < 256 ? NT : 256;
    // records of the next batch in q0..q5, list entries of the one after in nidx: the
    // gather never waits for the list load it depends on
    float4 q0, q1, q2, q3, q4, q5;
    uint32_t nidx = 0;
#define SS_FETCH_FWD(IDX)                                                              \
    {                                                                                  \
        const float4 *src_ = recv + (size_t)min((IDX), (uint32_t)(n - 1)) * RS;       \
        q0 = src_[0]; q1 = src_[1]; q2 = src_[2]; q3 = src_[3];                        \
        if (!DEPTH_ONLY) { q4 = src_[4]; q5 = src_[5]; }                               \
    }
    if (start < end && tid < (int)min((uint32_t)B, end - start)) SS_FETCH_FWD(lists[start + tid]);
    if (start + B < end && tid < (int)min((uint32_t)B, end - start - B)) nidx = lists[start + B + tid];
    const size_t wbase = (size_t)(start >> 6) + (size_t)tile;   // tiles' word ranges are disjoint
    unsigned long long wacc = 0ull;
    int wcur = -1;
    for (uint32_t b0 = start; b0 < end; b0 += B) {
        const int nb = (int)min((uint32_t)B, end - b0);
        __syncthreads();
        if (tid < nb) {
            lds[tid] = q0; lds[BS + tid] = q1; lds[2 * BS + tid] = q2; lds[3 * BS + tid] = q3;
            if (!DEPTH_ONLY) { lds[4 * BS + tid] = q4; lds[5 * BS + tid] = q5; }
        }
        __syncthreads();
        const uint32_t b1 = b0 + B, b2 = b1 + B;
        if (b1 < end && tid < (int)min((uint32_t)B, end - b1)) SS_FETCH_FWD(nidx);
        if (b2 < end && tid < (int)min((uint32_t)B, end - b2)) nidx = lists[b2 + tid];
        const int pos0 = (int)(b0 - start);
        for (int c0 = 0; c0 < nb; c0 += 64) {
            if (__ballot(!done) == 0) break;
            const int cnt = min(64, nb - c0);
            const float4 head = lds[c0 + (lane < cnt ? lane : 0)];
            uint64_t m = chunk_mask(head, lane < cnt, wx0, wy0, lane);
            if (done) m = 0;
            unsigned long long cmc = 0ull;
            while (m != 0) {
                const int jc = c0 + (int)__builtin_ctzll(m);
                m &= m - 1;
                const float4 r0 = lds[jc], r1 = lds[BS + jc], r2 = lds[2 * BS + jc], r3 = lds[3 * BS + jc];
                ++neval;
                const PairEval e = eval_pair(r0, r1, r2, r3, fx, fy, rc);
                // branch-free: a skipped pair accumulates with weight 0 (w * x + a == a
                // exactly for the finite record fields), so no exec-mask juggling per pair
                const bool hit = e.alpha >= rc.alpha_min;
                const float Tn = __fmul_rn(Tr, __fsub_rn(1.f, e.alpha));
                const bool stop = hit && Tn < rc.T_min;
                const bool take = hit && !stop;
                const float w = take ? __fmul_rn(e.alpha, Tr) : 0.f;
                const float z = e.ub ? __fmaf_rn(-r3.z, e.u0, __fmaf_rn(-r3.w, e.u1, r3.y)) : r3.y;
                aD = __fmaf_rn(w, z, aD);
                if (!DEPTH_ONLY) {
                    const float4 r4 = lds[4 * BS + jc], r5 = lds[5 * BS + jc];
                    a0 = __fmaf_rn(w, r4.x, a0);
                    a1 = __fmaf_rn(w, r4.y, a1);
                    a2 = __fmaf_rn(w, r4.z, a2);
                    if (HAS_VIS) aV = __fmaf_rn(w, r4.w, aV);
                    n0 = __fmaf_rn(w, r5.x, n0);
                    n1 = __fmaf_rn(w, r5.y, n1);
                    n2 = __fmaf_rn(w, r5.z, n2);
                }
                if (DIST) {
                    // sum_{j<i} w_j (m_i - m_j)^2 = m'(m' (1 - T) - 2 M1) + M2 with m' the
                    // depth relative to the first contributor
                    zref = (take && !has_ref) ? z : zref;
                    has_ref = has_ref || take;
                    const float mp = (z - zref) * da.ds;
                    dacc = fmaf(w, fmaf(mp, fmaf(mp, 1.f - Tr, -2.f * M1), M2), dacc);
                    M1 = fmaf(w, mp, M1);
                    M2 = fmaf(w * mp, mp, M2);
                }
                if (CM) cmc |= take ? 1ull << (jc - c0) : 0ull;
                Tr = take ? Tn : Tr;
                if (!CM) {   // with contributor masks both follow from cmc once per chunk
                    lastpos = take ? pos0 + jc + 1 : lastpos;
                    ncontrib += take ? 1 : 0;
                }
                done = done || stop;
                m = stop ? 0ull : m;
            }
            if (CM && cmc != 0ull) {
                lastpos = pos0 + c0 + 64 - (int)__builtin_clzll(cmc);
                ncontrib += (int)__popcll(cmc);
            }
            if (CM && cmask) {
                // chunk positions [P0, P0 + cnt) fall in word P0 / 64 and, when the batch
                // depth does not divide 64, also in the next word
                const int P0 = pos0 + c0, w = P0 >> 6, sh = P0 & 63;
                if (w != wcur) {
                    if (wcur >= 0) cmask[(wbase + wcur) * 64 + tid] = wacc;
                    wacc = 0ull;
                    wcur = w;
                }
                wacc |= cmc << sh;
                if (sh + cnt > 64) {
                    cmask[(wbase + wcur) * 64 + tid] = wacc;
                    wacc = cmc >> (64 - sh);
                    wcur = w + 1;
                }
            }
        }
        if (!__syncthreads_or(!done)) break;
    }
    if (CM && cmask && wcur >= 0) cmask[(wbase + wcur) * 64 + tid] = wacc;
#undef SS_FETCH_FWD
    {
        // work counters: one 64-bit atomic per wave and counter, into the tile's slot
        unsigned long long c = (unsigned long long)ncontrib, e = (unsigned long long)neval;
        for (int d = 32; d > 0; d >>= 1) {
            c += __shfl_xor(c, d, 64);
            e += __shfl_xor(e, d, 64);
        }
        if (lane == 0) {
            unsigned long long *slot = stats + (size_t)(tile % kStatSlots) * kStatStride;
            atomicAdd(slot, c);
            atomicAdd(slot + 1, e);
        }
    }
    if (!inside) return;
    const int64_t P = (int64_t)vd.W * vd.H;
    const int64_t local = (int64_t)py * vd.W + px;
    const int64_t g = vd.pix_off + local;
    if (DEPTH_ONLY) {
        Dout[g] = (float)((double)aD + (double)Tr * sun[v].zfar);
        return;
    }
    float C[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, cb[3] = {0, 0, 0}, La[3] = {0, 0, 0};
    if (colC) for (int k = 0; k < 9; ++k) C[k] = colC[9 * v + k];
    if (colc) for (int k = 0; k < 3; ++k) cb[k] = colc[3 * v + k];
    if (amb) for (int k = 0; k < 3; ++k) La[k] = amb[3 * v + k];
    const float Vp = HAS_VIS ? aV : 1.f;
    const float A[3] = {a0, a1, a2};
    const int64_t b3 = 3 * vd.pix_off + local;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float ca = C[3 * ch] * A[0] + C[3 * ch + 1] * A[1] + C[3 * ch + 2] * A[2] + cb[ch];
        image[b3 + ch * P] = ca * (Vp + (1.f - Vp) * La[ch]);
        Aout[b3 + ch * P] = A[ch];
    }
    Nout[b3] = n0; Nout[b3 + P] = n1; Nout[b3 + 2 * P] = n2;
    Vout[g] = Vp;
    Dout[g] = aD;
    Tout[g] = Tr;
    lastout[g] = lastpos;
    if (DIST) {
        da.dist[g] = dacc;
        da.aux[g] = zref;
        da.aux[da.P + g] = M1;
        da.aux[2 * da.P + g] = M2;
    }
}

template <int TS, bool DO, bool HV>
static void launch_fwd_t(dim3 grid, size_t lds, hipStream_t st, int32_t nv,
                         const ViewDesc *views, const uint32_t *ranges, const uint32_t *lists,
                         const float *rec, int64_t n, const RasterConsts &rc,
                         const float *colC, const float *colc, const float *amb,
                         const SunCam *sun, float *image, float *A, float *V, float *D,
                         float *N, float *T, int32_t *last, unsigned long long *stats,
                         unsigned long long *cmask, const DistArgs *dist)
{
    const DistArgs da = dist ? *dist : DistArgs{0.f, nullptr, nullptr, nullptr, 0};
    if (!DO && dist)
        hipLaunchKernelGGL((k_raster_fwd<TS, DO, HV, true>), grid, dim3(TS * TS), lds, st, nv,
                           views, ranges, lists, reinterpret_cast<const float4 *>(rec), n, rc,
                           colC, colc, amb, sun, image, A, V, D, N, T, last, stats, cmask, da);
    else
        hipLaunchKernelGGL((k_raster_fwd<TS, DO, HV, false>), grid, dim3(TS * TS), lds, st, nv,
                           views, ranges, lists, reinterpret_cast<const float4 *>(rec), n, rc,
                           colC, colc, amb, sun, image, A, V, D, N, T, last, stats, cmask, da);
}

size_t cmask_words(int64_t pair_cap, int32_t tiles)
{
    return ((size_t)(pair_cap > 0 ? pair_cap : 0) / 64 + (size_t)(tiles > 0 ? tiles : 0) + 1) * 64;
}

hipError_t launch_raster_fwd(int ts, bool depth_only, bool has_vis, int32_t total_tiles,
                             int32_t nv, const ViewDesc *views, const uint32_t *ranges,
                             const uint32_t *lists, const float *rec, int64_t n,
                             const RasterConsts &rc, const float *colC, const float *colc,
                             const float *amb, const SunCam *sun, float *image, float *A,
                             float *V, float *D, float *N, float *T, int32_t *last,
                             unsigned long long *stats, unsigned long long *cmask, hipStream_t st,
                             const DistArgs *dist)
{
    if (total_tiles <= 0) return hipSuccess;
    const dim3 grid((unsigned)total_tiles);
    // records staged at a fixed stride of min(ts^2, 256) float4 per field group; the
    // depth-only pass stages the first 4 of a record's 6 groups
    const size_t lds = (size_t)min(ts * ts, 256) * (depth_only ? 4 : kRecVec4) * sizeof(float4);
#define SS_FWD(TS_)                                                                              \
    if (ts == TS_) {                                                                             \
        if (depth_only)                                                                          \
            launch_fwd_t<TS_, true, false>(grid, lds, st, nv, views, ranges, lists, rec, n, rc,   \
                                           colC, colc, amb, sun, image, A, V, D, N, T, last, stats, cmask, dist);\
        else if (has_vis)                                                                        \
            launch_fwd_t<TS_, false, true>(grid, lds, st, nv, views, ranges, lists, rec, n, rc,   \
                                           colC, colc, amb, sun, image, A, V, D, N, T, last, stats, cmask, dist);\
        else                                                                                     \
            launch_fwd_t<TS_, false, false>(grid, lds, st, nv, views, ranges, lists, rec, n, rc,  \
                                            colC, colc, amb, sun, image, A, V, D, N, T, last, stats, cmask, dist);\
    }
    SS_FWD(8) else SS_FWD(16) else SS_FWD(32) else return hipErrorInvalidValue;
#undef SS_FWD
    return hipGetLastError();
}

// ------------------------------------------------------- wave transpose reduction
// 16 per-lane values -> lane l holds the wave sum of value (l >> 2) & 15 (lanes with
// l % 4 == 0 then hold all 16 sums).  Each level halves the vector a lane carries: the
// two cross-row levels use gfx950's lane swaps (permlane32 / permlane16: one VALU op
// exchanges half of two registers between the partner rows, then one add), the two
// in-row levels use DPP row mirrors, the last two are full DPP quad sums.  No LDS.
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __builtin_amdgcn_update_dpp(0.f, v, CTRL, 0xF, 0xF, true);
}

__device__ __forceinline__ void swap_rows32(float &a, float &b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}

__device__ __forceinline__ void swap_rows16(float &a, float &b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}

__device__ __forceinline__ float wave_transpose_reduce16(float (&x)[16], int lane)
{
    float y8[8], y4[4], y2[2];
#pragma unroll
    for (int k = 0; k < 8; ++k) {           // lanes 0-31 keep value k, 32-63 value k + 8
        float a = x[k], b = x[k + 8];
        swap_rows32(a, b);
        y8[k] = a + b;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {           // even rows keep k, odd rows k + 4
        float a = y8[k], b = y8[k + 4];
        swap_rows16(a, b);
        y4[k] = a + b;
    }
    const bool b3 = lane & 8, b2 = lane & 4;
#pragma unroll
    for (int k = 0; k < 2; ++k) {           // row mirror: partner 15 - i differs in bit 3
        const float keep = b3 ? y4[k + 2] : y4[k];
        const float send = b3 ? y4[k] : y4[k + 2];
        y2[k] = keep + dpp<0x140>(send);
    }
    // half-row mirror: partner 7 - i differs in bit 2
    float y = (b2 ? y2[1] : y2[0]) + dpp<0x141>(b2 ? y2[0] : y2[1]);
    y += dpp<0x4E>(y);                      // quad_perm [2,3,0,1]
    y += dpp<0xB1>(y);                      // quad_perm [1,0,3,2]
    return y;
}

// Within one 16-lane row: 16 per-lane values -> lane i holds the row sum of value i.
// Four levels, each pairing lanes that differ in one index bit (row mirror: bit 3,
// half-row mirror: bit 2, quad permutes: bits 1 and 0); every level keeps the half of
// the vector selected by that bit and adds the partner's copy of it.  The two halves of
// the first two levels are whole 4-lane DPP banks (bank b = lanes 4b..4b+3 of a row), so
// each kept value is one DPP add per half written under a bank mask; the compiler does
// not see into the asm, so each block waits out the VALU-write -> DPP-read hazard itself.
__device__ __forceinline__ float row_transpose_reduce16(const float (&x)[16], int lane)
{
    const bool b1 = lane & 2, b0 = lane & 1;
    float y8[8], y4[4], y2[2];
    // lanes 0-7 (banks 0, 1) keep values 0-7, lanes 8-15 (banks 2, 3) values 8-15; y8[k]
    // starts as x[k + 8] and is overwritten in place (an instruction reads its sources
    // before it writes)
#pragma unroll
    for (int k = 0; k < 8; ++k) y8[k] = x[k + 8];
    asm("s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_mirror row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %0, %8, %8 row_mirror row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %1, %1, %1 row_mirror row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %1, %9, %9 row_mirror row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %2, %2, %2 row_mirror row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %2, %10, %10 row_mirror row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %3, %3, %3 row_mirror row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %3, %11, %11 row_mirror row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %4, %4, %4 row_mirror row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %4, %12, %12 row_mirror row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %5, %5, %5 row_mirror row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %5, %13, %13 row_mirror row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %6, %6, %6 row_mirror row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %6, %14, %14 row_mirror row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %7, %7, %7 row_mirror row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %7, %15, %15 row_mirror row_mask:0xf bank_mask:0x3\n\t"
        : "+v"(y8[0]), "+v"(y8[1]), "+v"(y8[2]), "+v"(y8[3]), "+v"(y8[4]), "+v"(y8[5]),
          "+v"(y8[6]), "+v"(y8[7])
        : "v"(x[0]), "v"(x[1]), "v"(x[2]), "v"(x[3]), "v"(x[4]), "v"(x[5]), "v"(x[6]), "v"(x[7]));
    // lanes with bit 2 clear (banks 0, 2) keep values 0-3, the others 4-7
#pragma unroll
    for (int k = 0; k < 4; ++k) y4[k] = y8[k + 4];
    asm("s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xa\n\t"
        "v_add_f32_dpp %0, %4, %4 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
        "v_add_f32_dpp %1, %1, %1 row_half_mirror row_mask:0xf bank_mask:0xa\n\t"
        "v_add_f32_dpp %1, %5, %5 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
        "v_add_f32_dpp %2, %2, %2 row_half_mirror row_mask:0xf bank_mask:0xa\n\t"
        "v_add_f32_dpp %2, %6, %6 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
        "v_add_f32_dpp %3, %3, %3 row_half_mirror row_mask:0xf bank_mask:0xa\n\t"
        "v_add_f32_dpp %3, %7, %7 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
        "s_nop 1"
        : "+v"(y4[0]), "+v"(y4[1]), "+v"(y4[2]), "+v"(y4[3])
        : "v"(y8[0]), "v"(y8[1]), "v"(y8[2]), "v"(y8[3]));
#pragma unroll
    for (int k = 0; k < 2; ++k)
        y2[k] = (b1 ? y4[k + 2] : y4[k]) + dpp<0x4E>(b1 ? y4[k] : y4[k + 2]);
    return (b0 ? y2[1] : y2[0]) + dpp<0xB1>(b0 ? y2[0] : y2[1]);
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

// OR of a 64-bit mask over the 16 lanes of a row (same four partner patterns).
__device__ __forceinline__ uint64_t row_or64(uint64_t v)
{
    int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
    lo |= dpp_i<0x140>(lo); hi |= dpp_i<0x140>(hi);
    lo |= dpp_i<0x141>(lo); hi |= dpp_i<0x141>(hi);
    lo |= dpp_i<0x4E>(lo); hi |= dpp_i<0x4E>(hi);
    lo |= dpp_i<0xB1>(lo); hi |= dpp_i<0xB1>(hi);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Maximum over the 16 lanes of a row (same four partner patterns).
__device__ __forceinline__ int row_max(int v)
{
    v = max(v, dpp_i<0x140>(v));
    v = max(v, dpp_i<0x141>(v));
    v = max(v, dpp_i<0x4E>(v));
    v = max(v, dpp_i<0xB1>(v));
    return v;
}

// Per-pixel adjoints of Eq. image_formation: the upstream colour gradient through the
// colour transform and shading gives the gradients of the composited albedo (gA), of
// the composited visibility (gV), and the pixel's 15 per-view colour-parameter terms
// (cg[0..8] = dC, cg[9..11] = dc, cg[12..14] = dL_a, cg[15] = 0).
struct PixelAdjoint {
    float gA0, gA1, gA2, gV, gD, gN0, gN1, gN2, Tr;
    int last;
};

// Distortion state of a pixel in the backward: upstream gradient, reference depth, total
// weight 1 - T_final, shifted moments sum w m', sum w m'^2 over all its contributors.
struct DistPixel {
    float gDist, zref, At, M1, M2;
};

template <bool HAS_VIS>
__device__ __forceinline__ PixelAdjoint pixel_adjoint(
    bool inside, int v, int64_t g, int64_t b3, int64_t P, const float *__restrict__ colC,
    const float *__restrict__ colc, const float *__restrict__ amb, const float *__restrict__ Ain,
    const float *__restrict__ Vin, const float *__restrict__ Tin,
    const int32_t *__restrict__ lastin, const float *__restrict__ dI,
    const float *__restrict__ dD, const float *__restrict__ dN, float (&cg)[16])
{
    PixelAdjoint a{0, 0, 0, 0, 0, 0, 0, 0, 1.f, 0};
#pragma unroll
    for (int k = 0; k < 16; ++k) cg[k] = 0.f;
    if (!inside) return a;
    float C[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, cb[3] = {0, 0, 0}, La[3] = {0, 0, 0};
    if (colC) for (int k = 0; k < 9; ++k) C[k] = colC[9 * v + k];
    if (colc) for (int k = 0; k < 3; ++k) cb[k] = colc[3 * v + k];
    if (amb) for (int k = 0; k < 3; ++k) La[k] = amb[3 * v + k];
    const float A[3] = {Ain[b3], Ain[b3 + P], Ain[b3 + 2 * P]};
    const float Vp = HAS_VIS ? Vin[g] : 1.f;
    float gI[3] = {0, 0, 0};
    if (dI) { gI[0] = dI[b3]; gI[1] = dI[b3 + P]; gI[2] = dI[b3 + 2 * P]; }
    float gs[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float ca = C[3 * ch] * A[0] + C[3 * ch + 1] * A[1] + C[3 * ch + 2] * A[2] + cb[ch];
        const float shade = HAS_VIS ? Vp + (1.f - Vp) * La[ch] : 1.f;
        gs[ch] = gI[ch] * shade;
        if (HAS_VIS) {
            a.gV += gI[ch] * ca * (1.f - La[ch]);
            cg[12 + ch] = gI[ch] * ca * (1.f - Vp);
        }
        cg[9 + ch] = gs[ch];
#pragma unroll
        for (int q = 0; q < 3; ++q) cg[3 * ch + q] = gs[ch] * A[q];
    }
    a.gA0 = C[0] * gs[0] + C[3] * gs[1] + C[6] * gs[2];
    a.gA1 = C[1] * gs[0] + C[4] * gs[1] + C[7] * gs[2];
    a.gA2 = C[2] * gs[0] + C[5] * gs[1] + C[8] * gs[2];
    if (dD) a.gD = dD[g];
    if (dN) { a.gN0 = dN[b3]; a.gN1 = dN[b3 + P]; a.gN2 = dN[b3 + 2 * P]; }
    a.Tr = Tin[g];
    a.last = lastin[g];
    return a;
}

__device__ __forceinline__ DistPixel pixel_distortion_state(bool inside, int64_t g, float Tr,
                                                            const DistArgs &da)
{
    DistPixel d{0, 0, 0, 0, 0};
    if (!inside) return d;
    d.gDist = da.d_dist ? da.d_dist[g] : 0.f;
    d.zref = da.aux[g];
    d.M1 = da.aux[da.P + g];
    d.M2 = da.aux[2 * da.P + g];
    d.At = 1.f - Tr;
    return d;
}

// Per-pair terms of the walk: 1 / (1 - alpha), the pair's depth z (the centre depth on
// the low-pass branch), g . f (the upstream gradient dotted with the pair's composited
// features, plus the distortion's d dist / d w term) and the depth gradient per unit
// weight; u zeroed on the low-pass branch.
struct PairTerms {
    float rom, z, gf, gDe, u0, u1;
};

template <bool DIST>
__device__ __forceinline__ PairTerms pair_terms(const PairEval &e, float4 r3, float4 r4, float4 r5,
                                                const PixelAdjoint &pa, const DistPixel &dp,
                                                bool has_vis, float ds)
{
    PairTerms t;
    t.rom = __builtin_amdgcn_rcpf(1.f - e.alpha);
    t.u0 = e.ub ? e.u0 : 0.f;
    t.u1 = e.ub ? e.u1 : 0.f;
    t.z = __fmaf_rn(-r3.z, t.u0, __fmaf_rn(-r3.w, t.u1, r3.y));
    float gf = fmaf(pa.gA0, r4.x, fmaf(pa.gA1, r4.y, fmaf(pa.gA2, r4.z, fmaf(pa.gD, t.z,
               fmaf(pa.gN0, r5.x, fmaf(pa.gN1, r5.y, pa.gN2 * r5.z))))));
    if (has_vis) gf = fmaf(pa.gV, r4.w, gf);
    float gDe = pa.gD;
    if (DIST) {
        // d dist / d w_k = sum_j w_j (m'_k - m'_j)^2, d dist / d m_k = 2 w_k sum_j w_j (m'_k - m'_j)
        const float mp = (t.z - dp.zref) * ds;
        gf = fmaf(dp.gDist, fmaf(mp, fmaf(mp, dp.At, -2.f * dp.M1), dp.M2), gf);
        gDe = fmaf(2.f * dp.gDist * ds, fmaf(mp, dp.At, -dp.M1), pa.gD);
    }
    t.gf = gf;
    t.gDe = gDe;
    return t;
}

// The 16 record-gradient values of one pair from its weight w, dL/dalpha and dL/dz.
// The pair's branch enters once, through u (zero on the low-pass branch): the k, Q and
// u-centre terms vanish by multiplication, and the low-pass term of the centre gradient
// is zeroed on the u branch.  With rho2 = -oG dal (unclamped),
//   dL/dc = -(Q^T dL/du + delta rho2 / sigma^2 [low-pass branch]).
__device__ __forceinline__ void pair_record_grads(const PairEval &e, float w, float dal, float dz,
                                                  float u0, float u1, float4 r2, float4 r3,
                                                  const PixelAdjoint &pa, float inv_s2,
                                                  float alpha_max, float (&gr)[16])
{
    const float dzu = e.ub ? dz : 0.f;
    gr[G_AR] = w * pa.gA0; gr[G_AG] = w * pa.gA1; gr[G_AB] = w * pa.gA2;
    gr[G_NX] = w * pa.gN0; gr[G_NY] = w * pa.gN1; gr[G_NZ] = w * pa.gN2;
    gr[G_Z0] = dz;
    const float gd = e.oG < alpha_max ? dal : 0.f;       // zero where alpha is clamped
    gr[G_O] = e.G * gd;
    const float rho2 = -(e.oG * gd);
    const float du0 = fmaf(u0, rho2, -r3.z * dzu);
    const float du1 = fmaf(u1, rho2, -r3.w * dzu);
    gr[G_KU] = -u0 * dz;
    gr[G_KV] = -u1 * dz;
    gr[G_Q00] = du0 * e.dx;
    gr[G_Q01] = du0 * e.dy;
    gr[G_Q10] = du1 * e.dx;
    gr[G_Q11] = du1 * e.dy;
    const float nfd = e.ub ? 0.f : -(inv_s2 * rho2);
    gr[G_CX] = fmaf(-r2.x, du0, fmaf(-r2.z, du1, e.dx * nfd));
    gr[G_CY] = fmaf(-r2.y, du0, fmaf(-r2.w, du1, e.dy * nfd));
}

// Gradients of one (record, pixel) pair in the sequential back-to-front walk.  Updates
// the pixel's transmittance Tr and suffix gS when the pair contributes, returns the 16
// record gradient values in gr (zero when it does not).
template <bool DIST>
__device__ __forceinline__ void pair_gradients(const PairEval &e, bool contrib, float4 r2,
                                               float4 r3, float4 r4, float4 r5,
                                               const PixelAdjoint &pa, const DistPixel &dp,
                                               bool has_vis, float inv_s2, float alpha_max,
                                               float ds, float &Tr, float &gS, float (&gr)[16])
{
    const PairTerms t = pair_terms<DIST>(e, r3, r4, r5, pa, dp, has_vis, ds);
    const float Tb = Tr * t.rom;
    const float w = contrib ? e.alpha * Tb : 0.f;
    const float dal = contrib ? fmaf(Tb, t.gf, -gS * t.rom) : 0.f;
    gS = fmaf(w, t.gf, gS);
    Tr = contrib ? Tb : Tr;
    pair_record_grads(e, w, dal, w * t.gDe, t.u0, t.u1, r2, r3, pa, inv_s2, alpha_max, gr);
}

// --------------------------------------------------------------- raster backward
// Back to front over each pixel's contributors [0, last): transmittance before a
// surfel is recovered as T_i = T_{i+1} / (1 - alpha_i) from T_final, the suffix
// g . sum_{j>i} w_j f_j is accumulated on the way, and per pair
//   dL/dalpha_i = T_i (g . f_i) - (g . S_i) / (1 - alpha_i)           (Eq. rasterization)
// then through alpha = min(alpha_max, o G), G = exp(-rho/2), rho = |Q delta|^2 or
// |delta|^2 / sigma^2, delta = x - c, z = z0 - k . u.  Each 16-lane row of a wave owns a
// 4x4 quadrant of the wave's 8x8 pixels and walks, back to front, the staged records
// whose box meets the quadrant (4 ballots per chunk of 64).  A lane takes part in a pair
// only where the forward composited it - the forward's box and FP32 alpha tests and the
// pixel's `last` - so the walk revisits exactly the forward's pairs.  (8x8 tiles with
// the forward's contributor masks use the record-parallel kernel below.)
// The 16 record-gradient values are reduced within the row and added with one atomic per
// lane, so one instruction carries the sums of up to four records.
// The colour adjoint of Eq. image_formation runs first per pixel; its 15 per-view
// sums are reduced per tile into colour_partials.
template <int TS, bool HAS_VIS, bool DIST>
__global__ __launch_bounds__(TS *TS) __attribute__((amdgpu_waves_per_eu(TS == 8 ? 5 : 4))) void k_raster_bwd(
    int32_t nv, const ViewDesc *__restrict__ views, const uint32_t *__restrict__ ranges,
    const uint32_t *__restrict__ lists, const float4 *__restrict__ rec, int64_t n,
    RasterConsts rc, const float *__restrict__ colC, const float *__restrict__ colc,
    const float *__restrict__ amb, const float *__restrict__ Ain,
    const float *__restrict__ Vin, const float *__restrict__ Tin,
    const int32_t *__restrict__ lastin, const float *__restrict__ dI,
    const float *__restrict__ dD, const float *__restrict__ dN, float *__restrict__ recgrad,
    float *__restrict__ colour_partials, DistArgs da)
{
    constexpr int NT = TS * TS;
    constexpr int NW = NT / 64;
    // LDS: the staged batch (at offset 0, so a record's address is one multiply), its
    // ranks, the waves' colour sums, the tile's largest `last`
    extern __shared__ float4 lds[];
    uint32_t *lds_idx = reinterpret_cast<uint32_t *>(lds + min(rc.batch, NT) * kRecVec4);
    float(*red)[16] = reinterpret_cast<float(*)[16]>(lds_idx + min(rc.batch, NT));
    int &max_last = *reinterpret_cast<int *>(red + NW);
    const int tile = rc.torder ? (int)rc.torder[blockIdx.x] : xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int v = find_view(views, nv, tile);
    const ViewDesc vd = views[v];
    const int lt = tile - vd.tile_off;
    const int tx = lt % vd.tiles_x, ty = lt / vd.tiles_x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    constexpr int WPR = TS / 8;
    const int wx0 = tx * TS + (wave % WPR) * 8, wy0 = ty * TS + (wave / WPR) * 8;
    // 16-lane row `quad` owns the 4x4 quadrant (quad & 1, quad >> 1) of the wave's block
    const int quad = lane >> 4;
    const int px = wx0 + 4 * (quad & 1) + (lane & 3), py = wy0 + 4 * (quad >> 1) + ((lane >> 2) & 3);
    const bool inside = px < vd.W && py < vd.H;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const int64_t P = (int64_t)vd.W * vd.H;
    const int64_t local = (int64_t)py * vd.W + px;
    const int64_t g = vd.pix_off + local;
    const int64_t b3 = 3 * vd.pix_off + local;
    if (tid == 0) max_last = 0;

    // colour adjoint (Eq. image_formation)
    float cg[16];
    const PixelAdjoint pa = pixel_adjoint<HAS_VIS>(inside, v, g, b3, P, colC, colc, amb, Ain, Vin,
                                                   Tin, lastin, dI, dD, dN, cg);
    const DistPixel dp = DIST ? pixel_distortion_state(inside, g, pa.Tr, da) : DistPixel{0, 0, 0, 0, 0};
    float Tr = pa.Tr;
    const int mylast = pa.last;
    {
        const float s = wave_transpose_reduce16(cg, lane);
        if ((lane & 3) == 0) red[wave][lane >> 2] = s;
    }
    __syncthreads();
    if (tid < 16) {
        float s = 0.f;
        for (int w = 0; w < NW; ++w) s += red[w][tid];
        colour_partials[(int64_t)tile * 16 + tid] = s;
    }
    if (mylast > 0) atomicMax(&max_last, mylast);
    __syncthreads();

    const uint32_t start = ranges[2 * tile];
    const int tile_len = (int)(ranges[2 * tile + 1] - start);
    const float4 *recv = rec + (size_t)v * (size_t)n * kRecStride4;
    float *gv = recgrad + (size_t)v * (size_t)n * kGradFloats;
    float gS = 0.f;
    const int batch = min(rc.batch, NT);
    const float inv_s2 = rc.two_inv_s2 * 0.5f;
    const int blk_last = min(max_last, tile_len);   // a stale `last` cannot read past the list
    // the row walks records up to the largest `last` among its 16 pixels
    const int row_last = row_max(mylast);
    // one record per thread; the batch before the current one (back to front) is
    // fetched into registers while the current one is processed
    float4 q0, q1, q2, q3, q4, q5;
    uint32_t qidx = 0;
#define SS_FETCH_BWD(BB, CNT)                                                          \
    if (tid < (CNT)) {                                                                 \
        qidx = min(lists[start + (BB) + tid], (uint32_t)(n - 1));                      \
        const float4 *src_ = recv + (size_t)qidx * kRecStride4;                           \
        q0 = src_[0]; q1 = src_[1]; q2 = src_[2]; q3 = src_[3]; q4 = src_[4]; q5 = src_[5]; \
    }
    // batches on the forward's grid ([k * batch, (k + 1) * batch) from the list start),
    // back to front; the first one is cut at the tile's largest `last`
    const int nbat = (blk_last + batch - 1) / batch;
    if (nbat > 0) {
        const int bb0 = (nbat - 1) * batch;
        SS_FETCH_BWD(bb0, blk_last - bb0);
    }
    for (int kb = nbat - 1; kb >= 0; --kb) {
        const int bb = kb * batch;
        const int nb = min(bb + batch, blk_last) - bb;
        __syncthreads();
        if (tid < nb) {
            float4 *dst = lds + tid * kRecVec4;
            dst[0] = q0; dst[1] = q1; dst[2] = q2; dst[3] = q3; dst[4] = q4; dst[5] = q5;
            lds_idx[tid] = qidx;
        }
        __syncthreads();
        if (kb > 0) SS_FETCH_BWD(bb - batch, batch);
        for (int c0 = ((nb - 1) >> 6) << 6; c0 >= 0; c0 -= 64) {
            const int cnt = min(64, nb - c0);
            uint64_t m = 0;
            // lane t tests chunk record c0 + t against the wave's four 4x4 quadrants
            uint32_t qbits = 0;
            if (lane < cnt) {
                const float4 h = lds[(c0 + lane) * kRecVec4];
                const uint32_t x = __float_as_uint(h.x), y = __float_as_uint(h.y);
                const int xlo = (int)(int16_t)(x & 0xFFFFu), xhi = (int)(int16_t)(x >> 16);
                const int ylo = (int)(int16_t)(y & 0xFFFFu), yhi = (int)(int16_t)(y >> 16);
                const bool c0h = xlo <= wx0 + 3 && xhi >= wx0, c1h = xlo <= wx0 + 7 && xhi >= wx0 + 4;
                const bool r0h = ylo <= wy0 + 3 && yhi >= wy0, r1h = ylo <= wy0 + 7 && yhi >= wy0 + 4;
                qbits = (uint32_t)(c0h && r0h) | ((uint32_t)(c1h && r0h) << 1) |
                        ((uint32_t)(c0h && r1h) << 2) | ((uint32_t)(c1h && r1h) << 3);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint64_t bq = __ballot((qbits >> q) & 1u);
                m = quad == q ? bq : m;
            }
            const int lim = row_last - (bb + c0);        // chunk records j < lim can contribute
            m &= lim >= 64 ? ~0ull : (lim <= 0 ? 0ull : ((1ull << lim) - 1ull));
            // row-uniform walk, highest position first
            if (__ballot(m != 0) != 0) do {
                const bool act = m != 0;
                const int jl = act ? 63 - (int)__builtin_clzll(m) : 0;
                const int j = c0 + jl;
                if (act) m &= ~(1ull << jl);
                const float4 *R = lds + __mul24(j, kRecVec4);   // j < 256: 24-bit multiply
                const float4 r0 = R[0], r1 = R[1], r2 = R[2], r3 = R[3], r4 = R[4], r5 = R[5];
                // branch-free: every lane evaluates the row's record; lanes that do not
                // contribute (outside [0, last) or alpha < alpha_min) get zero gradients
                // and leave T and the suffix unchanged
                const PairEval e = eval_pair(r0, r1, r2, r3, fx, fy, rc);
                // the forward's own decision for this pair: the same FP32 alpha test inside
                // the pixel's FP64 box (the forward never evaluates a pair outside it)
                const uint32_t bx = __float_as_uint(r0.x), by = __float_as_uint(r0.y);
                const int xlo = (int)(int16_t)(bx & 0xFFFFu), xhi = (int)(int16_t)(bx >> 16);
                const int ylo = (int)(int16_t)(by & 0xFFFFu), yhi = (int)(int16_t)(by >> 16);
                const bool contrib = act && bb + j < mylast && px >= xlo && px <= xhi && py >= ylo &&
                                     py <= yhi && e.alpha >= rc.alpha_min;
                // a step where no lane of the wave contributes changes nothing (a branch
                // around the rest, and the loop test at the bottom, keep a single back edge:
                // no register copies per step)
                const uint64_t cb = __ballot(contrib);
                if (cb != 0) {
                    float gr[16];
                    pair_gradients<DIST>(e, contrib, r2, r3, r4, r5, pa, dp, HAS_VIS, inv_s2,
                                         rc.alpha_max, da.ds, Tr, gS, gr);
                    const float sum = row_transpose_reduce16(gr, lane);
                    // lane i of a row holds value i of its record's 16-lane sum
                    if (((cb >> (quad * 16)) & 0xFFFFull) != 0)
                        atomicAdd(gv + (size_t)lds_idx[j] * kGradFloats + (lane & 15), sum);
                }
            } while (__ballot(m != 0) != 0);
        }
    }
#undef SS_FETCH_BWD
}

// ------------------------------------------------- raster backward, 8x8 tiles
// Record-parallel rows.  With the forward's contributor masks the four 4x4 quadrants of
// an 8x8 tile are walked one after another, and all four 16-lane rows of the wave work
// on the *same* quadrant: lane i of every row holds pixel i of the quadrant, and each
// step takes the next four records of the quadrant's walk (the union of its 16 pixels'
// masks, back to front), one per row.  The pixel recursion of Eq. rasterization runs
// across the rows: with rom = 1 / (1 - alpha) for a contributing pair (1 otherwise) and
// x = w (g . f), row r needs T before its record = T_cur * prod_{k <= r} rom_k and the
// suffix g . S = gS_cur + sum_{k < r} x_k; both are scans over the four rows, done
// lane-wise with two lane swaps each (rows 0<->1, 2<->3, then 0,1<->2,3), which also
// give the totals that advance T_cur and gS_cur.  A step costs ~10 % more VALU than the
// quadrant-per-row walk but the walk takes sum_q |U_q| / 4 steps instead of
// sum over chunks of max_q |U_q|, a third fewer on the 2M-surfel views.  Per-pixel state
// (the adjoint inputs, T, the suffix, the distortion totals) lives in LDS between
// quadrants.
constexpr int kPstBase = 10, kPstDist = 5;

__device__ __forceinline__ float swap16_lo_hi(float v, float &hi)
{
    // rows [v0, v1, v2, v3] -> lo = [v0, v0, v2, v2], hi = [v1, v1, v3, v3]
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    hi = __uint_as_float(r[1]);
    return __uint_as_float(r[0]);
}

__device__ __forceinline__ float swap32_lo_hi(float v, float &hi)
{
    // rows [v0, v1, v2, v3] -> lo = [v0, v1, v0, v1], hi = [v2, v3, v2, v3]
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    hi = __uint_as_float(r[1]);
    return __uint_as_float(r[0]);
}

// Inclusive product over rows 0..r (per lane position), and the product of all four.
__device__ __forceinline__ float rows_prefix_mul(float f, bool odd, bool upper, float &total)
{
    float b;
    const float a = swap16_lo_hi(f, b);
    const float pair = a * b;                       // f0 f1 in rows 0, 1; f2 f3 in rows 2, 3
    const float p1 = odd ? pair : a;
    float d;
    const float c = swap32_lo_hi(pair, d);          // c = f0 f1, d = f2 f3 in every row
    total = c * d;
    return upper ? p1 * c : p1;
}

// Inclusive sum over rows 0..r, and the sum of all four.
__device__ __forceinline__ float rows_prefix_add(float x, bool odd, bool upper, float &total)
{
    float b;
    const float a = swap16_lo_hi(x, b);
    const float pair = a + b;
    const float p1 = odd ? pair : a;
    float d;
    const float c = swap32_lo_hi(pair, d);
    total = c + d;
    return upper ? p1 + c : p1;
}

template <bool HAS_VIS, bool DIST>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_raster_bwd_rp(
    int32_t nv, const ViewDesc *__restrict__ views, const uint32_t *__restrict__ ranges,
    const uint32_t *__restrict__ lists, const float4 *__restrict__ rec, int64_t n,
    RasterConsts rc, const float *__restrict__ colC, const float *__restrict__ colc,
    const float *__restrict__ amb, const float *__restrict__ Ain,
    const float *__restrict__ Vin, const float *__restrict__ Tin,
    const int32_t *__restrict__ lastin, const float *__restrict__ dI,
    const float *__restrict__ dD, const float *__restrict__ dN, float *__restrict__ recgrad,
    float *__restrict__ colour_partials, const unsigned long long *__restrict__ cmask,
    DistArgs da)
{
    constexpr int kPst = kPstBase + (DIST ? kPstDist : 0);
    // LDS: staged records (64 x 6 float4, a record's address is one multiply), their
    // ranks, the contributor words of the chunk, per-pixel state [field][pixel], the
    // quadrant's walk list, the tile's largest `last`
    extern __shared__ float4 lds[];
    const int batch = min(rc.batch, 64);
    uint32_t *lds_idx = reinterpret_cast<uint32_t *>(lds + batch * kRecVec4);
    unsigned long long *ownw = reinterpret_cast<unsigned long long *>(lds_idx + ((batch + 1) & ~1));
    float *pst = reinterpret_cast<float *>(ownw + 64);
    uint32_t *qlist = reinterpret_cast<uint32_t *>(pst + kPst * 64);
    int &max_last = *reinterpret_cast<int *>(qlist + 64);
    const int tile = rc.torder ? (int)rc.torder[blockIdx.x] : xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int v = find_view(views, nv, tile);
    const ViewDesc vd = views[v];
    const int lt = tile - vd.tile_off;
    const int tx = lt % vd.tiles_x, ty = lt / vd.tiles_x;
    const int lane = threadIdx.x;
    const int wx0 = tx * 8, wy0 = ty * 8;
    const int row = lane >> 4, li = lane & 15;
    const bool odd = lane & 16, upper = lane & 32;
    // prologue in the owner mapping: lane 16 q + i holds pixel i of quadrant q
    const int opx = wx0 + 4 * (row & 1) + (li & 3), opy = wy0 + 4 * (row >> 1) + (li >> 2);
    const bool inside = opx < vd.W && opy < vd.H;
    const int64_t P = (int64_t)vd.W * vd.H;
    const int64_t local = (int64_t)opy * vd.W + opx;
    const int64_t g = vd.pix_off + local;
    const int64_t b3 = 3 * vd.pix_off + local;
    if (lane == 0) max_last = 0;
    qlist[lane] = 0u;
    float cg[16];
    {
        const PixelAdjoint pa = pixel_adjoint<HAS_VIS>(inside, v, g, b3, P, colC, colc, amb, Ain, Vin,
                                                       Tin, lastin, dI, dD, dN, cg);
        const float s = wave_transpose_reduce16(cg, lane);
        if ((lane & 3) == 0) colour_partials[(int64_t)tile * 16 + (lane >> 2)] = s;
        pst[0 * 64 + lane] = pa.gA0; pst[1 * 64 + lane] = pa.gA1; pst[2 * 64 + lane] = pa.gA2;
        pst[3 * 64 + lane] = pa.gV;  pst[4 * 64 + lane] = pa.gD;
        pst[5 * 64 + lane] = pa.gN0; pst[6 * 64 + lane] = pa.gN1; pst[7 * 64 + lane] = pa.gN2;
        pst[8 * 64 + lane] = pa.Tr;  pst[9 * 64 + lane] = 0.f;
        if (DIST) {
            const DistPixel dp = pixel_distortion_state(inside, g, pa.Tr, da);
            pst[10 * 64 + lane] = dp.gDist; pst[11 * 64 + lane] = dp.zref;
            pst[12 * 64 + lane] = dp.At;    pst[13 * 64 + lane] = dp.M1;
            pst[14 * 64 + lane] = dp.M2;
        }
        if (pa.last > 0) atomicMax(&max_last, pa.last);
    }
    __syncthreads();
    const uint32_t start = ranges[2 * tile];
    const int tile_len = (int)(ranges[2 * tile + 1] - start);
    const float4 *recv = rec + (size_t)v * (size_t)n * kRecStride4;
    float *gv = recgrad + (size_t)v * (size_t)n * kGradFloats;
    const float inv_s2 = rc.two_inv_s2 * 0.5f;
    const int blk_last = min(max_last, tile_len);
    const size_t wbase = (size_t)(start >> 6) + (size_t)tile;
    const int pidx = ((opy - wy0) << 3) | (opx - wx0);
    // records of the next batch in q0..q5, list entries of the one after in nidx
    float4 q0, q1, q2, q3, q4, q5;
    uint32_t qidx = 0, nidx = 0;
#define SS_FETCH_RP(IDX)                                                               \
    {                                                                                  \
        qidx = min((IDX), (uint32_t)(n - 1));                                          \
        const float4 *src_ = recv + (size_t)qidx * kRecStride4;                        \
        q0 = src_[0]; q1 = src_[1]; q2 = src_[2]; q3 = src_[3]; q4 = src_[4]; q5 = src_[5]; \
    }
    const int nbat = (blk_last + batch - 1) / batch;
    if (nbat > 0) {
        const int bb0 = (nbat - 1) * batch;
        if (lane < blk_last - bb0) SS_FETCH_RP(lists[start + bb0 + lane]);
    }
    if (nbat > 1 && lane < batch) nidx = lists[start + (nbat - 2) * batch + lane];
    for (int kb = nbat - 1; kb >= 0; --kb) {
        const int bb = kb * batch;
        const int nb = min(bb + batch, blk_last) - bb;
        __syncthreads();
        if (lane < nb) {
            float4 *dst = lds + lane * kRecVec4;
            dst[0] = q0; dst[1] = q1; dst[2] = q2; dst[3] = q3; dst[4] = q4; dst[5] = q5;
            lds_idx[lane] = qidx;
        }
        // this lane's pixel's forward mask over the batch's positions [bb, bb + nb)
        uint64_t own = 0;
        {
            const int sh = bb & 63;
            const unsigned long long *wp = cmask + (wbase + (bb >> 6)) * 64 + pidx;
            if (inside) {
                own = wp[0] >> sh;
                if (sh != 0 && sh + nb > 64) own |= wp[64] << (64 - sh);
            }
            own &= nb >= 64 ? ~0ull : ((1ull << nb) - 1ull);
        }
        ownw[lane] = own;
        const uint64_t un = row_or64(own);          // row q: the union of quadrant q
        __syncthreads();
        if (kb > 0 && lane < batch) SS_FETCH_RP(nidx);
        if (kb > 1 && lane < batch) nidx = lists[start + bb - 2 * batch + lane];
        for (int q = 0; q < 4; ++q) {
            const uint64_t U = ((uint64_t)__builtin_amdgcn_readlane((int)(uint32_t)(un >> 32), 16 * q) << 32) |
                               (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)un, 16 * q);
            if (U == 0) continue;                     // uniform
            const int nq = __popcll(U);
            // walk list of the quadrant: position of the k-th set bit from the top
            {
                const bool set = (U >> lane) & 1ull;
                const int k = lane == 63 ? 0 : __popcll(U >> (lane + 1));
                if (set) qlist[k] = (uint32_t)lane;
            }
            const int p = 16 * q + li;               // the quadrant's pixel of this lane
            const float gA0 = pst[0 * 64 + p], gA1 = pst[1 * 64 + p], gA2 = pst[2 * 64 + p];
            const float gV = pst[3 * 64 + p], gD = pst[4 * 64 + p];
            const float gN0 = pst[5 * 64 + p], gN1 = pst[6 * 64 + p], gN2 = pst[7 * 64 + p];
            float Tr = pst[8 * 64 + p], gS = pst[9 * 64 + p];
            DistPixel dp{0, 0, 0, 0, 0};
            if (DIST) {
                dp.gDist = pst[10 * 64 + p]; dp.zref = pst[11 * 64 + p]; dp.At = pst[12 * 64 + p];
                dp.M1 = pst[13 * 64 + p]; dp.M2 = pst[14 * 64 + p];
            }
            const uint64_t ownq = ownw[p];
            const PixelAdjoint pa{gA0, gA1, gA2, gV, gD, gN0, gN1, gN2, Tr, 0};
            const int qpx = wx0 + 4 * (q & 1) + (li & 3), qpy = wy0 + 4 * (q >> 1) + (li >> 2);
            const float fx = (float)qpx + 0.5f, fy = (float)qpy + 0.5f;
            __syncthreads();                         // the walk list is complete
            // record positions are read one step ahead; k < 64, and entries past nq are
            // stale positions of earlier quadrants, all below the batch size
            int jl_next = (int)qlist[row];
            for (int s0 = 0; s0 < nq; s0 += 4) {
                const int k = s0 + row;
                const bool act = k < nq;
                const int jl = jl_next;
                jl_next = (int)qlist[min(k + 4, 63)];
                const float4 *R = lds + __mul24(jl, kRecVec4);
                const float4 r0 = R[0], r1 = R[1], r2 = R[2], r3 = R[3], r4 = R[4], r5 = R[5];
                const PairEval e = eval_pair(r0, r1, r2, r3, fx, fy, rc);
                const bool contrib = act && ((ownq >> jl) & 1ull);
                const PairTerms t = pair_terms<DIST>(e, r3, r4, r5, pa, dp, HAS_VIS, da.ds);
                const float f = contrib ? t.rom : 1.f;
                float ptot;
                const float Pinc = rows_prefix_mul(f, odd, upper, ptot);
                const float Tb = Tr * Pinc;          // T before this row's record
                const float w = contrib ? e.alpha * Tb : 0.f;
                const float x = w * t.gf;
                float stot;
                const float Sinc = rows_prefix_add(x, odd, upper, stot);
                const float gSb = gS + (Sinc - x);   // g . S after this row's record
                const float dal = contrib ? fmaf(Tb, t.gf, -gSb * t.rom) : 0.f;
                Tr *= ptot;
                gS += stot;
                // every walked record is composited by some pixel of the quadrant, so each
                // step has work; a row past the end of the list adds nothing
                float gr[16];
                pair_record_grads(e, w, dal, w * t.gDe, t.u0, t.u1, r2, r3, pa, inv_s2,
                                  rc.alpha_max, gr);
                const float sum = row_transpose_reduce16(gr, lane);
                const uint64_t cb = __ballot(contrib);
                if (((cb >> (row * 16)) & 0xFFFFull) != 0)
                    atomicAdd(gv + (size_t)lds_idx[jl] * kGradFloats + li, sum);
            }
            if (row == 0) {
                pst[8 * 64 + p] = Tr;
                pst[9 * 64 + p] = gS;
            }
            __syncthreads();                         // list and state reused by the next quadrant
        }
    }
#undef SS_FETCH_RP
}

template <int TS, bool HV, bool DIST>
static void launch_bwd_d(dim3 grid, size_t lds, hipStream_t st, int32_t nv,
                         const ViewDesc *views, const uint32_t *ranges, const uint32_t *lists,
                         const float *rec, int64_t n, const RasterConsts &rc,
                         const float *colC, const float *colc, const float *amb,
                         const float *A, const float *V, const float *T, const int32_t *last,
                         const float *dI, const float *dD, const float *dN, float *recgrad,
                         float *cp, const unsigned long long *cmask, const DistArgs &da)
{
    if constexpr (TS == 8) {
        if (cmask) {
            constexpr int kPst = kPstBase + (DIST ? kPstDist : 0);
            const int b = min(rc.batch, 64);
            const size_t lds_rp = (size_t)b * kRecVec4 * sizeof(float4) +
                                  (size_t)((b + 1) & ~1) * sizeof(uint32_t) +
                                  (size_t)64 * (sizeof(unsigned long long) + kPst * sizeof(float) +
                                                sizeof(uint32_t)) + sizeof(int);
            hipLaunchKernelGGL((k_raster_bwd_rp<HV, DIST>), grid, dim3(64), lds_rp, st, nv, views,
                               ranges, lists, reinterpret_cast<const float4 *>(rec), n, rc, colC,
                               colc, amb, A, V, T, last, dI, dD, dN, recgrad, cp, cmask, da);
            return;
        }
    }
    hipLaunchKernelGGL((k_raster_bwd<TS, HV, DIST>), grid, dim3(TS * TS), lds, st, nv, views,
                       ranges, lists, reinterpret_cast<const float4 *>(rec), n, rc, colC, colc, amb,
                       A, V, T, last, dI, dD, dN, recgrad, cp, da);
}

template <int TS, bool HV>
static void launch_bwd_t(dim3 grid, size_t lds, hipStream_t st, int32_t nv,
                         const ViewDesc *views, const uint32_t *ranges, const uint32_t *lists,
                         const float *rec, int64_t n, const RasterConsts &rc,
                         const float *colC, const float *colc, const float *amb,
                         const float *A, const float *V, const float *T, const int32_t *last,
                         const float *dI, const float *dD, const float *dN, float *recgrad,
                         float *cp, const unsigned long long *cmask, const DistArgs *dist)
{
    const DistArgs da = dist ? *dist : DistArgs{0.f, nullptr, nullptr, nullptr, 0};
    if (dist)
        launch_bwd_d<TS, HV, true>(grid, lds, st, nv, views, ranges, lists, rec, n, rc, colC, colc,
                                   amb, A, V, T, last, dI, dD, dN, recgrad, cp, cmask, da);
    else
        launch_bwd_d<TS, HV, false>(grid, lds, st, nv, views, ranges, lists, rec, n, rc, colC, colc,
                                    amb, A, V, T, last, dI, dD, dN, recgrad, cp, cmask, da);
}

hipError_t launch_raster_bwd(int ts, bool has_vis, int32_t total_tiles, int32_t nv,
                             const ViewDesc *views, const uint32_t *ranges,
                             const uint32_t *lists, const float *rec, int64_t n,
                             const RasterConsts &rc, const float *colC, const float *colc,
                             const float *amb, const float *A, const float *V,
                             const float *T, const int32_t *last, const float *dI,
                             const float *dD, const float *dN, float *recgrad,
                             float *colour_partials, const unsigned long long *cmask,
                             hipStream_t st, const DistArgs *dist)
{
    if (total_tiles <= 0) return hipSuccess;
    const dim3 grid((unsigned)total_tiles);
    const size_t lds = (size_t)min(rc.batch, ts * ts) * (kRecVec4 * sizeof(float4) + sizeof(uint32_t)) +
                       (size_t)(ts * ts / 64) * 16 * sizeof(float) + sizeof(int);
#define SS_BWD(TS_)                                                                          \
    if (ts == TS_) {                                                                         \
        if (has_vis)                                                                         \
            launch_bwd_t<TS_, true>(grid, lds, st, nv, views, ranges, lists, rec, n, rc,      \
                                    colC, colc, amb, A, V, T, last, dI, dD, dN, recgrad,     \
                                    colour_partials, cmask, dist);                                 \
        else                                                                                 \
            launch_bwd_t<TS_, false>(grid, lds, st, nv, views, ranges, lists, rec, n, rc,     \
                                     colC, colc, amb, A, V, T, last, dI, dD, dN, recgrad,    \
                                     colour_partials, cmask, dist);                                \
    }
    SS_BWD(8) else SS_BWD(16) else SS_BWD(32) else return hipErrorInvalidValue;
#undef SS_BWD
    return hipGetLastError();
}

// Per view: sum the per-tile colour partials -> dC (9), dc (3), dL_a (3).
__global__ void k_colour_reduce(const float *__restrict__ partials,
                                const ViewDesc *__restrict__ views, int32_t nv,
                                float *d_colC, float *d_colc, float *d_amb)
{
    const int v = blockIdx.x;
    __shared__ float red[256 / 64][16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int t0 = views[v].tile_off;
    const int t1 = t0 + views[v].tiles_x * views[v].tiles_y;
    float acc[16];
    for (int k = 0; k < 16; ++k) acc[k] = 0.f;
    for (int t = t0 + threadIdx.x; t < t1; t += blockDim.x)
        for (int k = 0; k < 16; ++k) acc[k] += partials[(int64_t)t * 16 + k];
    const float s = wave_transpose_reduce16(acc, lane);
    if ((lane & 3) == 0) red[w][lane >> 2] = s;
    __syncthreads();
    if (threadIdx.x < 15) {
        float tot = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                    red[3][threadIdx.x];
        const int k = threadIdx.x;
        if (k < 9) d_colC[9 * v + k] = tot;
        else if (k < 12) d_colc[3 * v + k - 9] = tot;
        else d_amb[3 * v + k - 12] = tot;
    }
}

hipError_t launch_colour_reduce(const float *partials, int32_t nv, const ViewDesc *views,
                                float *d_colC, float *d_colc, float *d_amb, hipStream_t st)
{
    hipLaunchKernelGGL(k_colour_reduce, dim3((unsigned)nv), dim3(256), 0, st, partials, views, nv,
                       d_colC, d_colc, d_amb);
    return hipGetLastError();
}

// ----------------------------------------------------------- projection backward
// One thread per rank, looping over views: record gradients -> parameter gradients
// (summed over views, written once, scattered back to surfel order), and per view the
// camera-delta gradient dF = [dB | db] reduced per block into dF_partials.
//   c = B p + b:        dp += B^T dc,  dB += dc p^T,  db += dc
//   Q = T^-1:           dT = -Q^T dQ Q^T
//   T = B M:            dB += dT M^T,  dM = B^T dT
//   z0 = b_z - p_z,  k = M[2,:]
//   M = [s_u t_u, s_v t_v],  n = nsign m / |m|,  m = t_u x t_v
constexpr int kPbThreads = 256;

__global__ __launch_bounds__(kPbThreads) void k_project_bwd(
    const float4 *__restrict__ sp, int64_t n, const uint32_t *__restrict__ order, int32_t nv,
    const float *__restrict__ Fxy, const float *__restrict__ dF, double det_rel_eps,
    const float4 *__restrict__ recgrad,
    float *__restrict__ d_mean, float *__restrict__ d_tu, float *__restrict__ d_tv,
    float *__restrict__ d_scale, float *__restrict__ d_opac, float *__restrict__ d_alb,
    float *__restrict__ dF_partials)
{
    __shared__ float red[kPbThreads / 64][16];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const bool valid = r < n;
    float p[3] = {0, 0, 0}, tu[3] = {0, 0, 0}, tv[3] = {0, 0, 0}, su = 0, sv = 0;
    if (valid) {
        const float4 a = sp[4 * r], b = sp[4 * r + 1], c = sp[4 * r + 2];
        p[0] = a.x; p[1] = a.y; p[2] = a.z;
        tu[0] = a.w; tu[1] = b.x; tu[2] = b.y;
        tv[0] = b.z; tv[1] = b.w; tv[2] = c.x;
        su = c.y; sv = c.z;
    }
    float M[3][2];
    for (int i = 0; i < 3; ++i) { M[i][0] = su * tu[i]; M[i][1] = sv * tv[i]; }
    float m[3] = {tu[1] * tv[2] - tu[2] * tv[1], tu[2] * tv[0] - tu[0] * tv[2],
                  tu[0] * tv[1] - tu[1] * tv[0]};
    const float mn = sqrtf(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    float gp[3] = {0, 0, 0}, gtu[3] = {0, 0, 0}, gtv[3] = {0, 0, 0}, gsu = 0, gsv = 0, go = 0;
    float ga[3] = {0, 0, 0};
    const double pd_tu[3] = {tu[0], tu[1], tu[2]}, pd_tv[3] = {tv[0], tv[1], tv[2]};
    for (int v = 0; v < nv; ++v) {
        float B[2][3];
        double Bd[2][3];
        for (int row = 0; row < 2; ++row)
            for (int q = 0; q < 3; ++q) {
                B[row][q] = Fxy[8 * v + 4 * row + q] + (dF ? dF[8 * v + 4 * row + q] : 0.f);
                Bd[row][q] = (double)Fxy[8 * v + 4 * row + q] +
                             (dF ? (double)dF[8 * v + 4 * row + q] : 0.0);
            }
        float x[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) x[k] = 0.f;
        if (valid) {
            const size_t slot = (size_t)v * (size_t)n + (size_t)r;
            const float4 g0 = recgrad[4 * slot], g1 = recgrad[4 * slot + 1];
            const float4 g2 = recgrad[4 * slot + 2], g3 = recgrad[4 * slot + 3];
            const float dc[2] = {g0.x, g0.y};
            const float dQ[2][2] = {{g0.z, g0.w}, {g1.x, g1.y}};
            const float dz0 = g1.z, dk0 = g1.w, dk1 = g2.x, dO = g2.y;
            // Q and the normal's sign exactly as the projection stored them in the record
            const SurfelAffine sa = surfel_affine(Bd, pd_tu, pd_tv, (double)su, (double)sv, det_rel_eps);
            const float nsign = (float)sa.nsign;
            const float Q[2][2] = {{(float)sa.Q[0][0], (float)sa.Q[0][1]},
                                   {(float)sa.Q[1][0], (float)sa.Q[1][1]}};
            float t1[2][2], dT[2][2];
            for (int a = 0; a < 2; ++a)
                for (int q = 0; q < 2; ++q) t1[a][q] = Q[0][a] * dQ[0][q] + Q[1][a] * dQ[1][q];
            for (int a = 0; a < 2; ++a)
                for (int q = 0; q < 2; ++q) dT[a][q] = -(t1[a][0] * Q[q][0] + t1[a][1] * Q[q][1]);
            float dM[3][2];
            for (int row = 0; row < 2; ++row) {
                for (int q = 0; q < 3; ++q)
                    x[4 * row + q] = dT[row][0] * M[q][0] + dT[row][1] * M[q][1] + dc[row] * p[q];
                x[4 * row + 3] = dc[row];
            }
            for (int q = 0; q < 3; ++q) {
                dM[q][0] = B[0][q] * dT[0][0] + B[1][q] * dT[1][0];
                dM[q][1] = B[0][q] * dT[0][1] + B[1][q] * dT[1][1];
                gp[q] += B[0][q] * dc[0] + B[1][q] * dc[1];
            }
            gp[2] -= dz0;
            dM[2][0] += dk0;
            dM[2][1] += dk1;
            float dtu[3], dtv[3];
            for (int q = 0; q < 3; ++q) {
                gsu += tu[q] * dM[q][0];
                gsv += tv[q] * dM[q][1];
                dtu[q] = su * dM[q][0];
                dtv[q] = sv * dM[q][1];
            }
            go += dO;
            ga[0] += g2.z; ga[1] += g2.w; ga[2] += g3.x;
            const float dn[3] = {g3.y, g3.z, g3.w};
            const float nn[3] = {nsign * m[0] / mn, nsign * m[1] / mn, nsign * m[2] / mn};
            const float ndn = nn[0] * dn[0] + nn[1] * dn[1] + nn[2] * dn[2];
            float dm[3];
            for (int q = 0; q < 3; ++q) dm[q] = nsign * (dn[q] - nn[q] * ndn) / mn;
            // dt_u += t_v x dm ; dt_v += dm x t_u
            dtu[0] += tv[1] * dm[2] - tv[2] * dm[1];
            dtu[1] += tv[2] * dm[0] - tv[0] * dm[2];
            dtu[2] += tv[0] * dm[1] - tv[1] * dm[0];
            dtv[0] += dm[1] * tu[2] - dm[2] * tu[1];
            dtv[1] += dm[2] * tu[0] - dm[0] * tu[2];
            dtv[2] += dm[0] * tu[1] - dm[1] * tu[0];
            for (int q = 0; q < 3; ++q) { gtu[q] += dtu[q]; gtv[q] += dtv[q]; }
        }
        const float s = wave_transpose_reduce16(x, lane);
        if ((lane & 3) == 0) red[w][lane >> 2] = s;
        __syncthreads();
        if (threadIdx.x < 8) {
            float tot = 0.f;
            for (int k = 0; k < kPbThreads / 64; ++k) tot += red[k][threadIdx.x];
            dF_partials[((int64_t)blockIdx.x * nv + v) * 8 + threadIdx.x] = tot;
        }
        __syncthreads();
    }
    if (!valid) return;
    const int64_t i = order[r];
    if (i >= n) return;
    for (int q = 0; q < 3; ++q) {
        d_mean[3 * i + q] = gp[q];
        d_tu[3 * i + q] = gtu[q];
        d_tv[3 * i + q] = gtv[q];
        d_alb[3 * i + q] = ga[q];
    }
    d_scale[2 * i] = gsu;
    d_scale[2 * i + 1] = gsv;
    d_opac[i] = go;
}

int project_bwd_blocks(int64_t n) { return (int)((n + kPbThreads - 1) / kPbThreads); }

hipError_t launch_project_bwd(const float *sorted, int64_t n, const uint32_t *order,
                              int32_t nv, const float *Fxy, const float *dF, double det_rel_eps,
                              const float *recgrad, float *d_mean, float *d_tu, float *d_tv,
                              float *d_scale, float *d_opac, float *d_alb, float *dF_partials,
                              hipStream_t st)
{
    const int nb = project_bwd_blocks(n);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_project_bwd, dim3((unsigned)nb), dim3(kPbThreads), 0, st,
                       reinterpret_cast<const float4 *>(sorted), n, order, nv, Fxy, dF, det_rel_eps,
                       reinterpret_cast<const float4 *>(recgrad), d_mean, d_tu, d_tv, d_scale,
                       d_opac, d_alb, dF_partials);
    return hipGetLastError();
}

__global__ void k_dF_reduce(const float *__restrict__ partials, int nblocks, int32_t nv,
                            float *__restrict__ d_dF)
{
    const int v = blockIdx.x;
    const int k = threadIdx.x & 7, part = threadIdx.x >> 3;    // 32 parts x 8 values
    float s = 0.f;
    for (int b = part; b < nblocks; b += 32) s += partials[((int64_t)b * nv + v) * 8 + k];
    __shared__ float red[32][8];
    red[part][k] = s;
    __syncthreads();
    if (threadIdx.x < 8) {
        float tot = 0.f;
        for (int q = 0; q < 32; ++q) tot += red[q][threadIdx.x];
        d_dF[8 * v + threadIdx.x] = tot;
    }
}

hipError_t launch_dF_reduce(const float *partials, int nblocks, int32_t nv, float *d_dF,
                            hipStream_t st)
{
    if (nblocks == 0) return fill_f32(d_dF, 0.f, 8 * (int64_t)nv, st);
    hipLaunchKernelGGL(k_dF_reduce, dim3((unsigned)nv), dim3(256), 0, st, partials, nblocks, nv,
                       d_dF);
    return hipGetLastError();
}

// Scatter per-(view, rank) rows back to per-(view, surfel) order for debug output.
__global__ void k_unpermute_rows(const uint32_t *__restrict__ order, int64_t n, int32_t nv,
                                 const uint32_t *__restrict__ in, int in_stride,
                                 int row_words, uint32_t *__restrict__ out)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (r >= n) return;
    if (order[r] >= n) return;
    const int64_t src = ((int64_t)v * n + r) * in_stride;
    const int64_t dst = ((int64_t)v * n + order[r]) * row_words;
    for (int k = 0; k < row_words; ++k) out[dst + k] = k < in_stride ? in[src + k] : 0u;
}

hipError_t launch_unpermute_rows(const uint32_t *order, int64_t n, int32_t nv,
                                 const uint32_t *in, int in_stride, int row_words,
                                 uint32_t *out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpermute_rows, dim3((unsigned)((n + 255) / 256), (unsigned)nv),
                       dim3(256), 0, st, order, n, nv, in, in_stride, row_words, out);
    return hipGetLastError();
}

// Per-(view, rank) short4 tile ranges -> int32 [view, surfel, 4] in surfel order.
__global__ void k_unpermute_tiles(const uint32_t *__restrict__ order, int64_t n,
                                  const short4 *__restrict__ t, int32_t *__restrict__ out)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (r >= n) return;
    if (order[r] >= n) return;
    const short4 s = t[(int64_t)v * n + r];
    int32_t *o = out + 4 * ((int64_t)v * n + order[r]);
    o[0] = s.x; o[1] = s.y; o[2] = s.z; o[3] = s.w;
}

hipError_t launch_unpermute_tiles(const uint32_t *order, int64_t n, int32_t nv, const short4 *t,
                                  int32_t *out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpermute_tiles, dim3((unsigned)((n + 255) / 256), (unsigned)nv),
                       dim3(256), 0, st, order, n, t, out);
    return hipGetLastError();
}

__global__ void k_map_through(const uint32_t *__restrict__ order, int64_t n_order,
                              const unsigned long long *n_dev, int64_t cap,
                              const uint32_t *__restrict__ in, uint32_t *__restrict__ out)
{
    unsigned long long nn = *n_dev;
    const int64_t n = nn < (unsigned long long)cap ? (int64_t)nn : cap;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = order[in[i] < n_order ? in[i] : 0];
}

hipError_t launch_map_through(const uint32_t *order, int64_t n_order,
                              const unsigned long long *n_dev, int64_t cap, const uint32_t *in,
                              uint32_t *out, hipStream_t st)
{
    if (cap <= 0 || n_order <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_map_through, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, st, order,
                       n_order, n_dev, cap, in, out);
    return hipGetLastError();
}

}  // namespace ss
