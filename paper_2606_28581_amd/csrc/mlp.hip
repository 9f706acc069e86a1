// Learned sun-visibility surrogate on gfx950 MFMA (not in the paper; a stand-in for the
// geometric shadow pass of Sec. 3.1 / 3.3, trained on that pass's labels).
//
// Network: Fourier features of the normalised surfel centre (16 frequencies x sin/cos
// x 3 coordinates) + (cos phi, sin phi, sin theta, cos theta) padded to 128, then
// 128 -> 64 -> 64 -> 64 (ReLU) -> 1.  BF16 weights and activations, FP32 accumulation
// with v_mfma_f32_16x16x32_bf16.  Parameters are one FP32 master vector
// [W1 (64x128), b1, W2 (64x64), b2, W3 (64x64), b3, w4 (64), b4].
//
// Forward: one wave step owns 64 points (four 16-point MFMA tiles, so that every weight
// fragment read from LDS feeds four independent accumulation chains).  Each lane computes
// exactly the 8 features its operand needs (point l%16, features 32 ks + 8 (l/16) .. +7),
// so the 96 sin/cos values of a point are spread over 4 lanes with no duplication and no
// LDS staging; the layers are computed transposed so that hidden activations stay in
// registers (see k_mlp_forward).  Weights live in LDS, row-major [out][in], so a weight
// operand is 16 contiguous bytes.  The backward kernels work on 32-point tiles.
#include "ss_internal.h"
#include "ss_mlp.h"

namespace ss {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kPtsPerWave = 32;
// the forward takes kFwdPT tiles of 16 points per wave step: each weight fragment read
// from LDS feeds kFwdPT independent MFMA chains
constexpr int kFwdPT = 4;
constexpr int kFwdPts = 16 * kFwdPT;
constexpr int kMlpThreads = 256;
constexpr int kMlpWaves = kMlpThreads / 64;

// FP32 -> BF16, round to nearest even (gfx950 converts in hardware, two values per
// instruction when the compiler pairs them)
__device__ __forceinline__ u16 f2bf(float x)
{
    const __bf16 h = (__bf16)x;
    return __builtin_bit_cast(u16, h);
}
__device__ __forceinline__ float bf2f(u16 b) { return __uint_as_float((uint32_t)b << 16); }

union Frag {
    bf16x8 v;
    u16 h[8];
    uint4 q;
};

__device__ __forceinline__ f32x4 mfma(const Frag &a, const Frag &b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, c, 0, 0, 0);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __builtin_amdgcn_update_dpp(0.f, v, CTRL, 0xF, 0xF, true);
}

// --------------------------------------------------------------- weight prep
// FP32 master -> BF16 copies (W1, W2, W3, w4) and FP32 biases, in the MLP workspace.
__global__ void k_mlp_prep(const float *__restrict__ w, u16 *__restrict__ wb, float *__restrict__ wf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kMlpW1 + kMlpW2 + kMlpW3 + kMlpWidth) {
        int src;
        if (i < kMlpW1) src = kOffW1 + i;
        else if (i < kMlpW1 + kMlpW2) src = kOffW2 + (i - kMlpW1);
        else if (i < kMlpW1 + kMlpW2 + kMlpW3) src = kOffW3 + (i - kMlpW1 - kMlpW2);
        else src = kOffW4 + (i - kMlpW1 - kMlpW2 - kMlpW3);
        wb[i] = f2bf(w[src]);
    }
    if (i < 3 * kMlpWidth + 1) {
        int src = i < 64 ? kOffB1 + i : i < 128 ? kOffB2 + i - 64 : i < 192 ? kOffB3 + i - 128 : kOffB4;
        wf[i] = w[src];
    }
}

// Feature chunk of one lane: point p_hat (3) and sun (phi, theta) -> 8 bf16 values for
// the k-step ks and lane group g (features 32 ks + 8 g .. + 7).
__device__ __forceinline__ void feature_chunk(const float ph[3], float cphi, float sphi,
                                              float sth, float cth, int ks, int g, Frag &out)
{
    if (ks < 3) {
        // frequency 4 g from the hardware sine and cosine: x = x0 2^(4g) is exact (a
        // power-of-two scaling), r = x - 2 rint(x / 2) in [-1, 1] too, and their argument
        // is in revolutions (r / 2, exact); frequencies 4 g + 1 .. 4 g + 3 by the double
        // angle, sin 2a = 2 sin a cos a, cos 2a = 1 - 2 sin^2 a, which grows the error at
        // most eightfold, still far below the BF16 rounding that follows
        const float x = ph[ks] * (float)(1u << (4 * g));
        const float r = x - 2.f * rintf(0.5f * x);
        float s = __builtin_amdgcn_sinf(0.5f * r);
        float c = __builtin_amdgcn_cosf(0.5f * r);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            out.h[2 * q] = f2bf(s);
            out.h[2 * q + 1] = f2bf(c);
            if (q < 3) {
                const float s2 = 2.f * s * c;
                c = __fmaf_rn(-2.f * s, s, 1.f);
                s = s2;
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) out.h[e] = 0;
        if (g == 0) {
            out.h[0] = f2bf(cphi); out.h[1] = f2bf(sphi);
            out.h[2] = f2bf(sth);  out.h[3] = f2bf(cth);
        }
    }
}

// Forward, transposed: every layer computes C^T = W X^T (rows = neurons, columns =
// points), so lane l of an accumulator tile holds neurons 4 (l / 16) + 0..3 of point
// l % 16 - four consecutive neurons of one point.  The next layer's B operand needs 8
// consecutive inputs of one point per lane; numbering that layer's inputs so that its
// k-step ks, lane group q, element e is neuron 16 (2 ks + e / 4) + 4 q + e % 4 (the
// columns of W2 and W3 are permuted once when they are copied to LDS) makes those 8 the
// lane's own accumulator values of tiles 2 ks and 2 ks + 1.  Hidden activations never
// leave registers.  Features are computed directly in the B layout (point l % 16,
// features 32 ks + 8 (l / 16) .. + 7), as for the first layer.
struct MlpLds {
    u16 W1[kMlpWidth * kMlpIn];
    u16 W2[kMlpWidth * kMlpWidth];   // columns permuted (see above)
    u16 W3[kMlpWidth * kMlpWidth];
    float b[3 * kMlpWidth + 1];
};

// input index k of a hidden layer -> neuron of the previous layer
__device__ __forceinline__ int hidden_input(int k)
{
    const int ks = k >> 5, q = (k >> 3) & 3, e = k & 7;
    return 16 * (2 * ks + (e >> 2)) + 4 * q + (e & 3);
}

__device__ __forceinline__ void load_weights(MlpLds &L, const u16 *wb, const float *wf)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(wb);
    uint4 *d1 = reinterpret_cast<uint4 *>(L.W1);
    for (int i = threadIdx.x; i < kMlpW1 / 8; i += blockDim.x) d1[i] = src[i];
    const u16 *w2 = wb + kMlpW1, *w3 = wb + kMlpW1 + kMlpW2;
    for (int i = threadIdx.x; i < kMlpW2; i += blockDim.x) {
        const int o = i / kMlpWidth, k = i % kMlpWidth;
        const int j = o * kMlpWidth + hidden_input(k);
        L.W2[i] = w2[j];
        L.W3[i] = w3[j];
    }
    for (int i = threadIdx.x; i < 3 * kMlpWidth + 1; i += blockDim.x) L.b[i] = wf[i];
}

// acc[rt][ct] (16x16 tiles) += A (32 x K, operand frags from `a`) * W^T
template <int KSTEPS>
__device__ __forceinline__ void layer_mfma(const Frag (&a)[2][KSTEPS], const u16 *W, int ldw,
                                           int lane, f32x4 (&acc)[2][4])
{
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            Frag b;
            b.q = *reinterpret_cast<const uint4 *>(W + (ct * 16 + (lane & 15)) * ldw + ks * 32 +
                                                   8 * (lane >> 4));
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) acc[rt][ct] = mfma(a[rt][ks], b, acc[rt][ct]);
        }
    }
}

// One layer, transposed: acc[ot][pt] (neurons 16 ot.., points 16 pt..) = bias +
// W[ot rows] x[pt] over KSTEPS k-steps; W row-major [out][in] (in LDS).
template <int KSTEPS, int PT>
__device__ __forceinline__ void layer_t(const u16 *W, int ldw, const float *bias,
                                        const Frag (&x)[PT][KSTEPS], int lane, f32x4 (&acc)[4][PT])
{
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        const float *bo = bias + ot * 16 + 4 * (lane >> 4);
        const f32x4 b0 = f32x4{bo[0], bo[1], bo[2], bo[3]};
#pragma unroll
        for (int pt = 0; pt < PT; ++pt) acc[ot][pt] = b0;
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            Frag w;
            w.q = *reinterpret_cast<const uint4 *>(W + (ot * 16 + (lane & 15)) * ldw + ks * 32 +
                                                   8 * (lane >> 4));
#pragma unroll
            for (int pt = 0; pt < PT; ++pt) acc[ot][pt] = mfma(w, x[pt][ks], acc[ot][pt]);
        }
    }
}

// ReLU + bf16 of a layer's accumulators into the next layer's B operands: two values are
// rounded to one packed bf16 pair, then the ReLU is one packed 16-bit integer max (a
// negative bf16, -0 included, is a negative int16 and becomes +0; rounding commutes with
// the ReLU, so the pair is bit-identical to bf16(max(x, 0))).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t relu_bf16x2(float a, float b)
{
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const bf16x2 v = __builtin_convertvector((f32x2){a, b}, bf16x2);
    const i16x2 z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(i16x2, v), z));
}

template <int PT>
__device__ __forceinline__ void relu_to_operand(const f32x4 (&acc)[4][PT], Frag (&h)[PT][2])
{
#pragma unroll
    for (int pt = 0; pt < PT; ++pt)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const f32x4 &lo = acc[2 * ks][pt], &hi = acc[2 * ks + 1][pt];
            h[pt][ks].q = make_uint4(relu_bf16x2(lo[0], lo[1]), relu_bf16x2(lo[2], lo[3]),
                                     relu_bf16x2(hi[0], hi[1]), relu_bf16x2(hi[2], hi[3]));
        }
}

// the activations of one layer for the backward, [M][64] in neuron order: 4 consecutive
// neurons (8 bytes) per lane and accumulator tile
template <int PT>
__device__ __forceinline__ void save_layer(const Frag (&h)[PT][2], u16 *dst, int64_t base, int64_t M,
                                           int lane)
{
#pragma unroll
    for (int pt = 0; pt < PT; ++pt) {
        const int64_t i = base + pt * 16 + (lane & 15);
        if (i >= M) continue;
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            const Frag &f = h[pt][ot >> 1];
            const int e0 = 4 * (ot & 1);
            uint2 v;
            v.x = (uint32_t)f.h[e0] | ((uint32_t)f.h[e0 + 1] << 16);
            v.y = (uint32_t)f.h[e0 + 2] | ((uint32_t)f.h[e0 + 3] << 16);
            *reinterpret_cast<uint2 *>(dst + i * kMlpWidth + ot * 16 + 4 * (lane >> 4)) = v;
        }
    }
}

// Forward over M points.  Point i uses position pts[i % G] and sun[i / G] when G > 0
// (every surfel under every sun), or pts[i] and sun[i] when G == 0.  When `saveF` /
// `saveH` are given the bf16 features [M,128] and hidden activations [3][M,64] are
// written for the backward.
__global__ __launch_bounds__(kMlpThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_mlp_forward(
    const u16 *__restrict__ wb, const float *__restrict__ wf, const float *__restrict__ pts,
    const float *__restrict__ sun, int64_t M, int64_t G, MlpNorm nz, int prob,
    float *__restrict__ out, u16 *__restrict__ saveF, u16 *__restrict__ saveH)
{
    __shared__ MlpLds L;
    load_weights(L, wb, wf);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int PT = kFwdPT;
    const int64_t ntile = (M + kFwdPts - 1) / kFwdPts;
    // output weights as an MFMA weight operand: row 0 (lanes n % 16 == 0) holds w4 in the
    // hidden layers' input numbering, rows 1..15 are zero
    Frag a4[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int e = 0; e < 8; ++e)
            a4[ks].h[e] = (lane & 15) == 0
                              ? wb[kMlpW1 + kMlpW2 + kMlpW3 + hidden_input(32 * ks + 8 * (lane >> 4) + e)]
                              : (u16)0;
    for (int64_t tile = (int64_t)blockIdx.x * kMlpWaves + wave; tile < ntile;
         tile += (int64_t)gridDim.x * kMlpWaves) {
        // weight fragments are read from LDS per tile (held across tiles they would take
        // 128 VGPRs)
        asm volatile("" ::: "memory");
        const int64_t base = tile * kFwdPts;
        // all-pairs mode: one division per tile; lanes carry into the next sun
        const int64_t is0 = G > 0 ? base / G : 0, ip0 = base - is0 * G;
        // ---- features in the B layout
        Frag fa[PT][4];
#pragma unroll
        for (int pt = 0; pt < PT; ++pt) {
            int64_t i = base + pt * 16 + (lane & 15);
            const bool valid = i < M;
            if (!valid) i = M - 1;
            int64_t ip = i, is = i;
            if (G > 0) {
                ip = ip0 + (i - base);
                is = is0;
                while (ip >= G) { ip -= G; ++is; }
            }
            float ph[3];
            ph[0] = __fmul_rn(__fsub_rn(pts[3 * ip], nz.cx), nz.inv_half);
            ph[1] = __fmul_rn(__fsub_rn(pts[3 * ip + 1], nz.cy), nz.inv_half);
            ph[2] = __fmul_rn(__fsub_rn(pts[3 * ip + 2], nz.cz), nz.inv_half);
            // sun angles through the hardware sine and cosine (argument in revolutions)
            constexpr float kRev = 0.15915494309189535f;   // 1 / (2 pi)
            const float phi = sun[2 * is] * kRev, th = sun[2 * is + 1] * kRev;
            const float sphi = __builtin_amdgcn_sinf(phi), cphi = __builtin_amdgcn_cosf(phi);
            const float sth = __builtin_amdgcn_sinf(th), cth = __builtin_amdgcn_cosf(th);
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                feature_chunk(ph, cphi, sphi, sth, cth, ks, lane >> 4, fa[pt][ks]);
                if (saveF && valid)
                    *reinterpret_cast<uint4 *>(saveF + i * kMlpIn + ks * 32 + 8 * (lane >> 4)) =
                        fa[pt][ks].q;
            }
        }
        f32x4 acc[4][PT];
        Frag h[PT][2];
        layer_t<4>(L.W1, kMlpIn, L.b, fa, lane, acc);
        relu_to_operand(acc, h);
        if (saveH) save_layer(h, saveH, base, M, lane);
        layer_t<2>(L.W2, kMlpWidth, L.b + kMlpWidth, h, lane, acc);
        relu_to_operand(acc, h);
        if (saveH) save_layer(h, saveH + M * kMlpWidth, base, M, lane);
        layer_t<2>(L.W3, kMlpWidth, L.b + 2 * kMlpWidth, h, lane, acc);
        relu_to_operand(acc, h);
        if (saveH) save_layer(h, saveH + 2 * M * kMlpWidth, base, M, lane);
        // ---- output: logit = w4 . h3 + b4, one more transposed MFMA layer whose weight
        // operand holds w4 in row 0: lane n < 16 gets point n's logit in element 0
        float part[PT];
#pragma unroll
        for (int pt = 0; pt < PT; ++pt) {
            f32x4 o = {0.f, 0.f, 0.f, 0.f};
            o = mfma(a4[0], h[pt][0], o);
            o = mfma(a4[1], h[pt][1], o);
            part[pt] = o[0];
        }
        if (lane < 16) {
#pragma unroll
            for (int pt = 0; pt < PT; ++pt) {
                const int64_t i = base + pt * 16 + lane;
                if (i < M) {
                    const float lg = part[pt] + L.b[3 * kMlpWidth];
                    out[i] = prob ? 1.f / (1.f + expf(-lg)) : lg;
                }
            }
        }
    }
}

// ------------------------------------------------------------- output backward
// Per point: dlogit, BCE loss, da3 = bf16(dlogit * w4 * [h3 > 0]); per block the sums
// of dlogit * h3 (dw4), dlogit (db4) and the loss -> part[blk][66].
__global__ __launch_bounds__(256) void k_mlp_out_bwd(
    const float *__restrict__ logits, const float *__restrict__ labels,
    const float *__restrict__ dlin, float scale, const u16 *__restrict__ wb,
    const u16 *__restrict__ H3, int64_t M, u16 *__restrict__ dA3, float *__restrict__ part)
{
    __shared__ float dl[256];
    __shared__ float red[4][66];
    __shared__ float w4s[kMlpWidth];
    if (threadIdx.x < kMlpWidth) w4s[threadIdx.x] = bf2f(wb[kMlpW1 + kMlpW2 + kMlpW3 + threadIdx.x]);
    const int64_t base = (int64_t)blockIdx.x * 256;
    const int64_t m = base + threadIdx.x;
    float d = 0.f, loss = 0.f;
    if (m < M) {
        const float lg = logits[m];
        if (labels) {
            const float y = labels[m];
            d = (1.f / (1.f + expf(-lg)) - y) * scale;
            loss = (fmaxf(lg, 0.f) - lg * y + log1pf(expf(-fabsf(lg)))) * scale;
        } else {
            d = dlin[m] * scale;
        }
    }
    dl[threadIdx.x] = d;
    __syncthreads();
    if (m < M) {
        const u16 *h = H3 + m * kMlpWidth;
        u16 *o = dA3 + m * kMlpWidth;
        for (int j = 0; j < kMlpWidth; ++j) {
            const u16 hj = h[j];
            o[j] = f2bf((hj != 0 && !(hj & 0x8000)) ? d * w4s[j] : 0.f);
        }
    }
    // column sums: thread t -> column j = t & 63 over points q = t >> 6 (+4)
    const int j = threadIdx.x & 63, q = threadIdx.x >> 6;
    float s = 0.f;
    for (int p = q; p < 256; p += 4)
        if (base + p < M) s += dl[p] * bf2f(H3[(base + p) * kMlpWidth + j]);
    red[q][j] = s;
    if (threadIdx.x < 4) {
        float a = 0.f, b = 0.f;
        for (int p = threadIdx.x; p < 256; p += 4) a += dl[p];
        red[threadIdx.x][64] = a;
        red[threadIdx.x][65] = 0.f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // loss: simple serial sum over the block (training-only path)
        float l = 0.f;
        for (int p = 0; p < 256; ++p) {
            const int64_t mm = base + p;
            if (mm < M && labels) {
                const float lg = logits[mm], y = labels[mm];
                l += (fmaxf(lg, 0.f) - lg * y + log1pf(expf(-fabsf(lg)))) * scale;
            }
        }
        red[0][65] = l;
    }
    (void)loss;
    __syncthreads();
    if (threadIdx.x < 66) {
        float t = red[0][threadIdx.x];
        if (threadIdx.x < 65) t += red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        part[(int64_t)blockIdx.x * 66 + threadIdx.x] = t;
    }
}

// ------------------------------------------------------------ weight gradients
// part_dw[blk][i][j] = sum over the block's kDwChunk points of dA[m][i] H[m][j] (MFMA,
// the point index is the contraction), part_db[blk][i] = sum of dA[m][i].
template <int N>
__global__ __launch_bounds__(256) void k_mlp_dw(const u16 *__restrict__ dA,
                                                const u16 *__restrict__ H, int64_t M,
                                                float *__restrict__ part_dw,
                                                float *__restrict__ part_db)
{
    __shared__ u16 sA[32 * kMlpWidth];
    __shared__ u16 sH[32 * N];
    const int lane = threadIdx.x & 63, rt = threadIdx.x >> 6;
    constexpr int NCT = N / 16;
    f32x4 acc[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
    float db = 0.f;
    const int64_t m0 = (int64_t)blockIdx.x * kDwChunk;
    for (int ks = 0; ks < kDwChunk / 32; ++ks) {
        const int64_t mb = m0 + ks * 32;
        __syncthreads();
        {   // 32 x 64 bf16 of dA: one uint4 per thread
            const int r = threadIdx.x >> 3, c = (threadIdx.x & 7) * 8;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (mb + r < M) v = *reinterpret_cast<const uint4 *>(dA + (mb + r) * kMlpWidth + c);
            *reinterpret_cast<uint4 *>(sA + r * kMlpWidth + c) = v;
        }
        for (int e = threadIdx.x; e < 32 * N / 8; e += 256) {
            const int r = e / (N / 8), c = (e % (N / 8)) * 8;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (mb + r < M) v = *reinterpret_cast<const uint4 *>(H + (mb + r) * N + c);
            *reinterpret_cast<uint4 *>(sH + r * N + c) = v;
        }
        __syncthreads();
        if (threadIdx.x < kMlpWidth)
            for (int r = 0; r < 32; ++r) db += bf2f(sA[r * kMlpWidth + threadIdx.x]);
        Frag a;
        const int i = rt * 16 + (lane & 15), g = lane >> 4;
#pragma unroll
        for (int q = 0; q < 8; ++q) a.h[q] = sA[(8 * g + q) * kMlpWidth + i];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            Frag b;
            const int j = ct * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 8; ++q) b.h[q] = sH[(8 * g + q) * N + j];
            acc[ct] = mfma(a, b, acc[ct]);
        }
    }
    float *out = part_dw + (int64_t)blockIdx.x * kMlpWidth * N;
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = rt * 16 + 4 * (lane >> 4) + r, j = ct * 16 + (lane & 15);
            out[i * N + j] = acc[ct][r];
        }
    if (threadIdx.x < kMlpWidth) part_db[(int64_t)blockIdx.x * kMlpWidth + threadIdx.x] = db;
}

// ------------------------------------------------------- propagated activations
// dA_prev[m][j] = bf16( sum_i dA[m][i] W[i][j] * [Hprev[m][j] > 0] ), W = [out i][in j].
__global__ __launch_bounds__(256) void k_mlp_dh(const u16 *__restrict__ dA,
                                                const u16 *__restrict__ Wb,
                                                const u16 *__restrict__ Hprev, int64_t M,
                                                u16 *__restrict__ dAp)
{
    __shared__ u16 Wt[kMlpWidth * kMlpWidth];   // Wt[j][i] = W[i][j]
    for (int e = threadIdx.x; e < kMlpWidth * kMlpWidth; e += 256) {
        const int i = e / kMlpWidth, j = e % kMlpWidth;
        Wt[j * kMlpWidth + i] = Wb[e];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4;
    const int64_t ntile = (M + kPtsPerWave - 1) / kPtsPerWave;
    for (int64_t tile = (int64_t)blockIdx.x * kMlpWaves + wave; tile < ntile;
         tile += (int64_t)gridDim.x * kMlpWaves) {
        const int64_t base = tile * kPtsPerWave;
        Frag a[2][2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const int64_t m = base + rt * 16 + (lane & 15);
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                a[rt][ks].q = m < M ? *reinterpret_cast<const uint4 *>(dA + m * kMlpWidth + ks * 32 + 8 * g)
                                    : make_uint4(0, 0, 0, 0);
        }
        f32x4 acc[2][4];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
        layer_mfma<2>(a, Wt, kMlpWidth, lane, acc);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t m = base + rt * 16 + 4 * g + r;
                    const int j = ct * 16 + (lane & 15);
                    if (m < M) {
                        const u16 hp = Hprev[m * kMlpWidth + j];
                        dAp[m * kMlpWidth + j] = f2bf((hp != 0 && !(hp & 0x8000)) ? acc[rt][ct][r] : 0.f);
                    }
                }
    }
}

__global__ void k_mlp_reduce(const float *__restrict__ part, int nblocks, int count, int stride,
                             float *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= count) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * stride + c];
    out[c] = s;
}

__global__ void k_mlp_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                           const float *__restrict__ g, int64_t n, float lr, float b1, float b2,
                           float eps, float bc1, float bc2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ------------------------------------------------------------------ launchers
int mlp_dw_blocks(int64_t M) { return (int)((M + kDwChunk - 1) / kDwChunk); }

hipError_t launch_mlp_prep(const float *w, uint16_t *wb, float *wf, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_prep, dim3((kMlpBf16 + 255) / 256), dim3(256), 0, st, w, wb, wf);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const uint16_t *wb, const float *wf, const float *pts,
                              const float *sun, int64_t M, int64_t G, MlpNorm nz, bool prob,
                              float *out, uint16_t *saveF, uint16_t *saveH, hipStream_t st)
{
    if (M <= 0) return hipSuccess;
    int64_t tiles = (M + kFwdPts - 1) / kFwdPts;
    int64_t blocks = (tiles + kMlpWaves - 1) / kMlpWaves;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(kMlpThreads), 0, st, wb, wf,
                       pts, sun, M, G, nz, prob ? 1 : 0, out, saveF, saveH);
    return hipGetLastError();
}

hipError_t launch_mlp_out_bwd(const float *logits, const float *labels, const float *dlogit_in,
                              float scale, const uint16_t *wb, const uint16_t *H3, int64_t M,
                              uint16_t *dA3, float *part, hipStream_t st)
{
    if (M <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_out_bwd, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, logits,
                       labels, dlogit_in, scale, wb, H3, M, dA3, part);
    return hipGetLastError();
}

hipError_t launch_mlp_dw(const uint16_t *dA, const uint16_t *H, int n, int64_t M, float *part_dw,
                         float *part_db, hipStream_t st)
{
    const int nb = mlp_dw_blocks(M);
    if (nb == 0) return hipSuccess;
    if (n == 64)
        hipLaunchKernelGGL(k_mlp_dw<64>, dim3(nb), dim3(256), 0, st, dA, H, M, part_dw, part_db);
    else if (n == 128)
        hipLaunchKernelGGL(k_mlp_dw<128>, dim3(nb), dim3(256), 0, st, dA, H, M, part_dw, part_db);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_mlp_dh(const uint16_t *dA, const uint16_t *Wb, const uint16_t *Hprev, int64_t M,
                         uint16_t *dA_prev, hipStream_t st)
{
    if (M <= 0) return hipSuccess;
    int64_t tiles = (M + kPtsPerWave - 1) / kPtsPerWave;
    int64_t blocks = (tiles + kMlpWaves - 1) / kMlpWaves;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_mlp_dh, dim3((unsigned)blocks), dim3(256), 0, st, dA, Wb, Hprev, M, dA_prev);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce(const float *part, int nblocks, int count, int stride, float *out,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_reduce, dim3((count + 255) / 256), dim3(256), 0, st, part, nblocks, count,
                       stride, out);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr,
                           float b1, float b2, float eps, int step, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, m, v, g, n,
                       lr, b1, b2, eps, bc1, bc2);
    return hipGetLastError();
}

}  // namespace ss
