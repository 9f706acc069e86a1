// Scans and the stable LSD radix sort used for the centre-depth order and for
// bucketing (tile, surfel) pairs by tile (Sec. 3.2 "Rasterization": sort by centre
// depth, organise into tiles).
//
// Radix sort: 8-bit digits, 256 threads x 16 items = 4096 items per block.
//   hist    : per-block digit histogram in LDS (one add per group of lanes holding the
//             same digit) -> hist[digit * nblocks + block], or per segment (below)
//   scan    : exclusive scan of hist (digit-major) -> global base of (digit, block)
//   scatter : per-wave stable multisplit with 8 ballots per item (lanes holding the
//             same digit form a mask; rank = popcount of lower lanes in the mask); the
//             group's lowest lane adds the group size to the wave's running count of
//             that digit in LDS and hands the old count to the group, then a prefix
//             over the 4 waves places each digit's run inside the block.
// Tile bucketing sorts within segments (one per view) on key minus the segment's base,
// so the number of passes follows the largest view's tile count; its last pass also
// writes each tile's [begin, end) range.
// Item counts may live in device memory (pair counts are data dependent), so grids
// are sized by capacity and blocks past the live count exit at once.
#include "ss_internal.h"

namespace ss {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // 4096
constexpr int kSortWaves = kSortThreads / kWave;

__device__ __forceinline__ int64_t live_count(const unsigned long long *n_dev, int64_t cap,
                                              int64_t n_host)
{
    if (!n_dev) return n_host;
    unsigned long long n = *n_dev;
    return n < (unsigned long long)cap ? (int64_t)n : cap;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

hipError_t fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, value, count);
    return hipGetLastError();
}

hipError_t fill_f32(float *p, float value, int64_t count, hipStream_t st)
{
    union { float f; uint32_t u; } cv;
    cv.f = value;
    return fill_u32(reinterpret_cast<uint32_t *>(p), cv.u, count, st);
}

// ------------------------------------------------------------------ block scan
// Exclusive scan of one uint32 per thread over a 256-thread block; returns the
// exclusive prefix, *total gets the block sum.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *lds_w,
                                                         uint32_t *total)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t inc = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(inc, d, kWave);
        if (lane >= d) inc += y;
    }
    if (lane == kWave - 1) lds_w[w] = inc;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
        uint32_t t = lds_w[i];
        if (i < w) wbase += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return wbase + inc - x;
}

// ------------------------------------------------------------- pair-count scan
// Each thread owns kSortItems consecutive entries; full groups are moved as uint4 (the
// arrays start 256-byte aligned and a group starts at a multiple of 16 entries).
__device__ __forceinline__ void load_items(const uint32_t *in, int64_t base, int64_t len,
                                           uint32_t (&v)[kSortItems])
{
    if (base + kSortItems <= len) {
        const uint4 *p = reinterpret_cast<const uint4 *>(in + base);
#pragma unroll
        for (int q = 0; q < kSortItems / 4; ++q) {
            const uint4 x = p[q];
            v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) v[i] = base + i < len ? in[base + i] : 0u;
    }
}

__device__ __forceinline__ void store_items(uint32_t *out, int64_t base, int64_t len,
                                            const uint32_t (&v)[kSortItems])
{
    if (base + kSortItems <= len) {
        uint4 *p = reinterpret_cast<uint4 *>(out + base);
#pragma unroll
        for (int q = 0; q < kSortItems / 4; ++q)
            p[q] = make_uint4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < kSortItems; ++i)
            if (base + i < len) out[base + i] = v[i];
    }
}

__global__ void k_scan_reduce(const uint32_t *in, int64_t len, uint32_t *partials)
{
    __shared__ uint32_t lds[kSortWaves];
    int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortItems;
    uint32_t v[kSortItems];
    load_items(in, base, len, v);
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) s += v[i];
    uint32_t tot;
    block_exclusive_scan(s, lds, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// One block: exclusive scan of the per-chunk sums in 64-bit, overflow detection.
constexpr int kScanPartialsThreads = 1024;

__global__ __launch_bounds__(kScanPartialsThreads) void k_scan_partials(
    uint32_t *partials, int64_t nparts, uint32_t *out_total, unsigned long long *counters,
    int which, uint32_t *flags, uint64_t cap)
{
    __shared__ unsigned long long lds[kScanPartialsThreads / kWave];
    __shared__ unsigned long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int64_t b0 = 0; b0 < nparts; b0 += blockDim.x) {
        int64_t i = b0 + threadIdx.x;
        unsigned long long x = i < nparts ? partials[i] : 0ull;
        unsigned long long inc = x;
        for (int d = 1; d < kWave; d <<= 1) {
            unsigned long long y = __shfl_up(inc, d, kWave);
            if (lane >= d) inc += y;
        }
        if (lane == kWave - 1) lds[w] = inc;
        __syncthreads();
        unsigned long long wbase = 0, tot = 0;
        for (int k = 0; k < (int)(blockDim.x / kWave); ++k) {
            if (k < w) wbase += lds[k];
            tot += lds[k];
        }
        unsigned long long excl = carry + wbase + inc - x;
        if (i < nparts) partials[i] = (uint32_t)(excl > 0xFFFFFFFFull ? 0xFFFFFFFFull : excl);
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsigned long long total = carry;
        counters[which] = total;
        *out_total = (uint32_t)(total > 0xFFFFFFFFull ? 0xFFFFFFFFull : total);
        if (total > 0xFFFFFFFFull || total > cap) flags[0] |= 1u;
    }
}

__global__ void k_scan_down(const uint32_t *in, int64_t len, const uint32_t *partials,
                            uint32_t *out)
{
    __shared__ uint32_t lds[kSortWaves];
    int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortItems;
    uint32_t v[kSortItems];
    load_items(in, base, len, v);
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) s += v[i];
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, lds, &tot) + partials[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const uint32_t x = v[i];
        v[i] = run;
        run += x;
    }
    store_items(out, base, len, v);
}

size_t scan_temp_elems(int64_t len)
{
    return (size_t)((len + kSortTile - 1) / kSortTile) + 1;
}

hipError_t scan_pair_counts(const uint32_t *counts, int64_t n, int32_t nv,
                            uint32_t *out, uint32_t *partials, unsigned long long *counters,
                            int which, uint32_t *flags, uint64_t cap, hipStream_t st)
{
    int64_t len = (int64_t)nv * n;
    int64_t nb = (len + kSortTile - 1) / kSortTile;
    if (nb > 0)
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kSortThreads), 0, st,
                           counts, len, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanPartialsThreads), 0, st, partials, nb,
                       out + len, counters, which, flags, cap);
    if (nb > 0)
        hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kSortThreads), 0, st, counts,
                           len, partials, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort
// Blocks never straddle a segment: block b of segment v covers items
// [start_v + j * kSortTile, ...) with j = b - blk0_v, and its digits are taken from
// key - base_v.  The histogram of block b sits at blk0_v * 256 + digit * nblk_v + j, so
// one exclusive scan over all blocks' histograms gives every (segment, digit, block) its
// output position inside its own segment.  Blocks past the last live one write zeros at
// b * 256 + digit, after every live block's entries.
struct SegDesc {
    uint32_t start, end, blk0, base;
};

struct BlockRange {
    int64_t lo, hi;
    uint32_t base;
    int64_t hidx0;      // histogram index of digit 0
    int64_t hstride;    // histogram index step per digit
    bool live;
};

__device__ __forceinline__ BlockRange block_range(const SegDesc *segs, int nseg,
                                                  const unsigned long long *n_dev, int64_t cap,
                                                  int64_t n_host, int64_t b)
{
    BlockRange r;
    if (!segs) {
        const int64_t n = live_count(n_dev, cap, n_host);
        const int64_t nb = (n + kSortTile - 1) / kSortTile;
        r.lo = b * kSortTile;
        r.hi = min(n, r.lo + kSortTile);
        r.base = 0;
        r.live = b < nb;
        r.hidx0 = r.live ? b : b * 256;
        r.hstride = r.live ? nb : 1;
        return r;
    }
    const int64_t total = segs[nseg].blk0;
    r.live = b < total;
    if (!r.live) {
        r.lo = r.hi = 0;
        r.base = 0;
        r.hidx0 = b * 256;
        r.hstride = 1;
        return r;
    }
    // last segment whose first block is <= b (segments without blocks share blk0 with
    // the next one and are skipped by taking the last)
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)segs[mid].blk0 <= b) lo = mid; else hi = mid - 1;
    }
    const SegDesc sd = segs[lo];
    const int64_t j = b - sd.blk0;
    const int64_t nblk = (int64_t)segs[lo + 1].blk0 - sd.blk0;
    r.lo = (int64_t)sd.start + j * kSortTile;
    r.hi = min((int64_t)sd.end, r.lo + kSortTile);
    r.base = sd.base;
    r.hidx0 = (int64_t)sd.blk0 * 256 + j;
    r.hstride = nblk;
    return r;
}

// Lanes of the wave whose `valid` item has the same digit as this lane (over the low
// `nbits` bits of d).
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid, int nbits)
{
    uint64_t m = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// One block: segment table from view-major pair offsets.  Segment v holds the items
// [offs[v * stride], offs[(v + 1) * stride]) clamped to the live count; its keys are
// based at views[v].tile_off.
constexpr int kSegThreads = 1024;

__global__ __launch_bounds__(kSegThreads) void k_seg_table(
    const uint32_t *offs, int64_t stride, int32_t nseg, const ViewDesc *views,
    const unsigned long long *n_dev, int64_t cap, SegDesc *segs)
{
    __shared__ uint32_t lds_w[kSegThreads / kWave];
    __shared__ uint32_t carry;
    const int64_t n = live_count(n_dev, cap, cap);
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int32_t v0 = 0; v0 <= nseg; v0 += kSegThreads) {
        const int32_t v = v0 + (int32_t)threadIdx.x;
        uint32_t st = 0, en = 0, nblk = 0;
        if (v <= nseg) {
            st = (uint32_t)min((int64_t)offs[(int64_t)v * stride], n);
            en = v < nseg ? (uint32_t)min((int64_t)offs[(int64_t)(v + 1) * stride], n) : st;
            en = max(en, st);
            nblk = v < nseg ? (en - st + kSortTile - 1) / kSortTile : 0u;
        }
        const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
        uint32_t inc = nblk;
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t y = __shfl_up(inc, d, kWave);
            if (lane >= d) inc += y;
        }
        if (lane == kWave - 1) lds_w[w] = inc;
        __syncthreads();
        uint32_t wbase = 0, tot = 0;
        for (int k = 0; k < kSegThreads / kWave; ++k) {
            if (k < w) wbase += lds_w[k];
            tot += lds_w[k];
        }
        if (v <= nseg)
            segs[v] = SegDesc{st, en, carry + wbase + inc - nblk,
                              v < nseg ? (uint32_t)views[v].tile_off : 0u};
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
}

// KT = uint16_t: tile keys local to their segment (the digit is taken from the key
// itself, the segment base only offsets the tile ranges); uint32_t: keys carry the
// segment base, which the digit subtracts.
template <typename KT>
__device__ __forceinline__ uint32_t key_digit(KT key, uint32_t base, int shift)
{
    constexpr bool kLocal = sizeof(KT) == 2;
    return (((uint32_t)key - (kLocal ? 0u : base)) >> shift) & 255u;
}

template <typename KT>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(
    const KT *keys, const SegDesc *segs, int nseg, const unsigned long long *n_dev,
    int64_t cap, int64_t n_host, int shift, uint32_t *hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const BlockRange br = block_range(segs, nseg, n_dev, cap, n_host, blockIdx.x);
    if (br.live) {
        const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
        const int64_t wbase = br.lo + (int64_t)w * (kSortItems * kWave);
        // all of the wave's keys are loaded before any is counted
        uint32_t key[kSortItems];
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            const int64_t i = wbase + it * kWave + lane;
            key[it] = i < br.hi ? (uint32_t)keys[i] : 0u;
        }
        // one LDS add per key: the LDS serialises lanes that hit the same counter, which
        // costs less than finding each digit's group of lanes with ballots
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            if (wbase + it * kWave + lane < br.hi)
                atomicAdd(&h[key_digit<KT>((KT)key[it], br.base, shift)], 1u);
        }
    }
    __syncthreads();
    hist[br.hidx0 + (int64_t)threadIdx.x * br.hstride] = h[threadIdx.x];
}

// Exclusive scan over the histograms, single pass per block chunk using the same
// three-kernel scheme as the pair counts but on a 32-bit total.
__global__ void k_hist_scan_reduce(uint32_t *hist, int64_t len, uint32_t *partials)
{
    __shared__ uint32_t lds[kSortWaves];
    int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortItems;
    uint32_t v[kSortItems];
    load_items(hist, base, len, v);
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) s += v[i];
    uint32_t tot;
    block_exclusive_scan(s, lds, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanPartialsThreads) void k_hist_scan_partials(uint32_t *partials,
                                                                             int64_t nparts)
{
    __shared__ uint32_t lds[kScanPartialsThreads / kWave];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nparts; b0 += blockDim.x) {
        int64_t i = b0 + threadIdx.x;
        uint32_t x = i < nparts ? partials[i] : 0u;
        const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
        uint32_t inc = x;
        for (int d = 1; d < kWave; d <<= 1) {
            uint32_t y = __shfl_up(inc, d, kWave);
            if (lane >= d) inc += y;
        }
        if (lane == kWave - 1) lds[w] = inc;
        __syncthreads();
        uint32_t wbase = 0, tot = 0;
        for (int k = 0; k < (int)(blockDim.x / kWave); ++k) {
            if (k < w) wbase += lds[k];
            tot += lds[k];
        }
        if (i < nparts) partials[i] = carry + wbase + inc - x;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
}

// With `ranges` (the last pass), every block also reports, per key, the first and last
// output position of its run: ranges[2k] = min over blocks, ranges[2k + 1] = max + 1.
// A block holds its items in LDS sorted by the whole key (stable on the top digit of
// items that the lower passes left sorted), so equal keys are adjacent there.
template <typename KT>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const KT *kin, const uint32_t *vin, KT *kout, uint32_t *vout,
    const uint32_t *offs, const SegDesc *segs, int nseg, const unsigned long long *n_dev,
    int64_t cap, int64_t n_host, int shift, int nbits, uint32_t *ranges, int64_t nkeys)
{
    constexpr bool kLocal = sizeof(KT) == 2;
    __shared__ uint32_t wcnt[kSortWaves][256];
    __shared__ uint32_t wsink[kSortWaves][kWave];  // target of the lanes that are not group leaders
    __shared__ uint32_t dbase[256];          // block-local start of each digit's run
    __shared__ uint32_t gshift[256];         // global start minus local start, per digit
    __shared__ uint32_t lds_w[kSortWaves];
    __shared__ KT skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    const BlockRange br = block_range(segs, nseg, n_dev, cap, n_host, blockIdx.x);
    if (!br.live) return;   // uniform over the block
    for (int i = threadIdx.x; i < kSortWaves * 256; i += kSortThreads) (&wcnt[0][0])[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t wbase = br.lo + (int64_t)w * (kSortItems * kWave);
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = wbase + it * kWave + lane;
        const bool valid = i < br.hi;
        key[it] = valid ? (uint32_t)kin[i] : 0u;
        val[it] = valid ? vin[i] : 0u;
    }
    // stable ranks: per item row, the lowest lane of each equal-digit group adds the group
    // size to the wave's running count of that digit and receives the count before it (LDS
    // atomics of one wave take effect in issue order, row after row); the other lanes add
    // to a private word so that no two lanes of an instruction share an address
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const bool valid = wbase + it * kWave + lane < br.hi;
        const uint32_t d = key_digit<KT>((KT)key[it], br.base, shift);
        const uint64_t m = digit_peers(d, valid, nbits);
        const uint32_t before = __popcll(m & lt_mask);
        const bool leader = valid && before == 0;
        uint32_t *cnt = leader ? &wcnt[w][d] : &wsink[w][lane];
        const uint32_t old = atomicAdd(cnt, leader ? (uint32_t)__popcll(m) : 0u);
        const int from = m != 0 ? (int)__builtin_ctzll(m) : lane;
        rank[it] = (uint32_t)__shfl((int)old, from, kWave) + before;
    }
    __syncthreads();
    {
        // per digit: prefix over the waves, then an exclusive scan over the digits gives
        // each digit's run inside the block; the run goes to offs[digit, block] globally
        const int d = threadIdx.x;
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < kSortWaves; ++k) {
            const uint32_t c = wcnt[k][d];
            wcnt[k][d] = run;
            run += c;
        }
        uint32_t tot;
        const uint32_t excl = block_exclusive_scan(run, lds_w, &tot);
        dbase[d] = excl;
        gshift[d] = offs[br.hidx0 + (int64_t)d * br.hstride] - excl;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = wbase + it * kWave + lane;
        if (i < br.hi) {
            const uint32_t d = key_digit<KT>((KT)key[it], br.base, shift);
            const uint32_t lp = dbase[d] + wcnt[w][d] + rank[it];
            if (lp < (uint32_t)kSortTile) {   // always true when the counts agree
                skey[lp] = (KT)key[it];
                sval[lp] = val[it];
            }
        }
    }
    __syncthreads();
    // digit runs are contiguous in LDS and in the output: consecutive threads write
    // consecutive addresses within a run
    const int nloc = (int)(br.hi - br.lo);
    const int64_t n_out = segs ? (int64_t)segs[nseg].end : live_count(n_dev, cap, n_host);
    for (int i = threadIdx.x; i < nloc; i += kSortThreads) {
        const KT k = skey[i];
        const uint32_t pos = gshift[key_digit<KT>(k, br.base, shift)] + (uint32_t)i;
        if (pos < n_out) {   // always true when histogram and scatter agree
            if (kout) kout[pos] = k;
            vout[pos] = sval[i];
            // the tile a key names: local keys sit on the segment's base
            const int64_t gk = kLocal ? (int64_t)br.base + (int64_t)k : (int64_t)k;
            if (ranges && gk < nkeys) {
                if (i == 0 || skey[i - 1] != k) atomicMin(&ranges[2 * gk], pos);
                if (i == nloc - 1 || skey[i + 1] != k) atomicMax(&ranges[2 * gk + 1], pos + 1);
            }
        }
    }
}

__global__ void k_ranges_init(uint32_t *ranges, int64_t nkeys)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nkeys) reinterpret_cast<uint2 *>(ranges)[k] = make_uint2(0xFFFFFFFFu, 0u);
}

__global__ void k_ranges_finish(uint32_t *ranges, int64_t nkeys)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nkeys) return;
    uint2 r = reinterpret_cast<uint2 *>(ranges)[k];
    if (r.x == 0xFFFFFFFFu) reinterpret_cast<uint2 *>(ranges)[k] = make_uint2(0u, 0u);
}

static int64_t sort_blocks(int64_t items) { return (items + kSortTile - 1) / kSortTile; }

size_t radix_temp_bytes(int64_t max_items, int32_t max_segs)
{
    const int64_t nb = sort_blocks(max_items > 0 ? max_items : 1) + max_segs;
    const int64_t hist = 256 * nb;
    const int64_t parts = (hist + kSortTile - 1) / kSortTile + 1;
    return (size_t)(hist + parts) * sizeof(uint32_t) + 256 +
           (size_t)(max_segs + 1) * sizeof(SegDesc) + 256;
}

template <typename KT>
hipError_t radix_sort_pairs(KT *keys_a, uint32_t *vals_a, KT *keys_b,
                            uint32_t *vals_b, int64_t cap, const unsigned long long *n_dev,
                            int64_t n_host, int bits, void *temp, bool *result_in_b,
                            hipStream_t st, const SortSegments *seg)
{
    *result_in_b = false;
    const int64_t items = n_dev ? cap : n_host;
    const int32_t nseg = seg ? seg->nseg : 0;
    const int64_t nb = sort_blocks(items) + nseg;
    if (sort_blocks(items) == 0) {
        if (seg && seg->ranges && seg->nkeys > 0)
            return fill_u32(seg->ranges, 0u, 2 * seg->nkeys, st);
        return hipSuccess;
    }
    uint32_t *hist = reinterpret_cast<uint32_t *>(temp);
    const int64_t hlen = 256 * nb;
    const int64_t nparts = (hlen + kSortTile - 1) / kSortTile;
    uint32_t *parts = hist + hlen;
    SegDesc *segs = nullptr;
    if (seg) {
        const size_t off = ((size_t)(hlen + nparts + 1) * sizeof(uint32_t) + 255) & ~size_t(255);
        segs = reinterpret_cast<SegDesc *>(static_cast<char *>(temp) + off);
        hipLaunchKernelGGL(k_seg_table, dim3(1), dim3(kSegThreads), 0, st, seg->offs, seg->stride,
                           nseg, seg->views, n_dev, cap, segs);
        if (seg->ranges && seg->nkeys > 0)
            hipLaunchKernelGGL(k_ranges_init, dim3((unsigned)((seg->nkeys + 255) / 256)), dim3(256),
                               0, st, seg->ranges, seg->nkeys);
    }
    uint32_t *ranges = seg && seg->nkeys > 0 ? seg->ranges : nullptr;
    const int passes = bits <= 8 ? 1 : (bits + 7) / 8;   // one pass at least: ranges come from it
    KT *ki = keys_a, *ko = keys_b;
    uint32_t *vi = vals_a, *vo = vals_b;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        const int nbits = std::max(1, std::min(8, bits - shift));
        hipLaunchKernelGGL(k_radix_hist<KT>, dim3((unsigned)nb), dim3(kSortThreads), 0, st, ki, segs,
                           nseg, n_dev, cap, n_host, shift, hist);
        hipLaunchKernelGGL(k_hist_scan_reduce, dim3((unsigned)nparts), dim3(kSortThreads), 0,
                           st, hist, hlen, parts);
        hipLaunchKernelGGL(k_hist_scan_partials, dim3(1), dim3(kScanPartialsThreads), 0, st, parts,
                           nparts);
        hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nparts), dim3(kSortThreads), 0, st,
                           hist, hlen, parts, hist);
        // the keys of the last pass are not read again once the ranges are out
        const bool last = p == passes - 1;
        hipLaunchKernelGGL(k_radix_scatter<KT>, dim3((unsigned)nb), dim3(kSortThreads), 0, st, ki,
                           vi, last && ranges ? nullptr : ko, vo, hist, segs, nseg, n_dev, cap,
                           n_host, shift, nbits, last ? ranges : nullptr, seg ? seg->nkeys : 0);
        std::swap(ki, ko);
        std::swap(vi, vo);
        *result_in_b = !*result_in_b;
    }
    if (ranges)
        hipLaunchKernelGGL(k_ranges_finish, dim3((unsigned)((seg->nkeys + 255) / 256)), dim3(256),
                           0, st, ranges, seg->nkeys);
    return hipGetLastError();
}

template hipError_t radix_sort_pairs<uint32_t>(uint32_t *, uint32_t *, uint32_t *, uint32_t *, int64_t,
                                               const unsigned long long *, int64_t, int, void *, bool *,
                                               hipStream_t, const SortSegments *);
template hipError_t radix_sort_pairs<uint16_t>(uint16_t *, uint32_t *, uint16_t *, uint32_t *, int64_t,
                                               const unsigned long long *, int64_t, int, void *, bool *,
                                               hipStream_t, const SortSegments *);

}  // namespace ss
