// build.hip -- tree construction on gfx950.
//
// Sec. 3 builds the tree top-down: a large cube enclosing all particles is
// split recursively into eight boxes until each box holds at most leaf_cap
// particles.  Here the same tree is produced bottom-up and in parallel:
//   1. enclosing cube per cloud (min/max reduction, side 2^e),
//   2. keys: the octant digits of the recursive subdivision (Morton order),
//      or the same boxes numbered along a Hilbert curve,
//   3. stable LSD radix sort of (key, index), 8-bit digits; the last pass
//      also gathers x and q into the sorted order,
//   4. per sorted position: the level of the common prefix with the previous
//      key and the level of the leaf holding it; the nodes that start at a
//      position are the levels in between, so a scan numbers all nodes in
//      preorder (node order = (first particle, level)),
//   5. node records (box centre, side, first particle, level),
//   6. moments (Q, p, S about the box centre, FP64), one level per launch from
//      the deepest up: a leaf sums its particles, an internal node sums its
//      children in key order with the exact shift of origin; the same pass
//      finds each node's particle count, skip link (first node after the
//      subtree) and its children's parent,
//   7. walk groups (node groups or consecutive runs of G particles).
// Every kernel first checks the device flag word and does nothing once a
// problem (capacity, non-finite input, bad offsets) has been flagged.
#include "internal.h"

namespace ucp {

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t n)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double *p, double v, int64_t n)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
}
void launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
}
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_f64, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
}

__device__ __forceinline__ int block_excl_scan(int v, int *total);
__device__ __forceinline__ bool grid_barrier(unsigned long long *bar, unsigned long long target);

// per-build state: cloud extents, counters (the walk's included), the walk's
// queue heads, the sort's tickets, digit counts and the look-back words of
// the sort's first pass and of the node offsets (every block); then block 0
// moves the last build's flags that ucp_get_stats has not yet reported
// (flags[2] holds the reported ones) into the sticky word (flags[1], cleared
// only by ucp_get_stats) and clears the flag word, sets the cloud offsets ({0, n} for one cloud, or a
// checked copy of the caller's) and, for chunk groups (G > 0), the first
// chunk group of each cloud and their total
__global__ __launch_bounds__(kScanBlock) void k_build_reset(
    unsigned long long *mm, int clouds, unsigned long long *ctr, uint32_t *sortctl,
    uint32_t *ghist, uint32_t *status0, int64_t nstatus, unsigned long long *offstat,
    int64_t noffstat, const int64_t *__restrict__ src_off,
    int64_t n, int G, int64_t *off, int32_t *gcl, int32_t *goff_n, unsigned long long *wq,
    int32_t *flags)
{
    __shared__ int tot;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t0 < clouds * 6) mm[t0] = (t0 % 6 < 3) ? ~0ull : 0ull;
    if (t0 < CTR_NCTR) ctr[t0] = 0;
    if (t0 < kWalkQueues) wq[kQStride * t0] = 0;
    if (t0 < kSortTickets) sortctl[t0] = 0;
    if (t0 < kSortPassesMax * 256) ghist[t0] = 0;
    for (int64_t t = t0; t < nstatus; t += (int64_t)gridDim.x * blockDim.x) status0[t] = 0;
    for (int64_t t = t0; t < noffstat; t += (int64_t)gridDim.x * blockDim.x) offstat[t] = 0;
    if (blockIdx.x != 0) return;
    if (threadIdx.x == 0) {
        flags[1] |= flags[0] & ~flags[2];
        flags[0] = 0;
        flags[2] = 0;
    }
    __syncthreads();
    if (src_off) {
        for (int c = threadIdx.x; c <= clouds; c += blockDim.x) {
            const int64_t v = src_off[c];
            const bool bad = (c == 0 && v != 0) || (c == clouds && v != n) ||
                             (c > 0 && v < src_off[c - 1]) || v < 0 || v > n;
            off[c] = bad ? (c == 0 ? 0 : n) : v;
            if (bad) atomicOr(flags, UCP_FLAG_BAD_OFFSETS);
        }
    } else if (threadIdx.x == 0) {
        off[0] = 0;
        off[1] = n;
    }
    __syncthreads();
    if (G <= 0) return;
    // offsets that failed the check may decrease; their counts are clamped at
    // 0, and the group emission, which sees the flag, publishes no groups
    const int per = (clouds + kScanBlock - 1) / kScanBlock;
    const int c0 = min(clouds, (int)threadIdx.x * per), c1 = min(clouds, c0 + per);
    int mine = 0;
    for (int c = c0; c < c1; ++c)
        mine += (int)max<int64_t>(0, (off[c + 1] - off[c] + G - 1) / G);
    int run = block_excl_scan(mine, &tot);
    for (int c = c0; c < c1; ++c) {
        gcl[c] = run;
        run += (int)max<int64_t>(0, (off[c + 1] - off[c] + G - 1) / G);
    }
    if (threadIdx.x == 0) {
        gcl[clouds] = tot;
        *goff_n = tot;
    }
}

// ---------------------------------------------------------------------------
// 1. enclosing cube
// ---------------------------------------------------------------------------
constexpr int kCubeItems = 16;    // particles per thread; a block covers 256 * 16

__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// per block: min/max of its chunk, reduced through LDS, one atomic per
// component and cloud (a chunk that straddles clouds is reduced cloud by cloud)
__global__ __launch_bounds__(256) void k_cube_reduce(const double *__restrict__ x, int64_t n,
                                                    const int64_t *__restrict__ off, int clouds,
                                                    unsigned long long *mm, int32_t *flags)
{
    __shared__ double red[6][4];
    if (*flags) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * 256 * kCubeItems;
    const int64_t last = min(base + (int64_t)256 * kCubeItems, n) - 1;
    const int c0 = cloud_of(off, clouds, base), c1 = cloud_of(off, clouds, last);
    bool bad = false;
    // the chunk's particles cloud by cloud (a chunk may straddle clouds): per
    // cloud one block reduction and one atomic per component
    for (int c = c0; c <= c1; ++c) {
        const int64_t lo = max(base, off[c]), hi = min(last + 1, off[c + 1]);
        if (lo >= hi) continue;   // the same on every thread of the block
        double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int it = 0; it < kCubeItems; ++it) {
            const int64_t i = base + it * 256 + threadIdx.x;
            if (i >= lo && i < hi) {
                for (int d = 0; d < 3; ++d) {
                    const double v = x[3 * i + d];
                    bad |= !isfinite(v);
                    mn[d] = fmin(mn[d], v);
                    mx[d] = fmax(mx[d], v);
                }
            }
        }
        for (int d = 0; d < 3; ++d) {
            mn[d] = wave_min(mn[d]);
            mx[d] = wave_max(mx[d]);
        }
        if (lane == 0)
            for (int d = 0; d < 3; ++d) {
                red[d][w] = mn[d];
                red[3 + d][w] = mx[d];
            }
        __syncthreads();
        if (threadIdx.x < 6) {
            const int d = threadIdx.x;
            double v = red[d][0];
            for (int j = 1; j < 4; ++j) v = d < 3 ? fmin(v, red[d][j]) : fmax(v, red[d][j]);
            if (d < 3) atomicMin(&mm[6 * c + d], f64_ordered(v));
            else atomicMax(&mm[6 * c + d], f64_ordered(v));
        }
        __syncthreads();   // red is reused by the next cloud
    }
    if (bad) atomicOr(flags, UCP_FLAG_NONFINITE);
}

// lo = minimum corner; side L = 2^e, e the smallest integer with 2^e > extent
// (frexp gives extent = m 2^e with m in [1/2, 1)); e = 0 for a zero extent.
// the cube of cloud c from its reduced extents: origin lo (the AABB minimum),
// side 2^e with e the least integer such that 2^e exceeds the largest extent;
// c1 = (2^(b-e), e).  Returns false when e is out of range.
__device__ __forceinline__ bool cloud_cube(const unsigned long long *__restrict__ mm,
                                           const int64_t *__restrict__ off, int c, int b,
                                           double4 *c0, double4 *c1)
{
    const bool empty = off[c + 1] == off[c];
    double lo[3], ext = 0.0;
    for (int d = 0; d < 3; ++d) {
        lo[d] = empty ? 0.0 : f64_from_ordered(mm[6 * c + d]);
        double hi = empty ? 0.0 : f64_from_ordered(mm[6 * c + 3 + d]);
        double w = hi - lo[d];
        ext = w > ext ? w : ext;
    }
    int e = 0;
    if (ext > 0.0) frexp(ext, &e);
    *c0 = make_double4(lo[0], lo[1], lo[2], ldexp(1.0, e));
    *c1 = make_double4(ldexp(1.0, b - e), (double)e, 0.0, 0.0);
    return e >= -1000 && e <= 1000;
}

// ---------------------------------------------------------------------------
// 2. keys from the quantised coordinates X_d = min(floor((x_d - lo_d) 2^(b-e)),
//    2^b - 1).  Morton: bits of X, Y, Z interleaved x-major (octant digit =
//    4 xbit + 2 ybit + zbit).  Hilbert: Skilling's transform (AIP Conf. Proc.
//    707, 381 (2004)) turns (X, Y, Z) into the transposed Hilbert index, which
//    is then interleaved the same way; the top 3l bits still name the level-l
//    box, so everything downstream works on either.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t quantise(double v, double lo, double scale, uint64_t top)
{
    double t = (v - lo) * scale;
    if (!(t >= 0.0)) return 0;
    double f = floor(t);
    if (f >= (double)top) return top;
    return (uint64_t)f;
}

__device__ __forceinline__ uint64_t hilbert_key(uint32_t x, uint32_t y, uint32_t z, int b)
{
    // from the top bit down: where a coordinate has the bit set, the lower
    // bits of x are inverted, otherwise they are exchanged with that
    // coordinate's lower bits (a no-op for x itself)
    for (uint32_t Q = 1u << (b - 1); Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        x = (x & Q) ? x ^ P : x;
        uint32_t t = (x ^ y) & P;
        const bool fy = (y & Q) != 0;
        x ^= fy ? P : t;
        y ^= fy ? 0u : t;
        t = (x ^ z) & P;
        const bool fz = (z & Q) != 0;
        x ^= fz ? P : t;
        z ^= fz ? 0u : t;
    }
    // Gray code across the coordinates
    y ^= x;
    z ^= y;
    // then every bit j takes the parity of z's bits above j
    uint32_t w = z >> 1;
    w ^= w >> 1;
    w ^= w >> 2;
    w ^= w >> 4;
    w ^= w >> 8;
    w ^= w >> 16;
    x ^= w;
    y ^= w;
    z ^= w;
    return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

// Each thread derives its cloud's cube from the reduced extents (the same
// arithmetic for every thread of the cloud); the first threads also store
// every cloud's cube for the later kernels.
__global__ __launch_bounds__(256) void k_keys(const double *__restrict__ x,
                                             const double *__restrict__ q, int64_t n,
                                             const int64_t *__restrict__ off, int clouds,
                                             const unsigned long long *__restrict__ mm,
                                             double4 *cube, int b, int curve, uint64_t *key,
                                             uint32_t *val, double4 *xin, int32_t *flags)
{
    if (*flags) return;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t cc = i; cc < clouds; cc += (int64_t)gridDim.x * blockDim.x) {
        double4 a0, a1;
        if (!cloud_cube(mm, off, (int)cc, b, &a0, &a1)) atomicOr(flags, UCP_FLAG_BAD_CUBE);
        cube[2 * cc] = a0;
        cube[2 * cc + 1] = a1;
    }
    if (i >= n) return;
    int c = cloud_of(off, clouds, i);
    double4 c0, c1;
    cloud_cube(mm, off, c, b, &c0, &c1);
    uint64_t top = (1ull << b) - 1;
    const double x0 = x[3 * i + 0], x1 = x[3 * i + 1], x2 = x[3 * i + 2];
    uint64_t X = quantise(x0, c0.x, c1.x, top);
    uint64_t Y = quantise(x1, c0.y, c1.x, top);
    uint64_t Z = quantise(x2, c0.z, c1.x, top);
    key[i] = curve == UCP_CURVE_HILBERT ? hilbert_key((uint32_t)X, (uint32_t)Y, (uint32_t)Z, b)
                                        : (spread3(X) << 2) | (spread3(Y) << 1) | spread3(Z);
    val[i] = (uint32_t)i;
    // position and charge packed in one 32-byte record, so that gathering
    // them into the sorted order reads one record per particle
    xin[i] = make_double4(x0, x1, x2, q[i]);
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan of int32 (three kernels)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// block-wide exclusive scan (blockDim = kScanBlock); returns the exclusive
// prefix of v and writes the block total to *total.
__device__ __forceinline__ int block_excl_scan(int v, int *total)
{
    __shared__ int ws[kScanBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = wave_incl_scan(v);
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    if (w == 0) {
        int t = lane < kScanBlock / 64 ? ws[lane] : 0;
        int ti = wave_incl_scan(t);
        if (lane < kScanBlock / 64) ws[lane] = ti - t;
        if (lane == kScanBlock / 64 - 1) *total = ti;
    }
    __syncthreads();
    int r = ws[w] + inc - v;
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const int32_t *__restrict__ in,
                                                           int64_t n, int32_t *blk)
{
    __shared__ int tot;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanItems;
    int s = 0;
    for (int j = 0; j < kScanItems; ++j) {
        int64_t e = base + (int64_t)threadIdx.x * kScanItems + j;
        if (e < n) s += in[e];
    }
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_blocks(int32_t *blk, int nb)
{
    __shared__ int tot;
    int carry = 0;
    for (int base = 0; base < nb; base += kScanBlock) {
        int i = base + threadIdx.x;
        int v = i < nb ? blk[i] : 0;
        int ex = block_excl_scan(v, &tot);
        if (i < nb) blk[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_down(const int32_t *__restrict__ in,
                                                         int32_t *out, int64_t n,
                                                         const int32_t *__restrict__ blk)
{
    __shared__ int tot;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanItems;
    int v[kScanItems];
    int s = 0;
    for (int j = 0; j < kScanItems; ++j) {
        int64_t e = base + (int64_t)threadIdx.x * kScanItems + j;
        v[j] = e < n ? in[e] : 0;
        s += v[j];
    }
    int ex = block_excl_scan(s, &tot) + blk[blockIdx.x];
    for (int j = 0; j < kScanItems; ++j) {
        int64_t e = base + (int64_t)threadIdx.x * kScanItems + j;
        if (e < n) out[e] = ex;
        ex += v[j];
    }
}

// one block scans a short array whose length is a multiple of 4: thread j
// holds elements [64 j, 64 j + 64) in registers (16-byte loads), the thread
// sums are scanned across the block, and the prefixes are written back
__global__ __launch_bounds__(kScanBlock) void k_scan_small(const int4 *__restrict__ in, int4 *out,
                                                          int n4)
{
    __shared__ int tot;
    constexpr int V = kScanSmallItems / 4;
    const int b0 = threadIdx.x * V;
    int4 v[V];
    int sum = 0;
#pragma unroll
    for (int j = 0; j < V; ++j) {
        v[j] = b0 + j < n4 ? in[b0 + j] : make_int4(0, 0, 0, 0);
        sum += v[j].x + v[j].y + v[j].z + v[j].w;
    }
    int ex = block_excl_scan(sum, &tot);
#pragma unroll
    for (int j = 0; j < V; ++j) {
        int4 o;
        o.x = ex;
        o.y = o.x + v[j].x;
        o.z = o.y + v[j].y;
        o.w = o.z + v[j].z;
        ex = o.w + v[j].w;
        if (b0 + j < n4) out[b0 + j] = o;
    }
}

static void scan_excl(const int32_t *in, int32_t *out, int64_t n, int32_t *blk, hipStream_t s)
{
    if (n <= kScanSmallLimit && n % 4 == 0) {
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kScanBlock), 0, s, (const int4 *)in,
                           (int4 *)out, (int)(n / 4));
        return;
    }
    const int64_t per = (int64_t)kScanBlock * kScanItems;
    int nb = (int)((n + per - 1) / per);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanBlock), 0, s, in, n, blk);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanBlock), 0, s, blk, nb);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanBlock), 0, s, in, out, n,
                       (const int32_t *)blk);
}

// ---------------------------------------------------------------------------
// 3. stable sort of (key, index): ordered by key, equal keys by index.
//    Stable LSD radix passes with 8-bit digits run over the top three (four
//    above 2^20 particles) digits of the key only, and then over the cloud
//    digits of a multi-cloud build, which restores the clouds' contiguity
//    while keeping the order inside each cloud.  After them, the elements of
//    a run of equal top digits lie together in index order, and one kernel
//    finishes the order inside every run by ranking (k_sort_finish, which
//    also gathers x and q).  The top three digits name boxes of level 7-8, so
//    runs are short for the clouds this library is for; a run longer than
//    kFinishMax raises a word that
//    turns on the full sort queued behind (all digits, least significant
//    first, from the keys in input order), whose passes otherwise return at
//    once.
//    The digit counts of every pass are found first, in one kernel (they do
//    not depend on the order).  Each pass is one kernel: a tile of kSortTile
//    elements (twice that above kSortWideN particles) is ranked (inside a
//    round of kSortThreads each wave ranks equal digits with ballots, and the
//    waves and rounds are ordered through LDS),
//    its digit counts are published, its digit prefixes over the earlier
//    tiles are found by a decoupled look-back, and the tile is scattered.
// ---------------------------------------------------------------------------
template <bool CLOUD>
__device__ __forceinline__ uint32_t sort_digit(uint64_t k, uint32_t v, int shift,
                                               const int64_t *__restrict__ off, int clouds)
{
    if (CLOUD) return ((uint32_t)cloud_of(off, clouds, v) >> shift) & 255u;
    return (uint32_t)(k >> shift) & 255u;
}

// digit counts of all passes: key passes first, then cloud passes (the
// values are still the identity here, so element e is particle e)
__global__ __launch_bounds__(kSortThreads) void k_radix_counts(
    const uint64_t *__restrict__ key, int64_t n, int key_passes, int cloud_passes,
    const int64_t *__restrict__ off, int clouds, uint32_t *ghist, const int32_t *flags)
{
    __shared__ uint32_t h[kSortPassesMax * 256];
    if (*flags) return;
    const int np = key_passes + cloud_passes;
    for (int j = threadIdx.x; j < np * 256; j += kSortThreads) h[j] = 0;
    __syncthreads();
    for (int64_t e = blockIdx.x * (int64_t)kSortThreads + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kSortThreads) {
        const uint64_t k = key[e];
        for (int ps = 0; ps < key_passes; ++ps)
            atomicAdd(&h[ps * 256 + (uint32_t)((k >> (8 * ps)) & 255u)], 1u);
        if (cloud_passes > 0) {
            const uint32_t cl = (uint32_t)cloud_of(off, clouds, e);
            for (int ps = 0; ps < cloud_passes; ++ps)
                atomicAdd(&h[(key_passes + ps) * 256 + ((cl >> (8 * ps)) & 255u)], 1u);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < np * 256; j += kSortThreads)
        if (h[j] != 0) atomicAdd(&ghist[j], h[j]);
}

// Status word of a (tile, digit): flag (2 bits) | count (30 bits).  A tile
// publishes its own count at once (flag AGG), then walks back over the earlier
// tiles adding published counts until one of them has published its inclusive
// prefix (flag INCL), and publishes its own.  Blocks take tiles in the order
// they start (a ticket), so a tile only waits for tiles that started before
// it and that publish before waiting: every wait ends.  A bounded spin turns a
// lost tile into an internal-error flag rather than a hang.
constexpr uint32_t kStAgg = 1u << 30, kStIncl = 2u << 30, kStMask = (1u << 30) - 1;
constexpr int kLookbackSpin = 1 << 18;
// look-back width: four lanes per digit, each reading kLbSeg consecutive
// earlier tiles per round, so a round covers 4 * kLbSeg tiles
constexpr int kLbSeg = 4;
static_assert(kSortThreads == 4 * 256, "the look-back takes four lanes per digit");

// LDS of one tile of a pass, ITEMS rounds of kSortThreads elements
template <int ITEMS>
struct SortLdsT {
    uint32_t wh[ITEMS][kSortThreads / 64][256];   // per-(round, wave) digit counts, then offsets
    uint32_t boff[256], rsh[256], bsh[256];
    int btot, tile_sh;
};
using SortLds = SortLdsT<kSortItems>;
// The passes of a build of more than kSortWideN particles take tiles of
// kSortWideItems rounds: half as many tiles, so the look-backs are
// half as long, while there are still more tiles than CUs (N = 4,194,304:
// 1024 tiles of 4096 keys).  Below it the tiles of kSortItems rounds keep
// every CU busy.  Status words stay laid out per tile of kSortTile elements
// (that is what the gated full sort uses), so a pass over wide tiles clears
// the next pass's words of every small tile it covers.
constexpr int kSortWideItems = 2 * kSortItems;
constexpr int64_t kSortWideN = int64_t(1) << 20;

// One tile of a pass: ranked, its counts published, its prefixes found by the
// look-back, scattered.  `below` is, on thread tid < 256, the exclusive prefix
// of digit tid over the pass's digit totals; L.wh is zero on entry.
template <bool CLOUD, int ITEMS>
__device__ __forceinline__ void radix_tile(
    SortLdsT<ITEMS> &L, int tile, int below, const uint64_t *__restrict__ kin,
    const uint32_t *__restrict__ vin, uint64_t *kout, uint32_t *vout, int64_t n, int shift,
    const int64_t *__restrict__ off, int clouds, uint32_t *status, uint32_t *status_next,
    const double4 *__restrict__ xin, double4 *xq, int32_t *flags)
{
    constexpr int NW = kSortThreads / 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t base = (int64_t)tile * (kSortThreads * ITEMS);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t k[ITEMS];
    uint32_t v[ITEMS], d[ITEMS], lrank[ITEMS];
    bool valid[ITEMS];
    double4 g[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int64_t e = base + it * kSortThreads + tid;
        valid[it] = e < n;
        k[it] = valid[it] ? kin[e] : 0ull;
        v[it] = valid[it] ? vin[e] : 0u;
        d[it] = valid[it] ? sort_digit<CLOUD>(k[it], v[it], shift, off, clouds) : 0u;
    }
    // the last pass also gathers each particle's position and charge into the
    // sorted order; the loads are issued here so that they overlap the ranking
    // and the look-back
    if (xq) {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int64_t i = v[it];
            const bool in = valid[it] && i < n;   // always, unless the records are inconsistent
            if (valid[it] && !in) atomicOr(flags, UCP_FLAG_INTERNAL);
            g[it] = in ? xin[i] : make_double4(0.0, 0.0, 0.0, 0.0);
        }
    }
    // rank equal digits inside each wave and round
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        uint64_t peers = __ballot(valid[it]);
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __ballot((d[it] >> bit) & 1u);
            peers &= ((d[it] >> bit) & 1u) ? bb : ~bb;
        }
        lrank[it] = (uint32_t)__popcll(peers & lt);
        if (valid[it] && lrank[it] == 0) L.wh[it][w][d[it]] = (uint32_t)__popcll(peers);
    }
    __syncthreads();
    if (tid < 256) {
        // the tile's count of digit tid, and each (round, wave)'s offset inside it
        uint32_t r = 0;
        for (int it = 0; it < ITEMS; ++it)
            for (int ww = 0; ww < NW; ++ww) {
                const uint32_t c = L.wh[it][ww][tid];
                L.wh[it][ww][tid] = r;
                r += c;
            }
        // publish the tile's count at once (tile 0's is already inclusive)
        __hip_atomic_store(status + (int64_t)tile * 256 + tid, (tile == 0 ? kStIncl : kStAgg) | r,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        L.rsh[tid] = r;
        L.bsh[tid] = (uint32_t)below;
        // the next pass's status words, for every tile of kSortTile elements
        // that this tile covers
#pragma unroll
        for (int h = 0; h < ITEMS / kSortItems; ++h)
            status_next[((int64_t)tile * (ITEMS / kSortItems) + h) * 256 + tid] = 0u;
    }
    __syncthreads();
    // look-back over the earlier tiles' published words, four lanes per digit
    // (lane q4 of the group takes tiles j - 4 q4 .. j - 4 q4 - 3 of a round): a
    // round adds the counts up to the first inclusive prefix it meets, or all
    // 4 kLbSeg of them and moves on; a round that meets an unpublished word
    // before that prefix is read again.  Before tile 0 the prefix is 0.
    {
        const int dg = tid >> 2, q4 = tid & 3;
        uint32_t excl = 0;
        if (tile > 0) {
            int j = tile - 1, spins = 0;
            for (;;) {
                uint32_t sv[kLbSeg];
#pragma unroll
                for (int m = 0; m < kLbSeg; ++m) {
                    const int jj = j - q4 * kLbSeg - m;
                    sv[m] = jj >= 0 ? __hip_atomic_load(status + (int64_t)jj * 256 + dg,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                    : kStIncl;
                }
                bool ok = true, found = false;
                uint32_t sum = 0;
#pragma unroll
                for (int m = 0; m < kLbSeg; ++m)
                    if (!found) {
                        ok = ok && (sv[m] & ~kStMask) != 0;
                        sum += sv[m] & kStMask;
                        found = (sv[m] & kStIncl) != 0;
                    }
                const int sh = lane & ~3;
                const uint32_t gf = (uint32_t)(__ballot(found) >> sh) & 0xFu;
                const uint32_t go = (uint32_t)(__ballot(ok) >> sh) & 0xFu;
                const int f = gf ? __builtin_ctz(gf) : 4;   // first lane that met a prefix
                const uint32_t need = f == 4 ? 0xFu : ((2u << f) - 1u);
                if ((go & need) != need) {
                    if (++spins > kLookbackSpin) {
                        atomicOr(flags, q4 == 0 ? UCP_FLAG_INTERNAL : 0);
                        break;
                    }
                    continue;
                }
                uint32_t add = q4 <= f ? sum : 0u;
                add += __shfl_xor(add, 1);
                add += __shfl_xor(add, 2);
                excl += add;
                if (f < 4) break;
                j -= 4 * kLbSeg;
            }
        }
        if (q4 == 0) {
            if (tile > 0)
                __hip_atomic_store(status + (int64_t)tile * 256 + dg, kStIncl | (excl + L.rsh[dg]),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            L.boff[dg] = L.bsh[dg] + excl;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITEMS; ++it)
        if (valid[it]) {
            const uint32_t dst = L.boff[d[it]] + L.wh[it][w][d[it]] + lrank[it];
            if ((int64_t)dst >= n) {   // only inconsistent prefixes lead here
                atomicOr(flags, UCP_FLAG_INTERNAL);
                continue;
            }
            kout[dst] = k[it];
            vout[dst] = v[it];
            if (xq) xq[dst] = g[it];
        }
}

// one pass, one tile of ITEMS rounds per block
template <bool CLOUD, int ITEMS>
__global__ __launch_bounds__(kSortThreads) void k_radix_pass(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *kout,
    uint32_t *vout, int64_t n, int shift, const int64_t *__restrict__ off, int clouds,
    const uint32_t *__restrict__ ghist, uint32_t *status, uint32_t *status_next,
    uint32_t *ticket, const double4 *__restrict__ xin, double4 *xq, int32_t *flags)
{
    __shared__ SortLdsT<ITEMS> L;
    if (*flags) return;
    const int tid = threadIdx.x;
    if (tid == 0) L.tile_sh = (int)atomicAdd(ticket, 1u);
    for (int j = tid; j < ITEMS * (kSortThreads / 64) * 256; j += kSortThreads)
        (&L.wh[0][0][0])[j] = 0;
    // digit totals of this pass and their exclusive prefix over the digits
    const uint32_t tot = tid < 256 ? ghist[tid] : 0u;
    const int below = block_excl_scan((int)tot, &L.btot);   // synchronises the block
    radix_tile<CLOUD, ITEMS>(L, L.tile_sh, below, kin, vin, kout, vout, n, shift, off, clouds,
                             status, status_next, xin, xq, flags);
}

// The passes of the full sort behind the finish, in one launch whose blocks
// are all resident at once: every block takes tiles of 4096 keys by ticket,
// pass after pass, with a grid barrier between passes (a tile's look-back
// then only waits for tiles of running blocks).  The whole launch returns at
// once unless the finish raised the gate, so the common build pays one empty
// launch.  Tiles of 4096 keys measured 212 us per full sort at N = 524,288
// against 254 us for 2048 (and 327 us with one block per CU instead of half
// as many: the grid barriers cost more than the shorter rounds save).
struct SortPassArgs {
    const uint64_t *kin;
    const uint32_t *vin;
    uint64_t *kout;
    uint32_t *vout;
    const uint32_t *ghist;
    uint32_t *status, *status_next, *ticket;
    double4 *xq;   // the last pass gathers x and q
    int shift, cloud;
};
struct SortPlan {
    SortPassArgs p[kSortPassesMax];
    int npass;
};

__global__ __launch_bounds__(kSortThreads) void k_sort_full(
    const SortPlan plan, int64_t n, const int64_t *__restrict__ off, int clouds,
    const double4 *__restrict__ xin, const unsigned long long *__restrict__ gate,
    unsigned long long *bar, int32_t *flags)
{
    __shared__ SortLdsT<kSortWideItems> L;
    __shared__ int go_s;
    const int tid = threadIdx.x;
    if (tid == 0) go_s = *gate != 0ull && *flags == 0;
    __syncthreads();
    if (!go_s) return;
    constexpr int kWide = kSortThreads * kSortWideItems;   // keys per tile
    const int ntiles = (int)((n + kWide - 1) / kWide);
    unsigned long long target = 0;
    bool wait = true;
    for (int ip = 0; ip < plan.npass; ++ip) {
        const SortPassArgs &P = plan.p[ip];
        const uint32_t tot = tid < 256 ? P.ghist[tid] : 0u;
        const int below = block_excl_scan((int)tot, &L.btot);
        for (;;) {
            if (tid == 0) L.tile_sh = (int)atomicAdd(P.ticket, 1u);
            for (int j = tid; j < kSortWideItems * (kSortThreads / 64) * 256; j += kSortThreads)
                (&L.wh[0][0][0])[j] = 0;
            __syncthreads();
            const int tile = L.tile_sh;
            if (tile >= ntiles) break;   // the same on every thread of the block
            if (P.cloud)
                radix_tile<true, kSortWideItems>(L, tile, below, P.kin, P.vin, P.kout, P.vout, n,
                                             P.shift, off, clouds, P.status, P.status_next, xin,
                                             P.xq, flags);
            else
                radix_tile<false, kSortWideItems>(L, tile, below, P.kin, P.vin, P.kout, P.vout, n,
                                              P.shift, off, clouds, P.status, P.status_next, xin,
                                              P.xq, flags);
            __syncthreads();
        }
        // every block passes every barrier, so that the count of arrivals
        // stays exact; a wait that times out flags the build and stops waiting
        if (ip + 1 < plan.npass && wait) {
            target += gridDim.x;
            if (!grid_barrier(bar, target)) {
                if (tid == 0) atomicOr(flags, UCP_FLAG_INTERNAL);
                wait = false;
            }
        }
    }
}
// The runs of equal top digits (bits from `shift` up, inside one cloud) after
// the passes over those digits: an element's place in its run is the number
// of elements of the run with a smaller key, or with an equal key and an
// earlier position (an earlier index: the passes were stable).  The run is
// scanned outwards from the element, four keys per round of loads, counting
// as it goes; a run longer than kFinishMax is not ranked but raises `full`,
// the word that gates the full sort.  The kernel writes the sorted keys and
// indices and gathers x and q.  Ranking costs each element the length of its
// run, so the limit is kept low: the longest runs of the initial clouds here
// hold 3-27 particles, while a cloud whose cube has grown (electrons thrown
// out by unresolved encounters) has many runs of hundreds to thousands, for
// which one full sort is cheaper (N = 4,194,304 after 50 steps: the finish
// took 2.4 ms with a limit of 2048, 0.16 ms with 256, the full sort 1.1 ms).
constexpr int kFinishMax = 256;
constexpr int kFinishThreads = 256, kFinishHalo = 64;   // keys staged in LDS on either side
__global__ __launch_bounds__(kFinishThreads) void k_sort_finish(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *kout,
    uint32_t *vout, int64_t n, int shift, const int64_t *__restrict__ off, int clouds,
    const double4 *__restrict__ xin, double4 *xq, unsigned long long *full, int32_t *flags)
{
    __shared__ uint64_t sk[kFinishThreads + 2 * kFinishHalo];
    if (*flags) return;
    const int64_t base = blockIdx.x * (int64_t)kFinishThreads;
    const int64_t wlo = base - kFinishHalo, whi = base + kFinishThreads + kFinishHalo;
    for (int t = threadIdx.x; t < kFinishThreads + 2 * kFinishHalo; t += kFinishThreads) {
        const int64_t q = wlo + t;
        sk[t] = q >= 0 && q < n ? kin[q] : 0ull;
    }
    __syncthreads();
    const int64_t p = base + threadIdx.x;
    if (p >= n) return;
    // key at position q (q inside the cloud): from LDS inside the window
    auto key = [&](int64_t q) -> uint64_t { return q >= wlo && q < whi ? sk[q - wlo] : kin[q]; };
    const int c = cloud_of(off, clouds, p);
    const int64_t c0 = off[c], c1 = off[c + 1];
    const uint64_t k = sk[p - wlo];
    const uint64_t top = k >> shift;
    // the top digits do not decrease inside a cloud, so equal tops at p and
    // p -+ kFinishMax mean a run longer than kFinishMax
    if ((p - kFinishMax >= c0 && (kin[p - kFinishMax] >> shift) == top) ||
        (p + kFinishMax < c1 && (kin[p + kFinishMax] >> shift) == top)) {
        *full = 1ull;
        return;
    }
    // earlier members (m of them): ranked before p when their key is not
    // larger; later members: when their key is smaller
    int64_t r = 0, m = 0;
    for (int64_t q = p - 1; q >= c0; --q) {
        const uint64_t kq = key(q);
        if ((kq >> shift) != top) break;
        r += kq <= k ? 1 : 0;
        ++m;
    }
    for (int64_t q = p + 1; q < c1; ++q) {
        const uint64_t kq = key(q);
        if ((kq >> shift) != top) break;
        r += kq < k ? 1 : 0;
    }
    const int64_t d = p - m + r;   // the run starts m positions before p
    const uint32_t v = vin[p];
    kout[d] = k;
    vout[d] = v;
    const int64_t i = v;
    if (i >= n) {   // only inconsistent records lead here
        atomicOr(flags, UCP_FLAG_INTERNAL);
        return;
    }
    xq[d] = xin[i];
}

// ---------------------------------------------------------------------------
// 4. per-position levels.
//    L(p): number of leading key digits shared with position p-1 (-1 at a
//    cloud edge).  A boundary at level l lies before p iff L(p) < l.
//    leaf(p): smallest level l at which the box holding p has <= leaf_cap
//    particles (b if none) -- found from running minima of L over the
//    leaf_cap positions on either side of p.
//    nodes starting at p: levels L(p)+1 .. leaf(p).
// ---------------------------------------------------------------------------
constexpr int kLvlTile = 256;

__device__ __forceinline__ int lcp_level(uint64_t a, uint64_t b2, int b)
{
    uint64_t x = a ^ b2;
    if (x == 0) return b;
    int lz = __clzll((long long)x) - (64 - 3 * b);
    return lz / 3;
}

__global__ __launch_bounds__(kLvlTile) void k_levels(const uint64_t *__restrict__ key, int64_t n,
                                                    const int64_t *__restrict__ off, int clouds,
                                                    int b, int cap, int8_t *Lout, int8_t *leafout,
                                                    int32_t *cnt, int32_t *lend, int32_t *blkmax,
                                                    const int32_t *flags)
{
    __shared__ int8_t sL[kLvlTile + 2 * kMaxLeafCap + 2];
    __shared__ int8_t sBM[kMaxLeafCap * kLvlTile];   // BM[j] of thread x at [j][x]
    __shared__ int wmax[kLvlTile / kWave];
    const int64_t base = (int64_t)blockIdx.x * kLvlTile;
    const int64_t wlo = base - cap;                 // sL[j - wlo] = L(j)
    const int wn = kLvlTile + 2 * cap + 1;
    const bool stop = *flags != 0;
    for (int t = threadIdx.x; t < wn; t += kLvlTile) {
        int64_t j = wlo + t;
        int v = -1;
        if (!stop && j > 0 && j < n) {
            int c1 = cloud_of(off, clouds, j);
            if (off[c1] != j) v = lcp_level(key[j - 1], key[j], b);
        }
        sL[t] = (int8_t)v;
    }
    __syncthreads();
    const int64_t p = base + threadIdx.x;
    int leaf = 0;   // deepest leaf level over the block, reduced below
    if (p < n && !stop) {
        auto Lw = [&](int64_t j) -> int { return (int)sL[j - wlo]; };
        // The box of level l holding p starts j* positions back (the first
        // j >= 0 with L(p - j) < l) and ends i* positions on (the first i >= 1
        // with L(p + i) < l); it holds at most cap particles iff j* + i* <= cap.
        // With BM[j] the least L over p - j .. p and FM[i] the least L over
        // p + 1 .. p + i, both non-increasing, that holds iff l > M with
        // M = min over j in [0, cap) of max(BM[j], FM[cap - j]).  The leaf is the
        // least such level, else the deepest.
        int run = 127;
        for (int j = 0; j < cap; ++j) {
            run = min(run, Lw(p - j));
            sBM[j * kLvlTile + threadIdx.x] = (int8_t)run;
        }
        int M = 127, fm = 127;
        for (int i = 1; i <= cap; ++i) {
            fm = min(fm, Lw(p + i));
            M = min(M, max((int)sBM[(cap - i) * kLvlTile + threadIdx.x], fm));
        }
        leaf = min(M + 1, b);
        int64_t tleaf = -1;   // -1: a max-depth leaf beyond the window, found by a scan
        if (M + 1 <= b) {
            int64_t t = p + 1;
            while (Lw(t) >= leaf) ++t;   // i* <= cap - j*, inside the window
            tleaf = t;
        }
        const int Lp = Lw(p);
        Lout[p] = (int8_t)Lp;
        leafout[p] = (int8_t)leaf;
        cnt[p] = leaf > Lp ? leaf - Lp : 0;
        lend[p] = (int32_t)tleaf;
    } else if (p <= n) {
        cnt[p] = 0;
        Lout[p] = -1;
        if (p < n) leafout[p] = -1;
    }
    // every position lies in one leaf, whose level its leaf(p) is
    for (int o = kWave / 2; o > 0; o >>= 1) leaf = max(leaf, __shfl_xor(leaf, o));
    if ((threadIdx.x & (kWave - 1)) == 0) wmax[threadIdx.x / kWave] = leaf;
    __syncthreads();
    if (threadIdx.x == 0) {
        int bm = 0;
        for (int w = 0; w < kLvlTile / kWave; ++w) bm = max(bm, wmax[w]);
        blkmax[blockIdx.x] = bm;
    }
}

// ---------------------------------------------------------------------------
// 5. node records: the nodes starting at position p are the boxes of levels
//    L(p)+1 .. leaf(p) holding p, numbered noff[p] + (l - L(p) - 1) in
//    preorder.  One kernel finds noff (below) and writes what follows from p
//    and l alone (box centre, side^2, first particle, level and leaf flag);
//    the box's integer coordinates are those of particle p, quantised again
//    exactly as the keys were, so no key is decoded and either curve works.
//    The particle count, the skip link and the parent of an internal node
//    are found by the moments pass below.
// ---------------------------------------------------------------------------
// The node offsets noff (the exclusive prefix of the per-position node
// counts) and the deepest leaf level come from one pass over tiles of
// kOffTile positions: a tile sums its counts and takes the maximum of its
// level blocks' deepest leaves, publishes both at once (kOffAgg), combines
// the earlier tiles' words, 64 at a time, back to the nearest one that holds
// the inclusive totals (kOffIncl) and publishes its own.  Tiles are taken in
// the order blocks start (a ticket), so every wait ends; a bounded spin
// turns a lost tile into an internal-error flag.  Word: flag (bits 62-63) |
// deepest level (bits 32-39) | count (bits 0-31).  The tile then writes the
// records of the nodes starting at its positions.
constexpr int kOffThreads = kScanBlock, kOffItems = 4, kOffTile = kOffThreads * kOffItems;
constexpr unsigned long long kOffAgg = 1ull << 62, kOffIncl = 2ull << 62;
static_assert(kOffTile % kLvlTile == 0, "a tile holds whole level blocks");

__global__ __launch_bounds__(kOffThreads) void k_offsets_nodes(
    const int32_t *__restrict__ cnt, const int32_t *__restrict__ blkmax, int nlvlblk,
    const double4 *__restrict__ xq, int64_t n, const int64_t *__restrict__ off, int clouds,
    const double4 *__restrict__ cube, int b, const int8_t *__restrict__ Lv,
    const int8_t *__restrict__ Lf, int64_t node_cap, int32_t *noff, double4 *ngeo, int4 *ninfo,
    int32_t *npar, uint8_t *nlev, unsigned long long *stat, unsigned long long *ctr,
    int32_t *flags)
{
    __shared__ int tile_s, tot_s, lmax_s;
    __shared__ unsigned long long excl_s;
    if (threadIdx.x == 0) tile_s = (int)atomicAdd(&ctr[CTR_OFFTICKET], 1ull);
    __syncthreads();
    const int tile = tile_s;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int64_t p0 = (int64_t)tile * kOffTile + kOffItems * threadIdx.x;
    int c[kOffItems];
    int mine = 0;
#pragma unroll
    for (int u = 0; u < kOffItems; ++u) {
        c[u] = p0 + u <= n ? cnt[p0 + u] : 0;
        mine += c[u];
    }
    // deepest leaf of the tile's level blocks
    int lm = 0;
    {
        const int64_t lb = (int64_t)tile * (kOffTile / kLvlTile) + threadIdx.x;
        if (threadIdx.x < kOffTile / kLvlTile && lb < nlvlblk) lm = blkmax[lb];
        for (int o = kWave / 2; o > 0; o >>= 1) lm = max(lm, __shfl_xor(lm, o));
    }
    int tot;
    const int ex = block_excl_scan(mine, &tot_s);   // barriers inside
    tot = tot_s;
    if (threadIdx.x == 0) {
        lmax_s = lm;   // wave 0 holds the level blocks
        __hip_atomic_store(stat + tile,
                           (tile == 0 ? kOffIncl : kOffAgg) | ((unsigned long long)(lm & 255) << 32) |
                               (uint32_t)tot,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // wave 0: the totals of the earlier tiles
    if (wv == 0) {
        unsigned long long cs = 0;
        int ms = 0;
        bool bad = false;
        for (int64_t j = (int64_t)tile - 1; j >= 0 && !bad; j -= kWave) {
            const int64_t jj = j - lane;
            unsigned long long w = jj >= 0 ? __hip_atomic_load(stat + jj, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT)
                                          : kOffIncl;
            int spins = 0;
            while (__ballot((w >> 62) == 0ull) != 0ull) {
                if (++spins > kLookbackSpin) {
                    bad = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                if ((w >> 62) == 0ull)
                    w = __hip_atomic_load(stat + jj, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (bad) break;
            // the words up to the nearest inclusive one (going back)
            const unsigned long long inc = __ballot((w >> 62) == 2ull);
            const int first = inc != 0ull ? __builtin_ctzll(inc) : kWave - 1;
            unsigned long long cc = lane <= first ? (w & 0xffffffffull) : 0ull;
            int mm = lane <= first ? (int)((w >> 32) & 255ull) : 0;
            for (int o = kWave / 2; o > 0; o >>= 1) {
                cc += __shfl_xor(cc, o);
                mm = max(mm, __shfl_xor(mm, o));
            }
            cs += cc;
            ms = max(ms, mm);
            if (inc != 0ull) break;
        }
        if (lane == 0) {
            if (bad) atomicOr(flags, UCP_FLAG_INTERNAL);
            excl_s = cs;
            const unsigned long long cin = cs + (unsigned long long)tot;
            const int min_ = max(ms, lmax_s);
            if (tile > 0)
                __hip_atomic_store(stat + tile,
                                   kOffIncl | ((unsigned long long)(min_ & 255) << 32) |
                                       (uint32_t)cin,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // the tile holding position n has the totals
            const int64_t tb = (int64_t)tile * kOffTile;
            if (tb <= n && n < tb + kOffTile) {
                ctr[CTR_MAXLEVEL] = (unsigned long long)min_;
                if (cin > (unsigned long long)node_cap) atomicOr(flags, UCP_FLAG_NODE_OVERFLOW);
            }
        }
    }
    __syncthreads();
    const int64_t k0t = (int64_t)excl_s + ex;
    int64_t kk = k0t;
#pragma unroll
    for (int u = 0; u < kOffItems; ++u) {
        if (p0 + u <= n) noff[p0 + u] = (int32_t)kk;
        kk += c[u];
    }
    // the records of the nodes starting at this thread's positions
    if (*flags) return;
    kk = k0t;
    for (int u = 0; u < kOffItems; ++u) {
        const int64_t p = p0 + u;
        const int k0 = (int)kk;
        kk += c[u];
        if (p >= n || c[u] == 0) continue;
        if (kk > node_cap) return;   // flagged by the tile holding position n
        const int Lp = Lv[p], lf = Lf[p];
        const int cl = cloud_of(off, clouds, p);
        const double4 xp = xq[p];
        const double4 c0 = cube[2 * cl], c1 = cube[2 * cl + 1];
        const int e = (int)c1.y;
        const uint64_t top = (1ull << b) - 1;
        const uint64_t X = quantise(xp.x, c0.x, c1.x, top), Y = quantise(xp.y, c0.y, c1.x, top),
                       Z = quantise(xp.z, c0.z, c1.x, top);
        for (int l = Lp + 1; l <= lf; ++l) {
            const int k = k0 + (l - Lp - 1);
            // box centre c_d = lo_d + (2 k_d + 1) 2^(e - l - 1); the product is exact
            const double h = ldexp(1.0, e - l - 1);
            const double cx = c0.x + (double)(2 * (X >> (b - l)) + 1) * h;
            const double cy = c0.y + (double)(2 * (Y >> (b - l)) + 1) * h;
            const double cz = c0.z + (double)(2 * (Z >> (b - l)) + 1) * h;
            ngeo[k] = make_double4(cx, cy, cz, ldexp(1.0, 2 * (e - l)));
            ninfo[k] = make_int4((int)p, 0, 0, l | (l == lf ? 256 : 0));
            nlev[k] = (uint8_t)(l | (l == lf ? kLeafBit : 0));
            if (l == 0) npar[k] = -1;   // other parents are set by the moments pass
        }
    }
}

// ---------------------------------------------------------------------------
// 6. moments about the box centre: the node (p, l) exists iff
//    L(p) < l <= leaf(p).  A leaf holds the positions p .. t-1 with t the
//    first later position whose L(t) < l (L is -1 at every cloud edge and at
//    n); it sums its particles (6a).  The range and children of an internal
//    node follow from the levels alone; a node of up to direct_max particles
//    sums its particles too (6b), a larger one sums its children's moments
//    with the exact shift of origin, from the deepest up (6c).
//    Every node records its count and its skip link noff[t]; every node but
//    a root records its parent.
//    Record per node, FP64 (16 doubles): cx cy cz Q px py pz trS Sxx Syy Szz
//    Sxy Sxz Syz 0 0; FP32 copy in the second line of the walk record:
//    Q px py pz, 1.5 trS 3Sxx 3Syy 3Szz, 3Sxy 3Sxz 3Syz 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void store_moments(double *mom64, float4 *nrec, int k, const double4 &g,
                                              const double *m)
{
    // m: Q, px, py, pz, Sxx, Syy, Szz, Sxy, Sxz, Syz
    const double trS = m[4] + m[5] + m[6];
    const double rec[16] = {g.x, g.y, g.z, m[0], m[1], m[2], m[3], trS,
                            m[4], m[5], m[6], m[7], m[8], m[9], 0.0, 0.0};
    double2 *d2 = (double2 *)(mom64 + 16 * (int64_t)k);
    for (int i = 0; i < 8; ++i) d2[i] = make_double2(rec[2 * i], rec[2 * i + 1]);
    // FP32 line of the walk record: Q, p, 1.5 trS and 3S (the factors the
    // expansion applies, folded in once per node)
    float4 *f4 = nrec + 8 * (int64_t)k + 4;
    f4[0] = make_float4((float)m[0], (float)m[1], (float)m[2], (float)m[3]);
    f4[1] = make_float4((float)(1.5 * trS), (float)(3.0 * m[4]), (float)(3.0 * m[5]),
                        (float)(3.0 * m[6]));
    f4[2] = make_float4((float)(3.0 * m[7]), (float)(3.0 * m[8]), (float)(3.0 * m[9]), 0.f);
}

// Per-species pseudo-particles of a box (Sec. 3, the paper's twig charges):
// the charge Q_s of its particles of one sign placed at their centre of
// charge c_s = c + mu_s / Q_s, mu_s = sum q_j (x_j - c) about the box centre c;
// delta_s = |c_s - c| enters the opening test.  Accumulators: Q+ mu+[3] Q-
// mu-[3]; record of kSpecVals doubles: c+[3] Q+ c-[3] Q- delta+ delta- 0 0.
// A box without particles of a sign has Q_s = 0 and c_s = c.
__device__ __forceinline__ void spec_add(double *sq, double q, double rx, double ry, double rz)
{
    if (q == 0.0) return;
    double *a = sq + (q > 0.0 ? 0 : 4);
    a[0] += q;
    a[1] += q * rx;
    a[2] += q * ry;
    a[3] += q * rz;
}

__device__ __forceinline__ void spec_store(double *spec, int k, const double4 &g, const double *sq)
{
    double *r = spec + kSpecVals * (int64_t)k;
    for (int sp = 0; sp < 2; ++sp) {
        const double Q = sq[4 * sp];
        const double ox = Q != 0.0 ? sq[4 * sp + 1] / Q : 0.0;
        const double oy = Q != 0.0 ? sq[4 * sp + 2] / Q : 0.0;
        const double oz = Q != 0.0 ? sq[4 * sp + 3] / Q : 0.0;
        *(double4 *)(r + 4 * sp) = make_double4(g.x + ox, g.y + oy, g.z + oz, Q);
        r[8 + sp] = sqrt(ox * ox + oy * oy + oz * oz);
    }
    r[10] = 0.0;
    r[11] = 0.0;
}

// v moved across lanes by the DPP control `ctrl` (rows outside row_mask read
// 0), each 32-bit half alike
template <int ctrl, int row_mask>
__device__ __forceinline__ double dpp_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, ctrl, row_mask, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), ctrl, row_mask, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// the sum of v over the wave, in lane 63, added in a fixed order: within
// each row of 16 lanes by swaps of lane pairs and quads and rotations by 4
// and 8 (every lane then holds its row's sum), then row 0 into row 1 and
// row 2 into row 3 (lane 15 and 47 broadcast), then rows 0-1 into rows 2-3
// (lane 31 broadcast).  All lanes must be active.
// the sum of v over each row of 16 lanes, in every lane of the row, added
// in a fixed order (swaps of lane pairs and quads, rotations by 4 and 8).
// All lanes must be active.
__device__ __forceinline__ double row_dsum(double v)
{
    v += dpp_d<0xB1, 0xf>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E, 0xf>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x124, 0xf>(v);   // row_ror 4
    v += dpp_d<0x128, 0xf>(v);   // row_ror 8
    return v;
}

__device__ __forceinline__ double wave_dsum(double v)
{
    v += dpp_d<0xB1, 0xf>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E, 0xf>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x124, 0xf>(v);   // row_ror 4
    v += dpp_d<0x128, 0xf>(v);   // row_ror 8
    v += dpp_d<0x142, 0xa>(v);   // row_bcast 15 into rows 1 and 3
    v += dpp_d<0x143, 0xc>(v);   // row_bcast 31 into rows 2 and 3
    return v;
}

// one particle's terms about the centre g: Q, p, S (m) and, by sign, Q and
// the first moment (sq)
__device__ __forceinline__ void moment_terms(const double4 &a, const double4 &g, double *m,
                                             double *sq, bool with_spec)
{
    const double r0 = a.x - g.x, r1 = a.y - g.y, r2 = a.z - g.z, qq = a.w;
    m[0] += qq;
    m[1] += qq * r0;
    m[2] += qq * r1;
    m[3] += qq * r2;
    m[4] += qq * r0 * r0;
    m[5] += qq * r1 * r1;
    m[6] += qq * r2 * r2;
    m[7] += qq * r0 * r1;
    m[8] += qq * r0 * r2;
    m[9] += qq * r1 * r2;
    if (with_spec) {
        const double qp = qq > 0.0 ? qq : 0.0, qm = qq < 0.0 ? qq : 0.0;
        sq[0] += qp;
        sq[1] += qp * r0;
        sq[2] += qp * r1;
        sq[3] += qp * r2;
        sq[4] += qm;
        sq[5] += qm * r0;
        sq[6] += qm * r1;
        sq[7] += qm * r2;
    }
}

// 6a. The leaves, every level at once (a leaf depends on nothing but its
// particles).  A wave takes 64 positions; the leaves starting there are handed
// out through LDS to groups of four lanes, 16 at a time, and lane s of a group
// takes the particles p + s, p + s + 4, ... of its leaf; the four sums are
// added by DPP in a fixed order.  A leaf's end was found by the level pass,
// or is -1 for a max-depth leaf wider than that pass's window (its starting
// lane then scans for it).
constexpr int kLeafThreads = 256, kLeafBatch = 4;
template <bool SPEC>
__global__ __launch_bounds__(kLeafThreads) void k_leaf_moments(
    const double4 *__restrict__ xq, int64_t n, const int8_t *__restrict__ Lv,
    const int8_t *__restrict__ Lf, const int32_t *__restrict__ lend,
    const int32_t *__restrict__ noff, const double4 *__restrict__ ngeo, int4 *ninfo,
    double *mom64, float4 *nrec, int32_t *leafof, double *spec, const int32_t *flags)
{
    __shared__ int4 slot[kLeafThreads / kWave][kWave];   // (p, k, t, level) of each start, by rank
    if (*flags) return;   // no other kernel runs meanwhile: the whole block reads the same word
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int64_t p = blockIdx.x * (int64_t)kLeafThreads + threadIdx.x;
    int Lp = 0, lf = 0, no = 0, le = 0;
    if (p < n) {
        Lp = Lv[p];
        lf = Lf[p];
        no = noff[p];
        le = lend[p];
    }
    const bool start = p < n && lf > Lp;
    const unsigned long long sm = __ballot(start);
    if (start) {
        int64_t t = le;
        if (t < 0) {
            t = p + 1;
            while ((int)Lv[t] >= lf) ++t;   // Lv[n] = -1 ends the scan
        }
        slot[wv][__popcll(sm & ((1ull << lane) - 1ull))] =
            make_int4((int)p, no + (lf - Lp - 1), (int)t, lf);
    }
    __syncthreads();
    const int ns = __popcll(sm);
    for (int b0 = 0; b0 < ns; b0 += kWave / 4) {
        const int gi = b0 + (lane >> 2), sub = lane & 3;
        const bool on = gi < ns;
        const int4 sl = on ? slot[wv][gi] : make_int4(0, 0, 0, 0);
        const double4 g = on ? ngeo[sl.y] : make_double4(0.0, 0.0, 0.0, 0.0);
        double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        double sq[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t q0 = (int64_t)sl.x + sub; on && q0 < sl.z; q0 += 4 * kLeafBatch) {
            double4 a[kLeafBatch];
#pragma unroll
            for (int u = 0; u < kLeafBatch; ++u) {
                const int64_t q = q0 + 4 * u;
                a[u] = xq[q < sl.z ? q : sl.x];
            }
#pragma unroll
            for (int u = 0; u < kLeafBatch; ++u) {
                if (q0 + 4 * u >= sl.z) break;
                leafof[q0 + 4 * u] = sl.y;
                moment_terms(a[u], g, m, sq, SPEC);
            }
        }
        // the group's four sums (every lane of the wave is active here)
#pragma unroll
        for (int i = 0; i < 10; ++i) {
            m[i] += dpp_d<0xB1, 0xf>(m[i]);   // quad_perm [1, 0, 3, 2]
            m[i] += dpp_d<0x4E, 0xf>(m[i]);   // quad_perm [2, 3, 0, 1]
        }
        if (SPEC) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                sq[i] += dpp_d<0xB1, 0xf>(sq[i]);
                sq[i] += dpp_d<0x4E, 0xf>(sq[i]);
            }
        }
        if (on && sub == 0) {
            const int k = sl.y, cnt = sl.z - sl.x, skip = noff[sl.z], info = sl.w | 256;
            if (SPEC) spec_store(spec, k, g, sq);
            ninfo[k] = make_int4(sl.x, cnt, skip, info);
            *(double4 *)(nrec + 8 * (int64_t)k) = g;
            *(int4 *)(nrec + 8 * (int64_t)k + 2) = make_int4(skip, sl.x, cnt, info);
            store_moments(mom64, nrec, k, g, m);
        }
    }
}

// High bit of each byte of x set where that byte (taken mod 128) is < v,
// for 0 < v <= 127; the bias 0x80 per byte keeps borrows inside each byte.
__device__ __forceinline__ uint32_t bytes_below(uint32_t x, uint32_t v)
{
    return ~((x & 0x7F7F7F7Fu) + 0x80808080u - v * 0x01010101u) & 0x80808080u;
}
// the four byte flags (bits 7, 15, 23, 31) gathered into bits 0..3
__device__ __forceinline__ uint32_t gather4(uint32_t m)
{
    return ((m >> 7) & 1u) | ((m >> 14) & 2u) | ((m >> 21) & 4u) | ((m >> 28) & 8u);
}

// ---------------------------------------------------------------------------
// 6b. internal nodes, each by one wave.  The node (p, l) holds the positions
//     p .. t-1, t the first later position with L(t) < l (L is -1 at every
//     cloud edge and at n).  Its children are the nodes of level l + 1 that
//     start at p (node k + 1) and at each position s in (p, t) with L(s) = l
//     (node noff[s], the first node there).  The wave reads the level bytes
//     of the next 1024 positions, 16 per lane; for a node that runs past
//     them, eight 8-ary searches over the sorted keys, eight lanes each, find
//     its end (the first key whose level-l prefix exceeds the node's prefix
//     P) and the start of each child octant o (the first key whose
//     level-(l + 1) prefix is at least 8 P + o).  It writes the count, the
//     skip link noff[t] (the node after the subtree in preorder), the walk
//     record's header, the children in order (-1 after the last) and each
//     child's parent.  A node of at most direct_max particles then sums its
//     particles' moments about its centre, lane j taking particles p + j,
//     p + j + 64, ..., and the lanes' sums are added in a fixed order; a
//     larger node is listed for 6c.
// ---------------------------------------------------------------------------
constexpr int kNodeThreads = 256, kNodeSpan = 16, kRangeWin = 16 * kWave;
// the largest node summed from its particles, for trees below and from
// kUpperWide particles on (measured from 256 to 2048 on 524,288 and
// 4,194,304 particles: 1024 and 2048 within a microsecond on the first,
// 1024 the faster on the second)
constexpr int kDirectMax = 1024, kDirectMaxWide = 1024;
constexpr int kDirectFirst = 4;   // particles per lane read with the level window

template <bool SPEC>
__global__ __launch_bounds__(kNodeThreads) void k_node_moments(
    const uint64_t *__restrict__ key, const int8_t *__restrict__ Lv,
    const double4 *__restrict__ xq, int64_t n, const int64_t *__restrict__ off, int clouds, int b,
    const int32_t *__restrict__ noff, const uint8_t *__restrict__ nlev,
    const double4 *__restrict__ ngeo, int4 *ninfo, float4 *nrec, double *mom64, int32_t *npar,
    int32_t *ctab, int32_t *uplist, double *spec, unsigned long long *ctr, int direct_max,
    int32_t *flags)
{
    if (*flags) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = (blockIdx.x * (int64_t)kNodeThreads + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * (kNodeThreads / kWave);
    const int nn = noff[n];
    constexpr bool with_spec = SPEC;
    // wave w takes kNodeSpan consecutive node slots at a time (the nodes of a
    // chain that start at one position, a node and its first child, read the
    // same particles); each lane reads its slot's first position, level and
    // centre
    for (int64_t s0 = wave * kNodeSpan; s0 < nn; s0 += kNodeSpan * nwaves) {
        const int64_t kl = lane < kNodeSpan ? s0 + lane : nn;
        // the three reads are issued together (a leaf's record is not used)
        const int64_t kr = kl < nn ? kl : 0;
        const uint8_t lv = nlev[kr];
        const int4 infl = ninfo[kr];
        const double4 gl = ngeo[kr];
        const bool inner = kl < nn && !(lv & kLeafBit);
        // Small nodes first, four at a time: row r (16 lanes) takes the r-th
        // of the next four internal nodes, reads the levels of the 256
        // positions after it, and when the node ends there it writes its
        // records and parents and sums its particles (lane j: p + j, p + j +
        // 16, ...), the row's sums added by DPP in a fixed order.  A node that
        // runs past those positions is left to the whole wave below.
        unsigned long long todo = __ballot(inner), big = 0ull;
        const int row = lane >> 4, rl = lane & 15;
        while (todo != 0ull) {
            unsigned long long mm = todo;
            for (int r = 0; r < row; ++r) mm &= mm - 1ull;
            const int src = mm != 0ull ? __builtin_ctzll(mm) : -1;
            for (int r = 0; r < 4; ++r) todo &= todo - 1ull;
            const int srcc = src >= 0 ? src : 0;
            const int k = (int)(s0 + srcc);
            const int64_t p = __shfl(infl.x, srcc);
            const int iw = __shfl(infl.w, srcc);
            const int l = iw & 255;
            const double4 g = make_double4(__shfl(gl.x, srcc), __shfl(gl.y, srcc),
                                           __shfl(gl.z, srcc), __shfl(gl.w, srcc));
            bool mine = src >= 0;
            if (mine && (p < 0 || p >= n || (iw & 256) || l >= b || k + 1 >= nn)) {
                if (rl == 0) atomicOr(flags, UCP_FLAG_INTERNAL);
                mine = false;
            }
            const int64_t pp = mine ? p : 0;
            // the row's particles, read with its level window
            double4 xa[kDirectFirst];
#pragma unroll
            for (int u = 0; u < kDirectFirst; ++u) {
                const int64_t q = pp + rl + 16 * u;
                xa[u] = xq[q < n ? q : pp];
            }
            const int64_t base = (pp + 1) & ~(int64_t)15;
            const int64_t q0 = base + 16 * rl;
            uint32_t endm = 0, eqm = 0;
            if (mine && q0 <= n) {
                const uint4 v = *(const uint4 *)(Lv + q0);
                const uint32_t d[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const uint32_t lt = bytes_below(d[w], (uint32_t)l) | (d[w] & 0x80808080u);
                    const uint32_t eq = bytes_below(d[w], (uint32_t)l + 1) & ~lt;
                    endm |= gather4(lt) << (4 * w);
                    eqm |= gather4(eq) << (4 * w);
                }
                const int lo = (int)max<int64_t>(0, pp + 1 - q0);
                const int hi = (int)min<int64_t>(16, n + 1 - q0);
                const uint32_t valid = ((1u << hi) - 1u) & ~((1u << lo) - 1u);
                endm &= valid;
                eqm &= valid;
            }
            const unsigned long long he = __ballot(endm != 0);
            const uint32_t rowend = (uint32_t)(he >> (16 * row)) & 0xFFFFu;
            const int f = rowend != 0u ? __builtin_ctz(rowend) : 0;
            const uint32_t ef = (uint32_t)__shfl((int)endm, 16 * row + f);
            const int64_t t = base + 16 * f + (ef != 0u ? __builtin_ctz(ef) : 0);
            const bool ok = mine && rowend != 0u;
            {
                // the nodes that run past their row's window, by span slot
                const unsigned long long bb = __ballot(mine && rowend == 0u && rl == 0);
                for (int r = 0; r < 4; ++r)
                    if ((bb >> (16 * r)) & 1ull) big |= 1ull << __shfl(srcc, 16 * r);
            }
            double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
            double sq[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (ok) {
                // parents of the children after the first (L == l before t)
                uint32_t cm = eqm;
                const int64_t lim = t - q0;
                if (lim <= 0) cm = 0;
                else if (lim < 16) cm &= (1u << lim) - 1u;
                while (cm != 0u) {
                    npar[noff[q0 + __builtin_ctz(cm)]] = k;
                    cm &= cm - 1u;
                }
#pragma unroll
                for (int u = 0; u < kDirectFirst; ++u)
                    if (pp + rl + 16 * u < t) moment_terms(xa[u], g, m, sq, with_spec);
                for (int64_t q = pp + rl + 16 * kDirectFirst; q < t; q += 16 * kDirectFirst) {
#pragma unroll
                    for (int u = 0; u < kDirectFirst; ++u) {
                        const int64_t qq = q + 16 * u;
                        xa[u] = xq[qq < t ? qq : pp];
                    }
#pragma unroll
                    for (int u = 0; u < kDirectFirst; ++u)
                        if (q + 16 * u < t) moment_terms(xa[u], g, m, sq, with_spec);
                }
            }
            // the row's sums (every lane of the wave is active here)
#pragma unroll
            for (int i = 0; i < 10; ++i) m[i] = row_dsum(m[i]);
            if (with_spec) {
#pragma unroll
                for (int i = 0; i < 8; ++i) sq[i] = row_dsum(sq[i]);
            }
            if (ok && rl == 0) {
                const int cntp = (int)(t - pp), skip = noff[t];
                npar[k + 1] = k;
                if (t < pp + 2) atomicOr(flags, UCP_FLAG_INTERNAL);
                ninfo[k] = make_int4((int)pp, cntp, skip, iw);
                *(double4 *)(nrec + 8 * (int64_t)k) = g;
                *(int4 *)(nrec + 8 * (int64_t)k + 2) = make_int4(skip, (int)pp, cntp, iw);
                if (with_spec) spec_store(spec, k, g, sq);
                store_moments(mom64, nrec, k, g, m);
            }
        }
        unsigned long long im = big;
        while (im != 0ull) {
            const int src = __builtin_ctzll(im);
            im &= im - 1ull;
            const int k = (int)(s0 + src);
            const int64_t p = __shfl(infl.x, src);
            const int iw = __shfl(infl.w, src);
            const int l = iw & 255;
            const double4 g = make_double4(__shfl(gl.x, src), __shfl(gl.y, src),
                                           __shfl(gl.z, src), __shfl(gl.w, src));
            if (p < 0 || p >= n || (iw & 256) || l >= b || k + 1 >= nn) {
                if (lane == 0) atomicOr(flags, UCP_FLAG_INTERNAL);
                continue;
            }
            // the node's first particles, read with the level window
            double4 xa[kDirectFirst];
#pragma unroll
            for (int u = 0; u < kDirectFirst; ++u) {
                const int64_t q = p + lane + u * kWave;
                xa[u] = xq[q < n ? q : p];
            }
            // level bytes of positions base .. base + 1023 (base: p + 1
            // rounded down to 16), flagged where the node ends (L < l, or a
            // cloud edge) or a child starts (L == l), over p + 1 .. n only
            const int64_t base = (p + 1) & ~(int64_t)15;
            const int64_t q0 = base + 16 * lane;
            uint32_t endm = 0, eqm = 0;
            if (q0 <= n) {
                const uint4 v = *(const uint4 *)(Lv + q0);
                const uint32_t d[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const uint32_t lt = bytes_below(d[w], (uint32_t)l) | (d[w] & 0x80808080u);
                    const uint32_t eq = bytes_below(d[w], (uint32_t)l + 1) & ~lt;
                    endm |= gather4(lt) << (4 * w);
                    eqm |= gather4(eq) << (4 * w);
                }
                const int lo = (int)max<int64_t>(0, p + 1 - q0);
                const int hi = (int)min<int64_t>(16, n + 1 - q0);
                const uint32_t valid = ((1u << hi) - 1u) & ~((1u << lo) - 1u);
                endm &= valid;
                eqm &= valid;
            }
            const unsigned long long hasend = __ballot(endm != 0);
            int64_t t = -1;
            if (hasend != 0ull) {
                const int f = __builtin_ctzll(hasend);
                t = base + 16 * f + __builtin_ctz((uint32_t)__shfl((int)endm, f));
            }
            int nch;
            if (t >= 0) {
                // the child starts are the flagged positions before t
                uint32_t cm = eqm;
                const int64_t lim = t - q0;
                if (lim <= 0) cm = 0;
                else if (lim < 16) cm &= (1u << lim) - 1u;
                const int c = __popc(cm);
                const int incl = wave_incl_scan(c);
                nch = 1 + __shfl(incl, kWave - 1);
                int j = 1 + incl - c;
                while (cm != 0u) {
                    const int s = noff[q0 + __builtin_ctz(cm)];
                    cm &= cm - 1u;
                    if (j < 8) ctab[8 * (int64_t)k + j] = s;
                    npar[s] = k;
                    ++j;
                }
                if (lane == 0) {
                    ctab[8 * (int64_t)k] = k + 1;
                    npar[k + 1] = k;
                }
            } else {
                // group g of eight lanes finds, over [p + 1, ce), the first
                // key past the node (g = 0) or the start of octant g (g >= 1);
                // the predicate is false then true along the sorted keys.
                // Each round probes 7 points splitting [a, e) into 8 parts, or
                // every point of a part of at most 8.
                const int64_t ce = off[cloud_of(off, clouds, p) + 1];
                const int g8 = lane >> 3, jj = lane & 7;
                const int sh = 3 * (b - l), sh1 = sh - 3;
                const uint64_t kp = key[p];
                const uint64_t P = kp >> sh, Po = (P << 3) | (uint64_t)g8;
                int64_t a = p + 1, e = ce;
                bool done = false;
                for (int it = 0; it < 64; ++it) {
                    const int64_t m = e - a;
                    const bool small = m <= 8;
                    const bool probe = !done && (small ? jj < m : jj < 7);
                    const int64_t q = small ? a + jj : a + ((m * (jj + 1)) >> 3);
                    bool pr = false;
                    if (probe) {
                        const uint64_t kq = key[q];
                        pr = g8 == 0 ? (kq >> sh) > P : (kq >> sh1) >= Po;
                    }
                    const unsigned long long fb = __ballot(probe && !pr);
                    const int nf = __popcll((fb >> (8 * g8)) & 0xFFull);
                    if (!done) {
                        if (small) {
                            a += nf;
                            e = a;
                            done = true;
                        } else {
                            const int64_t qlo = nf > 0 ? a + ((m * nf) >> 3) : a - 1;
                            const int64_t qhi = nf < 7 ? a + ((m * (nf + 1)) >> 3) : e;
                            a = qlo + 1;
                            e = qhi;
                        }
                    }
                    if (__ballot(!done) == 0ull) break;
                }
                if (__ballot(!done) != 0ull) {
                    if (lane == 0) atomicOr(flags, UCP_FLAG_INTERNAL);
                    continue;
                }
                const int ai = (int)a;
                t = __shfl(ai, 0);
                // lanes 0..7: S_o, the first position of octant o (p for the
                // octants up to that of particle p), and S_8 = t
                const int dig0 = (int)((kp >> sh1) & 7);
                int so = __shfl(ai, 8 * (lane & 7));
                if (lane <= dig0) so = (int)p;
                int snext = __shfl(so, (lane + 1) & (kWave - 1));
                if (lane == 7) snext = (int)t;
                const bool has = lane < 8 && so < snext;
                const unsigned long long hm = __ballot(has);
                nch = __popcll(hm);
                if (has) {
                    const int ch = so == (int)p ? k + 1 : noff[so];
                    ctab[8 * (int64_t)k + __popcll(hm & ((1ull << lane) - 1ull))] = ch;
                    npar[ch] = k;
                }
            }
            if (lane >= nch && lane < 8) ctab[8 * (int64_t)k + lane] = -1;
            const int cntp = (int)(t - p);
            if (lane == 0) {
                if (t < p + 2 || nch < 1 || nch > 8) atomicOr(flags, UCP_FLAG_INTERNAL);
                const int skip = noff[t];
                ninfo[k] = make_int4((int)p, cntp, skip, iw);
                *(double4 *)(nrec + 8 * (int64_t)k) = g;
                *(int4 *)(nrec + 8 * (int64_t)k + 2) = make_int4(skip, (int)p, cntp, iw);
            }
            if (cntp > direct_max) {
                // summed from its children (6c)
                if (lane == 0) {
                    const unsigned long long slot = atomicAdd(&ctr[CTR_UPCOUNT], 1ull);
                    if (slot < (unsigned long long)nn) uplist[slot] = k;
                    else atomicOr(flags, UCP_FLAG_INTERNAL);
                }
                continue;
            }
            // the moments of the particles p .. t-1 about the centre g
            double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
            double sq[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int u = 0; u < kDirectFirst; ++u)
                if (p + lane + u * kWave < t) moment_terms(xa[u], g, m, sq, with_spec);
            for (int64_t q = p + lane + kDirectFirst * kWave; q < t; q += kDirectFirst * kWave) {
#pragma unroll
                for (int u = 0; u < kDirectFirst; ++u) {
                    const int64_t qq = q + u * kWave;
                    xa[u] = xq[qq < t ? qq : p];
                }
#pragma unroll
                for (int u = 0; u < kDirectFirst; ++u)
                    if (q + u * kWave < t) moment_terms(xa[u], g, m, sq, with_spec);
            }
#pragma unroll
            for (int i = 0; i < 10; ++i) m[i] = wave_dsum(m[i]);
            if (with_spec) {
#pragma unroll
                for (int i = 0; i < 8; ++i) sq[i] = wave_dsum(sq[i]);
            }
            if (lane == kWave - 1) {
                if (with_spec) spec_store(spec, k, g, sq);
                store_moments(mom64, nrec, k, g, m);
            }
        }
    }
}

// Grid-wide barrier of a launch whose blocks are all resident at once (one
// block per CU).  Thread 0 of each block publishes the block's writes, counts
// itself in and waits for the count to reach `target`; the wait is bounded and
// returns false when the bound is hit.
constexpr int kBarrierSpin = 1 << 21;
__device__ __forceinline__ bool grid_barrier(unsigned long long *bar, unsigned long long target)
{
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(bar, 1ull);
        int spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target &&
               spins <= kBarrierSpin) {
            __builtin_amdgcn_s_sleep(2);
            ++spins;
        }
        ok = spins <= kBarrierSpin;
        __threadfence();
    }
    __syncthreads();
    return ok != 0;
}

// ---------------------------------------------------------------------------
// 6c. the internal nodes of more than direct_max particles (few, and near the
//     root), from the deepest up: a node sums its children's moments (read
//     through its child table) shifted to its centre, in order.  A small
//     tree takes one block, with a block barrier between levels; from
//     kUpperWide particles on, kUpperBlocks blocks (all resident at once)
//     with a grid barrier between levels.  Every block passes every barrier,
//     whatever it finds; few blocks keep the barrier cheap, since each
//     block's release writes back its L2.
// ---------------------------------------------------------------------------
constexpr int kUpperThreads = 512, kUpperBlocks = 16;
constexpr int64_t kUpperWide = int64_t(1) << 21;

struct UpperNode {
    int k, l;
    double4 g;
    int4 c0, c1;
};

// one child's moments shifted from its centre to the parent's centre g and
// added: p' = p + Q d, S' = S + p d^T + d p^T + Q d d^T with d = c_child - g
// (each component +-qd); c holds the child's FP64 record from cx on
__device__ __forceinline__ void add_child(double *m, const double4 &g, double qd, const double *c)
{
    const double d0 = c[0] > g.x ? qd : -qd;
    const double d1 = c[1] > g.y ? qd : -qd;
    const double d2 = c[2] > g.z ? qd : -qd;
    const double Q = c[3], p0 = c[4], p1 = c[5], p2 = c[6];
    m[0] += Q;
    m[1] += p0 + Q * d0;
    m[2] += p1 + Q * d1;
    m[3] += p2 + Q * d2;
    m[4] += c[8] + 2.0 * p0 * d0 + Q * d0 * d0;
    m[5] += c[9] + 2.0 * p1 * d1 + Q * d1 * d1;
    m[6] += c[10] + 2.0 * p2 * d2 + Q * d2 * d2;
    m[7] += c[11] + p0 * d1 + d0 * p1 + Q * d0 * d1;
    m[8] += c[12] + p0 * d2 + d0 * p2 + Q * d0 * d2;
    m[9] += c[13] + p1 * d2 + d1 * p2 + Q * d1 * d2;
}

// a child's pseudo-particles added to its parent's accumulators
__device__ __forceinline__ void spec_add_child(double *sq, const double *spec, int ch,
                                               const double4 &g)
{
    const double *r = spec + kSpecVals * (int64_t)ch;
    const double4 a = *(const double4 *)r, b = *(const double4 *)(r + 4);
    spec_add(sq, a.w, a.x - g.x, a.y - g.y, a.z - g.z);
    spec_add(sq, b.w, b.x - g.x, b.y - g.y, b.z - g.z);
}

__device__ __forceinline__ void moments_from_children(const UpperNode &nd, int nn, double *mom64,
                                                      float4 *nrec, double *spec, int32_t *flags)
{
    const int ch[8] = {nd.c0.x, nd.c0.y, nd.c0.z, nd.c0.w, nd.c1.x, nd.c1.y, nd.c1.z, nd.c1.w};
    bool bad = ch[0] < 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) bad = bad || ch[u] >= nn;
    if (bad) {
        atomicOr(flags, UCP_FLAG_INTERNAL);
        return;
    }
    const double4 g = nd.g;
    double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    double sq[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double qd = 0.25 * sqrt(g.w);   // |child centre - parent centre| per axis
    // four children's records (cx cy cz Q px py pz trS S[6]) per round of loads
#pragma unroll
    for (int r0 = 0; r0 < 8; r0 += 4) {
        if (ch[r0] < 0) break;
        double rc[4][14];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int cu = ch[r0 + u] >= 0 ? ch[r0 + u] : ch[r0];
            const double2 *r = (const double2 *)(mom64 + 16 * (int64_t)cu);
#pragma unroll
            for (int i = 0; i < 7; ++i) {
                const double2 v = r[i];
                rc[u][2 * i] = v.x;
                rc[u][2 * i + 1] = v.y;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (ch[r0 + u] < 0) break;
            add_child(m, g, qd, rc[u]);
            if (spec) spec_add_child(sq, spec, ch[r0 + u], g);
        }
    }
    if (spec) spec_store(spec, nd.k, g, sq);
    store_moments(mom64, nrec, nd.k, g, m);
}

__global__ __launch_bounds__(kUpperThreads) void k_moments_upper(
    int64_t n, const int32_t *__restrict__ noff, const uint8_t *__restrict__ nlev,
    const double4 *__restrict__ ngeo, const int32_t *__restrict__ ctab,
    const int32_t *__restrict__ uplist, unsigned long long *ctr, double *mom64, float4 *nrec,
    double *spec, int32_t *flags)
{
    __shared__ int go_s;
    const int maxl = (int)ctr[CTR_MAXLEVEL];   // deepest leaf; internal nodes lie above it
    const int nn = noff[n];
    const int cnt = (int)min(ctr[CTR_UPCOUNT], (unsigned long long)nn);
    const int t0 = blockIdx.x * kUpperThreads + threadIdx.x;
    auto node_at = [&](int i) -> UpperNode {
        UpperNode t;
        t.k = uplist[i];
        t.l = -1;
        if (t.k < 0 || t.k >= nn) {
            atomicOr(flags, UCP_FLAG_INTERNAL);
            t.k = -1;
            return t;
        }
        t.l = nlev[t.k];
        t.g = ngeo[t.k];
        t.c0 = *(const int4 *)(ctab + 8 * (int64_t)t.k);
        t.c1 = *(const int4 *)(ctab + 8 * (int64_t)t.k + 4);
        return t;
    };
    const int stride = gridDim.x * kUpperThreads;
    // this thread's first node, read once
    UpperNode held;
    held.k = -1;
    held.l = -1;
    if (t0 < cnt) held = node_at(t0);
    // the deepest level of a listed node: the levels below it hold none.
    // Every block reads the whole list, so all agree on the number of levels
    // (and of grid barriers).
    __shared__ int lbig_s;
    if (threadIdx.x == 0) lbig_s = -1;
    __syncthreads();
    int lb = -1;
    for (int i = threadIdx.x; i < cnt; i += kUpperThreads) {
        const int k = uplist[i];
        if (k >= 0 && k < nn) lb = max(lb, (int)nlev[k]);
    }
    for (int o = 32; o > 0; o >>= 1) lb = max(lb, __shfl_xor(lb, o));
    if ((threadIdx.x & 63) == 0) atomicMax(&lbig_s, lb);
    __syncthreads();
    const int ltop = min(lbig_s, maxl - 1);
    unsigned long long target = 0;
    bool wait = true;
    for (int l = ltop; l >= 0; --l) {
        // one reading of the flags for the whole block, so that its threads
        // agree on every loop bound below
        if (threadIdx.x == 0)
            go_s = __hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
        __syncthreads();
        const bool go = go_s != 0;
        __syncthreads();
        for (int i = t0; go && i < cnt; i += stride) {
            const UpperNode nd = i == t0 ? held : node_at(i);
            if (nd.k >= 0 && nd.l == l) moments_from_children(nd, nn, mom64, nrec, spec, flags);
        }
        if (gridDim.x == 1) {
            __syncthreads();
        } else if (l > 0 && wait) {
            // every block passes every barrier, so that the count of
            // arrivals stays exact; a wait that times out flags the build
            target += gridDim.x;
            if (!grid_barrier(&ctr[CTR_BARRIER], target)) {
                if (threadIdx.x == 0) atomicOr(flags, UCP_FLAG_INTERNAL);
                wait = false;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 7. walk groups
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_group_count(
    int64_t n, const int8_t *__restrict__ Lv, const int8_t *__restrict__ Lf,
    const int32_t *__restrict__ noff, const int4 *__restrict__ ninfo,
    const int32_t *__restrict__ npar, const int64_t *__restrict__ off, int clouds, int G,
    int mode, int32_t *cnt, int32_t *gnode, const int32_t *flags)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p > n) return;
    if (p == n || *flags) { cnt[p] = 0; return; }
    int ng = 0, gn = -1;
    if (mode == UCP_GROUP_CHUNK) {
        // a run of G starts at every G-th particle of the cloud
        const int64_t o = off[cloud_of(off, clouds, p)];
        if ((p - o) % G == 0) { ng = 1; gn = noff[o]; }
        cnt[p] = ng;
        gnode[p] = gn;
        return;
    }
    const int Lp = Lv[p], lf = Lf[p];
    if (lf > Lp) {
        const int k0 = noff[p];
        for (int l = Lp + 1; l <= lf; ++l) {
            const int k = k0 + (l - Lp - 1);
            const int c = ninfo[k].y;
            const int par = npar[k];
            const int cpar = par < 0 ? 0x7fffffff : ninfo[par].y;
            if (c <= G && cpar > G) { ng = 1; gn = k; break; }
        }
        if (ng == 0) {
            const int kl = k0 + (lf - Lp - 1);
            const int c = ninfo[kl].y;
            if (c > G) { ng = (c + G - 1) / G; gn = kl; }
        }
    }
    cnt[p] = ng;
    gnode[p] = gn;
}

// Chunk groups need no scan over positions: cloud c holds ceil(N_c / G)
// groups, the g-th from its first particle on.  The build's first kernel sets
// each cloud's first group and the total (read by the walk at goff[n]); here
// every group is written from its index alone.  A build that raised a flag
// publishes no groups (the walk and the statistics read the total).
__global__ __launch_bounds__(256) void k_group_chunk_emit(
    const int64_t *__restrict__ off, int clouds, int G, int32_t *gcl,
    const int32_t *__restrict__ noff, int4 *groups, int32_t *goff_n, const int32_t *flags)
{
    if (*flags) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            gcl[clouds] = 0;
            *goff_n = 0;
        }
        return;
    }
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= gcl[clouds]) return;
    // the cloud holding group g: the last c with gcl[c] <= g (it has groups)
    int lo = 0, hi = clouds;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (gcl[mid] <= g) lo = mid;
        else hi = mid;
    }
    const int64_t p = off[lo] + (int64_t)(g - gcl[lo]) * G;
    const int root = noff[off[lo]];
    groups[g] = make_int4((int)p, (int)min<int64_t>(G, off[lo + 1] - p), root, root);
}

__global__ __launch_bounds__(256) void k_group_emit(
    int64_t n, const int32_t *__restrict__ cnt, const int32_t *__restrict__ goff,
    const int32_t *__restrict__ gnode, const int4 *__restrict__ ninfo,
    const int32_t *__restrict__ noff, const int64_t *__restrict__ off, int clouds, int G,
    int mode, int4 *groups, const int32_t *flags)
{
    if (*flags) return;
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int ng = cnt[p];
    if (ng == 0) return;
    const int k = gnode[p];
    const int cl = cloud_of(off, clouds, p);
    const int root = noff[off[cl]];
    // particles left to cut from p on: the node's (node groups) or the cloud's (chunks)
    const int c = mode == UCP_GROUP_CHUNK ? (int)(off[cl + 1] - p) : ninfo[k].y;
    for (int j = 0; j < ng; ++j) {
        const int gc = min(G, c - j * G);
        groups[goff[p] + j] = make_int4((int)p + j * G, gc, k, root);
    }
}

// ---------------------------------------------------------------------------
// host driver of one build
// ---------------------------------------------------------------------------
static inline dim3 grid_for(int64_t n, int threads) { return dim3((unsigned)((n + threads - 1) / threads)); }

void launch_build(Ctx *c, const double *x, const double *q, const int64_t *offsets_in, int clouds,
                  int64_t n, hipStream_t s)
{
    const int b = c->p.key_bits == 30 ? 10 : 21;
    const int cap = c->p.leaf_cap;
    const int G = c->p.group_size;

    const int64_t nstatus = 256 * ((n + kSortTile - 1) / kSortTile);
    const bool chunk = c->p.group_mode == UCP_GROUP_CHUNK;
    hipLaunchKernelGGL(k_build_reset,
                       grid_for(std::max<int64_t>({6 * (int64_t)clouds + CTR_NCTR,
                                                   (int64_t)kSortPassesMax * 256, 1}),
                                kScanBlock),
                       dim3(kScanBlock), 0, s, c->d_mm, clouds, c->d_ctr, c->d_sortctl,
                       c->d_ghist, c->d_hist, nstatus, c->d_offstat,
                       (n + kOffTile) / kOffTile, offsets_in, n, chunk ? G : 0, c->d_off,
                       c->d_gcl, c->d_goff + n, c->d_wq, c->d_flags);
    c->walk_armed = true;

    // 1. cube
    hipLaunchKernelGGL(k_cube_reduce, grid_for(n, 256 * kCubeItems), dim3(256), 0, s, x, n,
                       (const int64_t *)c->d_off, clouds, c->d_mm, c->d_flags);
    // 2. keys (and each cloud's cube from the reduced extents)
    hipLaunchKernelGGL(k_keys, grid_for(n, 256), dim3(256), 0, s, x, q, n,
                       (const int64_t *)c->d_off, clouds, (const unsigned long long *)c->d_mm,
                       c->d_cube, b, c->p.curve, c->d_key[0], c->d_val[0], c->d_xin, c->d_flags);
    // 3. sort
    const int ntiles = (int)((n + kSortTile - 1) / kSortTile);
    const int key_passes = (3 * b + 7) / 8;
    // three top digits (boxes of level 7-8) leave runs of a few particles up
    // to about 2^20 particles; above that a fourth keeps ranking cheap
    const int top_passes = std::min(n > kSortWideN ? 4 : 3, key_passes);
    int cloud_passes = 0;
    if (clouds > 1) {
        int cbits = 0;
        while ((1 << cbits) < clouds) ++cbits;
        cloud_passes = (cbits + 7) / 8;
    }
    hipLaunchKernelGGL(k_radix_counts, dim3(std::max(1, std::min(ntiles, c->num_cu))),
                       dim3(kSortThreads), 0, s, (const uint64_t *)c->d_key[0], n, key_passes,
                       cloud_passes, (const int64_t *)c->d_off, clouds, c->d_ghist,
                       (const int32_t *)c->d_flags);
    int npass = 0;
    uint32_t *status[2] = {c->d_hist, c->d_histscan};
    // pass number npass from buffer `from` to `to` over key digit `digit` (or
    // cloud digit `digit` - key_passes); the counts of digit j are ghist[256 j]
    auto pass_args = [&](int from, int to, int digit, double4 *xq) {
        SortPassArgs a;
        a.kin = (const uint64_t *)c->d_key[from];
        a.vin = (const uint32_t *)c->d_val[from];
        a.kout = c->d_key[to];
        a.vout = c->d_val[to];
        a.ghist = c->d_ghist + 256 * digit;
        a.status = status[npass & 1];
        a.status_next = status[(npass + 1) & 1];
        a.ticket = c->d_sortctl + npass;
        a.xq = xq;
        a.cloud = digit >= key_passes;
        a.shift = 8 * (a.cloud ? digit - key_passes : digit);
        ++npass;
        return a;
    };
    // the digits of a sequence of passes, least significant first
    std::vector<int> digits;
    // passes over the top digits and the cloud digits, from buffer 0 to buffer 1
    for (int d = key_passes - top_passes; d < key_passes; ++d) digits.push_back(d);
    for (int d = 0; d < cloud_passes; ++d) digits.push_back(key_passes + d);
    int cur = 0;
    const bool wide = n > kSortWideN;
    constexpr int kWideTile = kSortThreads * kSortWideItems;
    const int ptiles = wide ? (int)((n + kWideTile - 1) / kWideTile) : ntiles;
    for (size_t i = 0; i < digits.size(); ++i) {
        // the first pass goes to the buffer that makes the last one land in 1
        const int to = i == 0 ? ((digits.size() - 1) % 2 == 0 ? 1 : 2) : (cur == 1 ? 2 : 1);
        const SortPassArgs a = pass_args(cur, to, digits[i], nullptr);
        auto kern = a.cloud ? (wide ? k_radix_pass<true, kSortWideItems>
                                    : k_radix_pass<true, kSortItems>)
                            : (wide ? k_radix_pass<false, kSortWideItems>
                                    : k_radix_pass<false, kSortItems>);
        hipLaunchKernelGGL(kern, dim3(ptiles), dim3(kSortThreads), 0, s, a.kin, a.vin, a.kout,
                           a.vout, n, a.shift, (const int64_t *)c->d_off, clouds, a.ghist, a.status,
                           a.status_next, a.ticket, (const double4 *)c->d_xin, a.xq, c->d_flags);
        cur = to;
    }
    // each run of equal top digits ordered by ranking, into buffer 2
    const int fin_shift = 8 * (key_passes - top_passes);
    hipLaunchKernelGGL(k_sort_finish, grid_for(n, kFinishThreads), dim3(kFinishThreads), 0, s,
                       (const uint64_t *)c->d_key[1], (const uint32_t *)c->d_val[1], c->d_key[2],
                       c->d_val[2], n, fin_shift, (const int64_t *)c->d_off, clouds,
                       (const double4 *)c->d_xin, c->d_xq, c->d_ctr + CTR_SORTFULL, c->d_flags);
    // the full sort, gated by the finish's word: every digit from buffer 0,
    // ending in buffer 2; its last pass gathers x and q
    SortPlan plan;
    plan.npass = key_passes + cloud_passes;
    cur = 0;
    for (int i = 0; i < plan.npass; ++i) {
        const int to = i == 0 ? ((plan.npass - 1) % 2 == 0 ? 2 : 1) : (cur == 1 ? 2 : 1);
        plan.p[i] = pass_args(cur, to, i, i + 1 == plan.npass ? c->d_xq : nullptr);
        cur = to;
    }
    const int wtiles = (int)((n + kSortThreads * kSortWideItems - 1) / (kSortThreads * kSortWideItems));
    hipLaunchKernelGGL(k_sort_full, dim3(std::max(1, std::min(wtiles, c->num_cu / 2))),
                       dim3(kSortThreads), 0, s, plan, n, (const int64_t *)c->d_off, clouds,
                       (const double4 *)c->d_xin, (const unsigned long long *)(c->d_ctr + CTR_SORTFULL),
                       c->d_ctr + CTR_SORTBAR, c->d_flags);
    c->d_skey = c->d_key[2];
    c->d_perm = c->d_val[2];
    // 4. levels and node numbering
    hipLaunchKernelGGL(k_levels, grid_for(n + 1, kLvlTile), dim3(kLvlTile), 0, s,
                       (const uint64_t *)c->d_skey, n, (const int64_t *)c->d_off, clouds, b, cap,
                       c->d_L, c->d_leaf, c->d_cnt, c->d_lend, c->d_lvlmax,
                       (const int32_t *)c->d_flags);
    // 5. node offsets, the deepest leaf level and the node records
    hipLaunchKernelGGL(k_offsets_nodes, grid_for(n + 1, kOffTile), dim3(kOffThreads), 0, s,
                       (const int32_t *)c->d_cnt, (const int32_t *)c->d_lvlmax,
                       (int)((n + 1 + kLvlTile - 1) / kLvlTile), (const double4 *)c->d_xq, n,
                       (const int64_t *)c->d_off, clouds, (const double4 *)c->d_cube, b,
                       (const int8_t *)c->d_L, (const int8_t *)c->d_leaf, c->node_cap, c->d_noff,
                       c->d_ngeo, c->d_ninfo, c->d_npar, c->d_nlev, c->d_offstat, c->d_ctr,
                       c->d_flags);
    // 6. moments: every leaf, then the internal levels from the deepest up
    //    (and the per-species pseudo-particles when the walk uses them)
    double *spec = c->p.expansion == UCP_EXPANSION_SPECIES ? c->d_spec : nullptr;
    auto leaf_kernel = spec ? k_leaf_moments<true> : k_leaf_moments<false>;
    hipLaunchKernelGGL(leaf_kernel, grid_for(n, kLeafThreads), dim3(kLeafThreads), 0, s,
                       (const double4 *)c->d_xq, n, (const int8_t *)c->d_L,
                       (const int8_t *)c->d_leaf, (const int32_t *)c->d_lend,
                       (const int32_t *)c->d_noff, (const double4 *)c->d_ngeo, c->d_ninfo,
                       c->d_mom64, c->d_nrec, c->d_leafof, spec, (const int32_t *)c->d_flags);
    // the internal nodes, one wave per node over a grid that fills the chip;
    // then the large ones from their children
    const int nwblocks = 8 * std::max(c->num_cu, 1);
    auto node_kernel = spec ? k_node_moments<true> : k_node_moments<false>;
    hipLaunchKernelGGL(node_kernel, dim3(nwblocks), dim3(kNodeThreads), 0, s,
                       (const uint64_t *)c->d_skey, (const int8_t *)c->d_L,
                       (const double4 *)c->d_xq, n, (const int64_t *)c->d_off, clouds, b,
                       (const int32_t *)c->d_noff, (const uint8_t *)c->d_nlev,
                       (const double4 *)c->d_ngeo, c->d_ninfo, c->d_nrec, c->d_mom64, c->d_npar,
                       c->d_ctab, c->d_uplist, spec, c->d_ctr,
                       n >= kUpperWide ? kDirectMaxWide : kDirectMax, c->d_flags);
    const int upper_blocks = n >= kUpperWide ? std::min(kUpperBlocks, std::max(c->num_cu, 1)) : 1;
    hipLaunchKernelGGL(k_moments_upper, dim3(upper_blocks), dim3(kUpperThreads), 0, s, n,
                       (const int32_t *)c->d_noff, (const uint8_t *)c->d_nlev,
                       (const double4 *)c->d_ngeo, (const int32_t *)c->d_ctab,
                       (const int32_t *)c->d_uplist, c->d_ctr, c->d_mom64, c->d_nrec, spec,
                       c->d_flags);
    // 7. groups
    if (chunk) {
        const int64_t gmax = (n + G - 1) / G + clouds;
        hipLaunchKernelGGL(k_group_chunk_emit, grid_for(gmax, 256), dim3(256), 0, s,
                           (const int64_t *)c->d_off, clouds, G, c->d_gcl,
                           (const int32_t *)c->d_noff, c->d_groups, c->d_goff + n,
                           (const int32_t *)c->d_flags);
        return;
    }
    hipLaunchKernelGGL(k_group_count, grid_for(n + 1, 256), dim3(256), 0, s, n,
                       (const int8_t *)c->d_L, (const int8_t *)c->d_leaf,
                       (const int32_t *)c->d_noff, (const int4 *)c->d_ninfo,
                       (const int32_t *)c->d_npar, (const int64_t *)c->d_off, clouds, G,
                       c->p.group_mode, c->d_cnt, c->d_gnode, (const int32_t *)c->d_flags);
    scan_excl((const int32_t *)c->d_cnt, c->d_goff, n + 1, c->d_scanblk, s);
    hipLaunchKernelGGL(k_group_emit, grid_for(n, 256), dim3(256), 0, s, n,
                       (const int32_t *)c->d_cnt, (const int32_t *)c->d_goff,
                       (const int32_t *)c->d_gnode, (const int4 *)c->d_ninfo,
                       (const int32_t *)c->d_noff, (const int64_t *)c->d_off, clouds, G,
                       c->p.group_mode, c->d_groups, (const int32_t *)c->d_flags);
}

}  // namespace ucp
