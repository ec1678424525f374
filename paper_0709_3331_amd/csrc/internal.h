// internal.h -- context layout, device helpers and kernel-launch declarations
// shared by the HIP translation units of the TREE library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ucp.h"

namespace ucp {

constexpr int kWave = 64;
constexpr int kMaxGroup = 64;      // one target particle per lane
constexpr int kMaxLeafCap = 64;
constexpr int kScanBlock = 1024;   // threads per scan block
constexpr int kScanItems = 4;      // elements per thread in the scan
constexpr int kSortThreads = 1024;  // 16 waves per sort block
constexpr int kSortItems = 2;       // rounds of kSortThreads elements per tile
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kSortTickets = 32;
constexpr int kSortPassesMax = 12;   // 8 key passes (63-bit keys) + up to 4 cloud passes
constexpr int kScanSmallItems = 64;            // elements per thread, one-block scan
// one block streams at most a few KB efficiently; longer arrays take the
// three-kernel scan
constexpr int64_t kScanSmallLimit = 4096;
constexpr uint8_t kLeafBit = 0x80;             // leaf flag of the per-node level byte
constexpr int kSpecVals = 12;                   // doubles per node of the species pseudo-particles

// device counter slots (unsigned long long)
enum { CTR_P2P = 0, CTR_M2P = 1, CTR_MAXLEVEL = 2, CTR_BARRIER = 3, CTR_VJPMAX = 4,
       CTR_UPCOUNT = 5, CTR_SORTFULL = 6, CTR_SORTBAR = 7, CTR_OFFTICKET = 8, CTR_NCTR = 9 };
// walk work queues: one per XCD, each on its own 128-byte line
constexpr int kWalkQueues = 8, kQStride = 16;

struct Ctx;

// ---------------------------------------------------------------------------
// Host-side launch helpers (defined in the .hip files).  All enqueue on `s`.
// ---------------------------------------------------------------------------
// build.hip
void launch_build(Ctx *c, const double *x, const double *q, const int64_t *offsets_in,
                  int clouds, int64_t n, hipStream_t s);
// walk.hip
void launch_forces(Ctx *c, double *f, double *phi, hipStream_t s);
// device scratch of the adjoint: sorted cotangents (n), source-side pair
// cotangents (4 n doubles), cell cotangents (10 doubles per node slot), and
// per cloud the cube-origin cotangent (4 doubles) and minimum particles (3)
struct VjpScratch {
    double4 *w;
    double *xsrc;
    double *cbar;
    double *lobar;
    uint32_t *lomin;
};
void launch_vjp(Ctx *c, const VjpScratch &sc, const double *u, double *xbar, hipStream_t s);
// integrate.hip
void launch_kick_drift(double *x, double *v, const double *f, const double *m, int64_t n,
                       double dt, hipStream_t s);
// the closing kick of one step and the opening kick and drift of the next
void launch_kick_kick_drift(double *x, double *v, const double *f, const double *m, int64_t n,
                            double dt, hipStream_t s);
void launch_kick(double *v, const double *f, const double *m, int64_t n, double dt,
                 hipStream_t s);
void launch_energy(Ctx *c, const double *v, const double *q, const double *m, int64_t n,
                   double *out, hipStream_t s);
void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s);
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// The context.  Every device buffer is sized at create time.
// ---------------------------------------------------------------------------
struct Ctx {
    int device = 0;
    int num_cu = 256;
    ucp_params p{};
    int64_t n_max = 0;
    int32_t clouds_max = 0;
    int64_t node_cap = 0;
    int64_t hist_cap = 0;

    // last build
    int built = 0;
    // the last enqueued build cleared the walk's counters and queue heads and
    // no walk has run since, so the next force walk needs no reset of its own
    bool walk_armed = false;
    int64_t n = 0;
    int32_t clouds = 0;
    ucp_params p_built{};

    // per cloud
    int64_t *d_off = nullptr;               // [clouds_max + 1]
    unsigned long long *d_mm = nullptr;     // [clouds_max][6] ordered min xyz, max xyz
    double4 *d_cube = nullptr;              // [clouds_max][2]: {lo xyz, L}, {scale, e, -, -}
    // sort
    // buffer 0: keys in input order; 1 and 2: the passes; the sorted keys end in 2
    uint64_t *d_key[3] = {nullptr, nullptr, nullptr};
    uint32_t *d_val[3] = {nullptr, nullptr, nullptr};
    // radix sort: per-(tile, digit) status words of the decoupled look-back
    // (two arrays, alternating by pass), the digit counts of every pass, and
    // one ticket counter per pass
    uint32_t *d_hist = nullptr;             // [256 * tiles] status, even passes
    uint32_t *d_histscan = nullptr;         // [256 * tiles] status, odd passes
    uint32_t *d_ghist = nullptr;            // [kSortPassesMax * 256]
    uint32_t *d_sortctl = nullptr;          // [kSortTickets]
    uint64_t *d_skey = nullptr;             // sorted keys (points into d_key[])
    uint32_t *d_perm = nullptr;             // sorted position -> caller index
    // particles: packed in input order by the key kernel, then sorted
    double4 *d_xin = nullptr;               // [n_max] x, y, z, q  (input order)
    double4 *d_xq = nullptr;                // [n_max] x, y, z, q  (sorted order)
    // per position
    int8_t *d_L = nullptr;                  // [n_max + 1] common-prefix level with predecessor
    int8_t *d_leaf = nullptr;               // [n_max + 1] level of the leaf holding the position
    int32_t *d_cnt = nullptr;               // [n_max + 1] per-position counts to scan
    int32_t *d_lend = nullptr;              // [n_max + 1] end of the leaf starting there (-1: scan)
    int32_t *d_lvlmax = nullptr;            // [n_max / 256 + 2] deepest leaf level per level-pass block
    unsigned long long *d_offstat = nullptr; // [n_max / 4096 + 2] look-back words of the node offsets
    int32_t *d_noff = nullptr;              // [n_max + 1] first node starting at the position
    int32_t *d_goff = nullptr;              // [n_max + 1] first group starting at the position
    int32_t *d_gnode = nullptr;             // [n_max]
    int32_t *d_gcl = nullptr;               // [clouds_max + 1] first chunk group of each cloud
    int32_t *d_scanblk = nullptr;           // scan block sums
    // nodes
    double4 *d_ngeo = nullptr;              // [node_cap] centre xyz, side^2
    int4 *d_ninfo = nullptr;                // [node_cap] first, count, skip, level | 256*leaf
    int32_t *d_npar = nullptr;              // [node_cap] parent (-1 for a root)
    uint8_t *d_nlev = nullptr;              // [node_cap + 128] level of each node, | kLeafBit for a leaf
    int32_t *d_uplist = nullptr;            // [node_cap] the internal nodes summed from their children
    int32_t *d_ctab = nullptr;              // [8 node_cap] an internal node's children in order, -1 after the last
    // per-species pseudo-particles (UCP_EXPANSION_SPECIES), allocated when that
    // expansion is first set: c+[3] Q+ c-[3] Q- delta+ delta- 0 0
    double *d_spec = nullptr;               // [node_cap][kSpecVals]
    double *d_mom64 = nullptr;              // [node_cap][16] cx cy cz Q p[3] trS S[6] 0 0
    // node record for the walk, two 64-byte lines per node:
    //   line 1: cx cy cz side^2 (double), skip first count level|256*leaf (int)
    //   line 2: Q px py pz | 1.5 trS 3Sxx 3Syy 3Szz | 3Sxy 3Sxz 3Syz 0   (float)
    float4 *d_nrec = nullptr;               // [node_cap][8]
    // groups
    int4 *d_groups = nullptr;               // [n_max] first, count, node, root
    int2 *d_gstat = nullptr;                // [n_max] accepted boxes, P2P sources
    int32_t *d_leafof = nullptr;            // [n_max] leaf holding each sorted position
    // results (sorted order)
    double4 *d_acc = nullptr;               // [n_max] E xyz, phi
    // adjoint, allocated by the first ucp_force_vjp
    double4 *d_w = nullptr;                 // [n_max] q_i u_i, sorted
    double *d_xsrc = nullptr;               // [n_max][4] source-side P2P cotangent
    double *d_cbar = nullptr;               // [node_cap][10] cell cotangents
    double *d_lobar = nullptr;              // [clouds_max][4] cube-origin cotangent per cloud
    uint32_t *d_lomin = nullptr;            // [clouds_max][3] caller index of each axis' minimum
    // counters, flags
    unsigned long long *d_ctr = nullptr;    // [CTR_NCTR]
    unsigned long long *d_wq = nullptr;     // [kWalkQueues * kQStride] walk queue heads
    int32_t *d_flags = nullptr;             // [1]
    // energy partials
    double *d_epart = nullptr;              // [256][8]

    // graphs of a Verlet step: every step but the last (ending in the closing
    // kick fused with the next step's opening kick and drift) and the last
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr, gexec_last = nullptr;
    hipGraph_t graph = nullptr, graph_last = nullptr;
    std::vector<uintptr_t> gkey;

    // timing
    int timing = 0;
    std::vector<hipEvent_t> ev;             // pairs
    int64_t ev_used = 0;
    unsigned long long *d_wclock = nullptr; // [3 * num_cu * 64] start, end and unit of every
                                            // wave of the last walk launched with timing on
    int64_t wclock_waves = 0;               // waves of that walk

    std::string err;
};

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long f64_ordered(double d)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(d);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ __forceinline__ double f64_from_ordered(unsigned long long u)
{
    u = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
    return __longlong_as_double((long long)u);
}

// bits 0..20 of v moved to bits 0, 3, 6, ..., 60
__device__ __forceinline__ uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// cloud holding particle i: largest c with off[c] <= i (off has clouds+1 entries)
__device__ __forceinline__ int cloud_of(const int64_t *__restrict__ off, int clouds, int64_t i)
{
    int lo = 0, hi = clouds;   // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

}  // namespace ucp
