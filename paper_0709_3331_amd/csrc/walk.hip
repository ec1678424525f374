// walk.hip -- the group tree walk of Sec. 3 on gfx950.
//
// One wavefront per walk group, one target particle per lane.  The wave walks
// the preorder node array of its cloud without a stack (first child = k + 1,
// next sibling / end of subtree = skip link).  At each node every lane
// evaluates the opening test of Eq. (5) with delta = 0 in FP64,
//     accept  iff  s^2 < theta^2 d^2,   d^2 = fma(dz,dz, fma(dy,dy, dx*dx)),
// and the wave opens the node iff any active lane fails (wave ballot).
// Accepted boxes go to an LDS-staged M2P list, opened leaves to an LDS-staged
// P2P list; a full list is evaluated (flushed) for all lanes at once.
//
// Precision (template PREC):
//   UCP_FP64  -- everything in FP64 (r = x_i - c and x_i - x_j in FP64).
//   UCP_SPLIT -- the offset of the target from a box centre is formed in FP64
//                and rounded once to FP32; source particles are stored as
//                FP32 offsets from their leaf centre, and the target offset
//                from the same leaf centre is formed in FP64 per leaf; the
//                interaction arithmetic is FP32 (FP32 moments rounded from the
//                FP64 ones), partial sums per flushed chunk are FP32 and are
//                accumulated into FP64 per-lane accumulators.
#include "internal.h"

namespace ucp {

struct WalkArgs {
    const double4 *xq;
    const float4 *xl;
    const double4 *ngeo;
    const int4 *ninfo;
    const double *mom64;
    const float4 *mom32;
    const int4 *groups;
    const int32_t *ngroups;
    const int32_t *nnodes;
    int32_t *flags_rw;
    int64_t n;
    int64_t n_spare;    // first of 64 spare accumulator slots (capacity n_max)
    int2 *gstat;
    double4 *acc;
    unsigned long long *ctr;
    const int32_t *flags;
    double th2;
    double eps2;
    float eps2f;
    int L;
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// evaluation of one accepted box (C-2.7 expansion of the softened kernel)
//   phi = Q/h + (p.r)/h^3 + (3 r.S.r/h^5 - trS/h^3)/2
//   E   = [Q/h^3 + 3(p.r)/h^5 + 7.5 r.S.r/h^7 - 1.5 trS/h^5] r - p/h^3 - 3 S r/h^5
// ---------------------------------------------------------------------------
template <typename T, bool PHI>
__device__ __forceinline__ void m2p_eval(T rx, T ry, T rz, T Q, T px, T py, T pz, T Sxx, T Syy,
                                         T Szz, T Sxy, T Sxz, T Syz, T trS, T eps2, T &ex, T &ey,
                                         T &ez, T &ph)
{
    const T h2 = rx * rx + ry * ry + rz * rz + eps2;
    T ih;
    if constexpr (sizeof(T) == 4) ih = __builtin_amdgcn_rsqf(h2);
    else ih = 1.0 / sqrt(h2);
    const T ih2 = ih * ih;
    const T ih3 = ih2 * ih;
    const T ih5 = ih3 * ih2;
    const T ih7 = ih5 * ih2;
    const T Srx = Sxx * rx + Sxy * ry + Sxz * rz;
    const T Sry = Sxy * rx + Syy * ry + Syz * rz;
    const T Srz = Sxz * rx + Syz * ry + Szz * rz;
    const T rSr = rx * Srx + ry * Sry + rz * Srz;
    const T pr = px * rx + py * ry + pz * rz;
    const T alpha = Q * ih3 + (T)3 * pr * ih5 + (T)7.5 * rSr * ih7 - (T)1.5 * trS * ih5;
    const T b3 = (T)3 * ih5;
    ex += alpha * rx - px * ih3 - b3 * Srx;
    ey += alpha * ry - py * ih3 - b3 * Sry;
    ez += alpha * rz - pz * ih3 - b3 * Srz;
    if (PHI) ph += Q * ih + pr * ih3 + (T)0.5 * ((T)3 * rSr * ih5 - trS * ih3);
}

template <int PREC, bool PHI>
__device__ __forceinline__ void flush_lists(const WalkArgs &a, const int *ml, int nm, const int *pl,
                                            int np, const double4 &xi, int i, double &E0,
                                            double &E1, double &E2, double &PH)
{
    // the list entries were written by lane 0; make them visible to the wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if constexpr (PREC == UCP_SPLIT) {
        float ex = 0.f, ey = 0.f, ez = 0.f, ph = 0.f;
        for (int e = 0; e < nm; ++e) {
            const int k = uni(ml[e]);
            const double4 g = a.ngeo[k];
            const float4 m0 = a.mom32[3 * k], m1 = a.mom32[3 * k + 1], m2 = a.mom32[3 * k + 2];
            const float rx = (float)(xi.x - g.x), ry = (float)(xi.y - g.y), rz = (float)(xi.z - g.z);
            m2p_eval<float, PHI>(rx, ry, rz, m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m2.x, m2.y,
                                 m2.z, m1.w, a.eps2f, ex, ey, ez, ph);
            if ((e & 7) == 7) {
                E0 += ex; E1 += ey; E2 += ez; PH += ph;
                ex = ey = ez = ph = 0.f;
            }
        }
        E0 += ex; E1 += ey; E2 += ez; PH += ph;
        for (int e = 0; e < np; ++e) {
            const int k = uni(pl[e]);
            const double4 g = a.ngeo[k];
            const int4 inf = a.ninfo[k];
            const float tx = (float)(xi.x - g.x), ty = (float)(xi.y - g.y), tz = (float)(xi.z - g.z);
            float sx = 0.f, sy = 0.f, sz = 0.f, sp = 0.f;
            const int j0 = uni(inf.x), j1 = uni(inf.x + inf.y);
            for (int j = j0; j < j1; ++j) {
                const float4 s = a.xl[j];
                const float rx = tx - s.x, ry = ty - s.y, rz = tz - s.z;
                const float h2 = rx * rx + ry * ry + rz * rz + a.eps2f;
                const float ih = __builtin_amdgcn_rsqf(h2);
                const float w = s.w * ih * ih * ih;
                sx += w * rx;
                sy += w * ry;
                sz += w * rz;
                if (PHI) sp += (j != i) ? s.w * ih : 0.f;
            }
            E0 += sx; E1 += sy; E2 += sz; PH += sp;
        }
    } else {
        for (int e = 0; e < nm; ++e) {
            const int k = uni(ml[e]);
            const double4 g = a.ngeo[k];
            const double *m = a.mom64 + 10 * (int64_t)k;
            const double rx = xi.x - g.x, ry = xi.y - g.y, rz = xi.z - g.z;
            m2p_eval<double, PHI>(rx, ry, rz, m[0], m[1], m[2], m[3], m[4], m[5], m[6], m[7], m[8],
                                  m[9], m[4] + m[5] + m[6], a.eps2, E0, E1, E2, PH);
        }
        for (int e = 0; e < np; ++e) {
            const int k = uni(pl[e]);
            const int4 inf = a.ninfo[k];
            const int j0 = uni(inf.x), j1 = uni(inf.x + inf.y);
            for (int j = j0; j < j1; ++j) {
                const double4 s = a.xq[j];
                const double rx = xi.x - s.x, ry = xi.y - s.y, rz = xi.z - s.z;
                const double h2 = rx * rx + ry * ry + rz * rz + a.eps2;
                const double ih = 1.0 / sqrt(h2);
                const double w = s.w * ih * ih * ih;
                E0 += w * rx;
                E1 += w * ry;
                E2 += w * rz;
                if (PHI) PH += (j != i) ? s.w * ih : 0.0;
            }
        }
    }
    // the lists are rewritten by lane 0 after this point
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int PREC, bool PHI>
__global__ __launch_bounds__(256) void k_walk(WalkArgs a)
{
    HIP_DYNAMIC_SHARED(int, lds)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int *ml = lds + wave * 2 * a.L;
    int *pl = ml + a.L;
    if (*a.flags) return;
    // every loop below is bounded by these totals, whatever the records hold
    const int ng = min(*a.ngroups, (int)a.n);
    const int nn = *a.nnodes;
    // No divergent branch anywhere in this loop: a divergent "if (lane == 0)"
    // around the queue atomic lets the compiler send only lane 0 back through
    // the atomic while the other lanes re-enter the body with a stale index.
    // Every lane executes the atomic; only lane 0 adds 1, so lane 0 receives
    // the queue value before its own increment.
    for (;;) {
        const unsigned long long old =
            atomicAdd(&a.ctr[CTR_QUEUE], lane == 0 ? 1ull : 0ull);
        const int g = uni((int)old);
        if (g >= ng) break;
        const int4 gr = a.groups[g];
        if (uni(gr.x) < 0 || uni(gr.y) < 1 || uni(gr.y) > kMaxGroup || (int64_t)uni(gr.x) + uni(gr.y) > a.n ||
            uni(gr.w) < 0 || uni(gr.w) >= nn) {
            atomicOr(a.flags_rw, UCP_FLAG_INTERNAL);
            continue;
        }
        const int gcount = uni(gr.y);
        const bool act = lane < gcount;
        const int i = gr.x + (act ? lane : 0);
        const double4 xi = a.xq[i];
        double E0 = 0.0, E1 = 0.0, E2 = 0.0, PH = 0.0;
        int nm = 0, np = 0, tot_m = 0, tot_src = 0;
        int k = uni(gr.w);
        const int kend = min(uni(a.ninfo[k].z), nn);
        while (k < kend) {
            const double4 geo = a.ngeo[k];
            const int4 inf = a.ninfo[k];
            const double dx = xi.x - geo.x, dy = xi.y - geo.y, dz = xi.z - geo.z;
            const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
            const bool fail = act && !(geo.w < a.th2 * d2);
            // the skip link always moves forward (k + 1 at least)
            const int skip = max(uni(inf.z), k + 1);
            if (__ballot(fail) == 0ull) {
                ml[nm] = k;   // every lane stores the same value
                ++nm;
                k = skip;
            } else if (inf.w & 256) {
                if (uni(inf.x) < 0 || (int64_t)uni(inf.x) + uni(inf.y) > a.n || uni(inf.y) < 0) {
                    atomicOr(a.flags_rw, UCP_FLAG_INTERNAL);
                } else {
                    pl[np] = k;
                    ++np;
                    tot_src += uni(inf.y);
                }
                k = skip;
            } else {
                ++k;
            }
            if (nm == a.L || np == a.L) {
                flush_lists<PREC, PHI>(a, ml, nm, pl, np, xi, i, E0, E1, E2, PH);
                tot_m += nm;
                nm = np = 0;
            }
        }
        flush_lists<PREC, PHI>(a, ml, nm, pl, np, xi, i, E0, E1, E2, PH);
        tot_m += nm;
        // inactive lanes store to a per-lane spare slot past the particles
        a.acc[act ? (int64_t)i : a.n_spare + lane] = make_double4(E0, E1, E2, PH);
        a.gstat[g] = make_int2(tot_m, tot_src);   // same value from every lane
        const unsigned long long zero = 0ull;
        atomicAdd(&a.ctr[CTR_P2P], lane == 0 ? (unsigned long long)gcount * (unsigned long long)tot_src : zero);
        atomicAdd(&a.ctr[CTR_M2P], lane == 0 ? (unsigned long long)gcount * (unsigned long long)tot_m : zero);
    }
}

__global__ void k_walk_reset(unsigned long long *ctr)
{
    if (threadIdx.x == 0) {
        ctr[CTR_QUEUE] = 0;
        ctr[CTR_P2P] = 0;
        ctr[CTR_M2P] = 0;
    }
}

// F_i = q_i E_i and phi_i back to the caller's order
__global__ __launch_bounds__(256) void k_scatter(const double4 *__restrict__ acc,
                                                const double4 *__restrict__ xq,
                                                const uint32_t *__restrict__ perm, int64_t n,
                                                double *f, double *phi, const int32_t *flags)
{
    if (*flags) return;
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t i = perm[p];
    const double qq = xq[p].w;
    const double4 e = acc[p];
    if (f) {
        f[3 * i + 0] = qq * e.x;
        f[3 * i + 1] = qq * e.y;
        f[3 * i + 2] = qq * e.z;
    }
    if (phi) phi[i] = e.w;
}

template <int PREC, bool PHI>
static void launch_walk_t(Ctx *c, const WalkArgs &wa, hipStream_t s)
{
    const int waves_per_cu = c->p.walk_waves > 0 ? c->p.walk_waves : 16;
    const int blocks = (c->num_cu * waves_per_cu + 3) / 4;
    const size_t lds = (size_t)4 * 2 * wa.L * sizeof(int);
    hipLaunchKernelGGL((k_walk<PREC, PHI>), dim3(blocks), dim3(256), lds, s, wa);
}

void launch_forces(Ctx *c, double *f, double *phi, hipStream_t s)
{
    const int64_t n = c->n;
    WalkArgs wa;
    wa.xq = c->d_xq;
    wa.xl = c->d_xl;
    wa.ngeo = c->d_ngeo;
    wa.ninfo = c->d_ninfo;
    wa.mom64 = c->d_mom64;
    wa.mom32 = c->d_mom32;
    wa.groups = c->d_groups;
    wa.ngroups = c->d_goff + n;
    wa.nnodes = c->d_noff + n;
    wa.flags_rw = c->d_flags;
    wa.n = n;
    wa.n_spare = c->n_max;
    wa.gstat = c->d_gstat;
    wa.acc = c->d_acc;
    wa.ctr = c->d_ctr;
    wa.flags = c->d_flags;
    wa.th2 = c->p_built.theta * c->p_built.theta;
    wa.eps2 = c->p_built.eps * c->p_built.eps;
    wa.eps2f = (float)wa.eps2;
    wa.L = c->p_built.list_len;
    hipLaunchKernelGGL(k_walk_reset, dim3(1), dim3(64), 0, s, c->d_ctr);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        if ((int64_t)c->ev.size() < 2 * (c->ev_used + 1)) {
            hipEvent_t a, b;
            (void)hipEventCreate(&a);
            (void)hipEventCreate(&b);
            c->ev.push_back(a);
            c->ev.push_back(b);
        }
        e0 = c->ev[2 * c->ev_used];
        e1 = c->ev[2 * c->ev_used + 1];
        c->ev_used++;
        (void)hipEventRecord(e0, s);
    }
    const bool want_phi = phi != nullptr || f == nullptr;
    if (c->p_built.precision == UCP_SPLIT) {
        if (want_phi) launch_walk_t<UCP_SPLIT, true>(c, wa, s);
        else launch_walk_t<UCP_SPLIT, false>(c, wa, s);
    } else {
        if (want_phi) launch_walk_t<UCP_FP64, true>(c, wa, s);
        else launch_walk_t<UCP_FP64, false>(c, wa, s);
    }
    if (c->timing) (void)hipEventRecord(e1, s);
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (const double4 *)c->d_acc, (const double4 *)c->d_xq,
                       (const uint32_t *)c->d_perm, n, f, phi, (const int32_t *)c->d_flags);
}

}  // namespace ucp
