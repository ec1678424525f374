// walk.hip -- the group tree walk of Sec. 3 on gfx950.
//
// One wavefront per walk group.  The wave keeps an LDS stack of sibling
// ranges [k, end) of the preorder node array (first child = k + 1, next
// sibling = skip link) and tests up to 64 nodes at once, one per lane.  For
// each node the opening test of Eq. (5) with delta = 0 is evaluated in FP64
// for every target of the group,
//     accept  iff  s^2 < theta^2 d^2,   d^2 = fma(dz,dz, fma(dy,dy, dx*dx)),
// and the node is opened iff any target fails.  Accepted boxes go to an LDS
// M2P list, opened leaves to an LDS P2P list; a full list is evaluated
// (flushed) at once.  At the end of a group the lane that owns a target
// writes F_i = q_i E_i and phi_i at the caller's index (or, for the energy
// and the adjoint, the sorted field).
//
// Node record (two 64-byte lines per node, written by the build): line 1
// holds the FP64 centre, side^2, skip, first, count and level|leaf flag and
// is all the traversal reads; line 2 holds the FP32 moments, read when an
// accepted box is staged.
//
// Lane layout: a group of c <= 64 targets gives each target lpt = floor(64/c)
// lanes.  The lanes of one target take the staged entries round-robin and
// their partial sums are added in fixed lane order at the end of the group
// (deterministic), so small groups still keep most lanes busy.
//
// Precision (template PREC):
//   UCP_FP64  -- staged entries are FP64 (absolute box centres and positions),
//                the interaction arithmetic is FP64 (r = x_i - c, x_i - x_j).
//   UCP_SPLIT -- staged entries are FP32 offsets from c_g, the centre of the
//                members' bounding box, formed in FP64 and rounded once (box
//                centre - c_g, source - c_g), with FP32 moments rounded from
//                the FP64 ones; the target offset x_i - c_g is also formed in
//                FP64 and rounded once.  The interaction arithmetic is FP32;
//                partial sums of each flushed list are FP32 and are
//                accumulated into FP64 per-lane accumulators.
//
// No divergent branch encloses a wave-level operation or the loop heads of
// the persistent loop: list staging writes one value per lane, idle lanes
// write to private spare slots.
#include <type_traits>

#include "internal.h"

namespace ucp {

// what a walk launch computes
enum { kWalkForce = 0, kWalkForcePhi = 1, kWalkVjp = 2 };
// at most this many waves share an adjoint group's evaluation
constexpr int kMaxParts = 4;

struct WalkArgs {
    const double4 *xq;
    const double4 *w;       // adjoint: sorted target cotangents q_i u_i
    double *cbar;           // adjoint: per node pbar[3], (Sbar + Sbar^T)[6], pad (10 doubles)
    double *xsrc;           // adjoint: per particle source-side P2P cotangent (4 doubles)
    double *lobar;          // adjoint: per cloud cotangent of the cube origin (4 doubles)
    const int64_t *off;     // cloud offsets [clouds + 1]
    int clouds;
    const float4 *nrec;
    const double *mom64;
    const int4 *groups;
    const int32_t *ngroups;
    const int32_t *nnodes;
    int2 *gstat;
    double4 *acc;           // per sorted target (E, phi), when fout and phiout are null
    double *fout;           // F_i = q_i E_i in the caller's order, or null
    double *phiout;         // phi_i in the caller's order, or null
    const uint32_t *perm;   // sorted position -> caller index
    unsigned long long *ctr;
    unsigned long long *wq;     // queue heads (kWalkQueues, kQStride apart)
    const int32_t *flags;
    int32_t *flags_rw;
    int64_t n;
    int64_t n_spare;    // first of 64 spare accumulator slots (capacity n_max)
    double th2;
    double eps2;
    float eps2f;
    double inv_lambda;      // 1 / lambda_ei under the Kelbg pair law
    float inv_lambdaf;
    const double *spec;     // per-species pseudo-particles (UCP_EXPANSION_SPECIES)
    double theta;
    int L;
    unsigned long long *wclock;   // or null: each wave's start, end (real-time counter) and unit
    int parts;              // adjoint: waves that share a group's evaluation (1 otherwise)
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Traversal stack entries per wave.  A batch pops at most kStackSoft - sp
// entries (at least one) and pushes at most two per popped entry, children on
// top, so the stack never passes kStackSoft by more than the depth of the
// tree (22 levels for 63-bit keys).
constexpr int kStackCap = 192;
constexpr int kStackSoft = kStackCap - 40;

// LDS layout of one wave (bytes): traversal stack (node, end of its sibling
// range), the M2P list (node, FP32 offset of its centre from the group centre),
// the P2P list (first particle, count of an opened leaf), a staging area (64
// M2P records of 16 values, or 64 P2P particles, or the final per-lane partial
// sums) and two 64-int tables for expanding leaves into particles.
// staged M2P records are kRec values apart: 80-byte (FP32) records put eight
// consecutive records on distinct LDS banks
constexpr int kRec = 20;
template <int PREC>
__host__ __device__ constexpr int walk_stage_bytes()
{
    return PREC == UCP_SPLIT ? 64 * kRec * 4 : 64 * kRec * 8;
}
template <int PREC>
__host__ __device__ constexpr int walk_wave_bytes(int L)
{
    return kStackCap * 8 + 16 * L + 8 * L + walk_stage_bytes<PREC>() + 2 * 64 * 4;
}

__device__ __forceinline__ int lanes_before(unsigned long long mask, int lane)
{
    return __popcll(mask & (lane == 0 ? 0ull : (~0ull >> (64 - lane))));
}

__device__ __forceinline__ double wave_fmin(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_fmax(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
// value of v held by lane src (src uniform over the wave)
__device__ __forceinline__ double readlane_d(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int wave_isum(int v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int wave_incl_scan_i(int v, int lane)
{
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o);
        v += lane >= o ? t : 0;
    }
    return v;
}

// ---------------------------------------------------------------------------
// evaluation of one accepted box: second-order expansion of the softened
// kernel about the box centre (r = target - centre, h^2 = |r|^2 + eps^2)
//   phi = Q/h + (p.r)/h^3 + (3 r.S.r/h^5 - trS/h^3)/2
//   E   = [Q/h^3 + 3(p.r)/h^5 + 7.5 r.S.r/h^7 - 1.5 trS/h^5] r - p/h^3 - 3 S r/h^5
// evaluated as E = h^-3 [ b r - u ] with u = p + h^-2 (3S) r and
// b = Q + h^-2 (3 p.r - 1.5 trS + 2.5 h^-2 r.(3S).r); the staged record holds
// c[3], Q, p[3], 1.5 trS and the six components of 3S.
// ---------------------------------------------------------------------------
// S3xx .. S3yz are the components of 3S.
template <typename T, bool PHI>
__device__ __forceinline__ void m2p_eval(T rx, T ry, T rz, T Q, T px, T py, T pz, T S3xx, T S3yy,
                                         T S3zz, T S3xy, T S3xz, T S3yz, T trS15, T eps2, T &ex,
                                         T &ey, T &ez, T &ph)
{
    const T h2 = fma(rx, rx, fma(ry, ry, fma(rz, rz, eps2)));
    T ih;
    if constexpr (sizeof(T) == 4) ih = __builtin_amdgcn_rsqf(h2);
    else ih = 1.0 / sqrt(h2);
    const T ih2 = ih * ih;
    const T ih3 = ih2 * ih;
    const T Srx = fma(S3xx, rx, fma(S3xy, ry, S3xz * rz));   // (3S) r
    const T Sry = fma(S3xy, rx, fma(S3yy, ry, S3yz * rz));
    const T Srz = fma(S3xz, rx, fma(S3yz, ry, S3zz * rz));
    const T rSr = fma(rx, Srx, fma(ry, Sry, rz * Srz));      // 3 r.S.r
    const T pr = fma(px, rx, fma(py, ry, pz * rz));
    const T ux = fma(ih2, Srx, px), uy = fma(ih2, Sry, py), uz = fma(ih2, Srz, pz);
    const T a = fma((T)2.5 * ih2, rSr, fma((T)3, pr, -trS15));
    const T b = fma(ih2, a, Q);
    ex = fma(ih3, fma(b, rx, -ux), ex);
    ey = fma(ih3, fma(b, ry, -uy), ey);
    ez = fma(ih3, fma(b, rz, -uz), ez);
    // phi = h^-1 [ Q + h^-2 (p.r - trS/2 + 1.5 h^-2 r.S.r) ]
    if (PHI) ph = fma(ih, fma(ih2, fma((T)0.5 * ih2, rSr, pr - trS15 * (T)(1.0 / 3.0)), Q), ph);
}

// one staged M2P record, read with 16-byte LDS loads.  FP32 record: dx dy dz 0,
// Q px py pz, 1.5 trS 3Sxx 3Syy 3Szz, 3Sxy 3Sxz 3Syz 0; FP64 record: cx cy cz Q
// px py pz 1.5 trS 3Sxx 3Syy 3Szz 3Sxy 3Sxz 3Syz.
template <typename T, bool PHI>
__device__ __forceinline__ void m2p_rec(const T *r, T tx, T ty, T tz, T eps2, T &ex, T &ey, T &ez,
                                        T &ph)
{
    if constexpr (sizeof(T) == 4) {
        const float4 a = ((const float4 *)r)[0], b = ((const float4 *)r)[1];
        const float4 c = ((const float4 *)r)[2], d = ((const float4 *)r)[3];
        m2p_eval<T, PHI>(tx - a.x, ty - a.y, tz - a.z, b.x, b.y, b.z, b.w, c.y, c.z, c.w, d.x, d.y,
                         d.z, c.x, eps2, ex, ey, ez, ph);
    } else {
        const double2 *v = (const double2 *)r;
        const double2 a = v[0], b = v[1], c = v[2], d = v[3], e = v[4], f = v[5], g = v[6];
        m2p_eval<T, PHI>(tx - a.x, ty - a.y, tz - b.x, b.y, c.x, c.y, d.x, e.x, e.y, f.x, f.y, g.x,
                         g.y, d.y, eps2, ex, ey, ez, ph);
    }
}

// the two per-species pseudo-particles of an accepted box (staged as c+ Q+
// c- Q-, offsets in FP32 or positions in FP64), each softened like a pair
template <typename T, bool PHI>
__device__ __forceinline__ void m2p_species(const T *r, T tx, T ty, T tz, T eps2, T &ex, T &ey,
                                            T &ez, T &ph)
{
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
        const T *v = r + 4 * sp;
        const T rx = tx - v[0], ry = ty - v[1], rz = tz - v[2], q = v[3];
        const T h2 = fma(rx, rx, fma(ry, ry, fma(rz, rz, eps2)));
        T ih;
        if constexpr (sizeof(T) == 4) ih = __builtin_amdgcn_rsqf(h2);
        else ih = 1.0 / sqrt(h2);
        const T w = q * (ih * ih * ih);
        ex = fma(w, rx, ex);
        ey = fma(w, ry, ey);
        ez = fma(w, rz, ez);
        if (PHI) ph = fma(q, ih, ph);
    }
}

template <typename T, bool PHI, bool SPEC>
__device__ __forceinline__ void m2p_entry(const T *r, T tx, T ty, T tz, T eps2, T &ex, T &ey,
                                          T &ez, T &ph)
{
    if constexpr (SPEC) m2p_species<T, PHI>(r, tx, ty, tz, eps2, ex, ey, ez, ph);
    else m2p_rec<T, PHI>(r, tx, ty, tz, eps2, ex, ey, ez, ph);
}

// ---------------------------------------------------------------------------
// adjoint of one accepted box.  With w the target's cotangent (q_i times the
// cotangent of F_i), r = target - centre and h^2 = |r|^2 + eps^2:
//   target side  g = d(w.E)/dr = g_QP + g_S,
//     g_QP = [(w.r)(-3 Q h^-5 - 15 (p.r) h^-7) + 3 (w.p) h^-5] r
//            + (Q h^-3 + 3 (p.r) h^-5) w + 3 (w.r) h^-5 p,
//     g_S  = [(w.r)(-52.5 (r.S.r) h^-9 + 7.5 trS h^-7) + 15 (w.S.r) h^-7] r
//            + (7.5 (r.S.r) h^-7 - 1.5 trS h^-5) w + 15 (w.r) h^-7 S r - 3 h^-5 S w;
//   source side  pbar += 3 (w.r) h^-5 r - h^-3 w,
//                sym  += 15 (w.r) h^-7 r r^T - 3 (w.r) h^-5 I - 3 h^-5 (w r^T + r w^T),
// sym being Sbar + Sbar^T; a particle j of the box then receives
// q_j (pbar + sym (x_j - c)).
//   Box centre.  Every centre is the cube origin plus a fixed offset, and the
// origin is the minimum particle of each axis.  The derivative of a Taylor
// expansion to order n with respect to its expansion point, the moments
// moving with it, telescopes to the order-n terms alone (the lower orders
// cancel): here d(w.E)/dc = (1/2) w_d S_ab d^4 G/dr_a dr_b dr_c dr_d with
// G = 1/h, which is -g_S.  So the centre's cotangent is -g_S, formed without
// the cancellation of the Q and p terms, and its sum over the boxes of a
// cloud goes to the cloud's minimum particles.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void m2p_adj_target(T rx, T ry, T rz, T Q, T px, T py, T pz, T Sxx,
                                               T Syy, T Szz, T Sxy, T Sxz, T Syz, T trS15, T wx,
                                               T wy, T wz, T eps2, T &gx, T &gy, T &gz, T &lx,
                                               T &ly, T &lz)
{
    const T h2 = fma(rx, rx, fma(ry, ry, fma(rz, rz, eps2)));
    T ih;
    if constexpr (sizeof(T) == 4) ih = __builtin_amdgcn_rsqf(h2);
    else ih = 1.0 / sqrt(h2);
    const T ih2 = ih * ih, ih3 = ih2 * ih, ih5 = ih3 * ih2, ih7 = ih5 * ih2, ih9 = ih7 * ih2;
    const T Srx = fma(Sxx, rx, fma(Sxy, ry, Sxz * rz));
    const T Sry = fma(Sxy, rx, fma(Syy, ry, Syz * rz));
    const T Srz = fma(Sxz, rx, fma(Syz, ry, Szz * rz));
    const T Swx = fma(Sxx, wx, fma(Sxy, wy, Sxz * wz));
    const T Swy = fma(Sxy, wx, fma(Syy, wy, Syz * wz));
    const T Swz = fma(Sxz, wx, fma(Syz, wy, Szz * wz));
    const T ur = fma(wx, rx, fma(wy, ry, wz * rz));
    const T pr = fma(px, rx, fma(py, ry, pz * rz));
    const T up = fma(wx, px, fma(wy, py, wz * pz));
    const T rSr = fma(rx, Srx, fma(ry, Sry, rz * Srz));
    const T uSr = fma(wx, Srx, fma(wy, Sry, wz * Srz));
    const T aS = ur * ((T)5 * trS15 * ih7 - (T)52.5 * rSr * ih9) + (T)15 * uSr * ih7;
    const T aQP = ur * (-(T)3 * Q * ih5 - (T)15 * pr * ih7) + (T)3 * up * ih5;
    const T bS = (T)7.5 * rSr * ih7 - trS15 * ih5;
    const T bQP = Q * ih3 + (T)3 * pr * ih5;
    const T cp = (T)3 * ur * ih5, cs = (T)15 * ur * ih7, cw = (T)3 * ih5;
    const T sx = aS * rx + bS * wx + cs * Srx - cw * Swx;
    const T sy = aS * ry + bS * wy + cs * Sry - cw * Swy;
    const T sz = aS * rz + bS * wz + cs * Srz - cw * Swz;
    gx += aQP * rx + bQP * wx + cp * px + sx;
    gy += aQP * ry + bQP * wy + cp * py + sy;
    gz += aQP * rz + bQP * wz + cp * pz + sz;
    lx -= sx;
    ly -= sy;
    lz -= sz;
}

template <typename T>
__device__ __forceinline__ void m2p_adj_source(T rx, T ry, T rz, T wx, T wy, T wz, T eps2, T *cb)
{
    const T h2 = fma(rx, rx, fma(ry, ry, fma(rz, rz, eps2)));
    T ih;
    if constexpr (sizeof(T) == 4) ih = __builtin_amdgcn_rsqf(h2);
    else ih = 1.0 / sqrt(h2);
    const T ih2 = ih * ih, ih3 = ih2 * ih, ih5 = ih3 * ih2, ih7 = ih5 * ih2;
    const T ur = fma(wx, rx, fma(wy, ry, wz * rz));
    const T a5 = (T)3 * ur * ih5, a7 = (T)15 * ur * ih7, c5 = (T)3 * ih5;
    cb[0] += a5 * rx - ih3 * wx;
    cb[1] += a5 * ry - ih3 * wy;
    cb[2] += a5 * rz - ih3 * wz;
    cb[3] += a7 * rx * rx - a5 - (T)2 * c5 * wx * rx;
    cb[4] += a7 * ry * ry - a5 - (T)2 * c5 * wy * ry;
    cb[5] += a7 * rz * rz - a5 - (T)2 * c5 * wz * rz;
    cb[6] += a7 * rx * ry - c5 * (wx * ry + rx * wy);
    cb[7] += a7 * rx * rz - c5 * (wx * rz + rx * wz);
    cb[8] += a7 * ry * rz - c5 * (wy * rz + ry * wz);
}

// adjoint of one particle pair: d(w.K)/dr with K = r h^-3 is w h^-3 - 3 (w.r) r h^-5
template <typename T>
__device__ __forceinline__ void p2p_adj(T rx, T ry, T rz, T sq, T wx, T wy, T wz, T eps2, T &gx,
                                        T &gy, T &gz)
{
    const T h2 = fma(rx, rx, fma(ry, ry, fma(rz, rz, eps2)));
    T ih;
    if constexpr (sizeof(T) == 4) ih = __builtin_amdgcn_rsqf(h2);
    else ih = 1.0 / sqrt(h2);
    const T ih3 = ih * ih * ih;
    const T c3 = sq * ih3, c5 = (T)3 * sq * fma(wx, rx, fma(wy, ry, wz * rz)) * ih3 * ih * ih;
    gx += c3 * wx - c5 * rx;
    gy += c3 * wy - c5 * ry;
    gz += c3 * wz - c5 * rz;
}

// one FP32 particle pair: source (offset, charge) in v; phi skips the self pair
template <bool PHI>
__device__ __forceinline__ void p2p_one(float tx, float ty, float tz, const float4 &v, float eps2,
                                        bool notself, float &ex, float &ey, float &ez, float &ph)
{
    const float rx = tx - v.x, ry = ty - v.y, rz = tz - v.z;
    const float h2 = fmaf(rx, rx, fmaf(ry, ry, fmaf(rz, rz, eps2)));
    const float ih = __builtin_amdgcn_rsqf(h2);
    const float w = v.w * (ih * ih * ih);
    ex = fmaf(w, rx, ex);
    ey = fmaf(w, ry, ey);
    ez = fmaf(w, rz, ez);
    if (PHI) ph += notself ? v.w * ih : 0.f;
}

// Kelbg electron-ion pair (Eq. (3)), u = r / lambda: the force bracket
// g = 1 - e^{-u}(1 + u) and the potential bracket p = 1 - e^{-u}.  Both vanish
// with u (as u^2/2 and u) and the exponential forms cancel there, so below
// u = 1/2 they are summed from their Taylor series in Horner form,
//   g = u^2 sum_{m>=2} (-1)^m (m-1)/m! u^(m-2),  p = u sum_{m>=1} (-1)^(m-1) u^(m-1)/m!,
// to the term below the type's rounding at u = 1/2 (FP32: m = 9 and 8; FP64:
// m = 16 and 15); above, from the exponential.
__host__ __device__ constexpr double inv_factorial(int m)
{
    double f = 1.0;
    for (int i = 2; i <= m; ++i) f *= (double)i;
    return 1.0 / f;
}

template <typename T>
__device__ __forceinline__ void kelbg_brackets(T u, T &g, T &p)
{
    constexpr int MG = sizeof(T) == 4 ? 9 : 16, MP = sizeof(T) == 4 ? 8 : 15;
    if (u < (T)0.5) {
        T sg = (T)((MG - 1) * inv_factorial(MG));
#pragma unroll
        for (int m = MG - 1; m >= 2; --m) sg = (T)((m - 1) * inv_factorial(m)) - u * sg;
        T sp = (T)inv_factorial(MP);
#pragma unroll
        for (int m = MP - 1; m >= 1; --m) sp = (T)inv_factorial(m) - u * sp;
        g = u * u * sg;
        p = u * sp;
    } else {
        T e;
        if constexpr (sizeof(T) == 4) e = __expf(-u);
        else e = exp(-u);
        g = (T)1 - e * ((T)1 + u);
        p = (T)1 - e;
    }
}

// one particle pair under the Kelbg law: the electron-ion pair (q_s q_t < 0)
// through the brackets above, a like pair through the softened Coulomb law
// (eps2 may be 0).  A pair at r = 0 exerts no force; its potential is
// q_s / lambda for an electron-ion pair and nothing for the self pair.
template <typename T, bool PHI>
__device__ __forceinline__ void p2p_kelbg(T rx, T ry, T rz, T sq, T qt, T eps2, T inv_lam,
                                          bool notself, T &ex, T &ey, T &ez, T &ph)
{
    const T r2 = fma(rx, rx, fma(ry, ry, rz * rz));
    const bool ei = sq * qt < (T)0;
    const T h2 = ei ? r2 : r2 + eps2;
    const bool live = h2 > (T)0;
    T ih;
    if constexpr (sizeof(T) == 4) ih = __builtin_amdgcn_rsqf(live ? h2 : (T)1);
    else ih = 1.0 / sqrt(live ? h2 : (T)1);
    T ga = (T)1, pa = (T)1;
    if (ei) kelbg_brackets<T>(r2 * ih * inv_lam, ga, pa);
    const T w = live ? sq * ga * (ih * ih * ih) : (T)0;
    ex = fma(w, rx, ex);
    ey = fma(w, ry, ey);
    ez = fma(w, rz, ez);
    if (PHI) ph += notself ? (live ? sq * pa * ih : (ei ? sq * inv_lam : (T)0)) : (T)0;
}

__device__ __forceinline__ float readlane_t(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double readlane_t(double v, int src) { return readlane_d(v, src); }

// record fields of a staged M2P entry (see m2p_rec for the two layouts)
template <typename T>
struct CellRec {
    T cx, cy, cz, Q, px, py, pz, trS15, Sxx, Syy, Szz, Sxy, Sxz, Syz;
};
template <typename T>
__device__ __forceinline__ CellRec<T> load_rec(const T *r)
{
    CellRec<T> c;
    if constexpr (sizeof(T) == 4) {
        const float4 a = ((const float4 *)r)[0], b = ((const float4 *)r)[1];
        const float4 d = ((const float4 *)r)[2], e = ((const float4 *)r)[3];
        c = {a.x, a.y, a.z, b.x, b.y, b.z, b.w, d.x, d.y, d.z, d.w, e.x, e.y, e.z};
    } else {
        c = {r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7], r[8], r[9], r[10], r[11], r[12], r[13]};
    }
    return c;
}

// staged record in adjoint mode: FP64 box centre, then the moments in T
// (UCP_SPLIT: 3 doubles then 11 floats, 68 bytes; UCP_FP64: the record of
// m2p_rec).  The adjoint's terms grow as h^-5 and h^-7, so its differences
// x_i - c are formed in FP64 and rounded once.
template <int PREC, typename T>
__device__ __forceinline__ void load_adj_rec(const T *r, CellRec<T> &m, double &cx, double &cy,
                                             double &cz)
{
    if constexpr (PREC == UCP_SPLIT) {
        const double *d = (const double *)r;
        cx = d[0];
        cy = d[1];
        cz = d[2];
        const float *f = (const float *)r + 6;
        m.Q = f[0]; m.px = f[1]; m.py = f[2]; m.pz = f[3];
        m.trS15 = f[4]; m.Sxx = f[5]; m.Syy = f[6]; m.Szz = f[7];
        m.Sxy = f[8]; m.Sxz = f[9]; m.Syz = f[10];
    } else {
        m = load_rec(r);
        cx = m.cx;
        cy = m.cy;
        cz = m.cz;
    }
    // the records hold 3S
    const T third = (T)(1.0 / 3.0);
    m.Sxx *= third; m.Syy *= third; m.Szz *= third;
    m.Sxy *= third; m.Sxz *= third; m.Syz *= third;
}

// Per-target state of a group in the walk: target offset (or position),
// cotangent (adjoint mode), and the FP64 per-lane accumulators.
template <typename T>
struct Target {
    T tx, ty, tz, wx, wy, wz;
    T qt;                        // target charge (the Kelbg law depends on the pair's signs)
    double px, py, pz;           // FP64 position (adjoint P2P differences)
    int i;                       // sorted index of the lane's target
    double E0, E1, E2, PH;       // field and potential, or the target-side adjoint
    double C0, C1, C2;           // adjoint: the lane's share of the cube-origin cotangent
    int part, ck;                // adjoint: this wave's share of the group, chunks seen
};

// Evaluate the M2P and P2P index lists of a group.  Entries are staged into
// LDS 64 at a time (one per lane), then the lpt lanes of each target take the
// staged entries round-robin.  In adjoint mode a second pass over the same
// staged entries gives each lane one entry, loops over the group's targets
// (broadcast from their lanes) and adds the entry's source-side cotangent to
// the global per-cell or per-particle arrays.
template <int PREC, int MODE, bool KELBG, bool SPEC, typename T>
__device__ __forceinline__ void flush_lists(const WalkArgs &a, const int4 *ml, int nm,
                                            const int2 *pl, int np, T *stage, int *pfx,
                                            int *lfirst, int lane, int sub, int lpt, int c,
                                            int gfirst, const double4 &cg, Target<T> &tg)
{
    constexpr bool PHI = MODE == kWalkForcePhi;
    constexpr bool ADJ = MODE == kWalkVjp;
    const T eps2 = PREC == UCP_SPLIT ? (T)a.eps2f : (T)a.eps2;
    const T inv_lam = PREC == UCP_SPLIT ? (T)a.inv_lambdaf : (T)a.inv_lambda;
    const T tx = tg.tx, ty = tg.ty, tz = tg.tz;
    wave_sync();   // the lists were written by other lanes
    // adjoint with the group shared by a.parts waves: every wave builds the
    // same lists, and each staged chunk of boxes or source particles is
    // evaluated by one of them, in turn
    auto mine = [&]() {
        if constexpr (ADJ) return a.parts == 1 || tg.ck++ % a.parts == tg.part;
        else return true;
    };
    for (int base = 0; base < nm; base += 64) {
        if (!mine()) continue;
        const int cnt = min(64, nm - base);
        const int4 ent = ml[base + (lane < cnt ? lane : cnt - 1)];
        const int k = ent.x;
        {
            T *rec = stage + kRec * lane;
            if constexpr (SPEC) {
                const double *sr = a.spec + kSpecVals * (int64_t)k;
                const double4 pp = *(const double4 *)sr, pm = *(const double4 *)(sr + 4);
                if constexpr (PREC == UCP_SPLIT) {
                    float4 *d4 = (float4 *)rec;
                    d4[0] = make_float4((float)(pp.x - cg.x), (float)(pp.y - cg.y),
                                        (float)(pp.z - cg.z), (float)pp.w);
                    d4[1] = make_float4((float)(pm.x - cg.x), (float)(pm.y - cg.y),
                                        (float)(pm.z - cg.z), (float)pm.w);
                } else {
                    double4 *d4 = (double4 *)rec;
                    d4[0] = pp;
                    d4[1] = pm;
                }
            } else if constexpr (PREC == UCP_SPLIT && ADJ) {
                const float4 *m4 = a.nrec + 8 * (int64_t)k;
                const double4 geo = *(const double4 *)m4;
                const float4 r1 = m4[4], r2 = m4[5], r3 = m4[6];
                double *dd = (double *)rec;
                dd[0] = geo.x;
                dd[1] = geo.y;
                dd[2] = geo.z;
                float *ff = (float *)rec + 6;
                ff[0] = r1.x; ff[1] = r1.y; ff[2] = r1.z; ff[3] = r1.w;
                ff[4] = r2.x; ff[5] = r2.y; ff[6] = r2.z; ff[7] = r2.w;
                ff[8] = r3.x; ff[9] = r3.y; ff[10] = r3.z;
            } else if constexpr (PREC == UCP_SPLIT) {
                const float4 *m4 = a.nrec + 8 * (int64_t)k + 4;
                const float4 r1 = m4[0], r2 = m4[1], r3 = m4[2];
                float4 *d4 = (float4 *)rec;
                d4[0] = make_float4(__int_as_float(ent.y), __int_as_float(ent.z),
                                    __int_as_float(ent.w), 0.f);
                d4[1] = r1;
                d4[2] = r2;
                d4[3] = r3;
            } else {
                const double2 *m2 = (const double2 *)(a.mom64 + 16 * (int64_t)k);
                double2 *d2 = (double2 *)rec;
                for (int q = 0; q < 4; ++q) d2[q] = m2[q];
                d2[3].y *= 1.5;
                for (int q = 4; q < 7; ++q) {
                    const double2 v = m2[q];
                    d2[q] = make_double2(3.0 * v.x, 3.0 * v.y);
                }
            }
        }
        wave_sync();
        if constexpr (!ADJ) {
            // two independent partial sums (records e and e + lpt) for ILP
            T ex = 0, ey = 0, ez = 0, ph = 0, fx = 0, fy = 0, fz = 0, fp = 0;
            if (lpt == 1) {
                // one lane per target (full groups): every lane takes every
                // record, so the record index is the same on all lanes
                int e = 0;
                for (; e + 1 < cnt; e += 2) {
                    const T *r0 = stage + kRec * e;
                    m2p_entry<T, PHI, SPEC>(r0, tx, ty, tz, eps2, ex, ey, ez, ph);
                    m2p_entry<T, PHI, SPEC>(r0 + kRec, tx, ty, tz, eps2, fx, fy, fz, fp);
                }
                if (e < cnt) m2p_entry<T, PHI, SPEC>(stage + kRec * e, tx, ty, tz, eps2, ex, ey, ez, ph);
            } else {
                int e = sub;
                for (; e + lpt < cnt; e += 2 * lpt) {
                    m2p_entry<T, PHI, SPEC>(stage + kRec * e, tx, ty, tz, eps2, ex, ey, ez, ph);
                    m2p_entry<T, PHI, SPEC>(stage + kRec * (e + lpt), tx, ty, tz, eps2, fx, fy, fz, fp);
                }
                if (e < cnt) m2p_entry<T, PHI, SPEC>(stage + kRec * e, tx, ty, tz, eps2, ex, ey, ez, ph);
            }
            tg.E0 += (double)(ex + fx);
            tg.E1 += (double)(ey + fy);
            tg.E2 += (double)(ez + fz);
            tg.PH += (double)(ph + fp);
        } else {
            T gx = 0, gy = 0, gz = 0, lx = 0, ly = 0, lz = 0;
            for (int e = sub; e < cnt; e += lpt) {
                CellRec<T> r;
                double cx, cy, cz;
                load_adj_rec<PREC>(stage + kRec * e, r, cx, cy, cz);
                m2p_adj_target<T>((T)(tg.px - cx), (T)(tg.py - cy), (T)(tg.pz - cz), r.Q, r.px,
                                  r.py, r.pz, r.Sxx, r.Syy, r.Szz, r.Sxy, r.Sxz, r.Syz, r.trS15,
                                  tg.wx, tg.wy, tg.wz, eps2, gx, gy, gz, lx, ly, lz);
            }
            tg.E0 += (double)gx;
            tg.E1 += (double)gy;
            tg.E2 += (double)gz;
            tg.C0 += (double)lx;
            tg.C1 += (double)ly;
            tg.C2 += (double)lz;
            // source side: lane e owns staged record e
            CellRec<T> r;
            double cx, cy, cz;
            load_adj_rec<PREC>(stage + kRec * lane, r, cx, cy, cz);
            T cb[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int t = 0; t < c; ++t) {
                const int src = t * lpt;
                m2p_adj_source<T>((T)(readlane_d(tg.px, src) - cx), (T)(readlane_d(tg.py, src) - cy),
                                  (T)(readlane_d(tg.pz, src) - cz), readlane_t(tg.wx, src),
                                  readlane_t(tg.wy, src), readlane_t(tg.wz, src), eps2, cb);
            }
            if (lane < cnt)
                for (int q = 0; q < 9; ++q) atomicAdd(a.cbar + 10 * (int64_t)k + q, (double)cb[q]);
        }
        wave_sync();
    }
    // staged sources are 16 bytes (FP32 offsets) or 32 bytes (FP64 positions)
    constexpr int kSrcBytes = (PREC == UCP_SPLIT && !ADJ) ? 16 : 32;
    int *sidx = (int *)((char *)stage + 64 * kSrcBytes);
    for (int base = 0; base < np; base += 64) {
        const int cntL = min(64, np - base);
        const int2 lf = pl[base + (lane < cntL ? lane : cntL - 1)];
        const int cl = lane < cntL ? lf.y : 0;
        const int incl = wave_incl_scan_i(cl, lane);
        const int total = uni(__shfl(incl, 63));
        pfx[lane] = incl;
        lfirst[lane] = lf.x - (incl - cl);   // particle j = lfirst[l] + (global offset)
        wave_sync();
        for (int pb = 0; pb < total; pb += 64) {
            if (!mine()) continue;
            const int ncur = min(64, total - pb);
            const int P = pb + (lane < ncur ? lane : ncur - 1);
            // leaf holding concatenated particle P: first l with pfx[l] > P
            int lo = -1, hi = cntL - 1;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (pfx[mid] > P) hi = mid;
                else lo = mid;
            }
            const int j = lfirst[hi] + P;
            const double4 s = a.xq[j];
            T *st = stage + 4 * lane;
            // the adjoint's pair terms grow as h^-3, so its pair differences
            // x_i - x_j are formed in FP64 (FP64 staging) and rounded once
            if constexpr (PREC == UCP_SPLIT && !ADJ) {
                *(float4 *)st = make_float4((float)(s.x - cg.x), (float)(s.y - cg.y),
                                            (float)(s.z - cg.z), (float)s.w);
            } else {
                *(double4 *)((double *)stage + 4 * lane) = s;
            }
            sidx[lane] = j;
            wave_sync();
            T ex = 0, ey = 0, ez = 0, ph = 0;
            bool done = false;
            if constexpr (!ADJ && sizeof(T) == 4) {
                if (lpt == 1) {
                    // one lane per target: every lane takes every staged
                    // source, in pairs with two partial sums
                    T fx = 0, fy = 0, fz = 0, fp = 0;
                    int e = 0;
                    auto one = [&](const float4 &v, bool notself, float &sx, float &sy,
                                   float &sz, float &sp) {
                        if constexpr (KELBG)
                            p2p_kelbg<float, PHI>(tx - v.x, ty - v.y, tz - v.z, v.w, tg.qt, eps2,
                                                  inv_lam, notself, sx, sy, sz, sp);
                        else p2p_one<PHI>(tx, ty, tz, v, eps2, notself, sx, sy, sz, sp);
                    };
                    for (; e + 1 < ncur; e += 2) {
                        const float4 v0 = ((const float4 *)stage)[e];
                        const float4 v1 = ((const float4 *)stage)[e + 1];
                        one(v0, sidx[e] != tg.i, ex, ey, ez, ph);
                        one(v1, sidx[e + 1] != tg.i, fx, fy, fz, fp);
                    }
                    if (e < ncur) one(((const float4 *)stage)[e], sidx[e] != tg.i, ex, ey, ez, ph);
                    ex += fx;
                    ey += fy;
                    ez += fz;
                    ph += fp;
                    done = true;
                }
            }
            for (int e = sub; !done && e < ncur; e += lpt) {
                if constexpr (ADJ) {
                    const double4 v = ((const double4 *)stage)[e];
                    if (sidx[e] != tg.i)
                        p2p_adj<T>((T)(tg.px - v.x), (T)(tg.py - v.y), (T)(tg.pz - v.z), (T)v.w,
                                   tg.wx, tg.wy, tg.wz, eps2, ex, ey, ez);
                } else {
                    T sx, sy, sz, sq;
                    if constexpr (sizeof(T) == 4) {
                        const float4 v = ((const float4 *)stage)[e];
                        sx = v.x; sy = v.y; sz = v.z; sq = v.w;
                    } else {
                        const double4 v = ((const double4 *)stage)[e];
                        sx = v.x; sy = v.y; sz = v.z; sq = v.w;
                    }
                    const T rx = tx - sx, ry = ty - sy, rz = tz - sz;
                    if constexpr (KELBG) {
                        p2p_kelbg<T, PHI>(rx, ry, rz, sq, tg.qt, eps2, inv_lam, sidx[e] != tg.i,
                                          ex, ey, ez, ph);
                    } else {
                        const T h2 = fma(rx, rx, fma(ry, ry, fma(rz, rz, eps2)));
                        T ih;
                        if constexpr (sizeof(T) == 4) ih = __builtin_amdgcn_rsqf(h2);
                        else ih = 1.0 / sqrt(h2);
                        const T w = sq * (ih * ih * ih);
                        ex = fma(w, rx, ex);
                        ey = fma(w, ry, ey);
                        ez = fma(w, rz, ez);
                        if (PHI) ph += (sidx[e] != tg.i) ? sq * ih : (T)0;
                    }
                }
            }
            tg.E0 += (double)ex;
            tg.E1 += (double)ey;
            tg.E2 += (double)ez;
            tg.PH += (double)ph;
            if constexpr (ADJ) {
                // source side: lane e owns staged source e (position s)
                T gx = 0, gy = 0, gz = 0;
                for (int t = 0; t < c; ++t) {
                    const int src = t * lpt;
                    const T rx = (T)(readlane_d(tg.px, src) - s.x);
                    const T ry = (T)(readlane_d(tg.py, src) - s.y);
                    const T rz = (T)(readlane_d(tg.pz, src) - s.z);
                    const T wx = readlane_t(tg.wx, src), wy = readlane_t(tg.wy, src),
                            wz = readlane_t(tg.wz, src);
                    if (gfirst + t != j) p2p_adj<T>(rx, ry, rz, (T)s.w, wx, wy, wz, eps2, gx, gy, gz);
                }
                if (lane < ncur) {
                    atomicAdd(a.xsrc + 4 * (int64_t)j + 0, -(double)gx);
                    atomicAdd(a.xsrc + 4 * (int64_t)j + 1, -(double)gy);
                    atomicAdd(a.xsrc + 4 * (int64_t)j + 2, -(double)gz);
                }
            }
            wave_sync();
        }
    }
}

template <int PREC, int MODE, bool KELBG, bool SPEC>
__device__ __forceinline__ void walk_body(const WalkArgs &a)
{
    using T = typename std::conditional<PREC == UCP_SPLIT, float, double>::type;
    HIP_DYNAMIC_SHARED(char, lds_raw)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int L = a.L;
    char *wbase = lds_raw + (size_t)wave * walk_wave_bytes<PREC>(L);
    int2 *stk = (int2 *)wbase;                                   // [kStackCap]
    int4 *ml = (int4 *)(wbase + kStackCap * 8);                   // [L]
    int2 *pl = (int2 *)(ml + L);                                  // [L]
    T *stage = (T *)(pl + L);                                     // [64][kRec]
    int *pfx = (int *)((char *)stage + walk_stage_bytes<PREC>()); // [64]
    int *lfirst = pfx + 64;                                       // [64]
    if (*a.flags) return;
    // every loop below is bounded by these totals, whatever the records hold
    const int ng = min(*a.ngroups, (int)a.n);
    const int nn = *a.nnodes;
    // the queues hand out units: group g, share `part` of its evaluation
    const int parts = MODE == kWalkVjp ? max(1, min(a.parts, kMaxParts)) : 1;
    const int nu = ng * parts;
    // Groups are split into kWalkQueues contiguous ranges, one per XCD (work
    // groups are dispatched to the XCDs in turn, so block b runs on XCD
    // b mod 8): neighbouring groups share most of their lists, and keeping
    // them on one XCD keeps those nodes in that XCD's L2.  A wave whose
    // queue is exhausted moves on to the next one, so all finish together.
    // No divergent branch anywhere around a queue: every lane executes the
    // atomic, only lane 0 adds 1, so lane 0 receives the value before its own
    // increment.  Queue heads only grow, so each wave passes each exhausted
    // queue once and the loop ends.
    int qx = (int)(blockIdx.x % kWalkQueues), exhausted = 0;
    for (;;) {
        const unsigned long long old =
            atomicAdd(&a.wq[kQStride * qx], lane == 0 ? 1ull : 0ull);
        const int g0 = (int)(((int64_t)nu * qx) / kWalkQueues);
        const int g1 = (int)(((int64_t)nu * (qx + 1)) / kWalkQueues);
        const int un = g0 + uni((int)min(old, (unsigned long long)nu));
        if (un >= g1) {
            if (++exhausted == kWalkQueues) break;
            qx = qx + 1 == kWalkQueues ? 0 : qx + 1;
            continue;
        }
        const int g = parts == 1 ? un : un / parts, part = un - g * parts;
        const int4 gr = a.groups[g];
        const int gfirst = uni(gr.x), c = uni(gr.y), gnode = uni(gr.z), root = uni(gr.w);
        if (gfirst < 0 || c < 1 || c > kMaxGroup || (int64_t)gfirst + c > a.n || gnode < 0 ||
            gnode >= nn || root < 0 || root >= nn) {
            atomicOr(a.flags_rw, lane == 0 ? UCP_FLAG_INTERNAL : 0);
            continue;
        }
        const int lpt = 64 / c;
        const int t = lane / lpt, sub = lane - t * lpt;
        const bool act = t < c;
        const int i = gfirst + (act ? t : 0);
        const double4 xi = a.xq[i];
        // bounding box of the members; its centre c_g is the origin of the
        // FP32 offsets
        const double bminx = wave_fmin(act ? xi.x : INFINITY), bmaxx = wave_fmax(act ? xi.x : -INFINITY);
        const double bminy = wave_fmin(act ? xi.y : INFINITY), bmaxy = wave_fmax(act ? xi.y : -INFINITY);
        const double bminz = wave_fmin(act ? xi.z : INFINITY), bmaxz = wave_fmax(act ? xi.z : -INFINITY);
        const double4 cg = make_double4(0.5 * (bminx + bmaxx), 0.5 * (bminy + bmaxy),
                                        0.5 * (bminz + bmaxz), 0.0);
        Target<T> tg;
        if constexpr (PREC == UCP_SPLIT) {
            tg.tx = (float)(xi.x - cg.x);
            tg.ty = (float)(xi.y - cg.y);
            tg.tz = (float)(xi.z - cg.z);
        } else {
            tg.tx = xi.x;
            tg.ty = xi.y;
            tg.tz = xi.z;
        }
        tg.wx = tg.wy = tg.wz = (T)0;
        if constexpr (MODE == kWalkVjp) {
            const double4 wi = a.w[i];
            tg.wx = act ? (T)wi.x : (T)0;   // idle lanes carry no cotangent
            tg.wy = act ? (T)wi.y : (T)0;
            tg.wz = act ? (T)wi.z : (T)0;
        }
        tg.px = xi.x;
        tg.py = xi.y;
        tg.pz = xi.z;
        tg.qt = (T)xi.w;
        tg.i = i;
        tg.E0 = tg.E1 = tg.E2 = tg.PH = 0.0;
        tg.C0 = tg.C1 = tg.C2 = 0.0;
        tg.part = part;
        tg.ck = 0;
        stk[0] = make_int2(root, min(((const int *)(a.nrec + 8 * (int64_t)root + 2))[0], nn));
        int sp = 1;
        wave_sync();
        int nm = 0, np = 0, my_m = 0, my_src = 0;
        bool overflow = false;
        const double th2 = a.th2;
        while (sp > 0) {
            if (nm > L - 64 || np > L - 64) {
                flush_lists<PREC, MODE, KELBG, SPEC>(a, ml, nm, pl, np, stage, pfx, lfirst, lane, sub, lpt, c,
                                        gfirst, cg, tg);
                nm = np = 0;
            }
            const int B = min(min(64, sp), max(1, kStackSoft - sp));
            const bool have = lane < B;
            const int2 ent = stk[sp - B + (have ? lane : B - 1)];
            wave_sync();
            sp -= B;
            const int k = (ent.x >= 0 && ent.x < nn) ? ent.x : 0;
            const int end = min(ent.y, nn);
            const float4 *rp = a.nrec + 8 * (int64_t)k;
            const double4 geo = *(const double4 *)rp;
            const int4 inf = *(const int4 *)(rp + 2);   // skip, first, count, level|256*leaf
            // distances from the group's bounding box to a point, nearest and
            // farthest, squared
            auto box_d2 = [&](double px, double py, double pz, double &dmin2, double &dmax2) {
                const double nx = fmax(0.0, fmax(bminx - px, px - bmaxx));
                const double ny = fmax(0.0, fmax(bminy - py, py - bmaxy));
                const double nz = fmax(0.0, fmax(bminz - pz, pz - bmaxz));
                const double fx = fmax(fabs(bminx - px), fabs(bmaxx - px));
                const double fy = fmax(fabs(bminy - py), fabs(bmaxy - py));
                const double fz = fmax(fabs(bminz - pz), fabs(bmaxz - pz));
                dmin2 = nx * nx + ny * ny + nz * nz;
                dmax2 = fx * fx + fy * fy + fz * fz;
            };
            // The group box bounds decide when a margin far above rounding
            // proves every member agrees; otherwise every member is tested.
            bool sure_acc, sure_open;
            double4 sp_p = make_double4(0, 0, 0, 0), sp_m = sp_p;   // c_s, Q_s
            double R2p = 0.0, R2m = 0.0;
            if constexpr (SPEC) {
                // Eq. (5) per species: accept iff (s/theta + delta_s)^2 < d_s^2
                // for every member and every sign the box holds (theta = 0:
                // s/theta is infinite and nothing is accepted)
                const double *sr = a.spec + kSpecVals * (int64_t)k;
                sp_p = *(const double4 *)sr;
                sp_m = *(const double4 *)(sr + 4);
                const double2 dl = *(const double2 *)(sr + 8);
                const double sth = sqrt(geo.w) / a.theta;
                R2p = (sth + dl.x) * (sth + dl.x);
                R2m = (sth + dl.y) * (sth + dl.y);
                double pmin2, pmax2, mmin2, mmax2;
                box_d2(sp_p.x, sp_p.y, sp_p.z, pmin2, pmax2);
                box_d2(sp_m.x, sp_m.y, sp_m.z, mmin2, mmax2);
                const bool hp = sp_p.w != 0.0, hm = sp_m.w != 0.0;
                sure_acc = (!hp || R2p < pmin2 * (1.0 - 1e-12)) &&
                           (!hm || R2m < mmin2 * (1.0 - 1e-12));
                sure_open = (hp && R2p >= pmax2 * (1.0 + 1e-12)) ||
                            (hm && R2m >= mmax2 * (1.0 + 1e-12));
            } else {
                // Eq. (5) about the box centre: accept iff s^2 < theta^2 d^2
                // for every member
                double dmin2, dmax2;
                box_d2(geo.x, geo.y, geo.z, dmin2, dmax2);
                sure_acc = geo.w < th2 * dmin2 * (1.0 - 1e-12);
                sure_open = geo.w >= th2 * dmax2 * (1.0 + 1e-12);
            }
            const bool band = have && !sure_acc && !sure_open;
            bool acc = sure_acc;
            // nodes in the band one at a time, every lane testing its own
            // member against the node
            unsigned long long bandm = __ballot(band);
            if constexpr (!SPEC) {
                // the popped nodes' centres and side^2 go through LDS (the
                // staging area is free during traversal), so a band node is
                // read by every lane with one broadcast load; the nodes that
                // every member accepts collect in a scalar mask
                double4 *bnode = (double4 *)stage;
                bnode[lane] = geo;
                wave_sync();
                unsigned long long okm = 0ull;
                while (bandm != 0ull) {
                    const int bl = __builtin_ctzll(bandm);
                    bandm &= bandm - 1ull;
                    const double4 nd = bnode[bl];
                    const double dx = xi.x - nd.x;
                    const double dy = xi.y - nd.y;
                    const double dz = xi.z - nd.z;
                    const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
                    // lanes without a target hold the group's first member
                    // (xi of i = gfirst), so they only repeat its test
                    const bool fail = !(nd.w < th2 * d2);
                    okm |= __builtin_amdgcn_ballot_w64(fail) == 0ull ? (1ull << bl) : 0ull;
                }
                acc = sure_acc || ((okm >> lane) & 1ull) != 0ull;
            }
            // the per-sign test of the species pseudo-particles broadcasts
            // each band node's centres of charge from its lane
            while (SPEC && bandm != 0ull) {
                const int bl = __builtin_ctzll(bandm);
                bandm &= bandm - 1ull;
                {
                    const double qp = readlane_d(sp_p.w, bl), qm = readlane_d(sp_m.w, bl);
                    const double px = xi.x - readlane_d(sp_p.x, bl);
                    const double py = xi.y - readlane_d(sp_p.y, bl);
                    const double pz = xi.z - readlane_d(sp_p.z, bl);
                    const double mx = xi.x - readlane_d(sp_m.x, bl);
                    const double my = xi.y - readlane_d(sp_m.y, bl);
                    const double mz = xi.z - readlane_d(sp_m.z, bl);
                    const double rp = readlane_d(R2p, bl), rm = readlane_d(R2m, bl);
                    const double dp = fma(pz, pz, fma(py, py, px * px));
                    const double dm = fma(mz, mz, fma(my, my, mx * mx));
                    const bool fail = act && ((qp != 0.0 && !(rp < dp)) || (qm != 0.0 && !(rm < dm)));
                    const bool ok = __ballot(fail) == 0ull;
                    acc = lane == bl ? ok : acc;
                }
            }
            const bool isleaf = (inf.w & 256) != 0;
            const bool leaf_ok = inf.y >= 0 && inf.z >= 0 && (int64_t)inf.y + inf.z <= a.n;
            const bool take_m = have && acc;
            const bool take_p = have && !acc && isleaf && leaf_ok;
            const bool push_c = have && !acc && !isleaf;
            const int skipk = max(inf.x, k + 1);
            const bool push_s = have && skipk < end;
            const unsigned long long bm = __ballot(take_m), bp = __ballot(take_p);
            const unsigned long long bc = __ballot(push_c), bs = __ballot(push_s);
            const int nc = __popcll(bc), ns = __popcll(bs);
            if (sp + nc + ns > kStackCap) { overflow = true; break; }
            if (take_m) {
                int4 e = make_int4(k, 0, 0, 0);
                if constexpr (PREC == UCP_SPLIT) {
                    e.y = __float_as_int((float)(geo.x - cg.x));
                    e.z = __float_as_int((float)(geo.y - cg.y));
                    e.w = __float_as_int((float)(geo.z - cg.z));
                }
                ml[nm + lanes_before(bm, lane)] = e;
            }
            if (take_p) pl[np + lanes_before(bp, lane)] = make_int2(inf.y, inf.z);
            // sibling ranges below, child ranges on top
            if (push_s) stk[sp + lanes_before(bs, lane)] = make_int2(skipk, end);
            if (push_c) stk[sp + ns + lanes_before(bc, lane)] = make_int2(k + 1, skipk);
            nm += __popcll(bm);
            np += __popcll(bp);
            sp += nc + ns;
            my_m += take_m ? 1 : 0;
            my_src += take_p ? inf.z : 0;
            wave_sync();
        }
        if (overflow) atomicOr(a.flags_rw, lane == 0 ? UCP_FLAG_WALK_STACK : 0);
        flush_lists<PREC, MODE, KELBG, SPEC>(a, ml, nm, pl, np, stage, pfx, lfirst, lane, sub, lpt, c, gfirst,
                                cg, tg);
        // sum the lpt partial results of each target in fixed lane order
        double *red = (double *)stage;   // 64 x 4 doubles
        red[4 * lane + 0] = tg.E0;
        red[4 * lane + 1] = tg.E1;
        red[4 * lane + 2] = tg.E2;
        red[4 * lane + 3] = tg.PH;
        wave_sync();
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int s = 0; s < lpt; ++s) {
            const int src = lane + s < 64 ? lane + s : 63;
            s0 += red[4 * src + 0];
            s1 += red[4 * src + 1];
            s2 += red[4 * src + 2];
            s3 += red[4 * src + 3];
        }
        wave_sync();
        // only lane sub == 0 of an active target owns the result.  Forces and
        // potentials go straight to the caller's order; otherwise (energy,
        // adjoint) the sorted field is kept, and the other lanes store to
        // their private spare slot past the particles
        if (a.fout || a.phiout) {
            if (act && sub == 0) {
                const int64_t ci = a.perm[i];
                if (a.fout) {
                    const double qq = a.xq[i].w;
                    a.fout[3 * ci + 0] = qq * s0;
                    a.fout[3 * ci + 1] = qq * s1;
                    a.fout[3 * ci + 2] = qq * s2;
                }
                if (a.phiout) a.phiout[ci] = s3;
            }
        } else if (parts > 1) {
            // a shared group's waves add their shares (acc cleared beforehand)
            if (act && sub == 0) {
                double *ac = (double *)(a.acc + i);
                atomicAdd(ac + 0, s0);
                atomicAdd(ac + 1, s1);
                atomicAdd(ac + 2, s2);
                atomicAdd(ac + 3, s3);
            }
        } else {
            a.acc[(act && sub == 0) ? (int64_t)i : a.n_spare + lane] =
                make_double4(s0, s1, s2, s3);
        }
        if constexpr (MODE == kWalkVjp) {
            // the group's share of its cloud's cube-origin cotangent (lanes
            // without a target carry w = 0 and add nothing)
            double c0 = tg.C0, c1 = tg.C1, c2 = tg.C2;
            for (int o = 32; o > 0; o >>= 1) {
                c0 += __shfl_xor(c0, o);
                c1 += __shfl_xor(c1, o);
                c2 += __shfl_xor(c2, o);
            }
            const int cl = cloud_of(a.off, a.clouds, gfirst);
            const double v = lane == 0 ? c0 : lane == 1 ? c1 : c2;
            if (lane < 3) atomicAdd(a.lobar + 4 * (int64_t)cl + lane, v);
        }
        // counts once per group (every wave of a shared group has the same)
        const int tot_m = wave_isum(my_m), tot_src = wave_isum(my_src);
        if (part == 0) a.gstat[g] = make_int2(tot_m, tot_src);   // same value from every lane
        const unsigned long long zero = 0ull;
        const bool count = lane == 0 && part == 0;
        atomicAdd(&a.ctr[CTR_P2P],
                  count ? (unsigned long long)c * (unsigned long long)tot_src : zero);
        atomicAdd(&a.ctr[CTR_M2P],
                  count ? (unsigned long long)c * (unsigned long long)tot_m : zero);
    }
}

// each wave's own busy span (start, end) and the compute unit it ran on, for
// the balance of the persistent waves, when the launch asks for it.  The unit
// is read at the start from the hardware registers HW_ID (CU, shader array and
// shader engine in bits 8-15) and XCC_ID (the XCD), kept as XCC_ID << 32 |
// HW_ID.
__device__ __forceinline__ void wave_stamp(unsigned long long *wclock, int end)
{
    if (wclock && (threadIdx.x & 63) == 0) {
        unsigned long long *w = wclock + 3 * (4 * (int64_t)blockIdx.x + (threadIdx.x >> 6));
        w[end] = __builtin_amdgcn_s_memrealtime();
        if (!end) {
            const unsigned hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);    // HW_ID, 32 bits
            const unsigned xcc = __builtin_amdgcn_s_getreg((31 << 11) | 20);  // XCC_ID, 32 bits
            w[2] = (unsigned long long)xcc << 32 | hw;
        }
    }
}

template <int PREC, int MODE, bool KELBG, bool SPEC>
__global__ __launch_bounds__(256) void k_walk(WalkArgs a)
{
    wave_stamp(a.wclock, 0);
    walk_body<PREC, MODE, KELBG, SPEC>(a);
    wave_stamp(a.wclock, 1);
}

// The split-precision force walks under the Plummer law with the quadrupole
// expansion fit in 128 VGPRs without spilling, so they can keep four waves
// per SIMD, as many as their LDS allows (the other variants would spill).
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_walk_w4(
    WalkArgs a)
{
    wave_stamp(a.wclock, 0);
    walk_body<UCP_SPLIT, MODE, false, false>(a);
    wave_stamp(a.wclock, 1);
}

__global__ void k_walk_reset(unsigned long long *ctr, unsigned long long *wq)
{
    if (threadIdx.x == 0) {
        ctr[CTR_P2P] = 0;
        ctr[CTR_M2P] = 0;
    }
    if (threadIdx.x < kWalkQueues) wq[kQStride * threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// adjoint: the cotangents are scaled by a power of two s >= max |q_i u_i| so
// that the FP32 arithmetic of the split walk cannot overflow however large
// they grow (a rollout's cotangents grow with its instability); s is exact,
// and the result is scaled back in FP64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_vjp_max(const double *__restrict__ u,
                                                const double4 *__restrict__ xq,
                                                const uint32_t *__restrict__ perm, int64_t n,
                                                unsigned long long *ctr, const int32_t *flags)
{
    __shared__ double red[4];
    if (*flags) return;
    double mx = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += stride) {
        const double a = fabs(xq[p].w);
        const int64_t i = perm[p];
        mx = fmax(mx, fmax(a * fabs(u[3 * i]), fmax(a * fabs(u[3 * i + 1]), a * fabs(u[3 * i + 2]))));
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        // non-negative doubles order like their bit patterns (NaN is largest)
        atomicMax(&ctr[CTR_VJPMAX], (unsigned long long)__double_as_longlong(mx));
    }
}

__device__ __forceinline__ double vjp_scale(const unsigned long long *ctr)
{
    const double mx = __longlong_as_double((long long)ctr[CTR_VJPMAX]);
    if (!(mx > 0.0) || !isfinite(mx)) return 1.0;
    int e;
    frexp(mx, &e);
    return ldexp(1.0, e);   // power of two > mx
}

// clears the scale and the per-cloud cube-origin cotangents, and marks every
// cloud's minimum particles as not yet found
__global__ void k_vjp_reset(unsigned long long *ctr, double *lobar, uint32_t *lomin, int clouds)
{
    if (threadIdx.x == 0) ctr[CTR_VJPMAX] = 0ull;
    for (int k = threadIdx.x; k < 4 * clouds; k += blockDim.x) lobar[k] = 0.0;
    for (int k = threadIdx.x; k < 3 * clouds; k += blockDim.x) lomin[k] = 0xffffffffu;
}

// ---------------------------------------------------------------------------
// adjoint: prepare the sorted cotangents and clear the accumulators
//   w_p = q_p u_{perm[p]} / s,  xsrc = 0,  cbar = 0 (nodes read from the device)
// ---------------------------------------------------------------------------
//   and, per cloud and axis, the lowest caller index among the particles on
//   the cube origin (the minimum of that axis)
__global__ __launch_bounds__(256) void k_vjp_prep(const double *__restrict__ u,
                                                 const double4 *__restrict__ xq,
                                                 const uint32_t *__restrict__ perm, int64_t n,
                                                 const int32_t *__restrict__ nnodes,
                                                 const unsigned long long *__restrict__ ctr,
                                                 const int64_t *__restrict__ off, int clouds,
                                                 const double4 *__restrict__ cube,
                                                 double4 *w, double *xsrc, double *cbar,
                                                 uint32_t *lomin, double4 *acc,
                                                 const int32_t *flags)
{
    if (*flags) return;
    const double inv = 1.0 / vjp_scale(ctr);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t p = t0; p < n; p += stride) {
        const int64_t i = perm[p];
        const double4 x = xq[p];
        const double qq = x.w * inv;
        w[p] = make_double4(qq * u[3 * i], qq * u[3 * i + 1], qq * u[3 * i + 2], 0.0);
        *(double4 *)(xsrc + 4 * p) = make_double4(0.0, 0.0, 0.0, 0.0);
        acc[p] = make_double4(0.0, 0.0, 0.0, 0.0);   // shared groups add their shares
        const int cl = cloud_of(off, clouds, p);
        const double4 lo = cube[2 * cl];
        if (x.x == lo.x) atomicMin(lomin + 3 * cl + 0, (uint32_t)i);
        if (x.y == lo.y) atomicMin(lomin + 3 * cl + 1, (uint32_t)i);
        if (x.z == lo.z) atomicMin(lomin + 3 * cl + 2, (uint32_t)i);
    }
    const int64_t nc = 10 * (int64_t)*nnodes;
    for (int64_t e = t0; e < nc; e += stride) cbar[e] = 0.0;
}

// ---------------------------------------------------------------------------
// adjoint: per particle j (sorted), the target side (walk accumulators), the
// P2P source side, and the cell cotangents of every box holding j:
//   xbar_j = g_j + xsrc_j + q_j sum_{C holding j} (pbar_C + sym_C (x_j - c_C)),
// plus, on each axis where j is its cloud's marked minimum particle, the
// cloud's cube-origin cotangent; then back to the caller's order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_vjp_down(const double4 *__restrict__ acc,
                                                 const double *__restrict__ xsrc,
                                                 const double *__restrict__ cbar,
                                                 const double4 *__restrict__ xq,
                                                 const double4 *__restrict__ ngeo,
                                                 const int32_t *__restrict__ npar,
                                                 const int32_t *__restrict__ leafof,
                                                 const int32_t *__restrict__ nnodes,
                                                 const uint32_t *__restrict__ perm, int64_t n,
                                                 const unsigned long long *__restrict__ ctr,
                                                 const int64_t *__restrict__ off, int clouds,
                                                 const uint32_t *__restrict__ lomin,
                                                 const double *__restrict__ lobar,
                                                 double *xbar, int32_t *flags)
{
    if (*flags) return;
    const double sc = vjp_scale(ctr);
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double4 x = xq[p];
    const double4 g = acc[p];
    double bx = 0.0, by = 0.0, bz = 0.0;
    const int nn = *nnodes;
    int k = leafof[p];
    for (int depth = 0; k >= 0; ++depth) {
        if (k >= nn || depth > 64) {   // inconsistent records
            atomicOr(flags, UCP_FLAG_INTERNAL);
            return;
        }
        const double *cb = cbar + 10 * (int64_t)k;
        const double4 c = ngeo[k];
        const double rx = x.x - c.x, ry = x.y - c.y, rz = x.z - c.z;
        bx += cb[0] + cb[3] * rx + cb[6] * ry + cb[7] * rz;
        by += cb[1] + cb[6] * rx + cb[4] * ry + cb[8] * rz;
        bz += cb[2] + cb[7] * rx + cb[8] * ry + cb[5] * rz;
        k = npar[k];
    }
    const int64_t i = perm[p];
    const int cl = cloud_of(off, clouds, p);
    const uint32_t *lm = lomin + 3 * cl;
    const double *lb = lobar + 4 * (int64_t)cl;
    xbar[3 * i + 0] = sc * (g.x + xsrc[4 * p + 0] + x.w * bx + (lm[0] == (uint32_t)i ? lb[0] : 0.0));
    xbar[3 * i + 1] = sc * (g.y + xsrc[4 * p + 1] + x.w * by + (lm[1] == (uint32_t)i ? lb[1] : 0.0));
    xbar[3 * i + 2] = sc * (g.z + xsrc[4 * p + 2] + x.w * bz + (lm[2] == (uint32_t)i ? lb[2] : 0.0));
}

template <int PREC, int MODE, bool KELBG = false, bool SPEC = false>
static void launch_walk_t(Ctx *c, const WalkArgs &wa, hipStream_t s)
{
    const int waves_per_cu = c->p_built.walk_waves > 0 ? c->p_built.walk_waves : 32;
    const int blocks = (c->num_cu * waves_per_cu + 3) / 4;
    const size_t lds = (size_t)4 * walk_wave_bytes<PREC>(wa.L);
    if constexpr (PREC == UCP_SPLIT && MODE != kWalkVjp && !KELBG && !SPEC)
        hipLaunchKernelGGL((k_walk_w4<MODE>), dim3(blocks), dim3(256), lds, s, wa);
    else
        hipLaunchKernelGGL((k_walk<PREC, MODE, KELBG, SPEC>), dim3(blocks), dim3(256), lds, s, wa);
}

// the force walks: precision x (forces | forces and potentials) x pair law x
// expansion
template <int PREC>
static void launch_force_walk(Ctx *c, const WalkArgs &wa, bool phi, bool kelbg, bool spec,
                              hipStream_t s)
{
    if (spec) {
        if (kelbg) {
            if (phi) launch_walk_t<PREC, kWalkForcePhi, true, true>(c, wa, s);
            else launch_walk_t<PREC, kWalkForce, true, true>(c, wa, s);
        } else {
            if (phi) launch_walk_t<PREC, kWalkForcePhi, false, true>(c, wa, s);
            else launch_walk_t<PREC, kWalkForce, false, true>(c, wa, s);
        }
    } else if (kelbg) {
        if (phi) launch_walk_t<PREC, kWalkForcePhi, true>(c, wa, s);
        else launch_walk_t<PREC, kWalkForce, true>(c, wa, s);
    } else {
        if (phi) launch_walk_t<PREC, kWalkForcePhi>(c, wa, s);
        else launch_walk_t<PREC, kWalkForce>(c, wa, s);
    }
}

static WalkArgs walk_args(Ctx *c)
{
    WalkArgs wa;
    wa.xq = c->d_xq;
    wa.w = nullptr;
    wa.cbar = nullptr;
    wa.xsrc = nullptr;
    wa.lobar = nullptr;
    wa.off = c->d_off;
    wa.clouds = c->clouds;
    wa.fout = nullptr;
    wa.phiout = nullptr;
    wa.perm = c->d_perm;
    wa.nrec = c->d_nrec;
    wa.mom64 = c->d_mom64;
    wa.groups = c->d_groups;
    wa.ngroups = c->d_goff + c->n;
    wa.nnodes = c->d_noff + c->n;
    wa.gstat = c->d_gstat;
    wa.acc = c->d_acc;
    wa.ctr = c->d_ctr;
    wa.wq = c->d_wq;
    wa.flags = c->d_flags;
    wa.flags_rw = c->d_flags;
    wa.n = c->n;
    wa.n_spare = c->n_max;
    wa.th2 = c->p_built.theta * c->p_built.theta;
    wa.eps2 = c->p_built.eps * c->p_built.eps;
    wa.eps2f = (float)wa.eps2;
    wa.inv_lambda = c->p_built.pair_law == UCP_PAIR_KELBG ? 1.0 / c->p_built.lambda_ei : 0.0;
    wa.inv_lambdaf = (float)wa.inv_lambda;
    wa.spec = c->d_spec;
    wa.theta = c->p_built.theta;
    wa.L = c->p_built.list_len;
    wa.wclock = nullptr;
    wa.parts = 1;
    return wa;
}

void launch_forces(Ctx *c, double *f, double *phi, hipStream_t s)
{
    WalkArgs wa = walk_args(c);
    // the walk writes F_i = q_i E_i and phi_i in the caller's order itself
    wa.fout = f;
    wa.phiout = phi;
    // right after a build its reset kernel has cleared the counters and queues
    if (!c->walk_armed) hipLaunchKernelGGL(k_walk_reset, dim3(1), dim3(64), 0, s, c->d_ctr, c->d_wq);
    c->walk_armed = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        if ((int64_t)c->ev.size() < 2 * (c->ev_used + 1)) {
            hipEvent_t ea, eb;
            (void)hipEventCreate(&ea);
            (void)hipEventCreate(&eb);
            c->ev.push_back(ea);
            c->ev.push_back(eb);
        }
        e0 = c->ev[2 * c->ev_used];
        e1 = c->ev[2 * c->ev_used + 1];
        c->ev_used++;
        (void)hipEventRecord(e0, s);
        // every wave stamps its start and end (the launch shape of launch_walk_t)
        const int wpc = c->p_built.walk_waves > 0 ? c->p_built.walk_waves : 32;
        wa.wclock = c->d_wclock;
        c->wclock_waves = 4 * (int64_t)((c->num_cu * wpc + 3) / 4);
    }
    const bool want_phi = phi != nullptr || f == nullptr;
    const bool kelbg = c->p_built.pair_law == UCP_PAIR_KELBG;
    const bool spec = c->p_built.expansion == UCP_EXPANSION_SPECIES;
    if (c->p_built.precision == UCP_SPLIT) {
        launch_force_walk<UCP_SPLIT>(c, wa, want_phi, kelbg, spec, s);
    } else {
        launch_force_walk<UCP_FP64>(c, wa, want_phi, kelbg, spec, s);
    }
    if (c->timing) (void)hipEventRecord(e1, s);
}

// Waves that share one group of the adjoint walk.  The adjoint's evaluation
// is four times the forward walk's, and a wave alone on its SIMD issues at
// about 0.4 of what several waves do together; so when the groups are fewer
// than the waves the device holds at once, each group's staged chunks are
// split between up to kMaxParts waves (each builds the same lists): with at
// least two resident waves per group, one more than that, so that units are
// left for the waves that finish first (N = 65,536, 1024 groups: 4 shares of a group with 3072
// resident SPLIT waves measured 1.14 ms per VJP against 1.22 ms for 3 and
// 1.42 ms for 2; in FP64, 2048 resident waves, 3 shares 1.66 ms against 1.71
// ms for 2 and 1.76 ms for 4).  The group count is estimated as n / G; it
// only sets the split.
template <int PREC>
static int vjp_parts(const Ctx *c)
{
    int blocks = 0;
    const size_t lds = (size_t)4 * walk_wave_bytes<PREC>(c->p_built.list_len);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &blocks, k_walk<PREC, kWalkVjp, false, false>, 256, lds) != hipSuccess ||
        blocks < 1)
        blocks = 1;
    const int64_t resident = (int64_t)4 * blocks * std::max(c->num_cu, 1);
    const int64_t groups = std::max<int64_t>(1, c->n / std::max(c->p_built.group_size, 1));
    const int64_t per = resident / groups;   // resident waves per group
    return per < 2 ? 1 : (int)std::min<int64_t>(kMaxParts, per + 1);
}

void launch_vjp(Ctx *c, const VjpScratch &sc, const double *u, double *xbar, hipStream_t s)
{
    const int64_t n = c->n;
    WalkArgs wa = walk_args(c);
    wa.parts = c->p_built.precision == UCP_SPLIT ? vjp_parts<UCP_SPLIT>(c) : vjp_parts<UCP_FP64>(c);
    wa.w = sc.w;
    wa.cbar = sc.cbar;
    wa.xsrc = sc.xsrc;
    wa.lobar = sc.lobar;
    hipLaunchKernelGGL(k_vjp_reset, dim3(1), dim3(256), 0, s, c->d_ctr, sc.lobar, sc.lomin,
                       c->clouds);
    hipLaunchKernelGGL(k_vjp_max, dim3(256), dim3(256), 0, s, u, (const double4 *)c->d_xq,
                       (const uint32_t *)c->d_perm, n, c->d_ctr, (const int32_t *)c->d_flags);
    hipLaunchKernelGGL(k_vjp_prep, dim3(1024), dim3(256), 0, s, u, (const double4 *)c->d_xq,
                       (const uint32_t *)c->d_perm, n, (const int32_t *)(c->d_noff + n),
                       (const unsigned long long *)c->d_ctr, (const int64_t *)c->d_off, c->clouds,
                       (const double4 *)c->d_cube, sc.w, sc.xsrc, sc.cbar, sc.lomin, c->d_acc,
                       (const int32_t *)c->d_flags);
    hipLaunchKernelGGL(k_walk_reset, dim3(1), dim3(64), 0, s, c->d_ctr, c->d_wq);
    c->walk_armed = false;
    if (c->p_built.precision == UCP_SPLIT) launch_walk_t<UCP_SPLIT, kWalkVjp>(c, wa, s);
    else launch_walk_t<UCP_FP64, kWalkVjp>(c, wa, s);
    hipLaunchKernelGGL(k_vjp_down, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (const double4 *)c->d_acc, (const double *)sc.xsrc,
                       (const double *)sc.cbar, (const double4 *)c->d_xq,
                       (const double4 *)c->d_ngeo, (const int32_t *)c->d_npar,
                       (const int32_t *)c->d_leafof, (const int32_t *)(c->d_noff + n),
                       (const uint32_t *)c->d_perm, n, (const unsigned long long *)c->d_ctr,
                       (const int64_t *)c->d_off, c->clouds, (const uint32_t *)sc.lomin,
                       (const double *)sc.lobar, xbar, c->d_flags);
}

}  // namespace ucp
