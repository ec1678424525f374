// integrate.hip -- velocity Verlet (Sec. 2) and FP64 energies on gfx950.
//
// Kick-drift-kick:  v += dt/2 F/m;  x += dt v;  (forces at the new x);
//                   v += dt/2 F/m.
// Energies: K = sum m|v|^2/2 (and per species), U = sum q phi/2, reduced in
// FP64 with a fixed grid and a fixed tree order, so the sums are bitwise
// reproducible for a given n.
#include "internal.h"

namespace ucp {

__global__ __launch_bounds__(256) void k_kick_drift(double *__restrict__ x, double *__restrict__ v,
                                                   const double *__restrict__ f,
                                                   const double *__restrict__ m, int64_t n,
                                                   double hdt, double dt)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= 3 * n) return;
    const double inv_m = 1.0 / m[t / 3];
    const double vv = v[t] + hdt * f[t] * inv_m;
    v[t] = vv;
    x[t] = x[t] + dt * vv;
}

__global__ __launch_bounds__(256) void k_kick(double *__restrict__ v, const double *__restrict__ f,
                                             const double *__restrict__ m, int64_t n, double hdt)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= 3 * n) return;
    v[t] = v[t] + hdt * f[t] / m[t / 3];
}

// between two steps of one call: the closing kick of the first, then the
// opening kick and drift of the second, each evaluated exactly as its own
// kernel evaluates it, in one pass over x, v, f and m
__global__ __launch_bounds__(256) void k_kick_kick_drift(double *__restrict__ x,
                                                        double *__restrict__ v,
                                                        const double *__restrict__ f,
                                                        const double *__restrict__ m, int64_t n,
                                                        double hdt, double dt)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= 3 * n) return;
    const double ft = f[t], mt = m[t / 3];
    const double vk = v[t] + hdt * ft / mt;
    const double inv_m = 1.0 / mt;
    const double vv = vk + hdt * ft * inv_m;
    v[t] = vv;
    x[t] = x[t] + dt * vv;
}

void launch_kick_kick_drift(double *x, double *v, const double *f, const double *m, int64_t n,
                            double dt, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_kick_kick_drift, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, s,
                       x, v, f, m, n, 0.5 * dt, dt);
}

void launch_kick_drift(double *x, double *v, const double *f, const double *m, int64_t n,
                       double dt, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_kick_drift, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, s, x, v,
                       f, m, n, 0.5 * dt, dt);
}

void launch_kick(double *v, const double *f, const double *m, int64_t n, double dt, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_kick, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, s, v, f, m, n,
                       0.5 * dt);
}

// ---------------------------------------------------------------------------
// energies: 256 blocks x 256 threads, grid-stride in a fixed order, then a
// fixed pairwise tree inside each block and a single block over the partials.
// slots: 0 K, 1 U, 2 K ion (q > 0), 3 K electron (q < 0)
// ---------------------------------------------------------------------------
constexpr int kEBlocks = 256;
constexpr int kEThreads = 256;

__device__ __forceinline__ void block_tree_sum4(double (*sh)[kEThreads], double *v)
{
    for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] = v[j];
    __syncthreads();
    for (int w = kEThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + w];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kEThreads) void k_energy_partial(
    const double *__restrict__ v, const double *__restrict__ q, const double *__restrict__ m,
    const double4 *__restrict__ acc, const double4 *__restrict__ xq, int64_t n, double *part,
    const int32_t *flags)
{
    __shared__ double sh[4][kEThreads];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    if (*flags == 0) {
        for (int64_t i = blockIdx.x * (int64_t)kEThreads + threadIdx.x; i < n;
             i += (int64_t)kEBlocks * kEThreads) {
            const double vx = v[3 * i], vy = v[3 * i + 1], vz = v[3 * i + 2];
            const double k = 0.5 * m[i] * (vx * vx + vy * vy + vz * vz);
            a[0] += k;
            if (q[i] > 0.0) a[2] += k;
            if (q[i] < 0.0) a[3] += k;
            a[1] += 0.5 * xq[i].w * acc[i].w;   // sorted order: q and phi of the same particle
        }
    }
    block_tree_sum4(sh, a);
    if (threadIdx.x == 0)
        for (int j = 0; j < 4; ++j) part[4 * blockIdx.x + j] = sh[j][0];
}

__global__ __launch_bounds__(kEThreads) void k_energy_final(const double *__restrict__ part,
                                                           double *out)
{
    __shared__ double sh[4][kEThreads];
    double a[4];
    for (int j = 0; j < 4; ++j) a[j] = part[4 * threadIdx.x + j];
    block_tree_sum4(sh, a);
    if (threadIdx.x == 0) {
        out[0] = sh[0][0];
        out[1] = sh[1][0];
        out[2] = sh[0][0] + sh[1][0];
        out[3] = sh[2][0];
        out[4] = sh[3][0];
    }
}

void launch_energy(Ctx *c, const double *v, const double *q, const double *m, int64_t n,
                   double *out, hipStream_t s)
{
    static_assert(kEBlocks == kEThreads, "final pass reads one partial per thread");
    hipLaunchKernelGGL(k_energy_partial, dim3(kEBlocks), dim3(kEThreads), 0, s, v, q, m,
                       (const double4 *)c->d_acc, (const double4 *)c->d_xq, n, c->d_epart,
                       (const int32_t *)c->d_flags);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kEThreads), 0, s, (const double *)c->d_epart,
                       out);
}

}  // namespace ucp
