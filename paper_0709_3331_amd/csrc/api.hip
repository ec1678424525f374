// api.hip -- the extern "C" entry points declared in include/ucp.h.
#include <string.h>

#include <cstdio>
#include <mutex>
#include <string>

#include "internal.h"

struct ucp_ctx : public ucp::Ctx {};

using ucp::Ctx;

namespace {

// ---------------------------------------------------------------------------
// Adjoint scratch of ucp_force_vjp_noalloc: one static device array per GPU
// (every GPU the library runs on holds its own copy until the process ends),
// sized for a context of at most kNoAllocN particles, kNoAllocNodes node
// slots and kNoAllocClouds clouds (n_max 65,536 and clouds_max 64 give
// node_cap 4 n_max + 64 clouds_max + 1024 = 267,264).  Layout (256-byte
// aligned parts): w double4[N], xsrc double[4 N], cbar double[10 nodes],
// lobar double[4 clouds], lomin uint32[3 clouds]; 25.6 MB in all.
// In host code the array's name only stands in for it: its device address
// is resolved per device with hipGetSymbolAddress and only that is used.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocN = 65536;
constexpr int kNoAllocClouds = 64;
constexpr int64_t kNoAllocNodes = 4 * kNoAllocN + 64 * kNoAllocClouds + 1024;
constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kOffW = 0;
constexpr size_t kOffXsrc = kOffW + align256(32 * (size_t)kNoAllocN);
constexpr size_t kOffCbar = kOffXsrc + align256(32 * (size_t)kNoAllocN);
constexpr size_t kOffLobar = kOffCbar + align256(80 * (size_t)kNoAllocNodes);
constexpr size_t kOffLomin = kOffLobar + align256(32 * (size_t)kNoAllocClouds);
constexpr size_t kNoAllocBytes = kOffLomin + align256(12 * (size_t)kNoAllocClouds);

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};   // device address of `scratch` per device

// the device address of this device's `scratch`, resolved once per device
// with that device current (no allocation is involved)
hipError_t scratch_address(int device, void **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_dev[device] = ptr;
    }
    *out = g_scratch_dev[device];
    return hipSuccess;
}

const char *kNoCtx = "ucp: NULL context";
thread_local std::string g_err;   // errors without a context

ucp_status fail(Ctx *c, ucp_status st, const std::string &msg)
{
    if (c) c->err = msg;
    else g_err = msg;
    return st;
}

#define HIP_TRY(c, call)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((c), UCP_EHIP, std::string("ucp: ") + #call + ": " + hipGetErrorString(e_)); \
    } while (0)

bool validate(const ucp_params *p, std::string &why)
{
    if (!p) { why = "params is NULL"; return false; }
    if (!(p->theta >= 0.0) || !(p->theta < 1.1547005383792515)) {
        why = "theta must satisfy 0 <= theta < 2/sqrt(3)";
        return false;
    }
    if (p->expansion != UCP_EXPANSION_QUADRUPOLE && p->expansion != UCP_EXPANSION_SPECIES) {
        why = "expansion must be UCP_EXPANSION_QUADRUPOLE or UCP_EXPANSION_SPECIES";
        return false;
    }
    if (p->curve != UCP_CURVE_MORTON && p->curve != UCP_CURVE_HILBERT) {
        why = "curve must be UCP_CURVE_MORTON or UCP_CURVE_HILBERT";
        return false;
    }
    if (p->pair_law != UCP_PAIR_PLUMMER && p->pair_law != UCP_PAIR_KELBG) {
        why = "pair_law must be UCP_PAIR_PLUMMER or UCP_PAIR_KELBG";
        return false;
    }
    if (p->pair_law == UCP_PAIR_KELBG) {
        if (!(p->lambda_ei > 0.0) || !(p->lambda_ei < 1e30)) {
            why = "lambda_ei must be > 0 and finite under UCP_PAIR_KELBG";
            return false;
        }
        if (!(p->eps >= 0.0) || !(p->eps < 1e30)) {
            why = "eps must be >= 0 and finite under UCP_PAIR_KELBG";
            return false;
        }
    } else if (!(p->eps > 0.0) || !(p->eps < 1e30)) {
        why = "eps must be > 0 and finite";
        return false;
    }
    if (p->key_bits != 30 && p->key_bits != 63) { why = "key_bits must be 30 or 63"; return false; }
    if (p->leaf_cap < 1 || p->leaf_cap > ucp::kMaxLeafCap) { why = "leaf_cap must be in 1..64"; return false; }
    if (p->group_size < 1 || p->group_size > ucp::kMaxGroup) { why = "group_size must be in 1..64"; return false; }
    if (p->list_len < 64 || p->list_len > 512) { why = "list_len must be in 64..512"; return false; }
    if (p->precision != UCP_FP64 && p->precision != UCP_SPLIT) { why = "precision must be UCP_FP64 or UCP_SPLIT"; return false; }
    if (p->walk_waves < 0 || p->walk_waves > 64) { why = "walk_waves must be in 0..64"; return false; }
    if (p->group_mode != UCP_GROUP_NODE && p->group_mode != UCP_GROUP_CHUNK) {
        why = "group_mode must be UCP_GROUP_NODE or UCP_GROUP_CHUNK";
        return false;
    }
    return true;
}

template <typename T>
hipError_t dalloc(T **p, size_t count)
{
    return hipMalloc((void **)p, count * sizeof(T) + 256);
}

void drop_graph(Ctx *c);

void free_all(Ctx *c)
{
    void *ptrs[] = {c->d_off,  c->d_mm,     c->d_cube,  c->d_key[0], c->d_key[1], c->d_key[2],
                    c->d_val[0], c->d_val[1], c->d_val[2], c->d_hist, c->d_histscan, c->d_xin, c->d_xq, c->d_L,
                    c->d_leaf, c->d_cnt,    c->d_lend, c->d_lvlmax, c->d_offstat, c->d_noff,  c->d_goff,   c->d_gnode,  c->d_gcl, c->d_scanblk,
                    c->d_ngeo, c->d_ninfo,  c->d_npar,  c->d_mom64,  c->d_nrec,
                    c->d_groups, c->d_gstat, c->d_acc,  c->d_ctr,    c->d_flags,  c->d_epart,
                    c->d_leafof, c->d_w,    c->d_xsrc,  c->d_cbar,  c->d_lobar, c->d_lomin, c->d_wq,
                    c->d_ghist,  c->d_sortctl, c->d_nlev, c->d_uplist, c->d_ctab, c->d_spec, c->d_wclock};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
}

void drop_graph(Ctx *c)
{
    for (hipGraphExec_t *e : {&c->gexec, &c->gexec_last}) {
        if (*e) (void)hipGraphExecDestroy(*e);
        *e = nullptr;
    }
    for (hipGraph_t *g : {&c->graph, &c->graph_last}) {
        if (*g) (void)hipGraphDestroy(*g);
        *g = nullptr;
    }
    c->gkey.clear();
}

bool ptr_ok(const void *p, int64_t n) { return n == 0 || p != nullptr; }

// the part of a Verlet step after its opening kick and drift: rebuild,
// forces, then the closing kick, or (more == true, another step follows in
// the same call) the closing kick fused with the next step's opening kick
// and drift
void enqueue_step_tail(Ctx *c, double *x, double *v, double *f, const double *q,
                       const double *m, const int64_t *offsets, int clouds, int64_t n, double dt,
                       bool more, hipStream_t s)
{
    ucp::launch_build(c, x, q, offsets, clouds, n, s);
    c->built = 1;
    c->n = n;
    c->clouds = clouds;
    c->p_built = c->p;
    ucp::launch_forces(c, f, nullptr, s);
    if (more) ucp::launch_kick_kick_drift(x, v, f, m, n, dt, s);
    else ucp::launch_kick(v, f, m, n, dt, s);
}

hipError_t capture_tail(Ctx *c, double *x, double *v, double *f, const double *q,
                        const double *m, const int64_t *offsets, int clouds, int64_t n, double dt,
                        bool more, hipGraph_t *g, hipGraphExec_t *ge)
{
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return e;
    enqueue_step_tail(c, x, v, f, q, m, offsets, clouds, n, dt, more, c->cap_stream);
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipStreamEndCapture(c->cap_stream, g);
    if (e1 != hipSuccess || e2 != hipSuccess || !*g) return e1 != hipSuccess ? e1 : e2;
    return hipGraphInstantiate(ge, *g, nullptr, nullptr, 0);
}

ucp_status run_steps(Ctx *c, double *x, double *v, double *f, const double *q, const double *m,
                     const int64_t *offsets, int clouds, int64_t n, double dt, int nsteps,
                     hipStream_t s)
{
    if (nsteps <= 0 || n == 0) return UCP_OK;
    if (c->timing || nsteps < 2) {
        ucp::launch_kick_drift(x, v, f, m, n, dt, s);   // the first step's opening kick and drift
        for (int t = 0; t < nsteps; ++t)
            enqueue_step_tail(c, x, v, f, q, m, offsets, clouds, n, dt, t + 1 < nsteps, s);
        HIP_TRY(c, hipGetLastError());
        return UCP_OK;
    }
    uint64_t dtb;
    memcpy(&dtb, &dt, sizeof dtb);
    // every parameter byte is part of the key
    uint64_t pb[(sizeof(ucp_params) + 7) / 8] = {};
    memcpy(pb, &c->p, sizeof c->p);
    std::vector<uintptr_t> key = {(uintptr_t)x, (uintptr_t)v, (uintptr_t)f, (uintptr_t)q,
                                  (uintptr_t)m, (uintptr_t)offsets, (uintptr_t)clouds,
                                  (uintptr_t)n, (uintptr_t)dtb};
    for (uint64_t w : pb) key.push_back((uintptr_t)w);
    if (!c->gexec || key != c->gkey) {
        drop_graph(c);
        hipError_t e = capture_tail(c, x, v, f, q, m, offsets, clouds, n, dt, true, &c->graph,
                                    &c->gexec);
        if (e == hipSuccess)
            e = capture_tail(c, x, v, f, q, m, offsets, clouds, n, dt, false, &c->graph_last,
                             &c->gexec_last);
        if (e != hipSuccess) {
            drop_graph(c);
            return fail(c, UCP_EHIP, std::string("ucp: step capture failed: ") +
                                         hipGetErrorString(e));
        }
        c->gkey = key;
    }
    ucp::launch_kick_drift(x, v, f, m, n, dt, s);   // the first step's opening kick and drift
    for (int t = 0; t + 1 < nsteps; ++t) HIP_TRY(c, hipGraphLaunch(c->gexec, s));
    HIP_TRY(c, hipGraphLaunch(c->gexec_last, s));
    c->built = 1;
    c->n = n;
    c->clouds = clouds;
    c->p_built = c->p;
    return UCP_OK;
}

}  // namespace

extern "C" {

int32_t ucp_version(void) { return 100; }

void ucp_default_params(ucp_params *p)
{
    if (!p) return;
    p->theta = 0.5;
    p->eps = 0.005;
    p->key_bits = 63;
    p->leaf_cap = 24;
    p->group_size = 64;
    p->list_len = 128;
    p->precision = UCP_SPLIT;
    p->walk_waves = 0;
    p->group_mode = UCP_GROUP_CHUNK;
    p->pair_law = UCP_PAIR_PLUMMER;
    p->lambda_ei = 0.0;
    p->expansion = UCP_EXPANSION_QUADRUPOLE;
    p->curve = UCP_CURVE_HILBERT;
}

const char *ucp_last_error(const ucp_ctx *c)
{
    if (!c) return g_err.c_str();
    return c->err.c_str();
}

ucp_status ucp_create(ucp_ctx **out, int64_t n_max, int32_t clouds_max, const ucp_params *p)
{
    if (!out) return fail(nullptr, UCP_EINVAL, "ucp_create: out is NULL");
    *out = nullptr;
    std::string why;
    if (n_max < 1 || n_max > (int64_t(1) << 28))
        return fail(nullptr, UCP_EINVAL, "ucp_create: n_max must be in 1..2^28");
    if (clouds_max < 1 || clouds_max > 65536)
        return fail(nullptr, UCP_EINVAL, "ucp_create: clouds_max must be in 1..65536");
    if (!validate(p, why)) return fail(nullptr, UCP_EINVAL, "ucp_create: " + why);
    ucp_ctx *c = new ucp_ctx();
    c->p = *p;
    c->n_max = n_max;
    c->clouds_max = clouds_max;
    c->node_cap = 4 * n_max + 64 * (int64_t)clouds_max + 1024;
    if (c->node_cap > 0x7fffffffLL) c->node_cap = 0x7fffffffLL;
    // status words of the sort: 256 per tile of kSortTile elements, and one
    // tile more, which a pass over the wide tiles clears when n is an odd
    // number of small tiles
    const int64_t ntiles = (n_max + ucp::kSortTile - 1) / ucp::kSortTile + 1;
    c->hist_cap = 256 * ntiles;
    const int64_t scan_items = (int64_t)ucp::kScanBlock * ucp::kScanItems;
    const int64_t nblk = ((n_max + 1 > c->hist_cap ? n_max + 1 : c->hist_cap) + scan_items - 1) / scan_items + 2;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device);
    const size_t N = (size_t)n_max, NC = (size_t)c->node_cap;
#define ALLOC(ptr, cnt) if (e == hipSuccess) e = dalloc(&(ptr), (size_t)(cnt))
    ALLOC(c->d_off, clouds_max + 1);
    ALLOC(c->d_gcl, clouds_max + 1);
    ALLOC(c->d_mm, 6 * (size_t)clouds_max);
    ALLOC(c->d_cube, 2 * (size_t)clouds_max);
    ALLOC(c->d_key[0], N);
    ALLOC(c->d_key[1], N);
    ALLOC(c->d_key[2], N);
    ALLOC(c->d_val[0], N);
    ALLOC(c->d_val[1], N);
    ALLOC(c->d_val[2], N);
    ALLOC(c->d_hist, c->hist_cap);
    ALLOC(c->d_histscan, c->hist_cap);
    ALLOC(c->d_ghist, ucp::kSortPassesMax * 256);
    ALLOC(c->d_sortctl, ucp::kSortTickets);
    ALLOC(c->d_xin, N);
    ALLOC(c->d_xq, N);
    ALLOC(c->d_L, N + 1);
    ALLOC(c->d_leaf, N + 1);
    ALLOC(c->d_cnt, N + 1);
    ALLOC(c->d_lend, N + 1);
    ALLOC(c->d_lvlmax, N / 256 + 2);
    ALLOC(c->d_offstat, N / 4096 + 2);
    ALLOC(c->d_noff, N + 1);
    ALLOC(c->d_goff, N + 1);
    ALLOC(c->d_gnode, N + 1);
    ALLOC(c->d_scanblk, nblk);
    ALLOC(c->d_ngeo, NC);
    ALLOC(c->d_ninfo, NC);
    ALLOC(c->d_npar, NC);
    ALLOC(c->d_nlev, NC + 128);
    ALLOC(c->d_uplist, NC);
    ALLOC(c->d_ctab, 8 * NC);
    if (p->expansion == UCP_EXPANSION_SPECIES) ALLOC(c->d_spec, ucp::kSpecVals * NC);
    ALLOC(c->d_mom64, 16 * NC);
    ALLOC(c->d_nrec, 8 * NC);
    ALLOC(c->d_groups, N);
    ALLOC(c->d_gstat, N);
    ALLOC(c->d_acc, N + 64);   // 64 spare slots for the walk's inactive lanes
    ALLOC(c->d_leafof, N);
    ALLOC(c->d_ctr, ucp::CTR_NCTR);
    ALLOC(c->d_wq, ucp::kWalkQueues * ucp::kQStride);
    ALLOC(c->d_flags, 4);
    ALLOC(c->d_epart, 4 * 256);
    ALLOC(c->d_wclock, 3 * ((size_t)std::max(c->num_cu, 1) * 64 + 4));
#undef ALLOC
    // set-up of this device's static adjoint scratch (ucp_force_vjp_noalloc)
    void *scratch_dev = nullptr;
    if (e == hipSuccess) e = scratch_address(c->device, &scratch_dev);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemset(c->d_flags, 0, 4 * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(c->d_ctr, 0, ucp::CTR_NCTR * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        ucp_status st = (e == hipErrorOutOfMemory) ? UCP_ENOMEM : UCP_EHIP;
        std::string msg = std::string("ucp_create: ") + hipGetErrorString(e);
        free_all(c);
        delete c;
        return fail(nullptr, st, msg);
    }
    *out = c;
    return UCP_OK;
}

void ucp_destroy(ucp_ctx *c)
{
    if (!c) return;
    (void)hipDeviceSynchronize();
    free_all(c);
    delete c;
}

ucp_status ucp_set_params(ucp_ctx *c, const ucp_params *p)
{
    if (!c) return fail(nullptr, UCP_EINVAL, kNoCtx);
    std::string why;
    if (!validate(p, why)) return fail(c, UCP_EINVAL, "ucp_set_params: " + why);
    // the expansion and the curve decide what the build computes, so they need
    // a new build
    const bool topo = p->key_bits != c->p.key_bits || p->leaf_cap != c->p.leaf_cap ||
                      p->group_size != c->p.group_size || p->group_mode != c->p.group_mode ||
                      p->expansion != c->p.expansion || p->curve != c->p.curve;
    if (p->expansion == UCP_EXPANSION_SPECIES && !c->d_spec) {
        const hipError_t e = dalloc(&c->d_spec, (size_t)c->node_cap * ucp::kSpecVals);
        if (e != hipSuccess) {
            c->d_spec = nullptr;
            return fail(c, UCP_ENOMEM, "ucp_set_params: no memory for the species pseudo-particles");
        }
    }
    c->p = *p;
    if (topo) c->built = 0;
    else if (c->built) {
        // theta, eps, list length, precision act at force time
        c->p_built.theta = p->theta;
        c->p_built.eps = p->eps;
        c->p_built.list_len = p->list_len;
        c->p_built.precision = p->precision;
        c->p_built.walk_waves = p->walk_waves;
        c->p_built.pair_law = p->pair_law;
        c->p_built.lambda_ei = p->lambda_ei;
    }
    drop_graph(c);
    return UCP_OK;
}

ucp_status ucp_get_params(const ucp_ctx *c, ucp_params *p)
{
    if (!c || !p) return fail(nullptr, UCP_EINVAL, "ucp_get_params: NULL argument");
    *p = c->p;
    return UCP_OK;
}

static ucp_status build_common(ucp_ctx *c, const double *x, const double *q, const int64_t *offsets,
                               int32_t clouds, int64_t n, void *stream, const char *who)
{
    if (!c) return fail(nullptr, UCP_EINVAL, kNoCtx);
    if (n < 0 || n > c->n_max)
        return fail(c, UCP_EINVAL, std::string(who) + ": n must be in 0..n_max");
    if (clouds < 1 || clouds > c->clouds_max)
        return fail(c, UCP_EINVAL, std::string(who) + ": clouds must be in 1..clouds_max");
    if (!ptr_ok(x, n) || !ptr_ok(q, n))
        return fail(c, UCP_EINVAL, std::string(who) + ": NULL particle array");
    hipStream_t s = (hipStream_t)stream;
    c->built = 1;
    c->n = n;
    c->clouds = clouds;
    c->p_built = c->p;
    if (n == 0) return UCP_OK;
    ucp::launch_build(c, x, q, offsets, clouds, n, s);
    HIP_TRY(c, hipGetLastError());
    return UCP_OK;
}

ucp_status ucp_build_tree(ucp_ctx *c, const double *x, const double *q, int64_t n, void *stream)
{
    return build_common(c, x, q, nullptr, 1, n, stream, "ucp_build_tree");
}

ucp_status ucp_build_tree_batched(ucp_ctx *c, const double *x, const double *q,
                                  const int64_t *offsets, int32_t clouds, int64_t n, void *stream)
{
    if (!offsets) return fail(c, UCP_EINVAL, "ucp_build_tree_batched: offsets is NULL");
    return build_common(c, x, q, offsets, clouds, n, stream, "ucp_build_tree_batched");
}

ucp_status ucp_compute_forces(ucp_ctx *c, double *f, double *phi, void *stream)
{
    if (!c) return fail(nullptr, UCP_EINVAL, kNoCtx);
    if (!c->built) return fail(c, UCP_ENOTBUILT, "ucp_compute_forces: no tree has been built");
    if (c->n == 0) return UCP_OK;
    if (!f) return fail(c, UCP_EINVAL, "ucp_compute_forces: f is NULL");
    ucp::launch_forces(c, f, phi, (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return UCP_OK;
}

static ucp_status step_common(ucp_ctx *c, double *x, double *v, double *f, const double *q,
                              const double *m, const int64_t *offsets, int32_t clouds, int64_t n,
                              double dt, int32_t nsteps, void *stream, const char *who)
{
    if (!c) return fail(nullptr, UCP_EINVAL, kNoCtx);
    if (n < 0 || n > c->n_max) return fail(c, UCP_EINVAL, std::string(who) + ": n must be in 0..n_max");
    if (clouds < 1 || clouds > c->clouds_max)
        return fail(c, UCP_EINVAL, std::string(who) + ": clouds must be in 1..clouds_max");
    if (nsteps < 0) return fail(c, UCP_EINVAL, std::string(who) + ": nsteps < 0");
    if (!(dt == dt) || dt > 1e300 || dt < -1e300) return fail(c, UCP_EINVAL, std::string(who) + ": dt not finite");
    if (!ptr_ok(x, n) || !ptr_ok(v, n) || !ptr_ok(f, n) || !ptr_ok(q, n) || !ptr_ok(m, n))
        return fail(c, UCP_EINVAL, std::string(who) + ": NULL particle array");
    return run_steps(c, x, v, f, q, m, offsets, clouds, n, dt, nsteps, (hipStream_t)stream);
}

ucp_status ucp_step(ucp_ctx *c, double *x, double *v, double *f, const double *q, const double *m,
                    int64_t n, double dt, int32_t nsteps, void *stream)
{
    return step_common(c, x, v, f, q, m, nullptr, 1, n, dt, nsteps, stream, "ucp_step");
}

ucp_status ucp_step_batched(ucp_ctx *c, double *x, double *v, double *f, const double *q,
                            const double *m, const int64_t *offsets, int32_t clouds, int64_t n,
                            double dt, int32_t nsteps, void *stream)
{
    if (!offsets) return fail(c, UCP_EINVAL, "ucp_step_batched: offsets is NULL");
    return step_common(c, x, v, f, q, m, offsets, clouds, n, dt, nsteps, stream, "ucp_step_batched");
}

ucp_status ucp_energy(ucp_ctx *c, const double *x, const double *v, const double *q,
                      const double *m, int64_t n, double *out, void *stream)
{
    if (!c) return fail(nullptr, UCP_EINVAL, kNoCtx);
    if (!out) return fail(c, UCP_EINVAL, "ucp_energy: out is NULL");
    if (!ptr_ok(v, n) || !ptr_ok(m, n)) return fail(c, UCP_EINVAL, "ucp_energy: NULL particle array");
    ucp_status st = build_common(c, x, q, nullptr, 1, n, stream, "ucp_energy");
    if (st != UCP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (n > 0) ucp::launch_forces(c, nullptr, nullptr, s);
    ucp::launch_energy(c, v, q, m, n, out, s);
    HIP_TRY(c, hipGetLastError());
    return UCP_OK;
}

// checks shared by both adjoint entry points; UCP_OK with *skip set when
// there is nothing to do (an empty cloud)
static ucp_status vjp_checks(ucp_ctx *c, const double *u, double *xbar, const char *who, bool *skip)
{
    *skip = false;
    if (!c) return fail(nullptr, UCP_EINVAL, kNoCtx);
    if (!c->built) return fail(c, UCP_ENOTBUILT, std::string(who) + ": no tree has been built");
    if (c->n == 0) {
        *skip = true;
        return UCP_OK;
    }
    if (!u || !xbar) return fail(c, UCP_EINVAL, std::string(who) + ": NULL argument");
    if (c->p_built.pair_law != UCP_PAIR_PLUMMER)
        return fail(c, UCP_EINVAL, std::string(who) + ": only the Plummer pair law has an adjoint");
    if (c->p_built.expansion != UCP_EXPANSION_QUADRUPOLE)
        return fail(c, UCP_EINVAL,
                    std::string(who) + ": only the quadrupole expansion has an adjoint");
    return UCP_OK;
}

ucp_status ucp_force_vjp(ucp_ctx *c, const double *u, double *xbar, void *stream)
{
    bool skip = false;
    const ucp_status st = vjp_checks(c, u, xbar, "ucp_force_vjp", &skip);
    if (st != UCP_OK || skip) return st;
    if (!c->d_w) {
        // the adjoint buffers are allocated on first use
        hipError_t e = hipMalloc((void **)&c->d_w, (size_t)c->n_max * sizeof(double4) + 256);
        if (e == hipSuccess) e = hipMalloc((void **)&c->d_xsrc, (size_t)c->n_max * 4 * sizeof(double) + 256);
        if (e == hipSuccess) e = hipMalloc((void **)&c->d_cbar, (size_t)c->node_cap * 10 * sizeof(double) + 256);
        if (e == hipSuccess) e = hipMalloc((void **)&c->d_lobar, (size_t)c->clouds_max * 4 * sizeof(double) + 256);
        if (e == hipSuccess) e = hipMalloc((void **)&c->d_lomin, (size_t)c->clouds_max * 3 * sizeof(uint32_t) + 256);
        if (e != hipSuccess) {
            for (void *q : {(void *)c->d_w, (void *)c->d_xsrc, (void *)c->d_cbar, (void *)c->d_lobar,
                            (void *)c->d_lomin})
                (void)hipFree(q);
            c->d_w = nullptr;
            c->d_xsrc = nullptr;
            c->d_cbar = nullptr;
            c->d_lobar = nullptr;
            c->d_lomin = nullptr;
            return fail(c, e == hipErrorOutOfMemory ? UCP_ENOMEM : UCP_EHIP,
                        std::string("ucp_force_vjp: ") + hipGetErrorString(e));
        }
    }
    const ucp::VjpScratch sc = {c->d_w, c->d_xsrc, c->d_cbar, c->d_lobar, c->d_lomin};
    ucp::launch_vjp(c, sc, u, xbar, (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return UCP_OK;
}

ucp_status ucp_force_vjp_noalloc(ucp_ctx *c, const double *u, double *xbar, void *stream)
{
    bool skip = false;
    const ucp_status st = vjp_checks(c, u, xbar, "ucp_force_vjp_noalloc", &skip);
    if (st != UCP_OK || skip) return st;
    if (c->n > kNoAllocN || c->node_cap > kNoAllocNodes || c->clouds > kNoAllocClouds)
        return fail(c, UCP_EINVAL,
                    "ucp_force_vjp_noalloc: the static scratch holds at most 65536 particles, "
                    "267264 node slots (a context of n_max <= 65536 and clouds_max <= 64) and 64 "
                    "clouds; this context has n " + std::to_string(c->n) + ", node_cap " +
                        std::to_string(c->node_cap) + ", clouds " + std::to_string(c->clouds) +
                        " (use ucp_force_vjp)");
    int dev = -1;
    HIP_TRY(c, hipGetDevice(&dev));
    if (dev != c->device)
        return fail(c, UCP_EINVAL, "ucp_force_vjp_noalloc: the context's device is not current");
    void *base = nullptr;
    HIP_TRY(c, scratch_address(c->device, &base));
    unsigned char *b = (unsigned char *)base;
    const ucp::VjpScratch sc = {(double4 *)(b + kOffW), (double *)(b + kOffXsrc),
                                (double *)(b + kOffCbar), (double *)(b + kOffLobar),
                                (uint32_t *)(b + kOffLomin)};
    ucp::launch_vjp(c, sc, u, xbar, (hipStream_t)stream);
    HIP_TRY(c, hipGetLastError());
    return UCP_OK;
}

ucp_status ucp_get_stats(ucp_ctx *c, ucp_stats *out, void *stream)
{
    if (!c || !out) return fail(c, UCP_EINVAL, "ucp_get_stats: NULL argument");
    HIP_TRY(c, hipStreamSynchronize((hipStream_t)stream));
    memset(out, 0, sizeof *out);
    out->n = c->n;
    out->clouds = c->clouds;
    if (!c->built || c->n == 0) return UCP_OK;
    unsigned long long ctr[ucp::CTR_NCTR];
    int32_t fl[2] = {0, 0}, nodes = 0, groups = 0;
    HIP_TRY(c, hipMemcpy(ctr, c->d_ctr, sizeof ctr, hipMemcpyDeviceToHost));
    // the current build's flags and those of every build since the last call;
    // the sticky word is cleared and the current build's flags are marked as
    // reported (they stay set, and stop its kernels, until the next build)
    HIP_TRY(c, hipMemcpy(fl, c->d_flags, sizeof fl, hipMemcpyDeviceToHost));
    const int32_t clear_and_mark[2] = {0, fl[0]};
    HIP_TRY(c, hipMemcpy(c->d_flags + 1, clear_and_mark, sizeof clear_and_mark,
                         hipMemcpyHostToDevice));
    const int32_t flags = fl[0] | fl[1];
    HIP_TRY(c, hipMemcpy(&nodes, c->d_noff + c->n, sizeof nodes, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(&groups, c->d_goff + c->n, sizeof groups, hipMemcpyDeviceToHost));
    out->nodes = nodes;
    out->groups = groups;
    out->max_level = (int64_t)ctr[ucp::CTR_MAXLEVEL];
    out->p2p = (int64_t)ctr[ucp::CTR_P2P];
    out->m2p = (int64_t)ctr[ucp::CTR_M2P];
    out->flags = flags;
    if (flags & UCP_FLAG_NODE_OVERFLOW)
        return fail(c, UCP_ECAPACITY, "ucp: node capacity exceeded (" + std::to_string(nodes) +
                                          " > " + std::to_string(c->node_cap) + ")");
    if (flags & UCP_FLAG_NONFINITE) return fail(c, UCP_ENONFINITE, "ucp: non-finite coordinate in the input");
    if (flags & UCP_FLAG_BAD_OFFSETS) return fail(c, UCP_EINVAL, "ucp: inconsistent cloud offsets");
    if (flags & UCP_FLAG_BAD_CUBE) return fail(c, UCP_EINVAL, "ucp: cloud extent out of range");
    if (flags & UCP_FLAG_INTERNAL) return fail(c, UCP_EHIP, "ucp: inconsistent tree records detected on the device");
    if (flags & UCP_FLAG_WALK_STACK)
        return fail(c, UCP_ECAPACITY, "ucp: walk traversal stack exceeded (use a smaller group_size)");
    return UCP_OK;
}

ucp_status ucp_debug_copy(ucp_ctx *c, int32_t which, void *dst, int64_t bytes, void *stream)
{
    if (!c || !dst) return fail(c, UCP_EINVAL, "ucp_debug_copy: NULL argument");
    if (!c->built) return fail(c, UCP_ENOTBUILT, "ucp_debug_copy: no tree has been built");
    HIP_TRY(c, hipStreamSynchronize((hipStream_t)stream));
    int32_t nodes = 0, groups = 0;
    if (c->n > 0) {
        HIP_TRY(c, hipMemcpy(&nodes, c->d_noff + c->n, sizeof nodes, hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemcpy(&groups, c->d_goff + c->n, sizeof groups, hipMemcpyDeviceToHost));
        if (nodes > c->node_cap) nodes = 0;
    }
    const void *src = nullptr;
    int64_t need = 0;
    switch (which) {
    case 0: src = c->d_skey; need = 8 * c->n; break;
    case 1: src = c->d_perm; need = 4 * c->n; break;
    case 2: src = c->d_ninfo; need = 16 * (int64_t)nodes; break;
    case 3: src = c->d_ngeo; need = 32 * (int64_t)nodes; break;
    case 4: src = c->d_mom64; need = 80 * (int64_t)nodes; break;   // repacked below
    case 5: src = c->d_groups; need = 16 * (int64_t)groups; break;
    case 6: src = c->d_gstat; need = 8 * (int64_t)groups; break;
    case 7: src = c->d_cube; need = 32 * (int64_t)c->clouds; break;
    case 8: src = c->d_wclock; need = 24 * c->wclock_waves; break;
    default: return fail(c, UCP_EINVAL, "ucp_debug_copy: unknown array");
    }
    if (bytes < need) return fail(c, UCP_EINVAL, "ucp_debug_copy: buffer too small, need " + std::to_string(need));
    if (need == 0) return UCP_OK;
    if (which == 4) {
        // Q, px, py, pz, Sxx, Syy, Szz, Sxy, Sxz, Syz from the 16-double records
        std::vector<double> rec(16 * (size_t)nodes);
        HIP_TRY(c, hipMemcpy(rec.data(), c->d_mom64, rec.size() * sizeof(double), hipMemcpyDeviceToHost));
        double *o = (double *)dst;
        static const int pick[10] = {3, 4, 5, 6, 8, 9, 10, 11, 12, 13};
        for (int32_t k = 0; k < nodes; ++k)
            for (int i = 0; i < 10; ++i) o[10 * (size_t)k + i] = rec[16 * (size_t)k + pick[i]];
        return UCP_OK;
    }
    if (which == 7) {
        // lo xyz and e per cloud, from the two double4 records
        std::vector<double4> cube(2 * (size_t)c->clouds);
        HIP_TRY(c, hipMemcpy(cube.data(), c->d_cube, cube.size() * sizeof(double4), hipMemcpyDeviceToHost));
        double *o = (double *)dst;
        for (int k = 0; k < c->clouds; ++k) {
            o[4 * k] = cube[2 * k].x;
            o[4 * k + 1] = cube[2 * k].y;
            o[4 * k + 2] = cube[2 * k].z;
            o[4 * k + 3] = cube[2 * k + 1].y;
        }
        return UCP_OK;
    }
    HIP_TRY(c, hipMemcpy(dst, src, (size_t)need, hipMemcpyDeviceToHost));
    return UCP_OK;
}

ucp_status ucp_set_timing(ucp_ctx *c, int32_t on)
{
    if (!c) return fail(nullptr, UCP_EINVAL, kNoCtx);
    c->timing = on ? 1 : 0;
    c->ev_used = 0;
    return UCP_OK;
}

ucp_status ucp_timing_read(ucp_ctx *c, double *walk_ms, int64_t *walk_launches)
{
    if (!c || !walk_ms || !walk_launches) return fail(c, UCP_EINVAL, "ucp_timing_read: NULL argument");
    double tot = 0.0;
    for (int64_t i = 0; i < c->ev_used; ++i) {
        HIP_TRY(c, hipEventSynchronize(c->ev[2 * i + 1]));
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
        tot += ms;
    }
    *walk_ms = tot;
    *walk_launches = c->ev_used;
    c->ev_used = 0;
    return UCP_OK;
}

}  // extern "C"
