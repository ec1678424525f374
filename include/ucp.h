/*
 * ucp.h -- C-ABI of the MI355X (gfx950) two-component plasma TREE library.
 *
 * The library evaluates the Barnes-Hut electrostatic forces of a cloud of
 * ions and electrons (Sec. 3 of Jeon, Kress, Collins, Gronbech-Jensen,
 * "Parallel TREE code for two-component ultracold plasma analysis") and
 * advances it by velocity Verlet (Sec. 2).  Everything runs on one GPU.
 *
 * Conventions for every entry point:
 *  - All particle arrays are DEVICE pointers owned by the caller, float64,
 *    C-contiguous.  Positions, velocities, forces and cotangents are [n][3]
 *    row-major; charges, masses and potentials are [n].  Results come back in
 *    the caller's particle order.
 *  - Reduced units: e^2/(4 pi eps0) = 1, k_B = 1.  The pair law is Eq. (1)-(2)
 *    with Plummer softening eps on every pair:
 *      F_i = q_i sum_j q_j (x_i - x_j) / (|x_i - x_j|^2 + eps^2)^{3/2}.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it; no entry point synchronises the stream unless
 *    it says so.  The context owns every scratch buffer, sized at create
 *    time.  Device memory is allocated by ucp_create, and besides only by the
 *    first ucp_force_vjp on a context (the adjoint's scratch) and by
 *    ucp_set_params when it first selects UCP_EXPANSION_SPECIES (the
 *    pseudo-particle records); ucp_force_vjp_noalloc never allocates.
 *  - Every entry point returns a ucp_status.  No C++ exception crosses the
 *    ABI.  ucp_last_error() returns a human-readable message for the last
 *    failure on that context.  Device-detected problems (node capacity
 *    exceeded, non-finite coordinates, inconsistent offsets) are raised as
 *    flags on the device and reported by the next synchronising call
 *    (ucp_get_stats); kernels launched after a flag is raised do no work
 *    until the next build.  A build starts with clear flags, but keeps every
 *    flag raised since the last ucp_get_stats in a sticky word, so a flag
 *    raised in any step of a multi-step call (or graph replay) is reported.
 *  - A context is not thread-safe; calls that overlap on one context race.
 */
#ifndef UCP_H
#define UCP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    UCP_OK = 0,
    UCP_EINVAL = -1,       /* invalid argument or parameter                    */
    UCP_ENOMEM = -2,       /* a device allocation failed (see the conventions) */
    UCP_EHIP = -3,         /* a HIP runtime call failed                        */
    UCP_ECAPACITY = -4,    /* a device capacity (nodes, particles) was exceeded */
    UCP_ENOTBUILT = -5,    /* forces/VJP requested before a tree was built     */
    UCP_ENONFINITE = -6    /* non-finite coordinate in the input               */
} ucp_status;

typedef enum {
    UCP_FP64 = 0,          /* all interaction arithmetic in FP64                       */
    UCP_SPLIT = 1          /* FP32 interaction arithmetic; FP64 cell moments, FP64
                              per-particle accumulators and FP64 energy sums          */
} ucp_precision;

/* Walk groups.  The targets of one group share one traversal of the tree;
 * each member still takes its own decision of Eq. (5), and a box is opened
 * for the group iff any member rejects it.  Both rules give the per-particle
 * walk of Sec. 3 at G = 1.                                                   */
typedef enum {
    UCP_GROUP_NODE = 0,    /* a node holding <= G particles whose parent holds > G
                              (a leaf holding > G is cut into runs of G)             */
    UCP_GROUP_CHUNK = 1    /* consecutive runs of G particles in key order, per
                              cloud; the last run of a cloud holds the remainder     */
} ucp_group_mode;

/* Pair law of the particle-particle (near-field) terms, Sec. 2.1.
 * UCP_PAIR_PLUMMER: every pair through q_i q_j / h, h^2 = r^2 + eps^2.
 * UCP_PAIR_KELBG: an electron-ion pair (q_i q_j < 0) through the modified
 *   potential of Eq. (3), q_i q_j (1 - exp(-r/lambda_ei)) / r, whose force is
 *   q_i q_j (1 - exp(-u)(1 + u)) r_ij / r^3 with u = r/lambda_ei (no force and
 *   potential q_i q_j / lambda_ei at r = 0); like pairs through the softened
 *   Coulomb law with eps (eps = 0: the bare law of Sec. 2.1).  The far field
 *   (accepted boxes) keeps the expansion of the softened kernel, which for
 *   boxes far beyond lambda_ei is the Coulomb far field.                     */
typedef enum {
    UCP_PAIR_PLUMMER = 0,
    UCP_PAIR_KELBG = 1
} ucp_pair_law;

/* What an accepted box contributes (its pseudo-particle, Sec. 3).
 * UCP_EXPANSION_QUADRUPOLE: charge, dipole and quadrupole about the box
 *   centre (the second-order expansion of the softened kernel), opening test
 *   s^2 < theta^2 d^2 with d to the box centre (delta = 0 in Eq. (5)).
 * UCP_EXPANSION_SPECIES: the paper's twig charges, one per sign: the charge
 *   Q_s of the box's particles of that sign at their centre of charge c_s,
 *   each evaluated like a particle (softened by eps); the box is accepted
 *   iff s/theta + delta_s < d_s for every member of the walk group and every
 *   sign the box holds, with delta_s = |c_s - box centre| and d_s the
 *   distance from the member to c_s (Eq. (5)).  Costs 96 bytes per node
 *   slot, allocated when the expansion is first selected.                  */
typedef enum {
    UCP_EXPANSION_QUADRUPOLE = 0,
    UCP_EXPANSION_SPECIES = 1
} ucp_expansion;

/* Order of the keys, and with it of the sorted particles and of the boxes
 * (Sec. 3's octasection gives the boxes; the order is free).  Both orders
 * give the same boxes and the same per-particle interaction lists; they
 * differ in which particles form a chunk group (UCP_GROUP_CHUNK) and in the
 * order of the nodes.
 * UCP_CURVE_MORTON: the octant digits of the recursive subdivision, most
 *   significant first (octant digit = 4 xbit + 2 ybit + zbit).
 * UCP_CURVE_HILBERT: the boxes visited along a Hilbert curve (Skilling's
 *   transform of the quantised coordinates, AIP Conf. Proc. 707, 381
 *   (2004)): consecutive boxes are face-adjacent, so runs of G consecutive
 *   particles are more compact and share shorter interaction lists.       */
typedef enum {
    UCP_CURVE_MORTON = 0,
    UCP_CURVE_HILBERT = 1
} ucp_curve;

/* Method parameters.  The opening test is Eq. (5), s/theta + delta < d, with
 * the pseudo-particle expanded about the box centre (delta = 0), s the box
 * side and d the distance from the target to the box centre; it is evaluated
 * in FP64 as s^2 < theta^2 d^2.  A walk group (below) opens a box iff any of
 * its members fails the test.                                                */
typedef struct {
    double theta;          /* opening parameter, 0 <= theta < 2/sqrt(3); 0 => direct sum */
    double eps;            /* Plummer softening, > 0 (>= 0 under UCP_PAIR_KELBG, where it
                              softens the like pairs and the far-field expansion only)   */
    int32_t key_bits;      /* 30 or 63 (key depth b = 10 or 21 levels)                   */
    int32_t leaf_cap;      /* a box holding more particles is split (Sec. 3 uses 1); 1..64 */
    int32_t group_size;    /* G: largest walk group, 1..64; see group_mode            */
    int32_t list_len;      /* capacity of each LDS interaction list of a walk group,
                              64..512; changes only the summation order                  */
    int32_t precision;     /* ucp_precision                                              */
    int32_t walk_waves;    /* resident waves per CU for the persistent walk, 0 = auto    */
    int32_t group_mode;    /* ucp_group_mode: how the sorted particles are cut into
                              walk groups                                                */
    int32_t pair_law;      /* ucp_pair_law: the pair law of the particle-particle terms  */
    double lambda_ei;      /* Kelbg length lambda_ei of Eq. (4), > 0 (UCP_PAIR_KELBG)     */
    int32_t expansion;     /* ucp_expansion: what an accepted box contributes            */
    int32_t curve;         /* ucp_curve: the order of the keys                           */
} ucp_params;

typedef struct ucp_ctx ucp_ctx;   /* opaque */

typedef struct {
    int64_t n;             /* particles of the last build                           */
    int64_t clouds;        /* independent clouds of the last build                  */
    int64_t nodes;         /* tree nodes (all clouds)                               */
    int64_t groups;        /* walk groups                                           */
    int64_t max_level;     /* deepest node level                                    */
    int64_t p2p;           /* particle-particle interactions of the last force call,
                              counted per (target, source) pair, self pair included   */
    int64_t m2p;           /* particle-cell interactions of the last force call     */
    int64_t flags;         /* raw device flag word (see UCP_FLAG_*)                  */
} ucp_stats;

#define UCP_FLAG_NODE_OVERFLOW   1
#define UCP_FLAG_NONFINITE       2
#define UCP_FLAG_BAD_OFFSETS     4
#define UCP_FLAG_BAD_CUBE        8
#define UCP_FLAG_INTERNAL       16   /* inconsistent tree records (a library defect) */
#define UCP_FLAG_WALK_STACK     32   /* a walk group overflowed its traversal stack     */

/* Default parameters: theta 0.5, eps 0.005, 63-bit keys, leaf_cap 24, G 64,
 * list_len 128, UCP_SPLIT, walk_waves 0, UCP_GROUP_CHUNK, UCP_PAIR_PLUMMER,
 * lambda_ei 0, UCP_EXPANSION_QUADRUPOLE, UCP_CURVE_HILBERT.                 */
void ucp_default_params(ucp_params *p);

/* Create a context on the current HIP device able to hold n_max particles in
 * up to clouds_max clouds.  Allocates all scratch (about 1 KB per particle).
 * Errors: UCP_EINVAL (n_max < 1, clouds_max < 1, bad params), UCP_ENOMEM,
 * UCP_EHIP.  *out is NULL on failure.                                       */
ucp_status ucp_create(ucp_ctx **out, int64_t n_max, int32_t clouds_max, const ucp_params *p);
void ucp_destroy(ucp_ctx *c);

/* Replace the parameters (validated as in ucp_create).  A tree built before
 * with other key_bits/leaf_cap/group_size/group_mode/expansion/curve must be
 * rebuilt.                                                                  */
ucp_status ucp_set_params(ucp_ctx *c, const ucp_params *p);
ucp_status ucp_get_params(const ucp_ctx *c, ucp_params *p);

/* Build the tree of one cloud (Sec. 3): enclosing cube, keys (ucp_curve), stable
 * radix sort, linear octree in preorder, cell moments (net charge, dipole and
 * quadrupole about each box centre, FP64) and walk groups.  x: [n][3], q: [n].
 * The library keeps sorted copies, so x and q may change after the call
 * returns (stream order).  n = 0 is allowed (empty tree).
 * Errors: UCP_EINVAL (n < 0 or n > n_max, NULL pointers with n > 0).        */
ucp_status ucp_build_tree(ucp_ctx *c, const double *x, const double *q, int64_t n, void *stream);

/* Build the trees of `clouds` independent clouds stored back to back: cloud k
 * holds particles [offsets[k], offsets[k+1]).  offsets is a DEVICE int64
 * array of clouds+1 entries with offsets[0] = 0, nondecreasing, and
 * offsets[clouds] = n (checked on the device: UCP_FLAG_BAD_OFFSETS).  Clouds
 * do not interact.  Errors as ucp_build_tree, plus clouds > clouds_max.    */
ucp_status ucp_build_tree_batched(ucp_ctx *c, const double *x, const double *q,
                                  const int64_t *offsets, int32_t clouds, int64_t n, void *stream);

/* Tree forces of the last build: the group walk of Sec. 3 with the opening
 * test of Eq. (5); accepted boxes contribute their expansion, opened leaves
 * their particles (Eq. (1)-(2), softened).  f: [n][3] out (caller order).
 * phi: [n] out or NULL; the potential excludes the self pair.  The walk
 * writes each target's F and phi as it finishes the target's group, so when
 * the walk raises a device flag (reported by the next ucp_get_stats) the
 * outputs may be partly written.
 * Errors: UCP_ENOTBUILT.                                                    */
ucp_status ucp_compute_forces(ucp_ctx *c, double *f, double *phi, void *stream);

/* nsteps velocity-Verlet (kick-drift-kick) steps, Sec. 2:
 *   v += dt/2 F/m;  x += dt v;  rebuild tree, F = F(x);  v += dt/2 F/m.
 * On entry f must hold F(x) (e.g. from ucp_build_tree + ucp_compute_forces);
 * on exit x, v, f hold the state after nsteps.  Within one call the closing
 * kick of a step and the opening kick and drift of the next run as one pass
 * (the same arithmetic, so the trajectory is bitwise that of nsteps calls of
 * one step).  Steps are captured once in hipGraphs and replayed (re-captured
 * when pointers, sizes or parameters change); a call of one step, and every
 * call while ucp_set_timing is on, enqueues the kernels directly instead.
 * Errors: UCP_EINVAL.                                                       */
ucp_status ucp_step(ucp_ctx *c, double *x, double *v, double *f, const double *q,
                    const double *m, int64_t n, double dt, int32_t nsteps, void *stream);

/* As ucp_step for the clouds of ucp_build_tree_batched (offsets on device). */
ucp_status ucp_step_batched(ucp_ctx *c, double *x, double *v, double *f, const double *q,
                            const double *m, const int64_t *offsets, int32_t clouds, int64_t n,
                            double dt, int32_t nsteps, void *stream);

/* Energies of one cloud at (x, v): builds the tree at x, evaluates the tree
 * potential, and writes to the DEVICE array out[5]:
 *   K = sum m|v|^2/2, U = sum q phi/2, E = K + U, K of ions (q > 0),
 *   K of electrons (q < 0)     (Sec. 5: <KE> = 3 k_B T/2 per species).
 * All sums are FP64 with a fixed reduction order (bitwise reproducible).
 * The tree of the last build is replaced.                                   */
ucp_status ucp_energy(ucp_ctx *c, const double *x, const double *v, const double *q,
                      const double *m, int64_t n, double *out, void *stream);

/* Vector-Jacobian product of the tree forces of the last build with respect
 * to positions, xbar = (dF/dx)^T u (the forces are those of Sec. 3 under the
 * expansion of ucp_compute_forces).  The topology, the interaction lists and
 * the cube's side are piecewise constant in x and held fixed (their jumps are
 * not differentiated).  The cube's origin is the per-axis minimum of each
 * cloud's positions and every box centre is that origin plus a fixed offset,
 * so the centres move with the minimum particles: the derivative through
 * them goes, per cloud and axis, to the particle holding the minimum (the
 * lowest caller index among equal minima).  The walk of the last build is
 * repeated, giving the same lists; each accepted box contributes through the
 * target position, through its dipole and quadrupole (their derivatives with
 * respect to the box's particles) and through its centre, each particle pair
 * through both positions.
 * u, xbar: device [n][3] FP64 (caller order), owned by the caller; u may not
 * alias xbar.  The positions given to the last build must be unchanged.
 * Precision as for the forces (UCP_SPLIT: FP32 arithmetic on offsets formed
 * in FP64, FP64 accumulation).  Contributions of different walk groups to one
 * box or particle are added with FP64 atomics, so xbar is reproducible to
 * rounding, not bitwise.  The first call allocates the adjoint scratch
 * (48 bytes per particle, 80 per node slot, 44 per cloud).
 * Errors: UCP_EINVAL (NULL argument, or a pair law other than
 * UCP_PAIR_PLUMMER or an expansion other than UCP_EXPANSION_QUADRUPOLE: only
 * those have an adjoint), UCP_ENOTBUILT, UCP_ENOMEM, UCP_EHIP; device flags
 * as for ucp_compute_forces.                                                */
ucp_status ucp_force_vjp(ucp_ctx *c, const double *u, double *xbar, void *stream);

/* As ucp_force_vjp, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels, with the adjoint scratch in a static device
 * array of the library (25.6 MB, held on every GPU the library runs on
 * until the process ends, its address resolved by ucp_create) instead of
 * buffers allocated by the first call.  It allocates nothing.  The array
 * serves contexts of at most 65,536 particles, 267,264 node slots (n_max <=
 * 65,536 with clouds_max <= 64) and 64 clouds; larger ones get UCP_EINVAL.
 * Every call on one GPU shares that GPU's array (each call clears what it
 * needs first), so calls that overlap on one GPU race, across contexts too.
 * The context's device must be current.
 * Errors: as ucp_force_vjp, plus UCP_EINVAL for the size limits above.      */
ucp_status ucp_force_vjp_noalloc(ucp_ctx *c, const double *u, double *xbar, void *stream);

/* Synchronise `stream`, read the device counters and flags.  Returns
 * UCP_ECAPACITY / UCP_ENONFINITE / UCP_EINVAL when a flag is raised by the
 * last build or any build since the previous ucp_get_stats (the stats are
 * still filled in; out->flags is their union), else UCP_OK.  Clears the
 * sticky flags; the last build's own flags stay until the next build.     */
ucp_status ucp_get_stats(ucp_ctx *c, ucp_stats *out, void *stream);

/* Introspection of the last build, for tests and tools: copies one internal
 * array to the HOST buffer dst of `bytes` bytes (synchronises `stream`).
 * which:  0 sorted keys (uint64[n])          1 permutation (uint32[n]: sorted
 *         position -> caller index)          2 node info (int32[nodes][4]:
 *         first, count, skip, level | 256*leaf)  3 node geometry
 *         (double[nodes][4]: centre xyz, side^2)  4 FP64 moments
 *         (double[nodes][10]: Q, px, py, pz, Sxx, Syy, Szz, Sxy, Sxz, Syz)
 *         5 groups (int32[groups][4]: first, count, node, root)
 *         6 per-group interaction counts of the last force call
 *         (int32[groups][2]: accepted boxes, P2P source particles)
 *         7 per-cloud cube (double[clouds][4]: lo xyz, e)
 *         8 the start, end and compute unit of every wave of the last force
 *         walk launched with ucp_set_timing on (uint64[waves][3]: start and
 *         end in ticks of the GPU's 100 MHz real-time counter, then
 *         XCC_ID << 32 | HW_ID as the hardware reports them, whose bits 8-15
 *         with the XCC_ID name the CU; waves = 4 * ceil(CUs * W / 4), W the
 *         walk_waves parameter or 32 when it is 0): the balance of the
 *         persistent walk
 * Errors: UCP_EINVAL (unknown `which`, buffer too small).                  */
ucp_status ucp_debug_copy(ucp_ctx *c, int32_t which, void *dst, int64_t bytes, void *stream);

/* Kernel timing with HIP events recorded on the launch stream around every
 * walk kernel (while enabled, ucp_step launches without a graph).
 * ucp_timing_read synchronises and returns the summed walk time in ms and the
 * number of walk launches since the last read, then resets.               */
ucp_status ucp_set_timing(ucp_ctx *c, int32_t on);
ucp_status ucp_timing_read(ucp_ctx *c, double *walk_ms, int64_t *walk_launches);

/* Message for the last error on this context ("" if none); c may be NULL. */
const char *ucp_last_error(const ucp_ctx *c);

/* Library version (major*10000 + minor*100 + patch).                       */
int32_t ucp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* UCP_H */
