/*
 * ucp_oracle.c -- plain, slow, FP64 CPU oracle for the two-component plasma
 * TREE force evaluation (Jeon, Kress, Collins, Gronbech-Jensen,
 * "Parallel TREE code for two-component ultracold plasma analysis").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library and never calls it.
 *
 * What it computes, and where each part comes from:
 *   - Direct sum (definition of the result): the Coulomb pair law of Eq. (1)-(2)
 *     in reduced units (e^2/4 pi eps0 = 1) with Plummer softening eps in place of
 *     the Kelbg form of Eq. (3), applied to every pair.  Neumaier-compensated.
 *   - TREE (the algorithm of Sec. 3, step by step): enclosing cube, recursive
 *     eight-way subdivision until a box holds at most leaf_cap particles, twig
 *     pseudo-particles carrying the charge of everything below them (read here as
 *     net charge, dipole and quadrupole about the box centre), and the opening
 *     criterion s/theta + delta < d of Eq. (5) with delta = 0.
 *   - The architecture series of Sec. 4.3 (node numbers with -1 as the back
 *     step) and a decoder that rebuilds the tree from it.
 *   - Velocity Verlet (Sec. 2), kinetic/potential energy, and the adjoint of the
 *     force map (direct-sum Hessian-vector product and frozen-list tree VJP).
 *
 * Everything is evaluated in FP64 in the plainest form; no blocking, fusion or
 * reordering beyond what the definitions state.  Build with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_VERSION 1

int orc_version(void) { return ORC_VERSION; }
int orc_max_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }

/* ------------------------------------------------------------------------- */
/* Neumaier compensated summation (keeps the direct sum at FP64 truth).       */
/* ------------------------------------------------------------------------- */
typedef struct { double s, c; } nsum;

static inline void nadd(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else                       a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nval(nsum a) { return a.s + a.c; }

/* ------------------------------------------------------------------------- */
/* Pair laws (Sec. 2.1).  ORC_PAIR_PLUMMER: every pair interacts through the  */
/* softened Coulomb potential q_i q_j / h, h^2 = r^2 + eps^2.                */
/* ORC_PAIR_KELBG: an electron-ion pair (q_i q_j < 0) through the modified   */
/* potential of Eq. (3), V = q_i q_j (1 - exp(-r/lambda)) / r; like pairs     */
/* through the softened Coulomb potential (eps = 0: bare, as in Sec. 2.1).   */
/* pair_factors gives the field factor a and the potential factor b of the   */
/* pair, E_i += q_j a (x_i - x_j) and phi_i += q_j b.  For the Kelbg pair,    */
/* -dV/dr gives a = (1 - e^{-u}(1 + u)) / r^3 and b = (1 - e^{-u}) / r with   */
/* u = r / lambda.  Both brackets cancel to O(u^2) and O(u) as u -> 0, so    */
/* below u = 1/4 they are taken from their Taylor series,                    */
/*   1 - e^{-u}(1+u) = sum_{m>=2} (-1)^m (m-1) u^m / m!,                      */
/*   1 - e^{-u}      = sum_{m>=1} (-1)^(m+1) u^m / m!,                        */
/* summed to m = 18 (the next term is below 1e-16 of the sum).  At r = 0 the  */
/* electron-ion pair exerts no force (a r = 0 by symmetry) and b = 1/lambda. */
/* ------------------------------------------------------------------------- */
enum { ORC_PAIR_PLUMMER = 0, ORC_PAIR_KELBG = 1 };
typedef struct { int law; double eps2, lambda; } orc_pair;

static void kelbg_brackets(double u, double *g, double *p)
{
    if (u < 0.25) {
        double term = u, sg = 0.0, sp = 0.0;   /* term = u^m / m! */
        for (int m = 1; m <= 18; ++m) {
            const double sgn = (m % 2) ? 1.0 : -1.0;   /* (-1)^(m+1) */
            sp += sgn * term;
            if (m >= 2) sg += -sgn * (double)(m - 1) * term;
            term *= u / (double)(m + 1);
        }
        *g = sg;
        *p = sp;
    } else {
        const double e = exp(-u);
        *g = 1.0 - e * (1.0 + u);
        *p = 1.0 - e;
    }
}

static void pair_factors(const orc_pair *pl, double qi, double qj, double r2, double *a, double *b)
{
    if (pl->law == ORC_PAIR_KELBG && qi * qj < 0.0) {
        if (r2 == 0.0) { *a = 0.0; *b = 1.0 / pl->lambda; return; }
        const double r = sqrt(r2);
        double g, p;
        kelbg_brackets(r / pl->lambda, &g, &p);
        *a = g / (r2 * r);
        *b = p / r;
        return;
    }
    const double h2 = r2 + pl->eps2;
    const double h = sqrt(h2);
    *a = 1.0 / (h2 * h);
    *b = 1.0 / h;
}

/* ------------------------------------------------------------------------- */
/* C-1  Direct sum.  Eq. (1)-(2) with e^2/(4 pi eps0) = 1 and softening:     */
/*   F_i   = q_i sum_{j!=i} q_j (x_i - x_j) / (|x_i - x_j|^2 + eps^2)^{3/2}  */
/*   phi_i =     sum_{j!=i} q_j / (|x_i - x_j|^2 + eps^2)^{1/2}              */
/* x is [n][3] row-major; f is [n][3]; phi may be NULL.                      */
/* ------------------------------------------------------------------------- */
static void direct_one(int64_t n, const double *x, const double *q, const orc_pair *pl,
                       int64_t i, double *fi, double *phii)
{
    nsum ex = {0, 0}, ey = {0, 0}, ez = {0, 0}, ph = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double rx = x[3 * i + 0] - x[3 * j + 0];
        double ry = x[3 * i + 1] - x[3 * j + 1];
        double rz = x[3 * i + 2] - x[3 * j + 2];
        double a, b;
        pair_factors(pl, q[i], q[j], rx * rx + ry * ry + rz * rz, &a, &b);
        double w = q[j] * a;
        nadd(&ex, w * rx);
        nadd(&ey, w * ry);
        nadd(&ez, w * rz);
        nadd(&ph, q[j] * b);
    }
    fi[0] = q[i] * nval(ex);
    fi[1] = q[i] * nval(ey);
    fi[2] = q[i] * nval(ez);
    if (phii) *phii = nval(ph);
}

void orc_direct(int64_t n, const double *x, const double *q, double eps,
                double *f, double *phi)
{
    const orc_pair pl = {ORC_PAIR_PLUMMER, eps * eps, 0.0};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i)
        direct_one(n, x, q, &pl, i, f + 3 * i, phi ? phi + i : NULL);
}

/* Direct sum under a given pair law (law: ORC_PAIR_*; lambda > 0 for Kelbg). */
int orc_direct_pair(int64_t n, const double *x, const double *q, double eps, int law,
                    double lambda, double *f, double *phi)
{
    if ((law != ORC_PAIR_PLUMMER && law != ORC_PAIR_KELBG) ||
        (law == ORC_PAIR_KELBG && !(lambda > 0.0)))
        return -1;
    const orc_pair pl = {law, eps * eps, lambda};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i)
        direct_one(n, x, q, &pl, i, f + 3 * i, phi ? phi + i : NULL);
    return 0;
}

/* Direct sum for a subset of targets (all n particles are sources).          */
void orc_direct_targets(int64_t n, const double *x, const double *q, double eps,
                        int64_t nt, const int64_t *targets, double *f, double *phi)
{
    const orc_pair pl = {ORC_PAIR_PLUMMER, eps * eps, 0.0};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t)
        direct_one(n, x, q, &pl, targets[t], f + 3 * t, phi ? phi + t : NULL);
}

/* Direct-sum vector-Jacobian product of the force map F(x):                 */
/*   xbar_k = sum_i (dF_i/dx_k)^T u_i = q_k sum_{j!=k} q_j K(r_kj) (u_k - u_j) */
/*   K(r) = I/h^3 - 3 r r^T / h^5,  h^2 = |r|^2 + eps^2.                      */
/* It is the negative Hessian of U applied to u.                             */
void orc_direct_vjp(int64_t n, const double *x, const double *q, double eps,
                    const double *u, double *xbar)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < n; ++k) {
        nsum a[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t j = 0; j < n; ++j) {
            if (j == k) continue;
            double r[3] = {x[3 * k] - x[3 * j], x[3 * k + 1] - x[3 * j + 1],
                           x[3 * k + 2] - x[3 * j + 2]};
            double du[3] = {u[3 * k] - u[3 * j], u[3 * k + 1] - u[3 * j + 1],
                            u[3 * k + 2] - u[3 * j + 2]};
            double h2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
            double h = sqrt(h2);
            double h3 = h2 * h, h5 = h3 * h2;
            double rdu = r[0] * du[0] + r[1] * du[1] + r[2] * du[2];
            for (int d = 0; d < 3; ++d)
                nadd(&a[d], q[j] * (du[d] / h3 - 3.0 * r[d] * rdu / h5));
        }
        for (int d = 0; d < 3; ++d) xbar[3 * k + d] = q[k] * nval(a[d]);
    }
}

/* ------------------------------------------------------------------------- */
/* C-2.1  Enclosing cube (Sec. 3: a large cube enclosing all particles).      */
/* Origin lo = per-axis minimum; side L = 2^e with e the smallest integer     */
/* such that 2^e > max_d (hi_d - lo_d); e = 0 when the extent is zero.        */
/* Returns 0, or -1 if a coordinate is not finite or n == 0.                  */
/* ------------------------------------------------------------------------- */
int orc_cube(int64_t n, const double *x, double *lo, int *e)
{
    if (n <= 0) return -1;
    double mn[3], mx[3];
    for (int d = 0; d < 3; ++d) mn[d] = mx[d] = x[d];
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            double v = x[3 * i + d];
            if (!isfinite(v)) return -1;
            if (v < mn[d]) mn[d] = v;
            if (v > mx[d]) mx[d] = v;
        }
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) {
        lo[d] = mn[d];
        double w = mx[d] - mn[d];
        if (w > ext) ext = w;
    }
    int ee = 0;
    if (ext > 0.0) {
        /* smallest e with 2^e > ext, found by stepping the exponent */
        while (ldexp(1.0, ee) <= ext) ++ee;
        while (ldexp(1.0, ee - 1) > ext) --ee;
    }
    *e = ee;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* C-2.2  Morton keys.  The recursive octasection of Sec. 3 labels each box by */
/* the sequence of octant digits on the path from the root; writing those    */
/* digits most-significant first gives the key.                              */
/*   X_d = min(floor((x_d - lo_d) * 2^(b-e)), 2^b - 1)                        */
/*   digit at depth t (from the leaves) = 4*xbit + 2*ybit + zbit              */
/* built here one bit at a time.                                             */
/* ------------------------------------------------------------------------- */
static uint64_t quantise(double v, double lo, int e, int b)
{
    double t = (v - lo) * ldexp(1.0, b - e);
    uint64_t top = (((uint64_t)1) << b) - 1;
    if (!(t >= 0.0)) return 0;
    double fl = floor(t);
    if (fl >= (double)top) return top;
    return (uint64_t)fl;
}

static uint64_t interleave_bits(uint64_t X, uint64_t Y, uint64_t Z, int b)
{
    uint64_t key = 0;
    for (int t = 0; t < b; ++t) {
        key |= ((X >> t) & 1u) << (3 * t + 2);
        key |= ((Y >> t) & 1u) << (3 * t + 1);
        key |= ((Z >> t) & 1u) << (3 * t + 0);
    }
    return key;
}

/* ------------------------------------------------------------------------- */
/* C-2.2b  Hilbert keys.  The same cells, with the children of every box     */
/* visited along a three-dimensional Hilbert curve instead of in octant      */
/* order, so that consecutive keys are always face-adjacent cells.  The      */
/* method is Skilling's transform (J. Skilling, "Programming the Hilbert     */
/* curve", AIP Conf. Proc. 707, 381 (2004)): from the top bit down, each    */
/* coordinate either flips the lower bits of the first coordinate or swaps   */
/* them with its own; a Gray code across the coordinates and a final         */
/* correction follow, and the three results, read bit level by bit level     */
/* (first coordinate most significant), are the index.  The top 3l bits of  */
/* the index name the level-l box, as the Morton digits do.                  */
/* ------------------------------------------------------------------------- */
static uint64_t hilbert_bits(uint64_t X, uint64_t Y, uint64_t Z, int b)
{
    uint64_t a[3] = {X, Y, Z};
    for (uint64_t Q = ((uint64_t)1) << (b - 1); Q > 1; Q >>= 1) {
        uint64_t P = Q - 1;                      /* the bits below Q */
        for (int i = 0; i < 3; ++i) {
            if (a[i] & Q) {
                a[0] ^= P;                       /* flip them in the first coordinate */
            } else {
                uint64_t t = (a[0] ^ a[i]) & P;  /* swap them between a[0] and a[i] */
                a[0] ^= t;
                a[i] ^= t;
            }
        }
    }
    for (int i = 1; i < 3; ++i) a[i] ^= a[i - 1];   /* Gray code */
    uint64_t t = 0;
    for (uint64_t Q = ((uint64_t)1) << (b - 1); Q > 1; Q >>= 1)
        if (a[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) a[i] ^= t;
    return interleave_bits(a[0], a[1], a[2], b);
}

/* curve 0: Morton order; curve 1: Hilbert order */
void orc_keys(int64_t n, const double *x, const double *lo, int e, int b, int curve, uint64_t *key)
{
    for (int64_t i = 0; i < n; ++i) {
        uint64_t X = quantise(x[3 * i + 0], lo[0], e, b);
        uint64_t Y = quantise(x[3 * i + 1], lo[1], e, b);
        uint64_t Z = quantise(x[3 * i + 2], lo[2], e, b);
        key[i] = curve == 1 ? hilbert_bits(X, Y, Z, b) : interleave_bits(X, Y, Z, b);
    }
}

/* ------------------------------------------------------------------------- */
/* Stable ordering of particles by key: ties keep ascending original index.   */
/* Plain top-down merge sort on (key, index).                                */
/* ------------------------------------------------------------------------- */
static void merge_sort_rec(const uint64_t *key, int64_t *a, int64_t *tmp, int64_t lo, int64_t hi)
{
    if (hi - lo < 2) return;
    int64_t mid = lo + (hi - lo) / 2;
    merge_sort_rec(key, a, tmp, lo, mid);
    merge_sort_rec(key, a, tmp, mid, hi);
    int64_t i = lo, j = mid, k = lo;
    while (i < mid && j < hi) {
        if (key[a[j]] < key[a[i]]) tmp[k++] = a[j++];
        else                       tmp[k++] = a[i++];
    }
    while (i < mid) tmp[k++] = a[i++];
    while (j < hi) tmp[k++] = a[j++];
    memcpy(a + lo, tmp + lo, (size_t)(hi - lo) * sizeof(int64_t));
}

void orc_sort(int64_t n, const uint64_t *key, int64_t *perm)
{
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    int64_t *tmp = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    merge_sort_rec(key, perm, tmp, 0, n);
    free(tmp);
}

/* ------------------------------------------------------------------------- */
/* The tree object.                                                          */
/* ------------------------------------------------------------------------- */
struct orc_tree {
    int64_t n;
    double theta, eps;
    int pair_law;          /* ORC_PAIR_*: the near-field (P2P) pair law           */
    int expansion;         /* ORC_EXP_*: what an accepted box contributes          */
    double lambda;         /* Kelbg length (ORC_PAIR_KELBG)                       */
    int b, leaf_cap, G;
    double lo[3];
    int e;
    int curve;         /* 0: Morton keys, 1: Hilbert keys     */
    uint64_t *skey;    /* keys in sorted order                */
    uint64_t *icoord;  /* [n][3] quantised coordinates, sorted order */
    int64_t *perm;     /* sorted position -> caller index     */
    /* nodes, preorder */
    int64_t M, Mcap;
    int32_t *level;
    int64_t *first, *count, *skip;
    double *centre;    /* [M][3] */
    /* groups, in preorder (= sorted position) order */
    int64_t ng, ngcap;
    int group_mode;    /* 0: node groups, 1: consecutive chunks */
    int64_t *gfirst, *gcount, *gnode;
    /* optional frozen interaction lists per group */
    int keep_lists;
    int64_t **m2p, **p2p;  /* per group: accepted cells / opened leaves */
    int64_t *nm2p, *np2p;  /* list lengths (cells, leaves)              */
    int64_t *nsrc;         /* number of P2P source particles per group  */
};
typedef struct orc_tree orc_tree;

static void node_grow(orc_tree *t)
{
    int64_t nc = t->Mcap ? 2 * t->Mcap : 1024;
    t->level = (int32_t *)realloc(t->level, (size_t)nc * sizeof(int32_t));
    t->first = (int64_t *)realloc(t->first, (size_t)nc * sizeof(int64_t));
    t->count = (int64_t *)realloc(t->count, (size_t)nc * sizeof(int64_t));
    t->skip = (int64_t *)realloc(t->skip, (size_t)nc * sizeof(int64_t));
    t->Mcap = nc;
}

/* C-2.3  Recursive subdivision (Sec. 3).  A box at depth lvl holding the     */
/* particles [f, f+c) of the stable key order is split into its eight         */
/* octants when it holds more than leaf_cap particles and lvl < b; empty      */
/* octants get no node.  Nodes are numbered in preorder, children in octant   */
/* order; skip[k] is the first node number after k's subtree.                */
static void build_rec(orc_tree *t, int lvl, int64_t f, int64_t c)
{
    if (t->M == t->Mcap) node_grow(t);
    int64_t k = t->M++;
    t->level[k] = lvl;
    t->first[k] = f;
    t->count[k] = c;
    if (c > t->leaf_cap && lvl < t->b) {
        int shift = 3 * (t->b - lvl - 1);
        int64_t s = f;
        for (uint64_t oct = 0; oct < 8; ++oct) {
            int64_t end = s;
            while (end < f + c && ((t->skey[end] >> shift) & 7u) == oct) ++end;
            if (end > s) build_rec(t, lvl + 1, s, end - s);
            s = end;
        }
    }
    t->skip[k] = t->M;
}

static int is_leaf(const orc_tree *t, int64_t k) { return t->skip[k] == k + 1; }

/* C-2.4  Box geometry: side s = L 2^-lvl and centre                          */
/*   c_d = lo_d + (2 k_d + 1) L 2^-(lvl+1),  k_d = X_d >> (b - lvl),          */
/* X_d the quantised coordinate of any particle of the box (its first).       */
static void node_centre(const orc_tree *t, int64_t k, double *c)
{
    const uint64_t *X = t->icoord + 3 * t->first[k];
    int lvl = t->level[k];
    uint64_t kk[3] = {X[0] >> (t->b - lvl), X[1] >> (t->b - lvl), X[2] >> (t->b - lvl)};
    for (int d = 0; d < 3; ++d)
        c[d] = t->lo[d] + (double)(2 * kk[d] + 1) * ldexp(1.0, t->e - lvl - 1);
}

static double node_side(const orc_tree *t, int64_t k) { return ldexp(1.0, t->e - t->level[k]); }

/* C-2.5  Walk groups.  Node groups (mode 0): a group is a node holding at    */
/* most G particles whose parent holds more than G (the root if it holds at  */
/* most G); a leaf holding more than G particles is cut into consecutive      */
/* chunks of G.  Chunk groups (mode 1): the key-sorted particles are cut into */
/* consecutive runs of G, the last run holding the remainder; the group node  */
/* recorded is the root.  In both modes G = 1 is the per-particle walk of     */
/* Sec. 3.  The group only decides which targets share one opening decision; */
/* the decision itself is made per member (see C-2.6).                       */
static void group_add(orc_tree *t, int64_t f, int64_t c, int64_t node)
{
    if (t->ng == t->ngcap) {
        int64_t nc = t->ngcap ? 2 * t->ngcap : 1024;
        t->gfirst = (int64_t *)realloc(t->gfirst, (size_t)nc * sizeof(int64_t));
        t->gcount = (int64_t *)realloc(t->gcount, (size_t)nc * sizeof(int64_t));
        t->gnode = (int64_t *)realloc(t->gnode, (size_t)nc * sizeof(int64_t));
        t->ngcap = nc;
    }
    t->gfirst[t->ng] = f;
    t->gcount[t->ng] = c;
    t->gnode[t->ng] = node;
    t->ng++;
}

static void groups_rec(orc_tree *t, int64_t k)
{
    if (t->count[k] <= t->G) { group_add(t, t->first[k], t->count[k], k); return; }
    if (is_leaf(t, k)) {
        for (int64_t o = 0; o < t->count[k]; o += t->G) {
            int64_t c = t->count[k] - o < t->G ? t->count[k] - o : t->G;
            group_add(t, t->first[k] + o, c, k);
        }
        return;
    }
    for (int64_t ch = k + 1; ch < t->skip[k]; ch = t->skip[ch]) groups_rec(t, ch);
}

static void groups_chunk(orc_tree *t)
{
    for (int64_t f = 0; f < t->n; f += t->G)
        group_add(t, f, t->n - f < t->G ? t->n - f : t->G, 0);
}

/* ------------------------------------------------------------------------- */
/* C-2.6  Opening criterion, Eq. (5) with delta = 0 (pseudo-particle at the   */
/* box centre): the box is accepted for target x iff s/theta < d, evaluated   */
/* as s^2 < theta^2 d^2 with d^2 = fma(dz,dz, fma(dy,dy, dx*dx)).             */
/* A group opens a box iff any of its members fails the test.                */
/* ------------------------------------------------------------------------- */
typedef struct { int64_t *v; int64_t n, cap; } ivec;
static void ivec_push(ivec *a, int64_t x)
{
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 256;
        a->v = (int64_t *)realloc(a->v, (size_t)a->cap * sizeof(int64_t));
    }
    a->v[a->n++] = x;
}

static int mac_accept(const orc_tree *t, int64_t k, const double *xs, int64_t gf, int64_t gc)
{
    double c[3];
    node_centre(t, k, c);
    double s = node_side(t, k);
    double s2 = s * s;
    double th2 = t->theta * t->theta;
    for (int64_t a = 0; a < gc; ++a) {
        const double *xi = xs + 3 * (gf + a);
        double dx = xi[0] - c[0], dy = xi[1] - c[1], dz = xi[2] - c[2];
        double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
        if (!(s2 < th2 * d2)) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------- */
/* Pseudo-particles as Sec. 3 has them (ORC_EXP_SPECIES): a box carries, per  */
/* species s (q > 0 and q < 0), the charge Q_s = sum q_j of its particles of  */
/* that sign placed at their centre of charge c_s = sum q_j x_j / Q_s (the    */
/* charge-ratio interpolation of the positions below it).  Eq. (5) then reads */
/* s/theta + delta_s < d_s with delta_s = |c_s - c| (c the box centre) and    */
/* d_s the distance from the member to c_s; the box is accepted for a group  */
/* iff every member passes for every species the box holds.  Layout per      */
/* node: Q+, c+[3], Q-, c-[3], delta+, delta- (a species the box does not    */
/* hold has Q_s = 0).  Sums run about the box centre, brute force over the   */
/* node's particles.                                                         */
/* ------------------------------------------------------------------------- */
enum { ORC_EXP_QUADRUPOLE = 0, ORC_EXP_SPECIES = 1 };

static void node_species(const orc_tree *t, int64_t k, const double *xs, const double *qs,
                         const double *c, double *ps)
{
    nsum Q[2], mu[2][3];
    memset(Q, 0, sizeof(Q));
    memset(mu, 0, sizeof(mu));
    for (int64_t p = t->first[k]; p < t->first[k] + t->count[k]; ++p) {
        if (qs[p] == 0.0) continue;
        const int sp = qs[p] > 0.0 ? 0 : 1;
        nadd(&Q[sp], qs[p]);
        for (int d = 0; d < 3; ++d) nadd(&mu[sp][d], qs[p] * (xs[3 * p + d] - c[d]));
    }
    for (int sp = 0; sp < 2; ++sp) {
        const double q = nval(Q[sp]);
        double off[3] = {0.0, 0.0, 0.0};
        if (q != 0.0)
            for (int d = 0; d < 3; ++d) off[d] = nval(mu[sp][d]) / q;
        ps[4 * sp] = q;
        for (int d = 0; d < 3; ++d) ps[4 * sp + 1 + d] = c[d] + off[d];
        ps[8 + sp] = sqrt(off[0] * off[0] + off[1] * off[1] + off[2] * off[2]);
    }
}

static int mac_accept_species(const orc_tree *t, int64_t k, const double *xs, int64_t gf,
                              int64_t gc, const double *ps)
{
    if (!(t->theta > 0.0)) return 0;
    const double s = node_side(t, k);
    for (int sp = 0; sp < 2; ++sp) {
        if (ps[4 * sp] == 0.0) continue;
        const double R = s / t->theta + ps[8 + sp];
        const double *cs = ps + 4 * sp + 1;
        for (int64_t a = 0; a < gc; ++a) {
            const double *xi = xs + 3 * (gf + a);
            double dx = xi[0] - cs[0], dy = xi[1] - cs[1], dz = xi[2] - cs[2];
            double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
            if (!(R * R < d2)) return 0;
        }
    }
    return 1;
}

/* field and potential at x of a box's two pseudo-particles (softened like   */
/* the pairs)                                                                */
static void cell_field_species(const double *ps, const double *x, double eps2, double *E,
                               double *phi)
{
    E[0] = E[1] = E[2] = 0.0;
    *phi = 0.0;
    for (int sp = 0; sp < 2; ++sp) {
        const double q = ps[4 * sp];
        if (q == 0.0) continue;
        double r[3] = {x[0] - ps[4 * sp + 1], x[1] - ps[4 * sp + 2], x[2] - ps[4 * sp + 3]};
        double h2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
        double h = sqrt(h2);
        for (int d = 0; d < 3; ++d) E[d] += q * r[d] / (h2 * h);
        *phi += q / h;
    }
}

/* ps: per-node pseudo-particles (ORC_EXP_SPECIES), NULL otherwise            */
static void walk_rec(const orc_tree *t, int64_t k, const double *xs, int64_t gf, int64_t gc,
                     const double *ps, ivec *M, ivec *P)
{
    const int acc = ps ? mac_accept_species(t, k, xs, gf, gc, ps + 10 * k)
                       : mac_accept(t, k, xs, gf, gc);
    if (acc) { ivec_push(M, k); return; }
    if (is_leaf(t, k)) { ivec_push(P, k); return; }
    for (int64_t ch = k + 1; ch < t->skip[k]; ch = t->skip[ch])
        walk_rec(t, ch, xs, gf, gc, ps, M, P);
}

/* ------------------------------------------------------------------------- */
/* Cell moments about the geometric centre c (pseudo-particle of Sec. 3, read */
/* as net charge, dipole and quadrupole):                                    */
/*   Q = sum q_j, p = sum q_j r'_j, S_ab = sum q_j r'_a r'_b, r' = x_j - c.    */
/* Layout per node: Q, px, py, pz, Sxx, Syy, Szz, Sxy, Sxz, Syz.             */
/* Brute force over the node's particles.                                    */
/* ------------------------------------------------------------------------- */
static void node_moments(const orc_tree *t, int64_t k, const double *xs, const double *qs,
                         const double *c, double *mom)
{
    nsum a[10];
    memset(a, 0, sizeof(a));
    for (int64_t p = t->first[k]; p < t->first[k] + t->count[k]; ++p) {
        double r0 = xs[3 * p] - c[0], r1 = xs[3 * p + 1] - c[1], r2 = xs[3 * p + 2] - c[2];
        double qq = qs[p];
        nadd(&a[0], qq);
        nadd(&a[1], qq * r0);
        nadd(&a[2], qq * r1);
        nadd(&a[3], qq * r2);
        nadd(&a[4], qq * r0 * r0);
        nadd(&a[5], qq * r1 * r1);
        nadd(&a[6], qq * r2 * r2);
        nadd(&a[7], qq * r0 * r1);
        nadd(&a[8], qq * r0 * r2);
        nadd(&a[9], qq * r1 * r2);
    }
    for (int i = 0; i < 10; ++i) mom[i] = nval(a[i]);
}

/* C-2.7  Field and potential of a cell at r = x - c, second-order Taylor     */
/* expansion of the softened kernel 1/h, h^2 = |r|^2 + eps^2:                 */
/*   phi = Q/h + (p.r)/h^3 + (3 r^T S r / h^5 - trS / h^3)/2                  */
/*   E   = [Q/h^3 + 3 (p.r)/h^5 + 7.5 r^T S r / h^7 - 1.5 trS / h^5] r         */
/*         - p/h^3 - 3 S r / h^5                                              */
static void cell_field(const double *mom, const double *r, double eps2, double *E, double *phi)
{
    double Q = mom[0];
    const double *p = mom + 1;
    double Sxx = mom[4], Syy = mom[5], Szz = mom[6], Sxy = mom[7], Sxz = mom[8], Syz = mom[9];
    double h2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
    double h = sqrt(h2);
    double ih = 1.0 / h;
    double ih2 = ih * ih;
    double ih3 = ih2 * ih, ih5 = ih3 * ih2, ih7 = ih5 * ih2;
    double Sr[3] = {Sxx * r[0] + Sxy * r[1] + Sxz * r[2],
                    Sxy * r[0] + Syy * r[1] + Syz * r[2],
                    Sxz * r[0] + Syz * r[1] + Szz * r[2]};
    double rSr = r[0] * Sr[0] + r[1] * Sr[1] + r[2] * Sr[2];
    double pr = p[0] * r[0] + p[1] * r[1] + p[2] * r[2];
    double trS = Sxx + Syy + Szz;
    double alpha = Q * ih3 + 3.0 * pr * ih5 + 7.5 * rSr * ih7 - 1.5 * trS * ih5;
    for (int d = 0; d < 3; ++d) E[d] = alpha * r[d] - p[d] * ih3 - 3.0 * Sr[d] * ih5;
    *phi = Q * ih + pr * ih3 + 0.5 * (3.0 * rSr * ih5 - trS * ih3);
}

/* ------------------------------------------------------------------------- */
/* Tree construction entry point.                                            */
/* ------------------------------------------------------------------------- */
static void tree_walk_group(const orc_tree *t, const double *xs, const double *ps, int64_t g,
                            ivec *M, ivec *P)
{
    M->n = 0;
    P->n = 0;
    if (t->M == 0) return;
    walk_rec(t, 0, xs, t->gfirst[g], t->gcount[g], ps, M, P);
}

static void sorted_copy(const orc_tree *t, const double *x, const double *q, double *xs, double *qs)
{
    for (int64_t p = 0; p < t->n; ++p) {
        int64_t i = t->perm[p];
        xs[3 * p] = x[3 * i];
        xs[3 * p + 1] = x[3 * i + 1];
        xs[3 * p + 2] = x[3 * i + 2];
        if (qs) qs[p] = q[i];
    }
}

void orc_tree_free(orc_tree *t);

orc_tree *orc_tree_new(int64_t n, const double *x, const double *q, double theta, double eps,
                       int b, int leaf_cap, int G, int group_mode, int keep_lists, int curve)
{
    (void)q;
    if (n < 0 || (b != 10 && b != 21) || leaf_cap < 1 || G < 1) return NULL;
    if (group_mode != 0 && group_mode != 1) return NULL;
    if (curve != 0 && curve != 1) return NULL;
    orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
    t->n = n;
    t->theta = theta;
    t->eps = eps;
    t->b = b;
    t->leaf_cap = leaf_cap;
    t->G = G;
    t->group_mode = group_mode;
    t->keep_lists = keep_lists;
    t->curve = curve;
    t->skey = (uint64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
    t->icoord = (uint64_t *)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(uint64_t));
    t->perm = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (n == 0) return t;
    if (orc_cube(n, x, t->lo, &t->e) != 0) { orc_tree_free(t); return NULL; }
    uint64_t *key = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    orc_keys(n, x, t->lo, t->e, b, curve, key);
    orc_sort(n, key, t->perm);
    for (int64_t p = 0; p < n; ++p) {
        t->skey[p] = key[t->perm[p]];
        for (int d = 0; d < 3; ++d)
            t->icoord[3 * p + d] = quantise(x[3 * t->perm[p] + d], t->lo[d], t->e, b);
    }
    free(key);
    build_rec(t, 0, 0, n);
    t->centre = (double *)malloc((size_t)t->M * 3 * sizeof(double));
    for (int64_t k = 0; k < t->M; ++k) node_centre(t, k, t->centre + 3 * k);
    if (group_mode == 0) groups_rec(t, 0);
    else groups_chunk(t);
    if (keep_lists) {
        double *xs = (double *)malloc((size_t)n * 3 * sizeof(double));
        sorted_copy(t, x, NULL, xs, NULL);
        t->m2p = (int64_t **)calloc((size_t)t->ng, sizeof(int64_t *));
        t->p2p = (int64_t **)calloc((size_t)t->ng, sizeof(int64_t *));
        t->nm2p = (int64_t *)calloc((size_t)t->ng, sizeof(int64_t));
        t->np2p = (int64_t *)calloc((size_t)t->ng, sizeof(int64_t));
        t->nsrc = (int64_t *)calloc((size_t)t->ng, sizeof(int64_t));
#pragma omp parallel
        {
            ivec M = {0, 0, 0}, P = {0, 0, 0};
#pragma omp for schedule(dynamic, 4)
            for (int64_t g = 0; g < t->ng; ++g) {
                tree_walk_group(t, xs, NULL, g, &M, &P);
                t->m2p[g] = (int64_t *)malloc((size_t)(M.n ? M.n : 1) * sizeof(int64_t));
                t->p2p[g] = (int64_t *)malloc((size_t)(P.n ? P.n : 1) * sizeof(int64_t));
                memcpy(t->m2p[g], M.v, (size_t)M.n * sizeof(int64_t));
                memcpy(t->p2p[g], P.v, (size_t)P.n * sizeof(int64_t));
                t->nm2p[g] = M.n;
                t->np2p[g] = P.n;
                int64_t s = 0;
                for (int64_t a = 0; a < P.n; ++a) s += t->count[P.v[a]];
                t->nsrc[g] = s;
            }
            free(M.v);
            free(P.v);
        }
        free(xs);
    }
    return t;
}

void orc_tree_free(orc_tree *t)
{
    if (!t) return;
    if (t->m2p) {
        for (int64_t g = 0; g < t->ng; ++g) { free(t->m2p[g]); free(t->p2p[g]); }
        free(t->m2p);
        free(t->p2p);
        free(t->nm2p);
        free(t->np2p);
        free(t->nsrc);
    }
    free(t->skey); free(t->perm); free(t->icoord);
    free(t->level); free(t->first); free(t->count); free(t->skip); free(t->centre);
    free(t->gfirst); free(t->gcount); free(t->gnode);
    free(t);
}

int64_t orc_tree_nnodes(const orc_tree *t) { return t->M; }
int64_t orc_tree_ngroups(const orc_tree *t) { return t->ng; }
/* Near-field pair law of the tree's P2P terms (ORC_PAIR_*; lambda > 0 for  */
/* Kelbg); the far field is the softened expansion either way.              */
/* What an accepted box contributes (ORC_EXP_*).  The species pseudo-       */
/* particles change the lists, so a tree that keeps lists (for the adjoint)  */
/* takes the expansion only.                                                 */
int orc_tree_set_expansion(orc_tree *t, int expansion)
{
    if (expansion != ORC_EXP_QUADRUPOLE && expansion != ORC_EXP_SPECIES) return -1;
    if (expansion != ORC_EXP_QUADRUPOLE && t->keep_lists) return -1;
    t->expansion = expansion;
    return 0;
}

int orc_tree_set_pair(orc_tree *t, int law, double lambda)
{
    if ((law != ORC_PAIR_PLUMMER && law != ORC_PAIR_KELBG) ||
        (law == ORC_PAIR_KELBG && !(lambda > 0.0)))
        return -1;
    t->pair_law = law;
    t->lambda = lambda;
    return 0;
}

void orc_tree_cube(const orc_tree *t, double *lo, int *e)
{
    for (int d = 0; d < 3; ++d) lo[d] = t->lo[d];
    *e = t->e;
}
void orc_tree_perm(const orc_tree *t, int64_t *perm) { memcpy(perm, t->perm, (size_t)t->n * sizeof(int64_t)); }
void orc_tree_sorted_keys(const orc_tree *t, uint64_t *k) { memcpy(k, t->skey, (size_t)t->n * sizeof(uint64_t)); }
void orc_tree_nodes(const orc_tree *t, int32_t *level, int64_t *first, int64_t *count, int64_t *skip)
{
    for (int64_t k = 0; k < t->M; ++k) {
        level[k] = t->level[k];
        first[k] = t->first[k];
        count[k] = t->count[k];
        skip[k] = t->skip[k];
    }
}
void orc_tree_centres(const orc_tree *t, double *c) { memcpy(c, t->centre, (size_t)t->M * 3 * sizeof(double)); }
void orc_tree_groups(const orc_tree *t, int64_t *first, int64_t *count, int64_t *node)
{
    for (int64_t g = 0; g < t->ng; ++g) {
        first[g] = t->gfirst[g];
        count[g] = t->gcount[g];
        node[g] = t->gnode[g];
    }
}

/* Moments of every node from positions x (caller order).                    */
void orc_tree_moments(const orc_tree *t, const double *x, const double *q, double *mom)
{
    if (t->n == 0) return;
    double *xs = (double *)malloc((size_t)t->n * 3 * sizeof(double));
    double *qs = (double *)malloc((size_t)t->n * sizeof(double));
    sorted_copy(t, x, q, xs, qs);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < t->M; ++k) node_moments(t, k, xs, qs, t->centre + 3 * k, mom + 10 * k);
    free(xs);
    free(qs);
}

/* ------------------------------------------------------------------------- */
/* C-2.8  Tree forces.  For each group, accepted cells contribute their       */
/* expansion (C-2.7) and opened leaves contribute their particles directly    */
/* (C-1 restricted to the leaf); F_i = q_i E_i.  phi skips the self pair.     */
/* With frozen lists (keep_lists) the lists of the build are reused and the   */
/* moments are recomputed from x; otherwise the walk runs on x.              */
/* stats[0] = P2P interactions (target-source pairs, self included),          */
/* stats[1] = M2P interactions.  gm2p/gp2p (optional, length ng) receive the  */
/* per-group number of accepted cells and of P2P source particles.           */
/* ------------------------------------------------------------------------- */
/* ------------------------------------------------------------------------- */
/* Size of the terms a target's field is summed from.  An evaluation that     */
/* forms every term in a working precision with unit roundoff u_w (FP32 or   */
/* FP64) and takes the offsets r from a point inside the bounding box of the */
/* target's walk group errs, per target, by at most a small multiple of      */
/*   u_w * A_i,   A_i = sum over the target's terms of                        */
/*                      |term|_+  +  ||d term / d r|| (2 |r| + D_g),          */
/* where |term|_+ is the term with every sum taken over magnitudes (no        */
/* cancellation inside a term), ||d term/d r|| a bound of its Jacobian, and   */
/* D_g the diagonal of the group's bounding box (offsets rounded relative to  */
/* a point of that box move r by at most u_w (2 |r| + D_g)).  This is the   */
/* first-order error analysis of a sum of rounded terms; it bounds each      */
/* particle's error separately instead of the norm over the cloud.           */
/* ------------------------------------------------------------------------- */
static double frob3(const double S[3][3])
{
    double s = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) s += S[a][c] * S[a][c];
    return sqrt(s);
}

static void cell_jacobian(const double *mom, const double *r, double eps2, double J[3][3]);

/* |term|_+ and the Jacobian term of one accepted box (C-2.7) */
static double cell_cond(const double *mom, const double *r, double eps2, double rho)
{
    const double S[3][3] = {{mom[4], mom[7], mom[8]}, {mom[7], mom[5], mom[9]},
                            {mom[8], mom[9], mom[6]}};
    const double Qa = fabs(mom[0]);
    const double pa = sqrt(mom[1] * mom[1] + mom[2] * mom[2] + mom[3] * mom[3]);
    const double Sa = frob3(S), trSa = fabs(mom[4]) + fabs(mom[5]) + fabs(mom[6]);
    const double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const double ih = 1.0 / sqrt(rn * rn + eps2);
    const double ih3 = ih * ih * ih, ih5 = ih3 * ih * ih, ih7 = ih5 * ih * ih;
    const double mag = (Qa * ih3 + 3.0 * pa * rn * ih5 + 7.5 * Sa * rn * rn * ih7 +
                        1.5 * trSa * ih5) * rn + pa * ih3 + 3.0 * Sa * rn * ih5;
    double J[3][3];
    cell_jacobian(mom, r, eps2, J);
    return mag + frob3(J) * rho;
}

/* the same for one particle pair: the field q_j a r has the Jacobian         */
/* q_j (a I + (da/dr) r r^T / r), of norm at most 2 |q_j| a for the softened  */
/* law and |q_j| (2 a + 1/(e lambda r^2)) for the Kelbg pair (its bracket's   */
/* derivative u e^-u is at most 1/e)                                          */
static double pair_cond(const orc_pair *pl, double qi, double qj, double r2, double a,
                        double rho)
{
    const double rn = sqrt(r2);
    double jac = 2.0 * fabs(a);
    if (pl->law == ORC_PAIR_KELBG && qi * qj < 0.0 && r2 > 0.0)
        jac += 1.0 / (exp(1.0) * pl->lambda * r2);
    return fabs(qj) * (fabs(a) * rn + jac * rho);
}

/* Forces and potentials of the members of group g (C-2.8), written in the   */
/* caller's order; returns the group's list lengths (cells, P2P sources).    */
/* cond (optional, caller order) receives A_i.                               */
static void eval_group(const orc_tree *t, const double *xs, const double *qs, const double *mom,
                       const double *ps, double eps2, const orc_pair *pl, int64_t g, ivec *M,
                       ivec *P, double *f, double *phi, double *cond, int64_t *mn_out,
                       int64_t *nsrc_out)
{
    const int64_t *mv, *pv;
    int64_t mn, pn;
    if (t->keep_lists) {
        mv = t->m2p[g]; mn = t->nm2p[g];
        pv = t->p2p[g]; pn = t->np2p[g];
    } else {
        tree_walk_group(t, xs, ps, g, M, P);
        mv = M->v; mn = M->n;
        pv = P->v; pn = P->n;
    }
    int64_t nsrc = 0;
    for (int64_t a = 0; a < pn; ++a) nsrc += t->count[pv[a]];
    *mn_out = mn;
    *nsrc_out = nsrc;
    /* diagonal of the members' bounding box */
    double bl[3] = {INFINITY, INFINITY, INFINITY}, bh[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t a = 0; a < t->gcount[g]; ++a)
        for (int d = 0; d < 3; ++d) {
            const double v = xs[3 * (t->gfirst[g] + a) + d];
            bl[d] = v < bl[d] ? v : bl[d];
            bh[d] = v > bh[d] ? v : bh[d];
        }
    const double Dg = sqrt((bh[0] - bl[0]) * (bh[0] - bl[0]) + (bh[1] - bl[1]) * (bh[1] - bl[1]) +
                           (bh[2] - bl[2]) * (bh[2] - bl[2]));
    for (int64_t a = 0; a < t->gcount[g]; ++a) {
        int64_t i = t->gfirst[g] + a;
        const double *xi = xs + 3 * i;
        nsum E[3] = {{0, 0}, {0, 0}, {0, 0}}, ph = {0, 0};
        double A = 0.0;
        for (int64_t m = 0; m < mn; ++m) {
            int64_t k = mv[m];
            const double *c = t->centre + 3 * k;
            double r[3] = {xi[0] - c[0], xi[1] - c[1], xi[2] - c[2]};
            double Ec[3], pc;
            if (ps) cell_field_species(ps + 10 * k, xi, eps2, Ec, &pc);
            else cell_field(mom + 10 * k, r, eps2, Ec, &pc);
            for (int d = 0; d < 3; ++d) nadd(&E[d], Ec[d]);
            nadd(&ph, pc);
            if (cond && !ps) {
                const double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                A += cell_cond(mom + 10 * k, r, eps2, 2.0 * rn + Dg);
            } else if (cond) {
                /* two softened monopoles at the centres of charge */
                for (int sp = 0; sp < 2; ++sp) {
                    const double *v = ps + 10 * k + 4 * sp;
                    double rs[3] = {xi[0] - v[1], xi[1] - v[2], xi[2] - v[3]};
                    const double r2 = rs[0] * rs[0] + rs[1] * rs[1] + rs[2] * rs[2];
                    const double ih = 1.0 / sqrt(r2 + eps2);
                    const orc_pair pp = {ORC_PAIR_PLUMMER, eps2, 0.0};
                    A += pair_cond(&pp, 1.0, v[0], r2, ih * ih * ih, 2.0 * sqrt(r2) + Dg);
                }
            }
        }
        for (int64_t m = 0; m < pn; ++m) {
            int64_t k = pv[m];
            for (int64_t j = t->first[k]; j < t->first[k] + t->count[k]; ++j) {
                double r[3] = {xi[0] - xs[3 * j], xi[1] - xs[3 * j + 1], xi[2] - xs[3 * j + 2]};
                if (j == i) continue;   /* the self pair: r = 0, no field, no potential */
                double a, b;
                const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                pair_factors(pl, qs[i], qs[j], r2, &a, &b);
                double w = qs[j] * a;
                for (int d = 0; d < 3; ++d) nadd(&E[d], w * r[d]);
                nadd(&ph, qs[j] * b);
                if (cond) A += pair_cond(pl, qs[i], qs[j], r2, a, 2.0 * sqrt(r2) + Dg);
            }
        }
        int64_t ci = t->perm[i];
        for (int d = 0; d < 3; ++d) f[3 * ci + d] = qs[i] * nval(E[d]);
        if (phi) phi[ci] = nval(ph);
        if (cond) cond[ci] = A;
    }
}

/* Tree forces of the groups gsel[0 .. ngs-1] only (all groups when gsel is  */
/* NULL); members of other groups are left untouched in f and phi.  gm2p and */
/* gp2p, when given, receive the list lengths per evaluated group, in the    */
/* order evaluated.                                                          */
static void eval_groups(const orc_tree *t, const double *x, const double *q, int64_t ngs,
                        const int64_t *gsel, double *f, double *phi, double *cond, int64_t *stats,
                        int64_t *gm2p, int64_t *gp2p)
{
    int64_t n = t->n;
    if (stats) { stats[0] = 0; stats[1] = 0; }
    if (n == 0) return;
    double *xs = (double *)malloc((size_t)n * 3 * sizeof(double));
    double *qs = (double *)malloc((size_t)n * sizeof(double));
    double *mom = (double *)malloc((size_t)t->M * 10 * sizeof(double));
    sorted_copy(t, x, q, xs, qs);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < t->M; ++k) node_moments(t, k, xs, qs, t->centre + 3 * k, mom + 10 * k);
    double *ps = NULL;
    if (t->expansion == ORC_EXP_SPECIES) {
        ps = (double *)malloc((size_t)t->M * 10 * sizeof(double));
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t k = 0; k < t->M; ++k)
            node_species(t, k, xs, qs, t->centre + 3 * k, ps + 10 * k);
    }
    const double eps2 = t->eps * t->eps;
    const orc_pair pl = {t->pair_law, eps2, t->lambda};
    int64_t sp2p = 0, sm2p = 0;
#pragma omp parallel reduction(+ : sp2p, sm2p)
    {
        ivec M = {0, 0, 0}, P = {0, 0, 0};
#pragma omp for schedule(dynamic, 4)
        for (int64_t e = 0; e < ngs; ++e) {
            const int64_t g = gsel ? gsel[e] : e;
            int64_t mn, nsrc;
            eval_group(t, xs, qs, mom, ps, eps2, &pl, g, &M, &P, f, phi, cond, &mn, &nsrc);
            if (gm2p) gm2p[e] = mn;
            if (gp2p) gp2p[e] = nsrc;
            sp2p += nsrc * t->gcount[g];
            sm2p += mn * t->gcount[g];
        }
        free(M.v);
        free(P.v);
    }
    if (stats) { stats[0] = sp2p; stats[1] = sm2p; }
    free(xs);
    free(qs);
    free(mom);
    free(ps);
}

/* cond (optional, [n], caller order) receives the term sizes A_i above.     */
void orc_tree_eval(const orc_tree *t, const double *x, const double *q, double *f, double *phi,
                   int64_t *stats, int64_t *gm2p, int64_t *gp2p, double *cond)
{
    eval_groups(t, x, q, t->ng, NULL, f, phi, cond, stats, gm2p, gp2p);
}

/* Tree forces of selected groups only (for checks of large clouds).  Returns */
/* -1 if a selected index is out of range.                                   */
int orc_tree_eval_groups(const orc_tree *t, const double *x, const double *q, int64_t ngs,
                         const int64_t *gsel, double *f, double *phi, int64_t *gm2p, int64_t *gp2p,
                         double *cond)
{
    for (int64_t e = 0; e < ngs; ++e)
        if (gsel[e] < 0 || gsel[e] >= t->ng) return -1;
    eval_groups(t, x, q, ngs, gsel, f, phi, cond, NULL, gm2p, gp2p);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Tree VJP: xbar = (dF/dx)^T u, the derivative of the forces of this build   */
/* with respect to the positions.  The topology, the interaction lists and    */
/* the cube's side are piecewise constant in x and held fixed (their jumps    */
/* are not differentiated).  The cube's origin lo is not: it is the per-axis  */
/* minimum of the positions (C-2.1), and every box centre is lo plus a fixed  */
/* offset (C-2.4), so the centres move with the particle that attains the     */
/* minimum.  Four contributions:                                             */
/*  (a) target side, J_C = dE_C/dr (symmetric, minus the Hessian of phi_C):   */
/*        xbar_i += q_i J_C(r) u_i                                            */
/*  (b) P2P source side: xbar_j -= q_i q_j K(r_ij) u_i                         */
/*  (c) M2P source side through the moments: per-cell cotangents              */
/*        pbar_C += q_i (dE_C/dp)^T u_i,  Sbar_C += q_i (dE_C/dS)^T u_i        */
/*      pushed to every particle j of C:                                     */
/*        xbar_j += q_j [pbar_C + (Sbar_C + Sbar_C^T)(x_j - c_C)]             */
/*  (d) the cube origin, by the chain rule through every accepted box's      */
/*      centre c_C (r = x_i - c_C, p = sum q_j (x_j - c_C) and S likewise):   */
/*        cbar_C = - sum_i q_i J_C u_i - Q_C pbar_C - (Sbar_C + Sbar_C^T) p_C, */
/*        lobar  = sum_C cbar_C,                                              */
/*      added on each axis d to the particle holding the minimum of that     */
/*      axis (the lowest caller index among equal minima).                   */
/* Requires keep_lists.  Returns 0, or -1 without lists.                     */
/* lobar (optional, [5]) receives the cube-origin cotangent (xyz), the size  */
/* of its terms (the part of each J u through S, which is what the centre's  */
/* derivative reduces to) and the size of the chain-rule terms summed above  */
/* (they cancel to the former, so this oracle's own rounding of lobar is a   */
/* small multiple of 2^-53 times that size).  cond (optional, [n], caller    */
/* order) receives B_j, the sum of the sizes of every term added to xbar_j,  */
/* each taken with its sums over magnitudes: an evaluation that forms each   */
/* term in a working precision with unit roundoff u_w from offsets rounded   */
/* once errs by at most a small multiple of u_w B_j.                         */
/* ------------------------------------------------------------------------- */
static void cell_jacobian(const double *mom, const double *r, double eps2, double J[3][3])
{
    double Q = mom[0];
    const double *p = mom + 1;
    double S[3][3] = {{mom[4], mom[7], mom[8]}, {mom[7], mom[5], mom[9]}, {mom[8], mom[9], mom[6]}};
    double h2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
    double ih = 1.0 / sqrt(h2);
    double ih2 = ih * ih;
    double ih3 = ih2 * ih, ih5 = ih3 * ih2, ih7 = ih5 * ih2, ih9 = ih7 * ih2;
    double Sr[3];
    for (int a = 0; a < 3; ++a) Sr[a] = S[a][0] * r[0] + S[a][1] * r[1] + S[a][2] * r[2];
    double rSr = r[0] * Sr[0] + r[1] * Sr[1] + r[2] * Sr[2];
    double pr = p[0] * r[0] + p[1] * r[1] + p[2] * r[2];
    double trS = S[0][0] + S[1][1] + S[2][2];
    double alpha = Q * ih3 + 3.0 * pr * ih5 + 7.5 * rSr * ih7 - 1.5 * trS * ih5;
    /* grad alpha */
    double ga[3];
    for (int a = 0; a < 3; ++a)
        ga[a] = -3.0 * Q * r[a] * ih5 + 3.0 * p[a] * ih5 - 15.0 * pr * r[a] * ih7 +
                15.0 * Sr[a] * ih7 - 52.5 * rSr * r[a] * ih9 + 7.5 * trS * r[a] * ih7;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
            J[a][c] = (a == c ? alpha : 0.0) + r[a] * ga[c] + 3.0 * p[a] * r[c] * ih5 -
                      3.0 * S[a][c] * ih5 + 15.0 * Sr[a] * r[c] * ih7;
}

int orc_tree_vjp(const orc_tree *t, const double *x, const double *q, const double *u, double *xbar,
                 double *lobar, double *cond)
{
    int64_t n = t->n;
    if (lobar) lobar[0] = lobar[1] = lobar[2] = lobar[3] = lobar[4] = 0.0;
    if (n == 0) return 0;
    if (!t->keep_lists || t->pair_law != ORC_PAIR_PLUMMER) return -1;
    double *xs = (double *)malloc((size_t)n * 3 * sizeof(double));
    double *qs = (double *)malloc((size_t)n * sizeof(double));
    double *us = (double *)malloc((size_t)n * 3 * sizeof(double));
    double *mom = (double *)malloc((size_t)t->M * 10 * sizeof(double));
    sorted_copy(t, x, q, xs, qs);
    sorted_copy(t, u, NULL, us, NULL);
    for (int64_t k = 0; k < t->M; ++k) node_moments(t, k, xs, qs, t->centre + 3 * k, mom + 10 * k);
    const double eps2 = t->eps * t->eps;
    /* per cell: pbar (3), full-matrix Sbar (9), target-side sum rbar (3); per
       particle xbar; and the term sizes (per cell: of pbar and of Sbar + Sbar^T;
       per particle: of xbar; of lobar) */
    double *cot = (double *)calloc((size_t)t->M * 15, sizeof(double));
    double *cab = (double *)calloc((size_t)t->M * 2, sizeof(double));
    double *xb = (double *)calloc((size_t)n * 3, sizeof(double));
    double *xa = (double *)calloc((size_t)n, sizeof(double));
    double loa = 0.0, lch = 0.0;
    /* serial accumulation: deterministic and plainly correct */
    for (int64_t g = 0; g < t->ng; ++g) {
        for (int64_t a = 0; a < t->gcount[g]; ++a) {
            int64_t i = t->gfirst[g] + a;
            const double *xi = xs + 3 * i, *ui = us + 3 * i;
            double qi = qs[i];
            const double wa = fabs(qi) * sqrt(ui[0] * ui[0] + ui[1] * ui[1] + ui[2] * ui[2]);
            for (int64_t m = 0; m < t->nm2p[g]; ++m) {
                int64_t k = t->m2p[g][m];
                const double *c = t->centre + 3 * k;
                double r[3] = {xi[0] - c[0], xi[1] - c[1], xi[2] - c[2]};
                double J[3][3];
                cell_jacobian(mom + 10 * k, r, eps2, J);
                double *pb = cot + 15 * k, *Sb = cot + 15 * k + 3, *rb = cot + 15 * k + 12;
                for (int d = 0; d < 3; ++d) {
                    const double Ju = qi * (J[d][0] * ui[0] + J[d][1] * ui[1] + J[d][2] * ui[2]);
                    xb[3 * i + d] += Ju;
                    rb[d] += Ju;
                }
                double h2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
                double ih = 1.0 / sqrt(h2);
                double ih2 = ih * ih, ih3 = ih2 * ih, ih5 = ih3 * ih2, ih7 = ih5 * ih2, ih9 = ih7 * ih2;
                double ur = ui[0] * r[0] + ui[1] * r[1] + ui[2] * r[2];
                for (int d = 0; d < 3; ++d) pb[d] += qi * (3.0 * r[d] * ur * ih5 - ui[d] * ih3);
                for (int b2 = 0; b2 < 3; ++b2)
                    for (int c2 = 0; c2 < 3; ++c2)
                        Sb[3 * b2 + c2] += qi * (7.5 * ur * r[b2] * r[c2] * ih7 -
                                                 (b2 == c2 ? 1.5 * ur * ih5 : 0.0) -
                                                 3.0 * ui[b2] * r[c2] * ih5);
                if (cond) {
                    const double *mm = mom + 10 * k;
                    const double S[3][3] = {{mm[4], mm[7], mm[8]}, {mm[7], mm[5], mm[9]},
                                            {mm[8], mm[9], mm[6]}};
                    const double Qa = fabs(mm[0]);
                    const double pa = sqrt(mm[1] * mm[1] + mm[2] * mm[2] + mm[3] * mm[3]);
                    const double Sa = frob3(S), tra = fabs(mm[4]) + fabs(mm[5]) + fabs(mm[6]);
                    const double rn = sqrt(h2 - eps2 > 0.0 ? h2 - eps2 : 0.0);
                    /* J u with every sum over magnitudes */
                    const double al = Qa * ih3 + 3.0 * pa * rn * ih5 + 7.5 * Sa * rn * rn * ih7 +
                                      1.5 * tra * ih5;
                    const double ga = 3.0 * Qa * rn * ih5 + 3.0 * pa * ih5 +
                                      15.0 * pa * rn * rn * ih7 + 15.0 * Sa * rn * ih7 +
                                      52.5 * Sa * rn * rn * rn * ih9 + 7.5 * tra * rn * ih7;
                    const double jua = wa * (al + rn * ga + 3.0 * pa * rn * ih5 + 3.0 * Sa * ih5 +
                                             15.0 * Sa * rn * rn * ih7);
                    xa[i] += jua;
                    lch += jua;
                    cab[2 * k] += wa * (3.0 * rn * rn * ih5 + ih3);
                    cab[2 * k + 1] += wa * (15.0 * rn * rn * rn * ih7 + 12.0 * rn * ih5);
                    /* the box's share of lobar, the part of J u through S */
                    loa += wa * ((52.5 * Sa * rn * rn * ih9 + 15.0 * Sa * ih7 + 7.5 * tra * ih7) *
                                     rn * rn +
                                 7.5 * Sa * rn * rn * ih7 + 1.5 * tra * ih5 +
                                 15.0 * Sa * rn * rn * ih7 + 3.0 * Sa * ih5);
                }
            }
            for (int64_t m = 0; m < t->np2p[g]; ++m) {
                int64_t k = t->p2p[g][m];
                for (int64_t j = t->first[k]; j < t->first[k] + t->count[k]; ++j) {
                    if (j == i) continue;
                    double r[3] = {xi[0] - xs[3 * j], xi[1] - xs[3 * j + 1], xi[2] - xs[3 * j + 2]};
                    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                    double h2 = r2 + eps2;
                    double ih = 1.0 / sqrt(h2);
                    double ih3 = ih * ih * ih, ih5 = ih3 * ih * ih;
                    double ur = ui[0] * r[0] + ui[1] * r[1] + ui[2] * r[2];
                    for (int d = 0; d < 3; ++d) {
                        double Ku = ui[d] * ih3 - 3.0 * r[d] * ur * ih5;
                        xb[3 * i + d] += qi * qs[j] * Ku;
                        xb[3 * j + d] -= qi * qs[j] * Ku;
                    }
                    if (cond) {
                        const double ka = wa * fabs(qs[j]) * (ih3 + 3.0 * r2 * ih5);
                        xa[i] += ka;
                        xa[j] += ka;
                    }
                }
            }
        }
    }
    /* push cell cotangents to the particles of each cell */
    for (int64_t k = 0; k < t->M; ++k) {
        const double *pb = cot + 15 * k, *Sb = cot + 15 * k + 3;
        const double *c = t->centre + 3 * k;
        for (int64_t j = t->first[k]; j < t->first[k] + t->count[k]; ++j) {
            double rp[3] = {xs[3 * j] - c[0], xs[3 * j + 1] - c[1], xs[3 * j + 2] - c[2]};
            for (int d = 0; d < 3; ++d) {
                double s = pb[d];
                for (int e2 = 0; e2 < 3; ++e2) s += (Sb[3 * d + e2] + Sb[3 * e2 + d]) * rp[e2];
                xb[3 * j + d] += qs[j] * s;
            }
            if (cond)
                xa[j] += fabs(qs[j]) *
                         (cab[2 * k] + cab[2 * k + 1] *
                                           sqrt(rp[0] * rp[0] + rp[1] * rp[1] + rp[2] * rp[2]));
        }
    }
    /* (d) the cube origin: chain rule through every box centre */
    double lob[3] = {0.0, 0.0, 0.0};
    for (int64_t k = 0; k < t->M; ++k) {
        const double *pb = cot + 15 * k, *Sb = cot + 15 * k + 3, *rb = cot + 15 * k + 12;
        const double Q = mom[10 * k], *pm = mom + 10 * k + 1;
        if (cond)
            lch += fabs(Q) * cab[2 * k] + cab[2 * k + 1] * sqrt(pm[0] * pm[0] + pm[1] * pm[1] +
                                                                   pm[2] * pm[2]);
        for (int d = 0; d < 3; ++d) {
            double s = -rb[d] - Q * pb[d];
            for (int e2 = 0; e2 < 3; ++e2) s -= (Sb[3 * d + e2] + Sb[3 * e2 + d]) * pm[e2];
            lob[d] += s;
        }
    }
    for (int64_t p = 0; p < n; ++p)
        for (int d = 0; d < 3; ++d) xbar[3 * t->perm[p] + d] = xb[3 * p + d];
    if (cond)
        for (int64_t p = 0; p < n; ++p) cond[t->perm[p]] = xa[p];
    for (int d = 0; d < 3; ++d) {
        int64_t jm = 0;
        for (int64_t i = 1; i < n; ++i)
            if (x[3 * i + d] < x[3 * jm + d]) jm = i;
        xbar[3 * jm + d] += lob[d];
        if (cond) cond[jm] += loa;
        if (lobar) lobar[d] = lob[d];
    }
    if (lobar && cond) {
        lobar[3] = loa;
        lobar[4] = lch;
    }
    free(xs); free(qs); free(us); free(mom); free(cot); free(cab); free(xb); free(xa);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Architecture series (Sec. 4.3): each node number (preorder index + 1, so   */
/* that every node number is a natural number) is followed by the series of   */
/* its children, then by -1, the back step.  Length 2 M.                     */
/* ------------------------------------------------------------------------- */
static void arch_rec(const orc_tree *t, int64_t k, int64_t *out, int64_t *pos)
{
    out[(*pos)++] = k + 1;
    for (int64_t ch = k + 1; ch < t->skip[k]; ch = t->skip[ch]) arch_rec(t, ch, out, pos);
    out[(*pos)++] = -1;
}

int64_t orc_tree_arch_series(const orc_tree *t, int64_t *out)
{
    int64_t pos = 0;
    if (t->M > 0) arch_rec(t, 0, out, &pos);
    return pos;
}

/* Decoder for the architecture series: rebuilds parent links and the number  */
/* of children of each node number (1-based) by reading the series left to   */
/* right -- a natural number opens a child of the current node, -1 closes it. */
/* parent[id-1] = parent node number (0 for the root).                       */
/* Returns the number of nodes, or -1 if the series is malformed.            */
static int64_t rebuild_rec(const int64_t *s, int64_t len, int64_t *pos, int64_t par,
                           int64_t *parent, int64_t *nchild, int64_t cap)
{
    if (*pos >= len || s[*pos] <= 0 || s[*pos] > cap) return -1;
    int64_t id = s[(*pos)++];
    parent[id - 1] = par;
    nchild[id - 1] = 0;
    int64_t nodes = 1;
    while (*pos < len && s[*pos] > 0) {
        int64_t sub = rebuild_rec(s, len, pos, id, parent, nchild, cap);
        if (sub < 0) return -1;
        nodes += sub;
        nchild[id - 1]++;
    }
    if (*pos >= len || s[*pos] != -1) return -1;
    (*pos)++;
    return nodes;
}

int64_t orc_rebuild(int64_t len, const int64_t *series, int64_t cap, int64_t *parent, int64_t *nchild)
{
    int64_t pos = 0;
    if (len == 0) return 0;
    int64_t m = rebuild_rec(series, len, &pos, 0, parent, nchild, cap);
    if (m < 0 || pos != len) return -1;
    return m;
}

/* ------------------------------------------------------------------------- */
/* C-3  Velocity Verlet, kick-drift-kick (Sec. 2):                            */
/*   v += dt/2 F(x)/m;  x += dt v;  v += dt/2 F(x')/m.                        */
/* mode 0: direct forces; mode 1: tree forces at (theta, eps, b, leaf_cap, G, */
/* group_mode), the tree rebuilt at every step.  f holds F(x_0) on entry     */
/* when f_valid, and F(x_n) on exit.                                         */
/* ------------------------------------------------------------------------- */
static int forces_any(int mode, int64_t n, const double *x, const double *q, double theta,
                      double eps, int b, int leaf_cap, int G, int group_mode, int curve, double *f)
{
    if (mode == 0) { orc_direct(n, x, q, eps, f, NULL); return 0; }
    orc_tree *t = orc_tree_new(n, x, q, theta, eps, b, leaf_cap, G, group_mode, 0, curve);
    if (!t) return -1;
    orc_tree_eval(t, x, q, f, NULL, NULL, NULL, NULL, NULL);
    orc_tree_free(t);
    return 0;
}

int orc_verlet(int64_t n, double *x, double *v, const double *q, const double *m, int mode,
               double theta, double eps, int b, int leaf_cap, int G, int group_mode, int curve,
               double dt, int nsteps, double *f, int f_valid)
{
    if (!f_valid && forces_any(mode, n, x, q, theta, eps, b, leaf_cap, G, group_mode, curve, f))
        return -1;
    for (int s = 0; s < nsteps; ++s) {
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) {
                v[3 * i + d] += 0.5 * dt * f[3 * i + d] / m[i];
                x[3 * i + d] += dt * v[3 * i + d];
            }
        if (forces_any(mode, n, x, q, theta, eps, b, leaf_cap, G, group_mode, curve, f)) return -1;
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) v[3 * i + d] += 0.5 * dt * f[3 * i + d] / m[i];
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Energies (Sec. 5: <KE> = 3 k_B T / 2 per species; total energy):          */
/*   out[0] K = sum m|v|^2/2, out[1] U = sum q phi / 2, out[2] E = K + U,     */
/*   out[3] K of the ions (q > 0), out[4] K of the electrons (q < 0).         */
/* ------------------------------------------------------------------------- */
void orc_energy(int64_t n, const double *v, const double *q, const double *m, const double *phi,
                double *out)
{
    nsum K = {0, 0}, U = {0, 0}, Ki = {0, 0}, Ke = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        double k = 0.5 * m[i] * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] +
                                 v[3 * i + 2] * v[3 * i + 2]);
        nadd(&K, k);
        if (q[i] > 0) nadd(&Ki, k);
        if (q[i] < 0) nadd(&Ke, k);
        nadd(&U, 0.5 * q[i] * phi[i]);
    }
    out[0] = nval(K);
    out[1] = nval(U);
    out[2] = out[0] + out[1];
    out[3] = nval(Ki);
    out[4] = nval(Ke);
}

/* ------------------------------------------------------------------------- */
/* Direct access for the pins: the C-2.7 expansion for one cell, its          */
/* Jacobian, and the frozen interaction lists of one group.                  */
/* ------------------------------------------------------------------------- */
void orc_cell_eval(const double *mom, const double *r, double eps, double *E, double *phi)
{
    cell_field(mom, r, eps * eps, E, phi);
}

void orc_cell_jacobian(const double *mom, const double *r, double eps, double *J)
{
    double JJ[3][3];
    cell_jacobian(mom, r, eps * eps, JJ);
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) J[3 * a + c] = JJ[a][c];
}

/* Lengths of group g's lists (cells, leaves); with non-NULL outputs, copies */
/* the accepted cells and opened leaves.  Requires keep_lists.               */
int orc_tree_lists(const orc_tree *t, int64_t g, int64_t *nm, int64_t *np, int64_t *m_out,
                   int64_t *p_out)
{
    if (!t->keep_lists || g < 0 || g >= t->ng) return -1;
    *nm = t->nm2p[g];
    *np = t->np2p[g];
    if (m_out) memcpy(m_out, t->m2p[g], (size_t)t->nm2p[g] * sizeof(int64_t));
    if (p_out) memcpy(p_out, t->p2p[g], (size_t)t->np2p[g] * sizeof(int64_t));
    return 0;
}
