/*
 * fmm_oracle.c -- CPU oracle for the PHANTOM-style kd-tree FMM gravity path.
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the package smoke check and the
 * CPU-baseline leg of the benchmark are the only callers.  The GPU library
 * shares no source, header, table or helper with this file and never loads it.
 *
 * Paper: Potashov & Yudin, "Non-conservation of linear momentum in widely used
 * hierarchical methods in gravitational gas dynamics", arXiv:2502.01496.
 *
 * Everything here is plain, serial FP64.  The file is compiled with
 * -O2 -ffp-contract=off and no fast-math, so every operation that feeds a
 * discrete decision (Morton quantisation, split axis, opening criteria) is one
 * IEEE-754 operation, in the order written.
 *
 * What is computed, and where it comes from:
 *   - the softened direct sum, the definition the FMM approximates
 *     (Sec. 2 eq. (3) with theta = 0; Sec. 3 eqs. (12)-(15));
 *   - the kd-tree (Sec. 2: longest-axis cut, leaf cells of a few particles),
 *     split at the count median of the longest axis of the particle bounding
 *     box, ties broken by (coordinate, Morton rank);
 *   - cell mass, centre of mass, size s, h_max and quadrupole (Sec. 2, eq. (7));
 *   - the two interaction criteria (Sec. 2 eqs. (4) and (5)) and the
 *     leaf <- cell walk of Sec. 4, plus the mutual walk recommended in Sec. 7;
 *   - the cell field to second order, eq. (6) and its first two r-derivatives,
 *     the Taylor evaluation at a particle, eq. (8), and the exact re-expansion
 *     of that quadratic polynomial to another centre; and the alternative
 *     expansion of Sec. 4, eqs. (25)-(26) with p = 3 (combined order of the
 *     source and sink offsets at most 2);
 *   - near-field softened pair sums, momentum diagnostics (Secs. 5-6) and the
 *     adjoint of the direct sum.
 *
 * Parity status per function is stated at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Softened pair kernel.                                                     */
/*                                                                           */
/* Sec. 3, eqs. (12)-(15): the pair Green's function is the mean of the two  */
/* softened potentials phi(r, h_i) and phi(r, h_j); beyond R_kern*h it is    */
/* exactly -1/r.  The smoothing kernel is the M4 cubic spline with           */
/* R_kern = 2 (Sec. 6).  phi solves the Poisson equation with W as source    */
/* (Sec. 3), so phi'(r) = M_W(<r) / r^2 with M_W the kernel mass inside r.   */
/* g(r,h) = phi'(r,h)/r, written without dividing by r so that g(0,h) is     */
/* finite.  Pinned by: numerical integration of W (tests), continuity at     */
/* q = 1, 2, and the exact Newtonian value beyond 2h.                        */
/* ------------------------------------------------------------------------ */
ORC_API double orc_m4_g(double r, double h)
{
    double q = r / h;
    double h3 = h * h * h;
    if (q < 1.0)
        return (4.0 / 3.0 - 1.2 * q * q + 0.5 * q * q * q) / h3;
    if (q < 2.0)
        return (8.0 / 3.0 - 3.0 * q + 1.2 * q * q - q * q * q / 6.0 - 1.0 / (15.0 * q * q * q)) / h3;
    return 1.0 / (r * r * r);
}

/* (dg/dr)/r, used only by the adjoint.  Finite at r = 0. */
ORC_API double orc_m4_dg_over_r(double r, double h)
{
    double q = r / h;
    double h5 = h * h * h * h * h;
    if (q < 1.0)
        return (-12.0 / 5.0 + 1.5 * q) / h5;
    if (q < 2.0) {
        double h4 = h * h * h * h;
        return (-3.0 + 2.4 * q - 0.5 * q * q + 1.0 / (5.0 * q * q * q * q)) / h4 / r;
    }
    return -3.0 / (r * r * r * r * r);
}

/* Mean of the two softened kernels: the symmetric pair factor G_ij. */
static double pair_g(double r, double hi, double hj)
{
    return 0.5 * (orc_m4_g(r, hi) + orc_m4_g(r, hj));
}

static double pair_dg_over_r(double r, double hi, double hj)
{
    return 0.5 * (orc_m4_dg_over_r(r, hi) + orc_m4_dg_over_r(r, hj));
}

/* ------------------------------------------------------------------------ */
/* Direct summation: the definition.                                         */
/* a_i = -G sum_{j != i} m_j G_ij (x_i - x_j)   (eq. (3) with theta = 0:     */
/* every interaction short-range; eqs. (12)-(16)).                           */
/* Pinned by: zero total force, the Plummer closed form, Newton's law beyond */
/* 2h.                                                                       */
/* ------------------------------------------------------------------------ */
static void direct_one(int64_t n, const double *x, const double *m, const double *h,
                       double G, int64_t i, double *ai)
{
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i)
            continue;
        double dx = x[3 * i + 0] - x[3 * j + 0];
        double dy = x[3 * i + 1] - x[3 * j + 1];
        double dz = x[3 * i + 2] - x[3 * j + 2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        double f = m[j] * pair_g(r, h[i], h[j]);
        ax -= f * dx;
        ay -= f * dy;
        az -= f * dz;
    }
    ai[0] = G * ax;
    ai[1] = G * ay;
    ai[2] = G * az;
}

ORC_API void orc_direct(int64_t n, const double *x, const double *m, const double *h,
                        double G, double *a)
{
    for (int64_t i = 0; i < n; ++i)
        direct_one(n, x, m, h, G, i, a + 3 * i);
}

/* Direct sum for a subset of sinks (rows of a), sources = all particles. */
ORC_API void orc_direct_sinks(int64_t n, const double *x, const double *m, const double *h,
                              double G, int64_t nsink, const int64_t *sink, double *a)
{
    for (int64_t k = 0; k < nsink; ++k)
        direct_one(n, x, m, h, G, sink[k], a + 3 * k);
}

/* Adjoint of the direct sum: xbar = (da/dx)^T abar, mbar = (da/dm)^T abar.
 * For the pair term f_ij = -G m_j G_ij(r) d, d = x_i - x_j:
 *   df/dd = -G m_j [G_ij I + (G_ij'/r) d d^T],   df/dm_j = -G G_ij d.
 * Pinned by central finite differences of orc_direct (tests). */
ORC_API void orc_direct_vjp(int64_t n, const double *x, const double *m, const double *h,
                            double G, const double *abar, double *xbar, double *mbar)
{
    for (int64_t i = 0; i < 3 * n; ++i)
        xbar[i] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        mbar[i] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *ab = abar + 3 * i;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double d[3] = {x[3 * i + 0] - x[3 * j + 0], x[3 * i + 1] - x[3 * j + 1],
                           x[3 * i + 2] - x[3 * j + 2]};
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double gij = pair_g(r, h[i], h[j]);
            double dgr = pair_dg_over_r(r, h[i], h[j]);
            double da = d[0] * ab[0] + d[1] * ab[1] + d[2] * ab[2];
            for (int c = 0; c < 3; ++c) {
                double db = -G * m[j] * (gij * ab[c] + dgr * da * d[c]);
                xbar[3 * i + c] += db;
                xbar[3 * j + c] -= db;
            }
            mbar[j] += -G * gij * da;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Morton order: the canonical particle order the kd-tree starts from.       */
/* Global box: lo_d = min x_d, ext = max_d (max x_d - lo_d) (1 if 0).        */
/* q_d = min(2^21 - 1, floor((x_d - lo_d) * (2^21 / ext))); bit b of q_d     */
/* goes to key bit 3b + d.  rank = position after sorting by (key, index).   */
/* Pinned by: brute-force interleaving in tests, power-of-two invariance.    */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t key;
    int64_t idx;
} key_idx;

static int cmp_key_idx(const void *pa, const void *pb)
{
    const key_idx *a = (const key_idx *)pa, *b = (const key_idx *)pb;
    if (a->key != b->key)
        return a->key < b->key ? -1 : 1;
    return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

ORC_API void orc_morton(int64_t n, const double *x, uint64_t *key, int32_t *order)
{
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d)
        lo[d] = hi[d] = x[d];
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            double v = x[3 * i + d];
            if (v < lo[d])
                lo[d] = v;
            if (v > hi[d])
                hi[d] = v;
        }
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) {
        double e = hi[d] - lo[d];
        if (e > ext)
            ext = e;
    }
    if (ext == 0.0)
        ext = 1.0;
    double scale = 2097152.0 / ext;
    key_idx *ki = (key_idx *)malloc((size_t)n * sizeof(key_idx));
    for (int64_t i = 0; i < n; ++i) {
        uint64_t k = 0;
        for (int d = 0; d < 3; ++d) {
            double t = floor((x[3 * i + d] - lo[d]) * scale);
            uint64_t q = t >= 2097151.0 ? 2097151u : (uint64_t)t;
            for (int b = 0; b < 21; ++b)
                k |= ((q >> b) & 1u) << (3 * b + d);
        }
        key[i] = k;
        ki[i].key = k;
        ki[i].idx = i;
    }
    qsort(ki, (size_t)n, sizeof(key_idx), cmp_key_idx);
    for (int64_t r = 0; r < n; ++r)
        order[r] = (int32_t)ki[r].idx;
    free(ki);
}

/* ------------------------------------------------------------------------ */
/* kd-tree (Sec. 2: cells are cut recursively along their longest axis into  */
/* two parts until a cell holds no more than leaf_size particles).           */
/* Reading used here: the longest axis of the node's particle bounding box   */
/* (ties -> lowest axis), cut at the count median: the left child takes the  */
/* ceil(n/2) smallest particles in the order (coordinate, Morton rank).      */
/* Both children keep ascending Morton rank.  Node ids are DFS pre-order;    */
/* tree order lists the leaves left to right.                                */
/* Pinned by: the invariants test (partition, median, axis) and brute force. */
/* ------------------------------------------------------------------------ */
static uint64_t ordbits(double v)
{
    uint64_t b;
    memcpy(&b, &v, sizeof b);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

typedef struct {
    const double *x;
    const int32_t *rank; /* rank[i]: Morton rank of particle i */
    int32_t *order;      /* tree order under construction */
    int32_t *tmp;
    uint8_t *goleft;
    int32_t leaf_size;
    int32_t nn;
    int32_t *first, *count, *left, *right, *axis;
    int cmp_axis;
} tree_ctx;

static tree_ctx *g_sort_ctx; /* qsort has no user pointer in C11 */

static int cmp_axis_rank(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    uint64_t ka = ordbits(g_sort_ctx->x[3 * a + g_sort_ctx->cmp_axis]);
    uint64_t kb = ordbits(g_sort_ctx->x[3 * b + g_sort_ctx->cmp_axis]);
    if (ka != kb)
        return ka < kb ? -1 : 1;
    int32_t ra = g_sort_ctx->rank[a], rb = g_sort_ctx->rank[b];
    return ra < rb ? -1 : (ra > rb ? 1 : 0);
}

static int32_t build_node(tree_ctx *t, int32_t lo, int32_t n)
{
    int32_t id = t->nn++;
    t->first[id] = lo;
    t->count[id] = n;
    t->left[id] = t->right[id] = -1;
    t->axis[id] = -1;
    if (n <= t->leaf_size)
        return id;
    double mn[3], mx[3];
    for (int d = 0; d < 3; ++d)
        mn[d] = mx[d] = t->x[3 * t->order[lo] + d];
    for (int32_t k = 0; k < n; ++k)
        for (int d = 0; d < 3; ++d) {
            double v = t->x[3 * t->order[lo + k] + d];
            if (v < mn[d])
                mn[d] = v;
            if (v > mx[d])
                mx[d] = v;
        }
    int ax = 0;
    double best = mx[0] - mn[0];
    for (int d = 1; d < 3; ++d)
        if (mx[d] - mn[d] > best) {
            best = mx[d] - mn[d];
            ax = d;
        }
    t->axis[id] = ax;
    int32_t nl = (n + 1) / 2;
    /* rank the node's particles along the axis, mark the first ceil(n/2) */
    memcpy(t->tmp, t->order + lo, (size_t)n * sizeof(int32_t));
    g_sort_ctx = t;
    t->cmp_axis = ax;
    qsort(t->tmp, (size_t)n, sizeof(int32_t), cmp_axis_rank);
    for (int32_t k = 0; k < n; ++k)
        t->goleft[t->tmp[k]] = (uint8_t)(k < nl);
    /* stable partition of the rank-ordered node list */
    int32_t w = 0;
    for (int32_t k = 0; k < n; ++k)
        if (t->goleft[t->order[lo + k]])
            t->tmp[w++] = t->order[lo + k];
    for (int32_t k = 0; k < n; ++k)
        if (!t->goleft[t->order[lo + k]])
            t->tmp[w++] = t->order[lo + k];
    memcpy(t->order + lo, t->tmp, (size_t)n * sizeof(int32_t));
    int32_t l = build_node(t, lo, nl);
    int32_t r = build_node(t, lo + nl, n - nl);
    t->left[id] = l;
    t->right[id] = r;
    return id;
}

/* Node arrays must hold 2n entries.  perm[p] = caller index of the particle at
 * tree position p.  Returns the number of nodes. */
ORC_API int32_t orc_build_tree(int64_t n, const double *x, int32_t leaf_size, int32_t *perm,
                               int32_t *first, int32_t *count, int32_t *left, int32_t *right,
                               int32_t *axis)
{
    uint64_t *key = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    int32_t *rank = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    tree_ctx t;
    memset(&t, 0, sizeof t);
    t.x = x;
    t.rank = rank;
    t.order = perm;
    t.tmp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    t.goleft = (uint8_t *)malloc((size_t)n);
    t.leaf_size = leaf_size;
    t.first = first;
    t.count = count;
    t.left = left;
    t.right = right;
    t.axis = axis;
    orc_morton(n, x, key, perm);
    for (int64_t r = 0; r < n; ++r)
        rank[perm[r]] = (int32_t)r;
    build_node(&t, 0, (int32_t)n);
    free(key);
    free(rank);
    free(t.tmp);
    free(t.goleft);
    return t.nn;
}

/* ------------------------------------------------------------------------ */
/* kd-tree cut through the centre of mass (Sec. 2 as written: cells are cut  */
/* through their centres of mass, across the longest axis, until a cell      */
/* holds no more than leaf_size particles).                                  */
/* Reading: positions are quantised on a grid of 2^32 steps over the largest */
/* extent of the global bounding box, q = floor((x - lo) 2^32 / ext) clamped  */
/* to 2^32 - 1 (the Morton quantisation with 32 bits), and masses to weights  */
/* w = floor(m / m_max 2^24) clamped to [1, 2^24] (all w = 1 without masses). */
/* Per cell: the longest axis d of the quantised bounding box (ties -> lowest */
/* axis); the cut is the weighted centre of mass of q_d, taken exactly in     */
/* integer arithmetic: a particle goes left iff q_d sum(w) < sum(w q_d).  So  */
/* the partition does not depend on any summation order.  A cell whose        */
/* particles share one grid point along d (then along every axis) is halved   */
/* in tree order (left: the first ceil(n/2)).  Both children keep the        */
/* parent's order (ascending Morton rank at the root); node ids are DFS       */
/* pre-order.  Pinned by: an exact big-integer re-implementation on small     */
/* inputs and the cut lying at the FP64 centre of mass to within the grid.    */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t *q;  /* [3][n] quantised coordinates by caller index */
    uint32_t *w;  /* [n] weights by caller index */
    int64_t n;
    int32_t *order, *tmp;
    int32_t leaf_size, nn;
    int32_t *first, *count, *left, *right, *axis;
} comtree_ctx;

static int32_t build_com_node(comtree_ctx *t, int32_t lo, int32_t n)
{
    int32_t id = t->nn++;
    t->first[id] = lo;
    t->count[id] = n;
    t->left[id] = t->right[id] = -1;
    t->axis[id] = -1;
    if (n <= t->leaf_size)
        return id;
    uint32_t mn[3], mx[3];
    for (int d = 0; d < 3; ++d)
        mn[d] = mx[d] = t->q[d * t->n + t->order[lo]];
    for (int32_t k = 0; k < n; ++k)
        for (int d = 0; d < 3; ++d) {
            uint32_t v = t->q[d * t->n + t->order[lo + k]];
            if (v < mn[d])
                mn[d] = v;
            if (v > mx[d])
                mx[d] = v;
        }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
        if (mx[d] - mn[d] > mx[ax] - mn[ax])
            ax = d;
    t->axis[id] = ax;
    int32_t nl;
    if (mx[ax] == mn[ax]) {
        nl = (n + 1) / 2; /* one grid point: halve in tree order */
    } else {
        uint64_t sw = 0;
        unsigned __int128 swq = 0;
        for (int32_t k = 0; k < n; ++k) {
            int32_t i = t->order[lo + k];
            sw += t->w[i];
            swq += (unsigned __int128)t->w[i] * t->q[ax * t->n + i];
        }
        int32_t w = 0;
        for (int32_t k = 0; k < n; ++k) {
            int32_t i = t->order[lo + k];
            if ((unsigned __int128)t->q[ax * t->n + i] * sw < swq)
                t->tmp[w++] = i;
        }
        nl = w;
        for (int32_t k = 0; k < n; ++k) {
            int32_t i = t->order[lo + k];
            if (!((unsigned __int128)t->q[ax * t->n + i] * sw < swq))
                t->tmp[w++] = i;
        }
        memcpy(t->order + lo, t->tmp, (size_t)n * sizeof(int32_t));
    }
    int32_t l = build_com_node(t, lo, nl);
    int32_t r = build_com_node(t, lo + nl, n - nl);
    t->left[id] = l;
    t->right[id] = r;
    return id;
}

/* m may be NULL (equal weights).  Node arrays must hold 2n entries.
 * Returns the number of nodes. */
ORC_API int32_t orc_build_tree_com(int64_t n, const double *x, const double *m, int32_t leaf_size,
                                   int32_t *perm, int32_t *first, int32_t *count, int32_t *left,
                                   int32_t *right, int32_t *axis)
{
    comtree_ctx t;
    memset(&t, 0, sizeof t);
    t.n = n;
    t.q = (uint32_t *)malloc((size_t)(3 * n) * sizeof(uint32_t));
    t.w = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    t.tmp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    t.order = perm;
    t.leaf_size = leaf_size;
    t.first = first;
    t.count = count;
    t.left = left;
    t.right = right;
    t.axis = axis;
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d)
        lo[d] = hi[d] = x[d];
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            double v = x[3 * i + d];
            if (v < lo[d])
                lo[d] = v;
            if (v > hi[d])
                hi[d] = v;
        }
    double ext = 0.0;
    for (int d = 0; d < 3; ++d)
        if (hi[d] - lo[d] > ext)
            ext = hi[d] - lo[d];
    if (ext == 0.0)
        ext = 1.0;
    double scale = 4294967296.0 / ext;
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            double v = floor((x[3 * i + d] - lo[d]) * scale);
            t.q[d * n + i] = v >= 4294967295.0 ? 4294967295u : (uint32_t)v;
        }
    double mmax = 0.0;
    if (m)
        for (int64_t i = 0; i < n; ++i)
            if (m[i] > mmax)
                mmax = m[i];
    for (int64_t i = 0; i < n; ++i) {
        uint32_t w = 1;
        if (m && mmax > 0.0) {
            double v = floor(m[i] / mmax * 16777216.0);
            w = v >= 1.0 ? (v <= 16777216.0 ? (uint32_t)v : 16777216u) : 1u;
        }
        t.w[i] = w;
    }
    uint64_t *key = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    orc_morton(n, x, key, perm); /* root order: ascending Morton rank */
    build_com_node(&t, 0, (int32_t)n);
    free(key);
    free(t.q);
    free(t.w);
    free(t.tmp);
    return t.nn;
}

/* ------------------------------------------------------------------------ */
/* Cell properties (Sec. 2): mass M, centre of mass c, size s = radius of    */
/* the smallest sphere about c holding all the cell's particles, h_max, and  */
/* the quadrupole of eq. (7) about c (per-particle masses).                  */
/* Leaf: M and sum(m x) accumulated left to right in tree order, c = S / M.  */
/* Internal: M = M_L + M_R, c = (M_L c_L + M_R c_R) / M, and the quadrupole  */
/* by the parallel-axis shift of the children's (exact: the dipole about a   */
/* centre of mass vanishes).  s is the exact maximum over the particles.     */
/* Pinned by: direct P2M of every node from its particles (tests).           */
/* ------------------------------------------------------------------------ */
static void quad_add_point(double *Q, double w, const double *y)
{
    double y2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    Q[0] += w * (3.0 * y[0] * y[0] - y2);
    Q[1] += w * (3.0 * y[0] * y[1]);
    Q[2] += w * (3.0 * y[0] * y[2]);
    Q[3] += w * (3.0 * y[1] * y[1] - y2);
    Q[4] += w * (3.0 * y[1] * y[2]);
    Q[5] += w * (3.0 * y[2] * y[2] - y2);
}

ORC_API void orc_moments(int64_t n, const double *x, const double *m, const double *h,
                         const int32_t *perm, int32_t nnodes, const int32_t *first,
                         const int32_t *count, const int32_t *left, const int32_t *right,
                         double *M, double *c, double *s, double *hmax, double *Q)
{
    (void)n;
    /* children have larger pre-order ids than their parent */
    for (int32_t v = nnodes - 1; v >= 0; --v) {
        double *cv = c + 3 * v, *Qv = Q + 6 * v;
        for (int k = 0; k < 6; ++k)
            Qv[k] = 0.0;
        if (left[v] < 0) {
            double Mv = 0.0, S[3] = {0.0, 0.0, 0.0};
            for (int32_t k = 0; k < count[v]; ++k) {
                int32_t i = perm[first[v] + k];
                Mv += m[i];
                for (int d = 0; d < 3; ++d)
                    S[d] += m[i] * x[3 * i + d];
            }
            M[v] = Mv;
            for (int d = 0; d < 3; ++d)
                cv[d] = S[d] / Mv;
            for (int32_t k = 0; k < count[v]; ++k) {
                int32_t i = perm[first[v] + k];
                double y[3] = {x[3 * i] - cv[0], x[3 * i + 1] - cv[1], x[3 * i + 2] - cv[2]};
                quad_add_point(Qv, m[i], y);
            }
        } else {
            int32_t l = left[v], r = right[v];
            double Mv = M[l] + M[r];
            M[v] = Mv;
            for (int d = 0; d < 3; ++d)
                cv[d] = (M[l] * c[3 * l + d] + M[r] * c[3 * r + d]) / Mv;
            int32_t ch[2] = {l, r};
            for (int k2 = 0; k2 < 2; ++k2) {
                int32_t u = ch[k2];
                double dd[3] = {c[3 * u] - cv[0], c[3 * u + 1] - cv[1], c[3 * u + 2] - cv[2]};
                for (int k = 0; k < 6; ++k)
                    Qv[k] += Q[6 * u + k];
                quad_add_point(Qv, M[u], dd);
            }
        }
        double s2 = 0.0, hm = 0.0;
        for (int32_t k = 0; k < count[v]; ++k) {
            int32_t i = perm[first[v] + k];
            double dx = x[3 * i] - cv[0], dy = x[3 * i + 1] - cv[1], dz = x[3 * i + 2] - cv[2];
            double d2 = (dx * dx + dy * dy) + dz * dz;
            if (d2 > s2)
                s2 = d2;
            if (h[i] > hm)
                hm = h[i];
        }
        s[v] = sqrt(s2);
        hmax[v] = hm;
    }
}

/* Quadrupole of an explicit particle set about its own centre of mass
 * (eq. (7)); used by the tests for pins on hand-built cells. */
ORC_API void orc_p2m(int64_t n, const double *x, const double *m, double *M, double *c, double *Q)
{
    double Mv = 0.0, S[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        Mv += m[i];
        for (int d = 0; d < 3; ++d)
            S[d] += m[i] * x[3 * i + d];
    }
    *M = Mv;
    for (int d = 0; d < 3; ++d)
        c[d] = S[d] / Mv;
    for (int k = 0; k < 6; ++k)
        Q[k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double y[3] = {x[3 * i] - c[0], x[3 * i + 1] - c[1], x[3 * i + 2] - c[2]};
        quad_add_point(Q, m[i], y);
    }
}

/* ------------------------------------------------------------------------ */
/* Interaction criteria (Sec. 2).  r = c_sink - c_source.                    */
/*   eq. (4), tree opening:  theta^2 < (s_source / r)^2, written             */
/*            s_source * s_source > theta^2 * r^2;                           */
/*   eq. (5), smoothing-sphere overlap:                                      */
/*            r^2 < (s_a + s_b + R_kern * max(h_a, h_b))^2.                  */
/* A pair meeting either is short-range (opened).                            */
/* ------------------------------------------------------------------------ */
static int opened_p(const double *ca, double sa, double ha, const double *cb, double sb,
                    double hb, double theta2, double r_kern)
{
    double dx = ca[0] - cb[0], dy = ca[1] - cb[1], dz = ca[2] - cb[2];
    double r2 = (dx * dx + dy * dy) + dz * dz;
    int open4 = sb * sb > theta2 * r2;
    double t = (sa + sb) + r_kern * (ha > hb ? ha : hb);
    int open5 = r2 < t * t;
    return open4 || open5;
}

/* Mutual criterion for the symmetric walk: well separated iff
 * (s_a + s_b)^2 <= theta^2 r^2 and eq. (5) fails. */
static int separated_m(const double *ca, double sa, double ha, const double *cb, double sb,
                       double hb, double theta2, double r_kern)
{
    double dx = ca[0] - cb[0], dy = ca[1] - cb[1], dz = ca[2] - cb[2];
    double r2 = (dx * dx + dy * dy) + dz * dz;
    double ss = sa + sb;
    int ok4 = theta2 * r2 >= ss * ss;
    double t = ss + r_kern * (ha > hb ? ha : hb);
    int ok5 = r2 >= t * t;
    return ok4 && ok5;
}

typedef struct {
    int32_t nnodes;
    const int32_t *left, *right;
    const double *c, *s, *hmax;
    double theta2, r_kern;
    int32_t *far_cnt, *near_cnt; /* running fill positions per sink node */
    const int32_t *far_off, *near_off;
    int32_t *far_src, *near_src; /* NULL in counting mode */
} walk_ctx;

static void emit(int32_t *cnt, const int32_t *off, int32_t *dst, int32_t sink, int32_t src)
{
    if (dst)
        dst[off[sink] + cnt[sink]] = src;
    cnt[sink]++;
}

/* Leaf <- cell walk (Sec. 4: partners are sought for leaf cells only, with
 * the one-sided criterion (4)).  DFS from the root, children pushed right
 * then left, so every list comes out in ascending tree order. */
static void walk_leaf(walk_ctx *w, int32_t a)
{
    int32_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    const double *ca = w->c + 3 * a;
    while (sp > 0) {
        int32_t b = stack[--sp];
        if (!opened_p(ca, w->s[a], w->hmax[a], w->c + 3 * b, w->s[b], w->hmax[b], w->theta2,
                      w->r_kern))
            emit(w->far_cnt, w->far_off, w->far_src, a, b);
        else if (w->left[b] < 0)
            emit(w->near_cnt, w->near_off, w->near_src, a, b);
        else {
            stack[sp++] = w->right[b];
            stack[sp++] = w->left[b];
        }
    }
}

/* Mutual walk (Sec. 7 recommendation): every accepted pair is used in both
 * directions, and sinks may be any cell. */
static void walk_pair(walk_ctx *w, int32_t a, int32_t b)
{
    if (separated_m(w->c + 3 * a, w->s[a], w->hmax[a], w->c + 3 * b, w->s[b], w->hmax[b],
                    w->theta2, w->r_kern)) {
        emit(w->far_cnt, w->far_off, w->far_src, a, b);
        emit(w->far_cnt, w->far_off, w->far_src, b, a);
        return;
    }
    int la = w->left[a] < 0, lb = w->left[b] < 0;
    if (la && lb) {
        emit(w->near_cnt, w->near_off, w->near_src, a, b);
        emit(w->near_cnt, w->near_off, w->near_src, b, a);
        return;
    }
    int split_a = lb || (!la && w->s[a] >= w->s[b]);
    if (split_a) {
        walk_pair(w, w->left[a], b);
        walk_pair(w, w->right[a], b);
    } else {
        walk_pair(w, a, w->left[b]);
        walk_pair(w, a, w->right[b]);
    }
}

static void walk_self(walk_ctx *w, int32_t a)
{
    if (w->left[a] < 0) {
        emit(w->near_cnt, w->near_off, w->near_src, a, a);
        return;
    }
    walk_self(w, w->left[a]);
    walk_self(w, w->right[a]);
    walk_pair(w, w->left[a], w->right[a]);
}

/* Lists are CSR over sink node ids: entries of sink v are
 * src[off[v] .. off[v+1]).  Call once with far_src == near_src == NULL to get
 * the offsets and totals, then again with buffers of those sizes.
 * policy 0 = leaf <- cell walk, 1 = mutual walk. */
ORC_API void orc_walk(int32_t policy, int32_t nnodes, const int32_t *left, const int32_t *right,
                      const double *c, const double *s, const double *hmax, double theta,
                      double r_kern, int32_t *far_off, int32_t *far_src, int32_t *near_off,
                      int32_t *near_src, int64_t *totals)
{
    walk_ctx w;
    w.nnodes = nnodes;
    w.left = left;
    w.right = right;
    w.c = c;
    w.s = s;
    w.hmax = hmax;
    w.theta2 = theta * theta;
    w.r_kern = r_kern;
    w.far_cnt = (int32_t *)calloc((size_t)nnodes, sizeof(int32_t));
    w.near_cnt = (int32_t *)calloc((size_t)nnodes, sizeof(int32_t));
    w.far_off = far_off;
    w.near_off = near_off;
    w.far_src = far_src;
    w.near_src = near_src;
    if (policy == 0) {
        for (int32_t a = 0; a < nnodes; ++a)
            if (left[a] < 0)
                walk_leaf(&w, a);
    } else {
        walk_self(&w, 0);
    }
    if (!far_src) {
        far_off[0] = near_off[0] = 0;
        for (int32_t v = 0; v < nnodes; ++v) {
            far_off[v + 1] = far_off[v] + w.far_cnt[v];
            near_off[v + 1] = near_off[v] + w.near_cnt[v];
        }
    }
    totals[0] = far_off[nnodes];
    totals[1] = near_off[nnodes];
    free(w.far_cnt);
    free(w.near_cnt);
}

/* ------------------------------------------------------------------------ */
/* Far field.                                                                */
/* Symmetric-tensor storage: vectors x,y,z; rank 2 (xx,xy,xz,yy,yz,zz);      */
/* rank 3 (xxx,xxy,xxz,xyy,xyz,xzz,yyy,yyz,yzz,zzz).  A local expansion is   */
/* L[19] = (L1[3], L2[6], L3[10]) with L1 = a(r), L2 = grad a, L3 = grad     */
/* grad a, so that eq. (8) reads a(y) = L1 + L2 y + 1/2 L3 : y y.            */
/* ------------------------------------------------------------------------ */
static int sym2(int i, int j)
{
    static const int t[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    return t[i][j];
}

static int sym3(int i, int j, int k)
{
    /* sort the three indices, then look up */
    int a = i, b = j, cc = k, tmp;
    if (a > b) { tmp = a; a = b; b = tmp; }
    if (b > cc) { tmp = b; b = cc; cc = tmp; }
    if (a > b) { tmp = a; a = b; b = tmp; }
    static const int t[3][3][3] = {
        {{0, 1, 2}, {-1, 3, 4}, {-1, -1, 5}},
        {{-1, -1, -1}, {-1, 6, 7}, {-1, -1, 8}},
        {{-1, -1, -1}, {-1, -1, -1}, {-1, -1, 9}},
    };
    return t[a][b][cc];
}

static double kd(int i, int j) { return i == j ? 1.0 : 0.0; }

/* M2L: the field of a source cell (mass M, quadrupole Q about its centre of
 * mass) at offset r = c_sink - c_source, to second order in the sink offset.
 * L1 is eq. (6) as printed:
 *   a_i = -M r_i / r^3 + (1/r^4) (rhat_k Q_ik - 5/2 rhat_i rhat_j rhat_k Q_jk).
 * L2 and L3 are its first and second r-derivatives in closed form, written
 * with g_n = (-1)^n (2n-1)!! r^-(2n+1) (the n-th radial factor of the
 * derivatives of 1/r, so that d/dr_i g_n = g_{n+1} r_i), q = Q r and
 * qq = r.Q.r:
 *   L2_ij  = M (g2 r_i r_j + g1 d_ij) + 1/6 [g4 qq r_i r_j + g3 qq d_ij
 *            + 2 g3 (r_i q_j + q_i r_j) + 2 g2 Q_ij]
 *   L3_ijk = M (g3 r_i r_j r_k + g2 (d_ij r_k + d_ik r_j + d_jk r_i))
 *            + 1/6 [g5 qq r_i r_j r_k + g4 qq (d_ij r_k + d_ik r_j + d_jk r_i)
 *            + 2 g4 (r_i r_j q_k + r_i r_k q_j + r_j r_k q_i)
 *            + 2 g3 (d_ij q_k + d_ik q_j + d_jk q_i)
 *            + 2 g3 (r_i Q_jk + r_j Q_ik + r_k Q_ij)]
 * Pinned by: symbolic differentiation of eq. (6), finite differences, the
 * direct field of explicit particle clusters, the pair-force closed form and
 * the three-cell expansion of Sec. 4 (eq. (31)).
 *
 * form = 1 selects the expansion of eqs. (25)-(26) with p = 3 and the
 * octupoles dropped: every term x^n y^m with |n| + |m| <= 2 is kept, so with
 * the dipole zero about the centre of mass the quadrupole enters L1 only
 * (L1 is eq. (6) again) and L2, L3 are the derivatives of the monopole field:
 *   L2_ij  = M (g2 r_i r_j + g1 d_ij)
 *   L3_ijk = M (g3 r_i r_j r_k + g2 (d_ij r_k + d_ik r_j + d_jk r_i)),
 * whose highest power of 1/r is 4 (against 6 for form 0).  Pinned by:
 * symbolic derivatives of the point-mass field, the truncated double Taylor
 * series of eqs. (25)-(26) built from explicit particle clusters, the
 * difference to form 0 being the (n, m) = (1, 2), (2, 2) terms of Sec. 4, and
 * the per-pair third law. */
ORC_API void orc_m2l(int32_t form, const double *rv, double M, const double *Q, double *L)
{
    double r2 = rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
    double r = sqrt(r2);
    double rh[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
    double Qf[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Qf[i][j] = Q[sym2(i, j)];
    /* L1: eq. (6) */
    double rQr = 0.0;
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k)
            rQr += rh[j] * rh[k] * Qf[j][k];
    double r4 = r2 * r2;
    for (int i = 0; i < 3; ++i) {
        double rq = 0.0;
        for (int k = 0; k < 3; ++k)
            rq += rh[k] * Qf[i][k];
        L[i] = -M / r2 * rh[i] + (rq - 2.5 * rh[i] * rQr) / r4;
    }
    /* radial factors */
    double u = 1.0 / r, u2 = u * u;
    double g1 = -u * u2;
    double g2 = -3.0 * g1 * u2;
    double g3 = -5.0 * g2 * u2;
    double g4 = -7.0 * g3 * u2;
    double g5 = -9.0 * g4 * u2;
    double q[3];
    for (int i = 0; i < 3; ++i) {
        q[i] = 0.0;
        for (int j = 0; j < 3; ++j)
            q[i] += Qf[i][j] * rv[j];
    }
    double qq = q[0] * rv[0] + q[1] * rv[1] + q[2] * rv[2];
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            double v = M * (g2 * rv[i] * rv[j] + g1 * kd(i, j));
            if (form == 0)
                v += (g4 * qq * rv[i] * rv[j] + g3 * qq * kd(i, j) +
                      2.0 * g3 * (rv[i] * q[j] + q[i] * rv[j]) + 2.0 * g2 * Qf[i][j]) /
                     6.0;
            L[3 + sym2(i, j)] = v;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j)
            for (int k = j; k < 3; ++k) {
                double rrr = rv[i] * rv[j] * rv[k];
                double dr = kd(i, j) * rv[k] + kd(i, k) * rv[j] + kd(j, k) * rv[i];
                double rrq = rv[i] * rv[j] * q[k] + rv[i] * rv[k] * q[j] + rv[j] * rv[k] * q[i];
                double dq = kd(i, j) * q[k] + kd(i, k) * q[j] + kd(j, k) * q[i];
                double rQ = rv[i] * Qf[j][k] + rv[j] * Qf[i][k] + rv[k] * Qf[i][j];
                double v = M * (g3 * rrr + g2 * dr);
                if (form == 0)
                    v += (g5 * qq * rrr + g4 * qq * dr + 2.0 * g4 * rrq + 2.0 * g3 * dq +
                          2.0 * g3 * rQ) /
                         6.0;
                L[9 + sym3(i, j, k)] = v;
            }
}

/* L2P, eq. (8): a_i(y) = L1_i + L2_ij y_j + 1/2 L3_ijk y_j y_k. */
ORC_API void orc_l2p(const double *L, const double *y, double *a)
{
    for (int i = 0; i < 3; ++i) {
        double v = L[i];
        for (int j = 0; j < 3; ++j)
            v += L[3 + sym2(i, j)] * y[j];
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                v += 0.5 * L[9 + sym3(i, j, k)] * y[j] * y[k];
        a[i] = v;
    }
}

/* L2L: the quadratic polynomial of eq. (8) re-expanded about a centre moved by
 * delta (exact for a quadratic):
 *   L1' = L1 + L2 delta + 1/2 L3 : delta delta,  L2' = L2 + L3 delta,  L3' = L3.
 * out may alias nothing.  Pinned by: L2P(shift(L), y - delta) = L2P(L, y). */
ORC_API void orc_l2l(const double *L, const double *delta, double *out)
{
    orc_l2p(L, delta, out);
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            double v = L[3 + sym2(i, j)];
            for (int k = 0; k < 3; ++k)
                v += L[9 + sym3(i, j, k)] * delta[k];
            out[3 + sym2(i, j)] = v;
        }
    for (int k = 0; k < 10; ++k)
        out[9 + k] = L[9 + k];
}

/* Local expansions of every sink node: M2L (expansion form `form`) over its
 * far list, in list order; with the mutual walk also the L2L pass from each
 * node into its children, parents first (pre-order).  L is nnodes x 19, zero
 * for nodes without a far field. */
/* M2L sum of one sink cell v over its far list src[0 .. nsrc), in list order. */
static void sink_far(int32_t form, int32_t v, const double *M, const double *c, const double *Q,
                     const int32_t *src, int64_t nsrc, double *Lv)
{
    double t[19];
    for (int k = 0; k < 19; ++k)
        Lv[k] = 0.0;
    for (int64_t e = 0; e < nsrc; ++e) {
        int32_t b = src[e];
        double rv[3] = {c[3 * v] - c[3 * b], c[3 * v + 1] - c[3 * b + 1],
                        c[3 * v + 2] - c[3 * b + 2]};
        orc_m2l(form, rv, M[b], Q + 6 * b, t);
        for (int k = 0; k < 19; ++k)
            Lv[k] += t[k];
    }
}

ORC_API void orc_far_field(int32_t policy, int32_t form, int32_t nnodes, const int32_t *left,
                           const int32_t *right, const double *M, const double *c,
                           const double *Q, const int32_t *far_off, const int32_t *far_src,
                           double *L)
{
    double t[19];
    for (int32_t v = 0; v < nnodes; ++v)
        sink_far(form, v, M, c, Q, far_src + far_off[v], far_off[v + 1] - far_off[v],
                 L + 19 * v);
    if (policy == 1) {
        for (int32_t v = 0; v < nnodes; ++v) {
            if (left[v] < 0)
                continue;
            int32_t ch[2] = {left[v], right[v]};
            for (int k2 = 0; k2 < 2; ++k2) {
                int32_t u = ch[k2];
                double dl[3] = {c[3 * u] - c[3 * v], c[3 * u + 1] - c[3 * v + 1],
                                c[3 * u + 2] - c[3 * v + 2]};
                orc_l2l(L + 19 * v, dl, t);
                for (int k = 0; k < 19; ++k)
                    L[19 * u + k] += t[k];
            }
        }
    }
}

/* L2P plus the near field for every particle, written in caller order:
 *   a_i = G (L2P(L_leaf, x_i - c_leaf)
 *            - sum_{b in near(leaf)} sum_{j in b, j != i} m_j G_ij (x_i - x_j)). */
/* L2P and the near field for the particles of leaf v, near list
 * src[0 .. nsrc), written in caller order:
 *   a_i = G (L2P(L_v, x_i - c_v) - sum_{b} sum_{j in b, j != i} m_j G_ij (x_i - x_j)). */
static void leaf_near_l2p(const double *x, const double *m, const double *h,
                          const int32_t *perm, const int32_t *first, const int32_t *count,
                          const double *c, int32_t v, const double *Lv, const int32_t *src,
                          int64_t nsrc, double G, double *a)
{
    for (int32_t k = 0; k < count[v]; ++k) {
        int32_t i = perm[first[v] + k];
        double y[3] = {x[3 * i] - c[3 * v], x[3 * i + 1] - c[3 * v + 1],
                       x[3 * i + 2] - c[3 * v + 2]};
        double af[3];
        orc_l2p(Lv, y, af);
        double an[3] = {0.0, 0.0, 0.0};
        for (int64_t e = 0; e < nsrc; ++e) {
            int32_t b = src[e];
            for (int32_t kk = 0; kk < count[b]; ++kk) {
                int32_t j = perm[first[b] + kk];
                if (j == i)
                    continue;
                double dx = x[3 * i] - x[3 * j], dy = x[3 * i + 1] - x[3 * j + 1],
                       dz = x[3 * i + 2] - x[3 * j + 2];
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                double f = m[j] * pair_g(r, h[i], h[j]);
                an[0] -= f * dx;
                an[1] -= f * dy;
                an[2] -= f * dz;
            }
        }
        for (int d = 0; d < 3; ++d)
            a[3 * i + d] = G * (af[d] + an[d]);
    }
}

ORC_API void orc_near_and_l2p(int64_t n, const double *x, const double *m, const double *h,
                              const int32_t *perm, int32_t nnodes, const int32_t *first,
                              const int32_t *count, const int32_t *left, const double *c,
                              const double *L, const int32_t *near_off, const int32_t *near_src,
                              double G, double *a)
{
    (void)n;
    for (int32_t v = 0; v < nnodes; ++v)
        if (left[v] < 0)
            leaf_near_l2p(x, m, h, perm, first, count, c, v, L + 19 * v,
                          near_src + near_off[v], near_off[v + 1] - near_off[v], G, a);
}

/* The leaf <- cell FMM (policy 0) for a chosen set of sink leaves only: for
 * each listed leaf, its own walk (the same DFS and criteria (4), (5) as
 * orc_walk), its M2L sum (eq. (6), orc_far_field's order) and L2P plus the
 * near field for its particles (orc_near_and_l2p's order).  The accelerations
 * of those particles are therefore identical to the full evaluation's; the
 * other rows of a are not written.  Lets a test or a timing run reach single
 * leaves of trees too large for the full O(N) list storage.
 *   leaves  node ids of leaf cells, nsel of them;
 *   counts  NULL or int64[2 nsel]: far and near list lengths per listed leaf.
 * Re-entrant: calls on disjoint leaf sets may run on several threads. */
ORC_API void orc_fmm_leaves(int64_t n, const double *x, const double *m, const double *h,
                            const int32_t *perm, int32_t nnodes, const int32_t *first,
                            const int32_t *count, const int32_t *left, const int32_t *right,
                            const double *M, const double *c, const double *s,
                            const double *hmax, const double *Q, double theta, double r_kern,
                            double G, int32_t form, int64_t nsel, const int32_t *leaves,
                            double *a, int64_t *counts)
{
    (void)n;
    walk_ctx w;
    w.nnodes = nnodes;
    w.left = left;
    w.right = right;
    w.c = c;
    w.s = s;
    w.hmax = hmax;
    w.theta2 = theta * theta;
    w.r_kern = r_kern;
    w.far_cnt = (int32_t *)calloc((size_t)nnodes, sizeof(int32_t));
    w.near_cnt = (int32_t *)calloc((size_t)nnodes, sizeof(int32_t));
    /* one sink at a time: its lists start at offset 0 */
    int32_t *zero_off = (int32_t *)calloc((size_t)nnodes + 1, sizeof(int32_t));
    w.far_off = zero_off;
    w.near_off = zero_off;
    int64_t cap_f = 0, cap_n = 0;
    int32_t *fs = NULL, *ns = NULL;
    double Lv[19];
    for (int64_t q = 0; q < nsel; ++q) {
        int32_t v = leaves[q];
        w.far_cnt[v] = w.near_cnt[v] = 0;
        w.far_src = w.near_src = NULL;
        walk_leaf(&w, v);
        int64_t nf = w.far_cnt[v], nn = w.near_cnt[v];
        if (nf > cap_f) {
            free(fs);
            cap_f = nf;
            fs = (int32_t *)malloc((size_t)cap_f * sizeof(int32_t));
        }
        if (nn > cap_n) {
            free(ns);
            cap_n = nn;
            ns = (int32_t *)malloc((size_t)cap_n * sizeof(int32_t));
        }
        w.far_cnt[v] = w.near_cnt[v] = 0;
        w.far_src = fs;
        w.near_src = ns;
        walk_leaf(&w, v);
        sink_far(form, v, M, c, Q, fs, nf, Lv);
        leaf_near_l2p(x, m, h, perm, first, count, c, v, Lv, ns, nn, G, a);
        if (counts) {
            counts[2 * q] = nf;
            counts[2 * q + 1] = nn;
        }
        w.far_cnt[v] = w.near_cnt[v] = 0;
    }
    free(fs);
    free(ns);
    free(zero_off);
    free(w.far_cnt);
    free(w.near_cnt);
}

/* ------------------------------------------------------------------------ */
/* Momentum diagnostics (Secs. 5-6): total force, its modulus sum, the       */
/* ratio |sum F| / sum |F|, total mass, centre of mass, momentum and angular */
/* momentum, accumulated in index order.  v may be NULL (P = L = 0).         */
/* out[16] = sumF[3], sumAbsF, ratio, mass, xcom[3], P[3], L[3], 0.          */
/* ------------------------------------------------------------------------ */
ORC_API void orc_stats(int64_t n, const double *x, const double *v, const double *m,
                       const double *a, double *out)
{
    double F[3] = {0, 0, 0}, Fa = 0.0, Mt = 0.0, X[3] = {0, 0, 0}, P[3] = {0, 0, 0},
           Lm[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        const double *ai = a + 3 * i, *xi = x + 3 * i;
        for (int d = 0; d < 3; ++d)
            F[d] += m[i] * ai[d];
        Fa += m[i] * sqrt(ai[0] * ai[0] + ai[1] * ai[1] + ai[2] * ai[2]);
        Mt += m[i];
        for (int d = 0; d < 3; ++d)
            X[d] += m[i] * xi[d];
        if (v) {
            const double *vi = v + 3 * i;
            for (int d = 0; d < 3; ++d)
                P[d] += m[i] * vi[d];
            Lm[0] += m[i] * (xi[1] * vi[2] - xi[2] * vi[1]);
            Lm[1] += m[i] * (xi[2] * vi[0] - xi[0] * vi[2]);
            Lm[2] += m[i] * (xi[0] * vi[1] - xi[1] * vi[0]);
        }
    }
    for (int d = 0; d < 3; ++d)
        out[d] = F[d];
    out[3] = Fa;
    out[4] = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]) / Fa;
    out[5] = Mt;
    for (int d = 0; d < 3; ++d) {
        out[6 + d] = X[d] / Mt;
        out[9 + d] = P[d];
        out[12 + d] = Lm[d];
    }
    out[15] = 0.0;
}

/* ------------------------------------------------------------------------ */
/* Asymmetric cell pairs and the total-force estimates of Sec. 4 (eq. (33))  */
/* and Sec. 6 (eq. (46)).                                                    */
/*                                                                           */
/* A pair "a receives the field of b" (b in the far list of sink a) is       */
/* asymmetric when the reverse pair (a in the far list of b) is absent.  For  */
/* a cell v with at least two leaves, v1 is its lightest leaf (smallest mass; */
/* among equal masses the one farthest from c_v, the "lightest distant        */
/* cell"), l_v = |c_v1 - c_v|, and                                           */
/*   T(v) = M_v1 l_v^3 / (M_v - M_v1) (1 - M_v1 / (M_v - M_v1));             */
/* T(v) = 0 for a leaf (zero size).  Per asymmetric pair, eq. (33) adds      */
/*   4 M_a M_b / r^5 (T(a) + T(b)),   r = |c_a - c_b|,                       */
/* and eq. (46), with N_v the number of leaves of v and m_leaf the mean leaf  */
/* mass, adds                                                                */
/*   4 m_leaf^2 N_a N_b / r^5 (U(a) + U(b)),                                 */
/*   U(v) = s_v^3 (N_v - 2) / (N_v - 1)^2 for N_v >= 2, 0 for a leaf.        */
/* out[0] = eq. (33) sum, out[1] = eq. (46) sum, out[2] = number of          */
/* asymmetric pairs, out[3] = those of them with a cell of >= 2 leaves.      */
/* Sums in sink order, then list order.  Pinned by: the two-leaf super-cell   */
/* of Sec. 4 (eq. (33) reduces to eq. (32)), equal leaf masses (eq. (33)     */
/* with l = s equals eq. (46)), brute-force lightest leaves and reverse-pair  */
/* checks on small trees, and zero for the mutual walk's lists.              */
/* ------------------------------------------------------------------------ */
static void asym_leaves(const int32_t *left, const int32_t *right, int32_t v, int32_t *out,
                        int32_t *k)
{
    if (left[v] < 0) {
        out[(*k)++] = v;
        return;
    }
    asym_leaves(left, right, left[v], out, k);
    asym_leaves(left, right, right[v], out, k);
}

static int asym_has(const int32_t *far_off, const int32_t *far_src, int32_t a, int32_t b)
{
    for (int32_t e = far_off[a]; e < far_off[a + 1]; ++e)
        if (far_src[e] == b)
            return 1;
    return 0;
}

ORC_API void orc_asym_estimate(int32_t nnodes, const int32_t *left, const int32_t *right,
                               const double *M, const double *c, const double *s,
                               const int32_t *far_off, const int32_t *far_src, double m_leaf,
                               double *out)
{
    double *T = (double *)calloc((size_t)nnodes, sizeof(double));
    double *U = (double *)calloc((size_t)nnodes, sizeof(double));
    double *N = (double *)calloc((size_t)nnodes, sizeof(double));
    int32_t *lv = (int32_t *)malloc((size_t)nnodes * sizeof(int32_t));
    for (int32_t v = 0; v < nnodes; ++v) {
        int32_t k = 0;
        asym_leaves(left, right, v, lv, &k);
        N[v] = (double)k;
        if (k < 2)
            continue;
        double m1 = M[lv[0]];
        for (int32_t j = 1; j < k; ++j)
            if (M[lv[j]] < m1)
                m1 = M[lv[j]];
        double d2 = -1.0;
        for (int32_t j = 0; j < k; ++j) {
            int32_t u = lv[j];
            if (M[u] != m1)
                continue;
            double dx = c[3 * u] - c[3 * v], dy = c[3 * u + 1] - c[3 * v + 1],
                   dz = c[3 * u + 2] - c[3 * v + 2];
            double e = dx * dx + dy * dy + dz * dz;
            if (e > d2)
                d2 = e;
        }
        double l = sqrt(d2);
        double rest = M[v] - m1;
        T[v] = m1 * l * l * l / rest * (1.0 - m1 / rest);
        U[v] = s[v] * s[v] * s[v] * (N[v] - 2.0) / ((N[v] - 1.0) * (N[v] - 1.0));
    }
    double f33 = 0.0, f46 = 0.0, nasym = 0.0, nsuper = 0.0;
    for (int32_t a = 0; a < nnodes; ++a)
        for (int32_t e = far_off[a]; e < far_off[a + 1]; ++e) {
            int32_t b = far_src[e];
            if (asym_has(far_off, far_src, b, a))
                continue;
            nasym += 1.0;
            if (N[a] >= 2.0 || N[b] >= 2.0)
                nsuper += 1.0;
            double dx = c[3 * a] - c[3 * b], dy = c[3 * a + 1] - c[3 * b + 1],
                   dz = c[3 * a + 2] - c[3 * b + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            double r5 = r2 * r2 * sqrt(r2);
            f33 += 4.0 * M[a] * M[b] / r5 * (T[a] + T[b]);
            f46 += 4.0 * m_leaf * m_leaf * N[a] * N[b] / r5 * (U[a] + U[b]);
        }
    out[0] = f33;
    out[1] = f46;
    out[2] = nasym;
    out[3] = nsuper;
    free(T);
    free(U);
    free(N);
    free(lv);
}
