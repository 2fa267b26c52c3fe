/*
 * fmm_mi355.h -- C ABI of the MI355X (gfx950) kd-tree FMM gravity library.
 *
 * The library evaluates self-gravity accelerations of N particles the way the
 * paper analyses it (Potashov & Yudin, arXiv:2502.01496, Sec. 2):
 *
 *     a_grav = a_short + a_long                                   eq. (3)
 *
 * Particles are grouped in a kd-tree; for every sink leaf cell the tree is
 * walked with the opening criterion eq. (4) and the smoothing-sphere overlap
 * criterion eq. (5).  Opened leaf cells are summed directly with the softened
 * pair kernel (Sec. 3, eqs. (12)-(15)); accepted cells act through their mass
 * and quadrupole (eq. (7)), the field eq. (6) and its Taylor evaluation at each
 * particle, eq. (8).
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers (HIP device memory), contiguous, in
 *     the caller's particle order: positions and accelerations are row-major
 *     [n][3], masses and smoothing lengths [n].  Exceptions say "host".
 *   - The caller owns its inputs and outputs; they must stay valid until the
 *     work enqueued on `stream` has completed.  The library owns the tree and
 *     its workspace until fmm_tree_free.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *     enqueues work on it, except where a call says it synchronises.
 *   - Arguments are validated on the host before any launch; a bad argument
 *     returns FMM_ERR_INVALID and enqueues nothing.  Data-dependent errors
 *     (non-finite coordinates, non-positive masses or smoothing lengths) are
 *     detected on the device and reported by the next call that synchronises
 *     (fmm_forces), which then returns FMM_ERR_INVALID.
 *   - A HIP runtime failure returns FMM_ERR_HIP.  fmm_last_error() returns the
 *     message of the last failure on the calling thread.
 *   - A tree is not thread-safe; distinct trees may be used concurrently on
 *     distinct streams.
 */
#ifndef FMM_MI355_H
#define FMM_MI355_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fmm_status {
    FMM_OK = 0,
    FMM_ERR_INVALID = -1,  /* bad argument or bad input data */
    FMM_ERR_ALLOC = -2,    /* device allocation failed */
    FMM_ERR_CAPACITY = -3, /* a size limit of the library was exceeded */
    FMM_ERR_HIP = -4,      /* HIP runtime error */
    FMM_ERR_STATE = -5     /* call out of order or unknown handle */
} fmm_status;

/* Arithmetic of the far and near field (M2L, L2P, P2P).  FMM_FP32 keeps the
 * tree build, the moments, the walk and the momentum reductions in FP64 and
 * runs M2L/L2P/P2P in FP32 with FP32 accumulation on leaf-relative offsets;
 * the output accelerations are then float[n][3]. */
enum { FMM_FP64 = 0, FMM_FP32 = 1 };

/* Interaction-list policy.
 * FMM_WALK_PHANTOM: partners are sought for leaf cells only, each with the
 *   one-sided criterion (4) (Sec. 4); pairs "leaf <- super-cell" are never
 *   formed in reverse.
 * FMM_WALK_MUTUAL: symmetric dual-tree walk (the remedy of Sec. 7): every
 *   accepted cell pair acts in both directions, cells of any level may be
 *   sinks, and local expansions are passed down the tree (L2L). */
enum { FMM_WALK_PHANTOM = 0, FMM_WALK_MUTUAL = 1 };

/* Expansion form of the far field (M2L), Sec. 4.
 * FMM_EXPANSION_PHANTOM: eq. (6) for the cell field and its first two
 *   r-derivatives for the sink offset (eq. (8)); the quadrupole enters every
 *   order, the highest power of 1/r is 6.
 * FMM_EXPANSION_DEHNEN: the series (25)-(26) with p = 3 and octupoles dropped:
 *   terms are kept while the combined order of the source and sink offsets is
 *   at most 2, so the quadrupole enters the field itself only and the two
 *   derivative orders come from the monopole; the highest power of 1/r is 4.
 * Both forms conserve momentum for every mutual cell pair; neither does with
 * the leaf <- cell lists. */
enum { FMM_EXPANSION_PHANTOM = 0, FMM_EXPANSION_DEHNEN = 1 };

/* Tree shape (Sec. 2).
 * FMM_TREE_MEDIAN: each cell is cut across its longest axis at the count
 *   median (the reading documented at fmm_build_tree); the shape depends on
 *   n and leaf_size only.
 * FMM_TREE_COM: each cell is cut across its longest axis through its centre
 *   of mass, as Sec. 2 describes (PHANTOM: leaf_size 10).  Positions are
 *   quantised on a grid of 2^32 steps over the largest extent of the global
 *   bounding box, q = floor((x - lo) 2^32 / ext), masses to weights
 *   w = floor(m / m_max 2^24) in [1, 2^24] (all 1 without masses); the axis
 *   is the longest of the quantised bounding box (ties -> lowest) and a
 *   particle goes left iff q_d sum(w) < sum(w q_d), exactly, in integer
 *   arithmetic.  A cell whose particles share one grid point is halved in
 *   tree order.  Children keep ascending Morton rank.  The shape depends on
 *   the data: node-sized buffers are allocated for the largest possible tree
 *   (2n - 1 nodes), and the build synchronises the stream once per level. */
enum { FMM_TREE_MEDIAN = 0, FMM_TREE_COM = 1 };

/* fmm_forces flags */
enum {
    FMM_REWALK = 1,  /* rebuild the interaction lists even if present */
    /* Prepare the tree for fmm_forces_vjp without evaluating the forces: the
     * walk (when due) and, for an FP64 tree, the far-field expansions the
     * reverse pass reads; the near field is not evaluated and a is neither
     * read nor written (it may be NULL).  For callers that need the reverse
     * pass at positions whose forces they already have, such as the
     * backward sweep through checkpointed time steps. */
    FMM_VJP_ONLY = 2
};

/* Device allocator hooks (fmm_params.dev_alloc / dev_free): every byte of
 * device memory a tree holds is taken with dev_alloc(bytes, alloc_ctx) and
 * returned with dev_free(ptr, alloc_ctx); NULL hooks use hipMalloc/hipFree.
 * dev_alloc returns NULL when it cannot serve the request, and the library
 * call then fails with FMM_ERR_ALLOC.  Pinned host staging buffers (a few
 * bytes per tree) are not device memory and do not go through the hooks. */
typedef void *(*fmm_alloc_fn)(size_t bytes, void *ctx);
typedef void (*fmm_free_fn)(void *ptr, void *ctx);

typedef struct fmm_params {
    double theta;      /* opening parameter of eq. (4), 0 <= theta <= 1 (default 0.5) */
    double r_kern;     /* kernel support radius in units of h, eq. (5); M4: 2 (default) */
    double G;          /* gravitational constant; G = 1 in the units of eq. (1) (default) */
    int32_t leaf_size; /* a cell with at most this many particles is a leaf; 1..64 (default 8) */
    int32_t walk;      /* FMM_WALK_* (default PHANTOM) */
    int32_t precision; /* FMM_FP64 or FMM_FP32 (default FP64) */
    int32_t expansion; /* FMM_EXPANSION_* (default PHANTOM) */
    int32_t tree;      /* FMM_TREE_* (default MEDIAN) */
    int32_t reserved;  /* must be 0 */
    /* Interaction-list capacity per sink list, in entries.  0 (default): the
     * per-sink slots grow on demand (a walk that overflows them is redone
     * with larger slots).  > 0: every sink list holds at most this many
     * cells; a walk that needs more returns FMM_ERR_CAPACITY and leaves the
     * tree without lists (its moments stay valid). */
    int64_t list_capacity;
    /* Upper bound on the device memory the tree may hold, in bytes (the
     * figure fmm_tree_device_bytes reports).  0 (default): no bound.  A call
     * whose allocation would exceed it returns FMM_ERR_ALLOC; memory the
     * failing call had taken for the same purpose is returned first, so the
     * tree holds what it held before the call. */
    int64_t device_bytes_limit;
    fmm_alloc_fn dev_alloc; /* NULL: hipMalloc (default) */
    fmm_free_fn dev_free;   /* NULL: hipFree; must be set iff dev_alloc is */
    void *alloc_ctx;        /* passed to both hooks */
} fmm_params;

/* Momentum diagnostics of Secs. 5-6, accumulated in FP64.
 * F_i = m_i a_i.  ratio = |sumF| / sumAbsF. */
typedef struct fmm_stats {
    double sumF[3];
    double sumAbsF;
    double ratio;
    double mass;
    double xcom[3];
    double P[3]; /* sum m v (0 if v == NULL) */
    double L[3]; /* sum m x cross v (0 if v == NULL) */
    double pad;
} fmm_stats;

typedef struct fmm_tree fmm_tree; /* opaque, library-owned */

/* Fill *p with the defaults listed in fmm_params. */
void fmm_default_params(fmm_params *p);

/* Build the kd-tree of x (Sec. 2: cells are cut along their longest axis until
 * a cell holds at most leaf_size particles).  Reading of the cut: the longest
 * axis of the cell's particle bounding box (ties -> lowest axis) is split at
 * the count median; the left child takes the ceil(n/2) particles that come
 * first in the order (coordinate, Morton rank), where the Morton rank orders
 * the particles by a 63-bit Morton key of their position quantised to 2^21
 * per axis in the global bounding box (ties by caller index).  Both children
 * keep ascending Morton rank.
 *   x      device, double[n][3]; read during the call's stream work only.
 *   n      1 <= n <= 2^31 - 1.
 *   p      host; copied.
 *   *tree  NULL: a new tree is allocated and returned; otherwise the given
 *          tree (built earlier with the same n and leaf_size) is rebuilt in
 *          place, reusing its memory.  Rebuilding invalidates the moments and
 *          the interaction lists.
 * A reused tree keeps its allocator: dev_alloc, dev_free, alloc_ctx and
 * device_bytes_limit must equal those it was created with.
 * Errors: FMM_ERR_INVALID (n, p out of range, NULL pointers, n/leaf_size or
 * the allocator differing from the reused tree's), FMM_ERR_ALLOC (nothing is
 * kept: a failed new tree returns all it took), FMM_ERR_HIP. */
fmm_status fmm_build_tree(const double *x, int64_t n, const fmm_params *p, void *stream,
                          fmm_tree **tree);

/* fmm_build_tree with particle masses, which the centre-of-mass cut
 * (FMM_TREE_COM) weighs the positions with:
 *   m  device, double[n], or NULL (equal weights); read during the call's
 *      stream work only; unused by FMM_TREE_MEDIAN.
 * A reused tree must also keep its tree shape (FMM_ERR_INVALID otherwise). */
fmm_status fmm_build_tree_weighted(const double *x, const double *m, int64_t n,
                                   const fmm_params *p, void *stream, fmm_tree **tree);

/* Cell properties for the current tree membership (Sec. 2): mass M, centre of
 * mass c, size s (radius of the smallest sphere about c that holds all the
 * cell's particles), the largest smoothing length h_max, and the quadrupole
 * of eq. (7) about c; leaves from their particles, parents by exact shifts of
 * their children (the dipole about a centre of mass vanishes).
 *   x, m, h  device, double[n][3], double[n], double[n]; m > 0, h > 0.
 * The positions may differ from those the tree was built on (the tree
 * membership is then held fixed).  The interaction lists are kept: the next
 * fmm_forces reuses them unless it is given FMM_REWALK (this is how forces
 * with a frozen tree and frozen lists are evaluated); fmm_build_tree discards
 * them. */
fmm_status fmm_moments(fmm_tree *tree, const double *x, const double *m, const double *h,
                       void *stream);

/* Accelerations a_grav = a_short + a_long (eq. (3)) for every particle.
 * Walks the tree (building the interaction lists) when there are none or
 * flags & FMM_REWALK, then evaluates M2L (eq. (6)), L2L (mutual walk only),
 * L2P (eq. (8)) and the softened near field, and writes
 *   a  device, double[n][3] (FMM_FP64) or float[n][3] (FMM_FP32), caller order;
 *      not used with FMM_VJP_ONLY (may then be NULL).
 *   flags  FMM_REWALK and / or FMM_VJP_ONLY; other bits: FMM_ERR_INVALID.
 * Synchronises `stream` once: to size the interaction lists when it walks,
 * else to read the data checks of the last fmm_moments.
 * Errors: FMM_ERR_STATE (no moments), FMM_ERR_INVALID (bad input data found
 * on the device by the last fmm_moments: non-finite positions, masses or
 * smoothing lengths not positive and finite; the lists are then dropped),
 * FMM_ERR_CAPACITY (a sink list needs more than params.list_capacity
 * entries), FMM_ERR_ALLOC, FMM_ERR_HIP. */
fmm_status fmm_forces(fmm_tree *tree, void *a, int32_t flags, void *stream);

/* Vector-Jacobian product of the accelerations of the last fmm_forces call
 * with respect to the positions and masses, with the tree membership and the
 * interaction lists held fixed (the moments do depend on x and m), for the
 * lists of either walk (after a mutual walk the reverse pass also runs the
 * L2L chain backwards).  The reverse pass is FP64 for both precisions:
 *   a_bar  device, [n][3] cotangent of a (double or float per precision);
 *   x_bar  device, [n][3] output, same precision;
 *   m_bar  device, [n] output, same precision.
 * Synchronises `stream` on the first call after a walk (sizes the transposed
 * lists).  Errors: FMM_ERR_STATE (no prior fmm_forces on this tree state),
 * FMM_ERR_ALLOC, FMM_ERR_HIP. */
fmm_status fmm_forces_vjp(fmm_tree *tree, const void *a_bar, void *x_bar, void *m_bar,
                          void *stream);

/* Census of the asymmetric cell pairs of the current interaction lists and the
 * total-force estimates built on them: Sec. 4, eq. (33), and Sec. 6, eq. (46).
 * A pair (sink a receives the field of source b) is asymmetric when the lists
 * lack the reverse pair.  For a cell v with N_v >= 2 leaves, v1 is its lightest
 * leaf (ties: the one farthest from c_v), l = |c_v1 - c_v|,
 *   T(v) = M_v1 l^3 / (M_v - M_v1) (1 - M_v1 / (M_v - M_v1)),
 *   U(v) = s_v^3 (N_v - 2) / (N_v - 1)^2   (T = U = 0 for a leaf);
 * per asymmetric pair eq. (33) adds 4 M_a M_b (T(a) + T(b)) / r^5 and
 * eq. (46) adds 4 m_leaf^2 N_a N_b (U(a) + U(b)) / r^5, r = |c_a - c_b|.
 *   m_leaf  the leaf mass M_l of eq. (46); <= 0 selects the mean leaf mass
 *           (total mass / number of leaves);
 *   out     HOST double[4]: eq. (33) sum, eq. (46) sum, number of asymmetric
 *           pairs, number of those with a cell of >= 2 leaves; written before
 *           the call returns (synchronises stream).
 * Works on the lists of either walk (the mutual walk's are symmetric by
 * construction: all four outputs 0).  With the leaf <- cell lists it builds
 * the transposed far lists (kept until the next walk, shared with the VJP).
 * Sums in a fixed order (bitwise reproducible).
 * Errors: FMM_ERR_STATE (no lists for the current moments), FMM_ERR_INVALID,
 * FMM_ERR_HIP. */
fmm_status fmm_asymmetry_estimate(fmm_tree *tree, double m_leaf, double *out, void *stream);

/* Momentum diagnostics (Secs. 5-6) in FP64 with a fixed reduction order
 * (bitwise reproducible run to run):
 *   x  device double[n][3];  v  device double[n][3] or NULL;  m  device double[n];
 *   a  device [n][3], double if a_precision == FMM_FP64, float if FMM_FP32;
 *   out  HOST pointer, written before the call returns (synchronises stream). */
fmm_status fmm_momentum_stats(const double *x, const double *v, const double *m, const void *a,
                              int32_t a_precision, int64_t n, fmm_stats *out, void *stream);

/* The same statistics written to DEVICE memory without waiting (Secs. 5-6),
 * for callers that gather them every step and read them once at the end.
 *   out  device pointer to one fmm_stats (16 doubles, caller-owned), written
 *        when the stream reaches the call; the values equal those of
 *        fmm_momentum_stats bit for bit.
 * The partial sums use a per-device library buffer: calls on one stream run
 * in order, calls on different streams of one device must not overlap.
 * Errors: FMM_ERR_INVALID for NULL x, m, a, out, n < 1 or an unknown
 * precision (nothing is launched); FMM_ERR_HIP for a failed launch. */
fmm_status fmm_momentum_stats_async(const double *x, const double *v, const double *m,
                                    const void *a, int32_t a_precision, int64_t n,
                                    fmm_stats *out, void *stream);

/* fmm_momentum_stats_async for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same 16 values, bit for bit, written to DEVICE memory
 * without waiting; the partial sums live in a fixed 64.1 KiB array of the
 * library's code object on each device (held until the process ends), so
 * the call allocates nothing, neither on its first call nor later.
 *   out  device pointer to one fmm_stats (caller-owned).
 * Calls that overlap on one device (other streams, other threads) race for
 * that array; calls on one stream run in order.
 * Errors: FMM_ERR_INVALID (NULL x, m, a or out, n < 1, unknown precision;
 * nothing is launched), FMM_ERR_CAPACITY (n above 2^31 - 1), FMM_ERR_HIP. */
fmm_status fmm_momentum_stats_noalloc(const double *x, const double *v, const double *m,
                                      const void *a, int32_t a_precision, int64_t n,
                                      fmm_stats *out, void *stream);

/* Leapfrog update for kick-drift-kick time stepping with fixed dt:
 *   v += kick * a;  then  x += drift * v      (elementwise, FP64 state)
 * A KDK step is fmm_kick_drift(kick = dt/2, drift = dt), new forces, then
 * fmm_kick_drift(kick = dt/2, drift = 0); consecutive half kicks may be merged.
 *   x, v  device double[n][3], updated in place;
 *   a     device [n][3], double if a_precision == FMM_FP64, float if FMM_FP32. */
fmm_status fmm_kick_drift(double *x, double *v, const void *a, int32_t a_precision, int64_t n,
                          double kick, double drift, void *stream);

/* Release a tree and its device memory (synchronises the device first).
 * NULL is a no-op. */
void fmm_tree_free(fmm_tree *tree);

/* Message of the last failure on the calling thread ("" if none). */
const char *fmm_last_error(void);

/* Sizes of a tree, host int64_t[8]: n, nodes, leaves, depth, far entries,
 * near entries, list sinks, has_lists. */
fmm_status fmm_tree_info(const fmm_tree *tree, int64_t *info);

/* The parameters a tree was last built with and its particle count, to host
 * memory (*p, *n; either may be NULL).  Never touches the device: callers use
 * it to check the shapes and precision of their buffers before a call. */
fmm_status fmm_tree_params(const fmm_tree *tree, fmm_params *p, int64_t *n);

/* Device memory the library holds for a tree (its topology, workspace,
 * interaction lists and VJP workspace), in bytes, to *bytes (host).  Memory
 * the caller owns (inputs, outputs) is not included. */
fmm_status fmm_tree_device_bytes(const fmm_tree *tree, int64_t *bytes);

/* Copy the tree, cell records and interaction lists to HOST buffers (test and
 * bring-up aid; synchronises).  Any pointer may be NULL to skip it.
 *   perm      int32[n]      tree position -> caller index
 *   first, count, left, right, axis   int32[nodes] (left = right = -1, axis = -1 for leaves)
 *   rec       double[nodes][12]: M, cx, cy, cz, s, h_max, Qxx, Qxy, Qxz, Qyy, Qyz, Qzz
 *   far_off   int64[nodes+1], far_src int32[far entries]  (CSR over sink node ids)
 *   near_off  int64[nodes+1], near_src int32[near entries]
 *   local     double[nodes][19]: local expansions L1(3), L2(6), L3(10) of the
 *             leaves in the last FP64 fmm_forces, about their centres of mass,
 *             with every far contribution (for the mutual walk also those
 *             passed down from the ancestors by L2L); zero for internal nodes.
 * Far lists are CSR over sink node ids: leaves only for the leaf <- cell walk,
 * every node for the mutual walk; near lists have leaf sinks only. */
fmm_status fmm_debug_export(const fmm_tree *tree, int32_t *perm, int32_t *first, int32_t *count,
                            int32_t *left, int32_t *right, int32_t *axis, double *rec,
                            int64_t *far_off, int32_t *far_src, int64_t *near_off,
                            int32_t *near_src, double *local);

/* Replace a tree's particle order, cell records and interaction lists with
 * given ones (test and bring-up aid, the inverse of fmm_debug_export), so that
 * the far field (M2L, eq. (6)), its Taylor evaluation (L2P, eq. (8)) and the
 * near field (Sec. 3, eqs. (12)-(15)) can be checked on structures that did
 * not come from this library's build, moments and walk.  Synchronises.
 *   tree         built with FMM_TREE_MEDIAN and FMM_WALK_PHANTOM;
 *   x, m, h      DEVICE, caller order, as for fmm_moments (the data checks of
 *                fmm_moments apply and are reported by the next fmm_forces);
 *   perm         HOST int32[n], tree position -> caller index (a permutation);
 *   first, count, left, right   HOST int32[nodes]: must equal the tree's own
 *                topology (FMM_ERR_INVALID otherwise; for a median-split tree
 *                the shape depends on n and leaf_size only);
 *   rec          HOST double[nodes][12], the layout of fmm_debug_export;
 *   far_off, near_off   HOST int64[nodes+1], far_src, near_src HOST int32:
 *                CSR over sink node ids, sinks are leaves; near entries are
 *                leaves, far entries any cell (may be NULL when empty).
 * After the call the tree holds moments and lists: fmm_forces without
 * FMM_REWALK evaluates M2L, L2P and the near field on exactly these, with
 * the tree's params (G, precision, expansion form); fmm_moments or a walk
 * replaces them again, and the imported perm stays until the next build.
 * Errors: FMM_ERR_STATE (no tree), FMM_ERR_INVALID (shape, permutation or
 * list checks fail; nothing is changed), FMM_ERR_CAPACITY (a list longer than
 * params.list_capacity), FMM_ERR_ALLOC, FMM_ERR_HIP. */
fmm_status fmm_debug_import(fmm_tree *tree, const double *x, const double *m, const double *h,
                            const int32_t *perm, const int32_t *first, const int32_t *count,
                            const int32_t *left, const int32_t *right, const double *rec,
                            const int64_t *far_off, const int32_t *far_src,
                            const int64_t *near_off, const int32_t *near_src, void *stream);

/* Stage timing.  fmm_set_timing(tree, 1) starts recording a pair of HIP
 * events around each stage on the caller's stream (no added synchronisation;
 * it also clears the accumulated times); fmm_stage_times (synchronises on the
 * last events) returns the MEAN device time per call since then, in
 * milliseconds, host double[8]: build, moments, walk (count + scan + fill),
 * far field (M2L, L2L), near field (P2P + L2P), vjp, stats (unused), and the
 * sum of the first seven.  The far and near stages are one kernel launch
 * each, so their means are per-launch kernel durations. */
fmm_status fmm_set_timing(fmm_tree *tree, int32_t on);
fmm_status fmm_stage_times(const fmm_tree *tree, double *ms);

#ifdef __cplusplus
}
#endif
#endif /* FMM_MI355_H */
