// Internal declarations of the gfx950 kd-tree FMM library: the tree object,
// device helpers shared by the kernel files, and the host-side launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fmm_mi355.h"

namespace fmm {

// Nodes with at most SUBTREE_MAX particles are split entirely inside one
// workgroup's LDS (all their descendants in one launch).
constexpr int SUBTREE_MAX = 2048;
constexpr int SUBTREE_MAXSEG = SUBTREE_MAX / 2;
constexpr int SUBTREE_THREADS = 1024;
constexpr int SM_MAXNODES = 1024;  // nodes of a subtree whose moments are combined in LDS
constexpr int SM_MAXL = 16;        // internal levels of such a subtree
// Positions handled by one workgroup in the per-level partition kernels.
constexpr int LVL_CHUNK = 2048;
constexpr int LVL_THREADS = 256;
// Radix sort: 16 waves x 4 rounds x 64 lanes = 4096 keys per tile, 8-bit digits.
constexpr int RS_THREADS = 1024;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_ROUNDS = 4;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;
constexpr int RS_SCAN_THREADS = 256;
constexpr int RS_PASSES = 8;
constexpr int MAX_LEAF = 64;
constexpr int COM_CHUNK = 4096;  // particles per chunk of the centre-of-mass build
constexpr int COM_MAX_DEPTH = 64; // deepest centre-of-mass tree accepted (walk stacks)
constexpr int NREC = 8;   // doubles per node record (geometry / quadrupole)
// Geometry record (recA) of a node: centre of mass 0..2, mass 3, size s 4,
// h_max 5; slot 6 holds the child ids (left in the low 32 bits, right in the
// high 32, -1 for a leaf) and slot 7 the leaf index (-1 for an internal
// node), so that a walk reads one 64-byte record per visited cell.
constexpr int REC_KIDS = 6, REC_LEAF = 7;
constexpr int NLOC = 20;  // doubles per local expansion (19 used)
constexpr int LLEAF = 24;  // doubles per leaf record of the reverse pass's M2L^T source side

// ------------------------------------------------------------------ device
__device__ __forceinline__ uint64_t ordbits(double v)
{
    uint64_t b = (uint64_t)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ double from_ordbits(uint64_t k)
{
    uint64_t b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// 1/sqrt(x) for finite x > 0: hardware estimate plus one second-order
// correction, y' = y + y e (1/2 + 3/8 e) with e = 1 - x y^2.
__device__ __forceinline__ double rsqrt_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// L2P, eq. (8)
template <typename T>
__device__ __forceinline__ void l2p(const T *L, T y0, T y1, T y2, T &a0, T &a1, T &a2)
{
    const T h = T(0.5);
    a0 = L[0] + L[3] * y0 + L[4] * y1 + L[5] * y2 +
         h * (L[9] * y0 * y0 + L[12] * y1 * y1 + L[14] * y2 * y2) +
         (L[10] * y0 * y1 + L[11] * y0 * y2 + L[13] * y1 * y2);
    a1 = L[1] + L[4] * y0 + L[6] * y1 + L[7] * y2 +
         h * (L[10] * y0 * y0 + L[15] * y1 * y1 + L[17] * y2 * y2) +
         (L[12] * y0 * y1 + L[13] * y0 * y2 + L[16] * y1 * y2);
    a2 = L[2] + L[5] * y0 + L[7] * y1 + L[8] * y2 +
         h * (L[11] * y0 * y0 + L[16] * y1 * y1 + L[18] * y2 * y2) +
         (L[13] * y0 * y1 + L[14] * y0 * y2 + L[17] * y1 * y2);
}

// L2L: re-expansion of the quadratic field about a point shifted by d (exact):
//   L1' = L1 + L2 d + 1/2 L3 : d d,  L2' = L2 + L3 d,  L3' = L3.
template <typename T>
__device__ __forceinline__ void l2l_shift(T *L, T d0, T d1, T d2)
{
    T a0, a1, a2;
    l2p<T>(L, d0, d1, d2, a0, a1, a2);
    const T s3 = L[3] + L[9] * d0 + L[10] * d1 + L[11] * d2;
    const T s4 = L[4] + L[10] * d0 + L[12] * d1 + L[13] * d2;
    const T s5 = L[5] + L[11] * d0 + L[13] * d1 + L[14] * d2;
    const T s6 = L[6] + L[12] * d0 + L[15] * d1 + L[16] * d2;
    const T s7 = L[7] + L[13] * d0 + L[16] * d1 + L[17] * d2;
    const T s8 = L[8] + L[14] * d0 + L[17] * d1 + L[18] * d2;
    L[0] = a0;
    L[1] = a1;
    L[2] = a2;
    L[3] = s3;
    L[4] = s4;
    L[5] = s5;
    L[6] = s6;
    L[7] = s7;
    L[8] = s8;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  This bijection of [0, nblocks) gives XCD x a contiguous range of
// logical block indices, so neighbouring leaves (which share most of their
// interaction partners) are processed behind the same L2.
__device__ __forceinline__ int xcd_block(int b, int nblocks)
{
    const int q = nblocks >> 3, r = nblocks & 7;
    const int x = b & 7, k = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Position of piece k of leaf lf in a piece list: the extra pieces (k >= 1)
// of split leaves come first, leaf by leaf (extra = off[nleaves] - nleaves of
// them, off the exclusive scan of the pieces per leaf), then the first piece
// of every leaf at extra + lf.  A leaf with one piece finishes in the kernel
// that evaluates it; the folds visit the extra entries only.
__device__ __forceinline__ int64_t piece_pos(const int64_t *__restrict__ off, int64_t extra,
                                             int lf, int k)
{
    return k == 0 ? extra + lf : off[lf] - lf + (k - 1);
}

// ------------------------------------------------------------------ host
// Data-independent shape of the median-split tree: with ceil(n/2) / floor(n/2)
// children, node sizes (and so first/count/left/right) depend on n and the
// leaf size only.  Computed once per (n, leaf_size) on the host.
struct Topology {
    int64_t n = 0;
    int leaf_size = 0;
    int nnodes = 0, nleaves = 0, depth = 0;
    // capacities of the node- and leaf-sized buffers: the sizes themselves for
    // the median tree; 2n - 1 and n for the centre-of-mass tree, whose shape
    // depends on the data
    int64_t node_cap = 0, leaf_cap = 0;
    bool com = false;
    int nbig = 0;                      // nodes of at least 64 particles
    std::vector<int32_t> first, count, left, right, parent, level, leaf_node, node_leaf;
    // level-synchronous partition of the nodes larger than SUBTREE_MAX
    int nlevels_up = 0;
    int max_lvl_blocks = 0;
    std::vector<int32_t> lvl_blk_off;  // nlevels_up + 1
    std::vector<int32_t> blk_node, blk_start, blk_end, blk_first;
    std::vector<int32_t> sub_root;     // roots of the LDS subtrees
    // internal nodes grouped by level (for the bottom-up moment pass)
    std::vector<int32_t> lvl_int_off;  // depth + 1
    std::vector<int32_t> int_nodes;
    std::vector<int32_t> big_nodes;    // nodes of at least 64 particles
    // moments of the LDS subtrees in one launch (sub_moments): per subtree
    // its leaf range, its internal nodes as (node, right child) grouped by
    // level, deepest first (group k of subtree s starts at
    // sm_lvl[s * (SM_MAXL + 1) + k]), and the nodes above the subtrees by
    // level; sub_moments is false when a subtree has more than SM_MAXNODES
    // nodes
    bool sub_moments = false;
    std::vector<int32_t> sm_leaf, sm_lvl, sm_nodes;
    std::vector<int32_t> top_lvl_off;  // depth + 1
    std::vector<int32_t> top_nodes;
    // the cells above the subtrees combined by one workgroup through LDS
    // (when the subtree roots and those cells fit SM_MAXNODES slots): slots
    // [0, nsub) hold the subtree roots, then the cells above them deepest
    // level first; per such cell (node, left slot, right slot), grouped by
    // level (top_grp offsets)
    bool top_fused = false;
    std::vector<int32_t> top_slot_node;  // node id per slot
    std::vector<int32_t> top_task;       // (node, left slot, right slot) per cell
    std::vector<int32_t> top_grp;        // group offsets into top_task / 3
};

void build_topology(int64_t n, int leaf_size, Topology &t);

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Tree;
// Device memory of a tree.  Every allocation and release of a tree's device
// memory goes through these two: they apply the caller's allocator hooks and
// byte limit (fmm_params) and keep the count fmm_tree_device_bytes reports.
// tree_malloc returns hipErrorOutOfMemory when the limit would be exceeded
// or a hook returns NULL; tree_free(nullptr) is a no-op.
hipError_t tree_malloc(Tree &t, void **p, size_t bytes);
void tree_free(Tree &t, void *p);

// Mutual walk state: pair frontier, far / near pair buffers (sorted by
// (sink, source) keys), CSR ranges of the far lists, and the counters
//   cnt[MW_NFAR], cnt[MW_NNEAR]  pairs appended,
//   cnt[MW_FLAGS]                overflow bits (1 frontier, 2 far, 4 near),
//   cnt[MW_MAXNEAR]              largest near count of a leaf,
//   cnt[MW_IT + k]               size of the frontier at recursion level k.
constexpr int MW_NFAR = 0, MW_NNEAR = 1, MW_FLAGS = 2, MW_MAXNEAR = 3, MW_IT = 8, MW_CNT = 160;
struct MutualLists {
    int2 *task[2] = {nullptr, nullptr};
    uint64_t *fkeys[2] = {nullptr, nullptr};
    uint64_t *nkeys[2] = {nullptr, nullptr};
    int64_t cap_task = 0, cap_far = 0, cap_near = 0;
    const uint64_t *far_sorted = nullptr;  // fkeys[0] or fkeys[1] after the sort
    int64_t *fstart = nullptr, *fend = nullptr;  // per node (fend = fstart + nnodes)
    int64_t *nstart = nullptr;                   // per leaf
    uint32_t *hist = nullptr, *tot = nullptr;
    unsigned long long *cnt = nullptr;           // device, MW_CNT
    unsigned long long *h_cnt = nullptr;         // pinned host mirror
    double *Lown = nullptr;                      // NLOC per node: M2L sums only
    float *Lownf = nullptr;
    DevBuf b_task, b_fkeys, b_nkeys, b_hist;
    std::vector<DevBuf> owned;                   // fixed-size parts
    int64_t n_far = 0, n_near = 0;
};

struct Tree {
    uint32_t magic = 0;
    fmm_params p{};
    Topology topo;
    std::vector<DevBuf> owned;
    int64_t held_bytes = 0;         // device memory held (tree_malloc - tree_free)
    std::vector<std::pair<void *, size_t>> held;  // every live allocation

    // topology on the device
    int32_t *first = nullptr, *count = nullptr, *left = nullptr, *right = nullptr;
    int32_t *parent = nullptr, *level = nullptr, *leaf_node = nullptr, *node_leaf = nullptr;
    int32_t *blk_node = nullptr, *blk_start = nullptr, *blk_end = nullptr, *blk_first = nullptr;
    int32_t *sub_root = nullptr, *axis = nullptr, *int_nodes = nullptr;
    int32_t *sm_leaf = nullptr, *sm_lvl = nullptr, *sm_nodes = nullptr, *top_nodes = nullptr;
    int32_t *top_slot_node = nullptr, *top_task = nullptr, *top_grp = nullptr;

    // build workspace
    uint64_t *keys0 = nullptr, *keys1 = nullptr;  // 3n each (batched sorts)
    uint32_t *vals0 = nullptr, *vals1 = nullptr;
    uint32_t *rs_hist = nullptr, *rs_tot = nullptr;
    uint32_t *run_cnt = nullptr;  // long runs of equal high key halves: count, list
    int64_t *run_list = nullptr;
    int32_t *r2o = nullptr;       // Morton rank -> caller index
    double *xr = nullptr;         // coordinates by Morton rank, 3 x n SoA
    uint32_t *lists = nullptr;    // 2 buffers x 4 lists x n
    uint8_t *side = nullptr;      // 4 x n: side of each list entry at the current level,
                                  // then n: the sides by Morton rank
    int32_t *lvl_cnt = nullptr;
    uint64_t *bbox = nullptr;     // ordered bits: min xyz, max xyz
    // device error flags: err[0] from the build (bit 0 non-finite x, bit 3
    // internal), err[1] from the last moments call (bit 0 x, bit 1 m, bit 2 h;
    // cleared at the start of every moments call)
    uint32_t *err = nullptr;
    int32_t *perm = nullptr;      // tree position -> caller index

    // particles in tree order
    double4 *pm = nullptr;        // x, y, z, m
    double *hs = nullptr;         // h
    double4 *ph = nullptr;        // 1/h, 1/h^3, 4 h^2, h
    float4 *pf = nullptr;         // FP32 form: offset from the leaf centre of mass, m
    float4 *pfh = nullptr;        // FP32 form: 1/h, 1/h^3, 4 h^2, 0

    // nodes
    double *recA = nullptr;       // per node: cx, cy, cz, M, s, hmax, 0, 0
    double *recQ = nullptr;       // per node: Qxx, Qxy, Qxz, Qyy, Qyz, Qzz, 0, 0
    float *recF = nullptr;        // per node FP32 mirror: M, Q[6], 0
    uint64_t *s2bits = nullptr;
    uint64_t *s2part = nullptr;   // depth x ceil(n/64) per-wavefront maxima
    int32_t *big_nodes = nullptr;
    int32_t *upcnt = nullptr;

    // interaction lists: fixed-capacity slots per sink leaf
    //   far:  far_src[leaf * cap_far + k],  k < far_cnt[leaf]
    //   near: near_src[leaf * cap_near + k], k < near_cnt[leaf]
    int32_t *far_src = nullptr, *near_src = nullptr;
    int64_t cap_far = 0, cap_near = 0;
    DevBuf far_buf, near_buf;
    int32_t *far_cnt = nullptr, *near_cnt = nullptr;
    int32_t *walk_flags = nullptr;  // device: max far, max near, stack overflow, queued groups
    int32_t *walk_heavy = nullptr;  // groups of four leaves queued for the workgroup walk
    int32_t *h_flags = nullptr;     // pinned host mirror of walk_flags + error bits
    int wide_stack_limit = 1 << 30; // test hook: FMM_MI355_WIDE_STACK lowers it
    int walk_budget = 256;          // steps of a group walk before it is queued (FMM_MI355_WALK_BUDGET)
    int nsinks = 0;
    int64_t n_far = 0, n_near = 0;
    double *L = nullptr;          // local expansions, NLOC per node
    float *Lf = nullptr;          // FP32 form, NLOC per node

    // reductions
    double *red = nullptr;
    double *h_red = nullptr;

    // VJP workspace (allocated on first use, grown on demand)
    struct Transposed {
        int64_t *off = nullptr;   // nnodes + 1, CSR over target node ids
        uint32_t *src = nullptr;  // sink node ids, ascending per target
        int64_t npairs = 0;
        int64_t src_cap = 0;      // entries src holds
    } farT, nearT;
    bool has_transposed = false;
    std::vector<DevBuf> vjp_owned;
    int64_t vjp_pair_cap = 0;
    uint32_t *vk0 = nullptr, *vk1 = nullptr;
    uint32_t *vv0 = nullptr, *vv1 = nullptr, *vhist = nullptr, *vtot = nullptr;
    int64_t *pair_off = nullptr;   // nleaves + 1 offsets of the compacted pairs
    int64_t *vscan = nullptr;
    double *abt = nullptr;         // G * abar, tree order, 3 per particle
    double *xbt = nullptr;         // xbar accumulator, tree order, 3 per particle
    double *mbt = nullptr;         // mbar accumulator, tree order
    double *Lbar = nullptr;        // NLOC per node
    double *Lleaf = nullptr;       // LLEAF per leaf: Lbar[19], leaf centre[3], 0, 0
    double *nadj = nullptr;        // 16 per node: cbar_sink[3], cbar_src[3], Mbar, Qbar[6]
    int64_t *h_pairs = nullptr;    // pinned: pair totals, piece total
    // pieces of the transposed far lists (source side of M2L^T)
    int32_t *pcnt = nullptr;       // pieces per cell
    int64_t *poff = nullptr;       // nnodes + 1 piece offsets
    int64_t *pscan = nullptr;      // scan workspace
    int32_t *pnode = nullptr;      // cell of each piece
    double *ppart = nullptr;       // 10 sums per piece
    int64_t npieces = 0, piece_cap = 0;

    MutualLists mw;
    int64_t mw_init_cap = 0;        // test hook: FMM_MI355_MW_CAP sets small first capacities
    bool morton_full = false;       // Morton keys sorted on all eight digits

    // centre-of-mass tree build (FMM_TREE_COM)
    struct ComWork {
        uint32_t *q = nullptr, *q_tmp = nullptr;   // [4][n]: q0, q1, q2, w in tree order
        int32_t *perm_tmp = nullptr;
        int32_t *node = nullptr;   // [8][node_cap] BFS: first, count, parent, level, axis,
                                   // left, right, internal rank
        int32_t *ren = nullptr;    // [4][node_cap] subtree nodes, leaves, pre-order id, leaf offset
        int32_t *act[2] = {nullptr, nullptr};     // active BFS ids per level
        int64_t *act_choff[2] = {nullptr, nullptr};
        int32_t *chk[2] = {nullptr, nullptr};     // [3][cap_c]: active index, start, end
        uint64_t *cpart = nullptr;                 // 16 per chunk
        int32_t *cleft = nullptr;                  // left count per chunk, then its base
        int32_t *cbase = nullptr;                  // right base per chunk
        uint64_t *split = nullptr;                 // 4 per active node: axis|flag, sw, swq lo, hi
        int32_t *nl = nullptr;                     // left count per active node
        int32_t *big = nullptr;                    // BFS ids of nodes of >= 64 particles
        int64_t *ctl = nullptr, *h_ctl = nullptr;  // next level's A, C; big count; m_max bits
        int64_t cap_a = 0, cap_c = 0;
        std::vector<int32_t> lev_off;              // BFS id range per level
    } cw;
    int64_t s2part_depth = 0;       // levels the s^2 partial buffer holds
    int64_t slots_nl = 0;           // leaves the list slots were allocated for

    // asymmetric-pair census: T, U, N per node, then partial sums per sink
    double *asym = nullptr;
    double *h_asym = nullptr;       // pinned, 4

    // Long interaction lists are split into pieces of bounded work, one
    // wavefront (near field) or 16-lane group (far field) each, with partial
    // sums folded per leaf in piece order; used when the last walk found a
    // list longer than one piece (trees with a few very long lists).
    struct Pieces {
        int32_t *np = nullptr;    // pieces per leaf
        int64_t *off = nullptr;   // nleaves + 1, first piece of each leaf
        int64_t *tsum = nullptr;  // scan workspace
        int2 *list = nullptr;     // (leaf, piece index) per piece
        void *part = nullptr;     // partial sums per piece
        int64_t cap = 0;          // pieces the list and partial buffers hold
        int64_t n = 0;            // pieces of the current lists
        size_t part_stride = 0;   // bytes of partial sums per piece
    } pnear, pfar, pnearT;  // forward near and far lists; transposed near lists
    bool split_lists = false;     // the last walk's lists are split (predicted for the next)
    bool lists_seen = false;      // a walk's list maxima were read back (until then a walk
                                  // reads them before the lists are evaluated)
    bool pieces_valid = false;    // pnear / pfar describe the current lists
    int64_t near_piece_blocks = 512, far_piece_entries = 1024;  // test hook: FMM_MI355_PIECE
    // pieces of the transposed near lists (reverse pass, source side): the
    // source-side P2P^T has more work per block than the forward kernel and
    // balances better with shorter pieces
    int64_t vjp_src_piece_blocks = 256;
    int32_t max_far = 0, max_near = 0;  // longest lists of the last walk
    int64_t *h_piece = nullptr;         // pinned: piece totals (near, far)

    bool has_tree = false, has_moments = false, has_lists = false, has_forces = false;
    int lists_policy = -1;

    // stage timers: an event pair per stage, harvested lazily (no added syncs)
    bool timing = false;
    hipEvent_t sev[8][2] = {};
    bool pending[8] = {};
    double acc_ms[8] = {};
    int64_t acc_n[8] = {};
};

// Stable LSD radix sorts, digit_bits = 8 or 10 bits per pass (hist: B 2^digit_bits
// words per 4096-key tile; tot: passes B 2^digit_bits words).
constexpr int RS_MAX_DIGITS = 1024;
hipError_t radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n,
                          int B, int passes, uint32_t *hist, uint32_t *tot, hipStream_t s,
                          int digit_bits);
hipError_t radix_sort_u32(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n,
                          int B, int passes, uint32_t *hist, uint32_t *tot, hipStream_t s,
                          int digit_bits);
void radix_plan(int bits, int &passes, int &digit_bits);


// launchers (return hipError_t of the last launch / runtime call)
hipError_t launch_build(Tree &t, const double *x, hipStream_t s);
hipError_t launch_morton_order(Tree &t, const double *x, hipStream_t s);
hipError_t launch_build_com(Tree &t, const double *x, const double *m, hipStream_t s);
hipError_t launch_moments(Tree &t, const double *x, const double *m, const double *h,
                          hipStream_t s);
hipError_t launch_import(Tree &t, const double *x, const double *m, const double *h,
                         const double *rec12, hipStream_t s);
hipError_t launch_walk(Tree &t, hipStream_t s);
hipError_t launch_walk_fallback(Tree &t, hipStream_t s);
hipError_t launch_far(Tree &t, hipStream_t s);
hipError_t launch_near(Tree &t, void *a, hipStream_t s);
hipError_t launch_count_scan(const int32_t *cnt, int cap, int n, int64_t *tsum, int64_t *off,
                             hipStream_t s);
int64_t count_scan_workspace(int n);
hipError_t launch_piece_counts(Tree &t, hipStream_t s);
hipError_t launch_piece_fill(Tree &t, hipStream_t s);
hipError_t launch_piece_table(const int64_t *off, const int32_t *np, int nleaves, int2 *list,
                              hipStream_t s);

// The forward lists are split into pieces (the last walk found a list
// longer than one piece, and the piece tables describe the current lists).
inline bool use_pieces(const Tree &t)
{
    return t.split_lists && t.pieces_valid && t.lists_policy == FMM_WALK_PHANTOM;
}
hipError_t launch_stats(const double *x, const double *v, const double *m, const void *a,
                        int a_fp32, int64_t n, double *red, double *d_out, double *h_out,
                        hipStream_t s);
hipError_t stats_noalloc_scratch(double **ptr);
constexpr int64_t NOALLOC_MAX_N = INT32_MAX;  // particles fmm_momentum_stats_noalloc accepts
hipError_t launch_far_f64(Tree &t, hipStream_t s);
int mutual_key_bits(const Tree &t);
int mutual_iterations(const Tree &t);
hipError_t launch_mutual_walk(Tree &t, hipStream_t s);
hipError_t launch_mutual_lists(Tree &t, int64_t n_far, int64_t n_near, hipStream_t s);
hipError_t launch_far_mutual(Tree &t, hipStream_t s);
hipError_t launch_l2l_internal(Tree &t, hipStream_t s);
hipError_t launch_vjp(Tree &t, const void *abar, void *xbar, void *mbar, hipStream_t s);
hipError_t ensure_transposed(Tree &t, hipStream_t s);
void release_vjp(Tree &t);
hipError_t launch_asym(Tree &t, double m_leaf, double *out, hipStream_t s);
void release_asym(Tree &t);
hipError_t launch_kick_drift(double *x, double *v, const void *a, int a_fp32, int64_t n,
                             double kick, double drift, hipStream_t s);

}  // namespace fmm
