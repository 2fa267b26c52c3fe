// Host side of the C ABI declared in include/fmm_mi355.h: argument checks,
// the data-independent tree shape, device memory, and the order of launches.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "fmm_internal.h"

namespace fmm {

static constexpr uint32_t TREE_MAGIC = 0x464d4d33u;
static thread_local std::string g_err;

static fmm_status fail(fmm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(e_ == hipErrorOutOfMemory ? FMM_ERR_ALLOC : FMM_ERR_HIP, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                     \
    } while (0)

void build_topology(int64_t n, int leaf_size, Topology &T)
{
    T = Topology();
    T.n = n;
    T.leaf_size = leaf_size;
    struct E {
        int64_t f, c;
        int32_t parent;
        int32_t side;
        int32_t lvl;
    };
    std::vector<E> st;
    st.push_back({0, n, -1, 0, 0});
    int64_t est = 2 * (n / std::max(1, leaf_size)) + 16;
    T.first.reserve(est);
    T.count.reserve(est);
    T.left.reserve(est);
    T.right.reserve(est);
    T.parent.reserve(est);
    T.level.reserve(est);
    while (!st.empty()) {
        E e = st.back();
        st.pop_back();
        int32_t id = (int32_t)T.first.size();
        T.first.push_back((int32_t)e.f);
        T.count.push_back((int32_t)e.c);
        T.left.push_back(-1);
        T.right.push_back(-1);
        T.parent.push_back(e.parent);
        T.level.push_back(e.lvl);
        if (e.parent >= 0)
            (e.side == 0 ? T.left : T.right)[e.parent] = id;
        if (e.c > leaf_size) {
            int64_t nl = (e.c + 1) / 2;
            st.push_back({e.f + nl, e.c - nl, id, 1, e.lvl + 1});
            st.push_back({e.f, nl, id, 0, e.lvl + 1});
        }
    }
    T.nnodes = (int)T.first.size();
    T.node_leaf.assign(T.nnodes, -1);
    int maxlvl = 0;
    for (int v = 0; v < T.nnodes; ++v) {
        maxlvl = std::max(maxlvl, T.level[v]);
        if (T.left[v] < 0) {
            T.node_leaf[v] = (int32_t)T.leaf_node.size();
            T.leaf_node.push_back(v);
        }
    }
    T.nleaves = (int)T.leaf_node.size();
    T.depth = maxlvl + 1;
    // level-synchronous part: nodes larger than SUBTREE_MAX, left to right per level
    std::vector<std::vector<int32_t>> up(T.depth);
    for (int v = 0; v < T.nnodes; ++v)
        if (T.count[v] > SUBTREE_MAX)
            up[T.level[v]].push_back(v);
    T.lvl_blk_off.push_back(0);
    for (int l = 0; l < T.depth && !up[l].empty(); ++l) {
        int nb = 0;
        for (int v : up[l]) {
            int bf = nb;
            for (int64_t s = T.first[v]; s < (int64_t)T.first[v] + T.count[v]; s += LVL_CHUNK) {
                T.blk_node.push_back(v);
                T.blk_start.push_back((int32_t)s);
                T.blk_end.push_back((int32_t)std::min<int64_t>(s + LVL_CHUNK,
                                                               (int64_t)T.first[v] + T.count[v]));
                T.blk_first.push_back(bf);
                ++nb;
            }
        }
        T.lvl_blk_off.push_back((int32_t)T.blk_node.size());
        T.max_lvl_blocks = std::max(T.max_lvl_blocks, nb);
        ++T.nlevels_up;
    }
    for (int v = 0; v < T.nnodes; ++v)
        if (T.count[v] <= SUBTREE_MAX && (T.parent[v] < 0 || T.count[T.parent[v]] > SUBTREE_MAX))
            T.sub_root.push_back(v);
    std::vector<std::vector<int32_t>> byl(T.depth);
    for (int v = 0; v < T.nnodes; ++v)
        if (T.left[v] >= 0)
            byl[T.level[v]].push_back(v);
    for (int v = 0; v < T.nnodes; ++v)
        if (T.count[v] >= 64)
            T.big_nodes.push_back(v);
    T.lvl_int_off.assign(1, 0);
    for (int l = 0; l < T.depth; ++l) {
        T.int_nodes.insert(T.int_nodes.end(), byl[l].begin(), byl[l].end());
        T.lvl_int_off.push_back((int32_t)T.int_nodes.size());
    }
    T.nbig = (int)T.big_nodes.size();
    // subtree moments: a subtree's nodes are the pre-order ids [r, r + size)
    // and its leaves a contiguous run of leaf indices
    T.sub_moments = true;
    for (int32_t r : T.sub_root) {
        int32_t lo = r, hi = r;
        while (T.left[lo] >= 0)
            lo = T.left[lo];
        while (T.right[hi] >= 0)
            hi = T.right[hi];
        const int32_t size = hi - r + 1;
        if (size > SM_MAXNODES) {
            T.sub_moments = false;
            break;
        }
        T.sm_leaf.push_back(T.node_leaf[lo]);
        T.sm_leaf.push_back(T.node_leaf[hi] + 1);
        std::vector<std::vector<int32_t>> g(SM_MAXL);
        for (int32_t v = r; v <= hi; ++v)
            if (T.left[v] >= 0) {
                const int d = T.level[v] - T.level[r];
                if (d >= SM_MAXL) {
                    T.sub_moments = false;
                    break;
                }
                g[d].push_back(v);
            }
        if (!T.sub_moments)
            break;
        for (int d = SM_MAXL - 1; d >= 0; --d) {
            T.sm_lvl.push_back((int32_t)(T.sm_nodes.size() / 2));
            for (int32_t v : g[d]) {
                T.sm_nodes.push_back(v);
                T.sm_nodes.push_back(T.right[v]);
            }
        }
        T.sm_lvl.push_back((int32_t)(T.sm_nodes.size() / 2));
    }
    T.top_lvl_off.assign(1, 0);
    for (int l = 0; l < T.depth; ++l) {
        for (int32_t v : byl[l])
            if (T.count[v] > SUBTREE_MAX)
                T.top_nodes.push_back(v);
        T.top_lvl_off.push_back((int32_t)T.top_nodes.size());
    }
    {
        const size_t nslots = T.sub_root.size() + T.top_nodes.size();
        T.top_fused = T.sub_moments && nslots <= (size_t)SM_MAXNODES;
        if (T.top_fused) {
            std::vector<int32_t> slot(T.nnodes, -1);
            for (int32_t r : T.sub_root) {
                slot[r] = (int32_t)T.top_slot_node.size();
                T.top_slot_node.push_back(r);
            }
            for (int l = T.depth - 1; l >= 0; --l)
                for (int k = T.top_lvl_off[l]; k < T.top_lvl_off[l + 1]; ++k) {
                    slot[T.top_nodes[k]] = (int32_t)T.top_slot_node.size();
                    T.top_slot_node.push_back(T.top_nodes[k]);
                }
            for (int l = T.depth - 1; l >= 0; --l) {
                if (T.top_lvl_off[l + 1] == T.top_lvl_off[l])
                    continue;
                T.top_grp.push_back((int32_t)(T.top_task.size() / 3));
                for (int k = T.top_lvl_off[l]; k < T.top_lvl_off[l + 1]; ++k) {
                    const int32_t v = T.top_nodes[k];
                    // a child is either above the subtrees or a subtree root
                    if (slot[T.left[v]] < 0 || slot[T.right[v]] < 0)
                        T.top_fused = false;
                    T.top_task.push_back(v);
                    T.top_task.push_back(slot[T.left[v]]);
                    T.top_task.push_back(slot[T.right[v]]);
                }
            }
            T.top_grp.push_back((int32_t)(T.top_task.size() / 3));
        }
    }
    T.node_cap = T.nnodes;
    T.leaf_cap = T.nleaves;
}

hipError_t tree_malloc(Tree &t, void **p, size_t bytes)
{
    *p = nullptr;
    bytes = std::max<size_t>(bytes, 256);
    if (t.p.device_bytes_limit > 0 &&
        t.held_bytes + (int64_t)bytes > t.p.device_bytes_limit)
        return hipErrorOutOfMemory;
    void *q = nullptr;
    if (t.p.dev_alloc) {
        q = t.p.dev_alloc(bytes, t.p.alloc_ctx);
        if (!q)
            return hipErrorOutOfMemory;
    } else {
        hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess)
            return e;
    }
    t.held.push_back({q, bytes});
    t.held_bytes += (int64_t)bytes;
    *p = q;
    return hipSuccess;
}

void tree_free(Tree &t, void *p)
{
    if (!p)
        return;
    for (size_t k = 0; k < t.held.size(); ++k)
        if (t.held[k].first == p) {
            t.held_bytes -= (int64_t)t.held[k].second;
            t.held[k] = t.held.back();
            t.held.pop_back();
            if (t.p.dev_free)
                t.p.dev_free(p, t.p.alloc_ctx);
            else
                (void)hipFree(p);
            return;
        }
}

template <typename P>
static hipError_t dalloc(Tree &t, P **out, size_t elems)
{
    void *p = nullptr;
    hipError_t e = tree_malloc(t, &p, elems * sizeof(P));
    if (e != hipSuccess)
        return e;
    t.owned.push_back({p, std::max<size_t>(elems * sizeof(P), 256)});
    *out = (P *)p;
    return hipSuccess;
}

template <typename P>
static hipError_t upload(Tree &t, P **out, const std::vector<P> &v)
{
    hipError_t e = dalloc(t, out, v.size());
    if (e != hipSuccess || v.empty())
        return e;
    return hipMemcpy(*out, v.data(), v.size() * sizeof(P), hipMemcpyHostToDevice);
}

static void release(Tree *t)
{
    (void)hipDeviceSynchronize();
    release_vjp(*t);
    release_asym(*t);
    if (t->cw.h_ctl)
        (void)hipHostFree(t->cw.h_ctl);
    t->owned.clear();
    t->mw.owned.clear();
    // every device allocation still held, newest first
    while (!t->held.empty())
        tree_free(*t, t->held.back().first);
    if (t->mw.h_cnt)
        (void)hipHostFree(t->mw.h_cnt);
    if (t->h_piece)
        (void)hipHostFree(t->h_piece);
    if (t->h_flags)
        (void)hipHostFree(t->h_flags);
    if (t->h_red)
        (void)hipHostFree(t->h_red);
    for (auto &pr : t->sev)
        for (auto &e : pr)
            if (e)
                (void)hipEventDestroy(e);
    t->magic = 0;
    delete t;
}

static fmm_status create_tree(int64_t n, const fmm_params &p, Tree **out)
{
    Tree *t = new Tree();
    t->magic = TREE_MAGIC;
    t->p = p;
    // Test hook: a smaller stack for the wide walk sends more leaves through
    // the exact narrow-stack walk.
    if (const char *e = std::getenv("FMM_MI355_WIDE_STACK"))
        t->wide_stack_limit = std::atoi(e);
    // Test hook: a smaller step budget sends more leaf groups through the
    // workgroup walk.
    if (const char *e = std::getenv("FMM_MI355_WALK_BUDGET"))
        t->walk_budget = std::max(1, std::atoi(e));
    // Test hook: small first capacities for the mutual walk's frontier and
    // pair buffers exercise their overflow-and-retry path.
    if (const char *e = std::getenv("FMM_MI355_MW_CAP"))
        t->mw_init_cap = std::max<int64_t>(1, std::atoll(e));
    // Test hook: small list pieces (near-field blocks and far-field entries
    // per piece) put the split evaluation to work on ordinary trees; "a,b"
    // sets the near and far piece sizes apart.
    if (const char *e = std::getenv("FMM_MI355_PIECE")) {
        t->near_piece_blocks = t->far_piece_entries = t->vjp_src_piece_blocks =
            std::max<int64_t>(1, std::atoll(e));
        if (const char *c = std::strchr(e, ','))
            t->far_piece_entries = std::max<int64_t>(1, std::atoll(c + 1));
    }
    // Test hook: the full-key Morton sort from the first build on.
    if (const char *e = std::getenv("FMM_MI355_MORTON_FULL"))
        t->morton_full = std::atoi(e) != 0;
    hipError_t e = hipSuccess;
#define A(expr)                \
    if (e == hipSuccess)       \
        e = (expr);
    if (p.tree == FMM_TREE_COM) {
        // shape set by each build; node-sized buffers for the largest tree
        Topology &T = t->topo;
        T = Topology();
        T.n = n;
        T.leaf_size = p.leaf_size;
        T.com = true;
        T.node_cap = 2 * n - 1;
        T.leaf_cap = n;
        const int64_t nc = T.node_cap;
        A(dalloc(*t, &t->first, nc));
        A(dalloc(*t, &t->count, nc));
        A(dalloc(*t, &t->left, nc));
        A(dalloc(*t, &t->right, nc));
        A(dalloc(*t, &t->parent, nc));
        A(dalloc(*t, &t->level, nc));
        A(dalloc(*t, &t->leaf_node, T.leaf_cap));
        A(dalloc(*t, &t->node_leaf, nc));
        A(dalloc(*t, &t->int_nodes, nc));
        A(dalloc(*t, &t->big_nodes, nc));
        Tree::ComWork &W = t->cw;
        W.cap_a = n / (p.leaf_size + 1) + 2;
        W.cap_c = (n + COM_CHUNK - 1) / COM_CHUNK + W.cap_a + 2;
        A(dalloc(*t, &W.q, 4 * n));
        A(dalloc(*t, &W.q_tmp, 4 * n));
        A(dalloc(*t, &W.perm_tmp, n));
        A(dalloc(*t, &W.node, 8 * nc));
        A(dalloc(*t, &W.ren, 4 * nc));
        for (int k = 0; k < 2; ++k) {
            A(dalloc(*t, &W.act[k], W.cap_a));
            A(dalloc(*t, &W.act_choff[k], W.cap_a + 1));
            A(dalloc(*t, &W.chk[k], 3 * W.cap_c));
        }
        A(dalloc(*t, &W.cpart, 16 * W.cap_c));
        A(dalloc(*t, &W.cleft, W.cap_c));
        A(dalloc(*t, &W.cbase, W.cap_c));
        A(dalloc(*t, &W.split, 4 * W.cap_a));
        A(dalloc(*t, &W.nl, W.cap_a));
        A(dalloc(*t, &W.big, nc));
        A(dalloc(*t, &W.ctl, 8));
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&W.h_ctl, 8 * sizeof(int64_t), hipHostMallocDefault);
    } else {
        build_topology(n, p.leaf_size, t->topo);
        const Topology &T = t->topo;
        A(upload(*t, &t->first, T.first));
        A(upload(*t, &t->count, T.count));
        A(upload(*t, &t->left, T.left));
        A(upload(*t, &t->right, T.right));
        A(upload(*t, &t->parent, T.parent));
        A(upload(*t, &t->level, T.level));
        A(upload(*t, &t->leaf_node, T.leaf_node));
        A(upload(*t, &t->node_leaf, T.node_leaf));
        A(upload(*t, &t->blk_node, T.blk_node));
        A(upload(*t, &t->blk_start, T.blk_start));
        A(upload(*t, &t->blk_end, T.blk_end));
        A(upload(*t, &t->blk_first, T.blk_first));
        A(upload(*t, &t->sub_root, T.sub_root));
        A(upload(*t, &t->int_nodes, T.int_nodes));
        A(upload(*t, &t->big_nodes, T.big_nodes));
        A(upload(*t, &t->sm_leaf, T.sm_leaf));
        A(upload(*t, &t->sm_lvl, T.sm_lvl));
        A(upload(*t, &t->sm_nodes, T.sm_nodes));
        A(upload(*t, &t->top_nodes, T.top_nodes));
        A(upload(*t, &t->top_slot_node, T.top_slot_node));
        A(upload(*t, &t->top_task, T.top_task));
        A(upload(*t, &t->top_grp, T.top_grp));
    }
    const Topology &T = t->topo;
    const int64_t nn = T.node_cap;
    const int64_t nblk = (n + RS_TILE - 1) / RS_TILE;
    t->s2part_depth = T.com ? 64 : T.depth;
    A(dalloc(*t, &t->axis, nn));
    A(dalloc(*t, &t->keys0, 3 * n));
    A(dalloc(*t, &t->keys1, 3 * n));
    A(dalloc(*t, &t->vals0, 3 * n));
    A(dalloc(*t, &t->vals1, 3 * n));
    A(dalloc(*t, &t->rs_hist, 3 * 256 * nblk));
    A(dalloc(*t, &t->rs_tot, (size_t)RS_PASSES * 3 * 256));
    A(dalloc(*t, &t->run_cnt, 4));  // axis sorts: [0..1], Morton sort: [2..3]
    A(dalloc(*t, &t->run_list, 3 * (n / 65 + 1)));
    A(dalloc(*t, &t->r2o, n));
    A(dalloc(*t, &t->xr, 3 * n));
    A(dalloc(*t, &t->lists, 8 * n));
    A(dalloc(*t, &t->side, 5 * n));  // 4 lists by position, then one byte per rank
    A(dalloc(*t, &t->lvl_cnt, 4 * (size_t)std::max(1, T.max_lvl_blocks)));
    A(dalloc(*t, &t->bbox, 8));
    A(dalloc(*t, &t->err, 4));
    A(dalloc(*t, &t->perm, n));
    A(dalloc(*t, &t->pm, n + 1));  // + the null source record
    A(dalloc(*t, &t->hs, n));
    A(dalloc(*t, &t->ph, n + 1));
    A(dalloc(*t, &t->pf, n));
    A(dalloc(*t, &t->pfh, n));
    A(dalloc(*t, &t->recA, NREC * nn));
    A(dalloc(*t, &t->recQ, NREC * nn));
    A(dalloc(*t, &t->recF, NREC * nn));
    A(dalloc(*t, &t->s2bits, nn));
    // per-level partial maxima of s^2: grown by deeper centre-of-mass trees,
    // so kept apart from the fixed allocations
    A(tree_malloc(*t, (void **)&t->s2part,
                  std::max<size_t>((size_t)t->s2part_depth * ((n + 63) / 64), 32) * sizeof(uint64_t)));
    A(dalloc(*t, &t->upcnt, nn));
    A(dalloc(*t, &t->far_cnt, nn));
    A(dalloc(*t, &t->near_cnt, nn));
    A(dalloc(*t, &t->walk_flags, 4));
    A(dalloc(*t, &t->walk_heavy, (size_t)(n + 3) / 4 + 1));  // groups of four leaves
    A(dalloc(*t, &t->L, NLOC * nn));
    A(dalloc(*t, &t->Lf, NLOC * nn));
    A(dalloc(*t, &t->red, 16 + 16 * 512));
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&t->h_flags, 16 * sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&t->h_red, 16 * sizeof(double), hipHostMallocDefault);
    for (int k = 0; k < 8 && e == hipSuccess; ++k)
        for (int j = 0; j < 2 && e == hipSuccess; ++j)
            e = hipEventCreate(&t->sev[k][j]);
#undef A
    if (e != hipSuccess) {
        fmm_status st = fail(e == hipErrorOutOfMemory ? FMM_ERR_ALLOC : FMM_ERR_HIP,
                             "tree allocation failed: %s", hipGetErrorString(e));
        release(t);
        return st;
    }
    *out = t;
    return FMM_OK;
}

static bool tree_ok(const fmm_tree *h)
{
    return h && reinterpret_cast<const Tree *>(h)->magic == TREE_MAGIC;
}

static fmm_status check_params(const fmm_params *p)
{
    if (!p)
        return fail(FMM_ERR_INVALID, "params is NULL");
    if (!(p->theta >= 0.0 && p->theta <= 1.0))
        return fail(FMM_ERR_INVALID, "theta must lie in [0, 1] (got %g)", p->theta);
    if (!(p->r_kern > 0.0 && std::isfinite(p->r_kern)))
        return fail(FMM_ERR_INVALID, "r_kern must be positive and finite");
    if (!std::isfinite(p->G))
        return fail(FMM_ERR_INVALID, "G must be finite");
    if (p->leaf_size < 1 || p->leaf_size > MAX_LEAF)
        return fail(FMM_ERR_INVALID, "leaf_size must lie in [1, %d]", MAX_LEAF);
    if (p->walk != FMM_WALK_PHANTOM && p->walk != FMM_WALK_MUTUAL)
        return fail(FMM_ERR_INVALID, "unknown walk policy %d", p->walk);
    if (p->precision != FMM_FP64 && p->precision != FMM_FP32)
        return fail(FMM_ERR_INVALID, "unknown precision %d", p->precision);
    if (p->expansion != FMM_EXPANSION_PHANTOM && p->expansion != FMM_EXPANSION_DEHNEN)
        return fail(FMM_ERR_INVALID, "unknown expansion form %d", p->expansion);
    if (p->tree != FMM_TREE_MEDIAN && p->tree != FMM_TREE_COM)
        return fail(FMM_ERR_INVALID, "unknown tree shape %d", p->tree);
    if (p->reserved != 0)
        return fail(FMM_ERR_INVALID, "reserved must be 0");
    if (p->list_capacity < 0)
        return fail(FMM_ERR_INVALID, "list_capacity must be >= 0");
    if (p->device_bytes_limit < 0)
        return fail(FMM_ERR_INVALID, "device_bytes_limit must be >= 0");
    if ((p->dev_alloc == nullptr) != (p->dev_free == nullptr))
        return fail(FMM_ERR_INVALID, "dev_alloc and dev_free must be given together");
    return FMM_OK;
}

// Stage timing (only when enabled): a start/stop event pair per stage on the
// caller's stream.  The previous pair of a stage is read when the stage runs
// again (by then it has normally completed) or by fmm_stage_times, so timing
// adds no synchronisation to the steady state.
static void harvest(Tree &t, int slot)
{
    if (!t.pending[slot])
        return;
    (void)hipEventSynchronize(t.sev[slot][1]);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.sev[slot][0], t.sev[slot][1]) == hipSuccess) {
        t.acc_ms[slot] += ms;
        t.acc_n[slot] += 1;
    }
    t.pending[slot] = false;
}

struct StageTimer {
    Tree &t;
    hipStream_t s;
    int slot;
    StageTimer(Tree &tt, hipStream_t ss, int sl) : t(tt), s(ss), slot(sl)
    {
        if (t.timing) {
            harvest(t, slot);
            (void)hipEventRecord(t.sev[slot][0], s);
        }
    }
    void done()
    {
        if (!t.timing)
            return;
        (void)hipEventRecord(t.sev[slot][1], s);
        t.pending[slot] = true;
    }
};

// (Re)allocate the per-leaf list slots for capacities cap_far / cap_near
// (both fixed at params.list_capacity when that is set).  Slots that are
// reallocated lose their lists; on failure the tree is left without lists.
static fmm_status ensure_slots(Tree &t, int64_t cap_far, int64_t cap_near)
{
    const int64_t nl = t.topo.nleaves;
    if (t.p.list_capacity > 0)
        cap_far = cap_near = t.p.list_capacity;
    struct Want {
        DevBuf *b;
        int32_t **ptr;
        int64_t *cap;
        int64_t want;
    } w[2] = {{&t.far_buf, &t.far_src, &t.cap_far, cap_far},
              {&t.near_buf, &t.near_src, &t.cap_near, cap_near}};
    const bool more_leaves = nl > t.slots_nl;
    for (auto &x : w) {
        if (x.b->p && *x.cap == x.want && !more_leaves)
            continue;
        if (x.b->p) {
            HIP_TRY(hipDeviceSynchronize());
            tree_free(t, x.b->p);
            x.b->p = nullptr;
            x.b->bytes = 0;
            *x.ptr = nullptr;
            *x.cap = 0;
            t.has_lists = false;
        }
        size_t bytes = (size_t)std::max<int64_t>(1, nl * x.want) * sizeof(int32_t);
        void *p = nullptr;
        hipError_t e = tree_malloc(t, &p, bytes);
        if (e != hipSuccess) {
            t.has_lists = false;
            return fail(e == hipErrorOutOfMemory ? FMM_ERR_ALLOC : FMM_ERR_HIP,
                        "interaction-list slots of %lld bytes: %s", (long long)bytes,
                        hipGetErrorString(e));
        }
        x.b->p = p;
        x.b->bytes = bytes;
        *x.ptr = (int32_t *)p;
        *x.cap = x.want;
    }
    t.slots_nl = std::max(t.slots_nl, nl);
    return FMM_OK;
}

// Release the per-leaf list slots (and with them the lists).
static fmm_status drop_slots(Tree &t)
{
    if (!t.far_buf.p && !t.near_buf.p)
        return FMM_OK;
    HIP_TRY(hipDeviceSynchronize());
    for (DevBuf *b : {&t.far_buf, &t.near_buf}) {
        tree_free(t, b->p);
        b->p = nullptr;
        b->bytes = 0;
    }
    t.far_src = t.near_src = nullptr;
    t.cap_far = t.cap_near = 0;
    t.slots_nl = 0;
    t.has_lists = t.has_forces = false;
    t.pieces_valid = false;
    return FMM_OK;
}

static int64_t round_cap(int64_t need) { return ((need + need / 4 + 64) + 63) / 64 * 64; }

// (Re)allocate a growable device buffer to at least `bytes` (contents lost).
static fmm_status grow(Tree &t, DevBuf &b, size_t bytes)
{
    if (b.p && b.bytes >= bytes)
        return FMM_OK;
    if (b.p) {
        HIP_TRY(hipDeviceSynchronize());
        tree_free(t, b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    HIP_TRY(tree_malloc(t, &b.p, bytes));
    b.bytes = std::max<size_t>(bytes, 256);
    return FMM_OK;
}

static fmm_status mw_alloc(Tree &t, void **out, size_t bytes)
{
    void *p = nullptr;
    HIP_TRY(tree_malloc(t, &p, bytes));
    t.mw.owned.push_back({p, bytes});
    *out = p;
    return FMM_OK;
}

// Buffers of the mutual walk for the given capacities (pairs / frontier).
static fmm_status ensure_mutual(Tree &t, int64_t cap_task, int64_t cap_far, int64_t cap_near)
{
    MutualLists &M = t.mw;
    const Topology &T = t.topo;
    fmm_status st = FMM_OK;
    if (!M.cnt) {
        void *p = nullptr;
        if ((st = mw_alloc(t, &p, MW_CNT * sizeof(unsigned long long))) != FMM_OK)
            return st;
        M.cnt = (unsigned long long *)p;
        if ((st = mw_alloc(t, &p, 2 * (size_t)T.node_cap * sizeof(int64_t))) != FMM_OK)
            return st;
        M.fstart = (int64_t *)p;
        M.fend = M.fstart + T.node_cap;
        if ((st = mw_alloc(t, &p, (size_t)T.leaf_cap * sizeof(int64_t))) != FMM_OK)
            return st;
        M.nstart = (int64_t *)p;
        if ((st = mw_alloc(t, &p, (size_t)RS_PASSES * 256 * sizeof(uint32_t))) != FMM_OK)
            return st;
        M.tot = (uint32_t *)p;
        HIP_TRY(hipHostMalloc((void **)&M.h_cnt, MW_CNT * sizeof(unsigned long long),
                              hipHostMallocDefault));
    }
    if (t.p.precision == FMM_FP64 && !M.Lown) {
        void *p = nullptr;
        if ((st = mw_alloc(t, &p, (size_t)NLOC * T.node_cap * sizeof(double))) != FMM_OK)
            return st;
        M.Lown = (double *)p;
    }
    if (t.p.precision == FMM_FP32 && !M.Lownf) {
        void *p = nullptr;
        if ((st = mw_alloc(t, &p, (size_t)NLOC * T.node_cap * sizeof(float))) != FMM_OK)
            return st;
        M.Lownf = (float *)p;
    }
    if (cap_task > M.cap_task) {
        M.task[0] = M.task[1] = nullptr;
        M.cap_task = 0;
        if ((st = grow(t, M.b_task, 2 * (size_t)cap_task * sizeof(int2))) != FMM_OK)
            return st;
        M.task[0] = (int2 *)M.b_task.p;
        M.task[1] = M.task[0] + cap_task;
        M.cap_task = cap_task;
    }
    if (cap_far > M.cap_far) {
        M.fkeys[0] = M.fkeys[1] = nullptr;
        M.far_sorted = nullptr;
        M.cap_far = 0;
        t.has_lists = false;
        if ((st = grow(t, M.b_fkeys, 2 * (size_t)cap_far * sizeof(uint64_t))) != FMM_OK)
            return st;
        M.fkeys[0] = (uint64_t *)M.b_fkeys.p;
        M.fkeys[1] = M.fkeys[0] + cap_far;
        M.cap_far = cap_far;
    }
    if (cap_near > M.cap_near) {
        M.nkeys[0] = M.nkeys[1] = nullptr;
        M.cap_near = 0;
        if ((st = grow(t, M.b_nkeys, 2 * (size_t)cap_near * sizeof(uint64_t))) != FMM_OK)
            return st;
        M.nkeys[0] = (uint64_t *)M.b_nkeys.p;
        M.nkeys[1] = M.nkeys[0] + cap_near;
        M.cap_near = cap_near;
    }
    const int64_t tiles = (std::max(M.cap_far, M.cap_near) + RS_TILE - 1) / RS_TILE;
    M.hist = nullptr;
    if ((st = grow(t, M.b_hist, (size_t)256 * tiles * sizeof(uint32_t))) != FMM_OK)
        return st;
    M.hist = (uint32_t *)M.b_hist.p;
    return FMM_OK;
}

// After a readback that included the Morton sort's long-run entry count
// (h_flags[6]): data whose keys mostly share their high halves switches the
// tree's later builds to the full-key sort.
static void note_long_runs(Tree &t)
{
    if (!t.morton_full && (uint32_t)t.h_flags[6] > (uint64_t)t.topo.n / 16)
        t.morton_full = true;
}

// Enqueue the readback of both data-check words (build, moments) to
// h_flags[8..9]; their OR after the stream has synchronised.
static hipError_t read_err_async(Tree &t, hipStream_t s)
{
    return hipMemcpyAsync(t.h_flags + 8, t.err, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
}

static uint32_t err_bits(const Tree &t) { return (uint32_t)t.h_flags[8] | (uint32_t)t.h_flags[9]; }

static fmm_status bad_input(uint32_t errbits)
{
    if (!(errbits & 7u))
        return fail(FMM_ERR_HIP, "internal error in the tree build (flags 0x%x)", errbits);
    return fail(FMM_ERR_INVALID, "bad input data:%s%s%s",
                (errbits & 1) ? " non-finite positions" : "",
                (errbits & 2) ? " masses not positive and finite" : "",
                (errbits & 4) ? " smoothing lengths not positive and finite" : "");
}

// Workspace of the list pieces that does not depend on the lists: pieces per
// leaf, their offsets and the scan workspace (all or nothing).
static fmm_status ensure_piece_base(Tree &t)
{
    if (t.pnear.np)
        return FMM_OK;
    const int64_t nl = t.topo.leaf_cap;
    hipError_t e = hipSuccess;
    for (Tree::Pieces *P : {&t.pnear, &t.pfar}) {
        if (e == hipSuccess)
            e = tree_malloc(t, (void **)&P->np, nl * sizeof(int32_t));
        if (e == hipSuccess)
            e = tree_malloc(t, (void **)&P->off, (nl + 1) * sizeof(int64_t));
        if (e == hipSuccess)
            e = tree_malloc(t, (void **)&P->tsum, count_scan_workspace((int)nl) * sizeof(int64_t));
    }
    if (e == hipSuccess && !t.h_piece)
        e = hipHostMalloc((void **)&t.h_piece, 2 * sizeof(int64_t), hipHostMallocDefault);
    if (e != hipSuccess) {
        for (Tree::Pieces *P : {&t.pnear, &t.pfar}) {
            tree_free(t, P->np);
            tree_free(t, P->off);
            tree_free(t, P->tsum);
            P->np = nullptr;
            P->off = P->tsum = nullptr;
        }
        return fail(FMM_ERR_ALLOC, "list pieces: %s", hipGetErrorString(e));
    }
    return FMM_OK;
}

// The piece totals (near, far) to the pinned host buffer.
static hipError_t read_piece_totals_async(Tree &t, hipStream_t s)
{
    const int nl = t.topo.nleaves;
    hipError_t e = hipMemcpyAsync(t.h_piece, t.pnear.off + nl, sizeof(int64_t),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(t.h_piece + 1, t.pfar.off + nl, sizeof(int64_t), hipMemcpyDeviceToHost,
                           s);
    return e;
}

// Lay out the pieces of the current lists: counts and offsets (unless the
// totals were already read back with them, have_totals), buffers for the
// pieces and their partial sums, and the piece lists.
static fmm_status build_pieces(Tree &t, hipStream_t s, bool have_totals)
{
    fmm_status st = ensure_piece_base(t);
    if (st != FMM_OK)
        return st;
    if (!have_totals) {
        HIP_TRY(launch_piece_counts(t, s));
        HIP_TRY(read_piece_totals_async(t, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    const size_t strides[2] = {(size_t)3 * t.topo.leaf_size * sizeof(double),
                               (size_t)NLOC * sizeof(double)};
    Tree::Pieces *Ps[2] = {&t.pnear, &t.pfar};
    for (int k = 0; k < 2; ++k) {
        Tree::Pieces &P = *Ps[k];
        const int64_t np = t.h_piece[k];
        if (np > P.cap) {
            HIP_TRY(hipStreamSynchronize(s));
            tree_free(t, P.list);
            tree_free(t, P.part);
            P.list = nullptr;
            P.part = nullptr;
            P.cap = 0;
            const int64_t cap = np + np / 4 + 64;
            hipError_t e = tree_malloc(t, (void **)&P.list, cap * sizeof(int2));
            if (e == hipSuccess)
                e = tree_malloc(t, &P.part, cap * strides[k]);
            if (e != hipSuccess) {
                tree_free(t, P.list);
                P.list = nullptr;
                return fail(FMM_ERR_ALLOC, "list pieces: %s", hipGetErrorString(e));
            }
            P.cap = cap;
        }
        P.n = np;
        P.part_stride = strides[k];
    }
    HIP_TRY(launch_piece_fill(t, s));
    t.pieces_valid = true;
    return FMM_OK;
}

// Forces on kept lists: the data checks of the last moments call are read
// back (one synchronisation); bad data drops the lists.
static fmm_status check_data_after(Tree &t, hipStream_t s)
{
    HIP_TRY(read_err_async(t, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint32_t errbits = err_bits(t);
    if (errbits) {
        t.has_lists = t.has_forces = false;
        return bad_input(errbits);
    }
    t.has_forces = true;
    return FMM_OK;
}

// fmm_forces for the mutual walk: walk (one readback of the pair counts,
// buffers grown and the walk redone if they overflowed), sort into lists,
// then M2L + L2L and the near field.
static fmm_status forces_mutual(Tree &t, void *a, bool walk, bool vjp_only, hipStream_t s)
{
    MutualLists &M = t.mw;
    const Topology &T = t.topo;
    if (walk) {
        // the lists are replaced: none until the walk has succeeded
        t.has_lists = t.has_forces = false;
        // first capacities: above the frontier and pair counts of theta = 0.5
        // with 58-neighbour smoothing lengths (grown on overflow, then kept)
        const int64_t c0 = t.mw_init_cap;
        fmm_status st = ensure_mutual(t, c0 ? c0 : 48 * (int64_t)T.nnodes + 4096,
                                      c0 ? c0 : 96 * (int64_t)T.nnodes + 4096,
                                      c0 ? c0 : 192 * (int64_t)T.nleaves + 4096);
        if (st != FMM_OK)
            return st;
        if (!t.far_buf.p && (st = ensure_slots(t, 1, 128)) != FMM_OK)
            return st;
        const int nit = mutual_iterations(t);
        if (MW_IT + nit + 1 > MW_CNT)
            return fail(FMM_ERR_INVALID, "tree too deep for the mutual walk (%d levels)", T.depth);
        bool done = false;
        for (int attempt = 0; attempt < 8 && !done; ++attempt) {
            StageTimer tm(t, s, 2);
            HIP_TRY(launch_mutual_walk(t, s));
            HIP_TRY(hipMemcpyAsync(M.h_cnt, M.cnt, (MW_IT + nit + 1) * sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(read_err_async(t, s));
            HIP_TRY(hipMemcpyAsync(t.h_flags + 5, t.run_cnt + 2, 2 * sizeof(uint32_t),
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            note_long_runs(t);
            const uint32_t errbits = err_bits(t);
            if (errbits) {
                t.has_lists = false;
                return bad_input(errbits);
            }
            const uint64_t flags = M.h_cnt[MW_FLAGS];
            const int64_t nf = (int64_t)M.h_cnt[MW_NFAR], nn = (int64_t)M.h_cnt[MW_NNEAR];
            if (flags) {
                int64_t mt = 0;
                for (int k = 0; k <= nit; ++k)
                    mt = std::max<int64_t>(mt, (int64_t)M.h_cnt[MW_IT + k]);
                st = ensure_mutual(t, (flags & 1) ? std::max(2 * M.cap_task, round_cap(mt)) : 0,
                                   (flags & 2) ? round_cap(nf) : 0,
                                   (flags & 4) ? round_cap(nn) : 0);
                if (st != FMM_OK)
                    return st;
                continue;
            }
            if (M.h_cnt[MW_IT + nit] != 0)
                return fail(FMM_ERR_CAPACITY, "mutual walk did not finish in %d levels", nit);
            const int64_t mx = (int64_t)M.h_cnt[MW_MAXNEAR];
            if (t.p.list_capacity > 0 && mx > t.p.list_capacity)
                return fail(FMM_ERR_CAPACITY,
                            "a near list needs %lld entries; list_capacity is %lld",
                            (long long)mx, (long long)t.p.list_capacity);
            if (mx > t.cap_near && (st = ensure_slots(t, t.cap_far, round_cap(mx))) != FMM_OK)
                return st;
            HIP_TRY(launch_mutual_lists(t, nf, nn, s));
            tm.done();
            M.n_far = nf;
            M.n_near = nn;
            done = true;
        }
        if (!done)
            return fail(FMM_ERR_CAPACITY, "mutual walk buffers did not fit after resizing");
        t.has_lists = true;
        t.has_transposed = false;
        t.lists_policy = FMM_WALK_MUTUAL;
        t.nsinks = T.nnodes;
        t.n_far = M.n_far;
        t.n_near = M.n_near;
    } else {
        fmm_status st = ensure_mutual(t, 0, 0, 0);  // Lown of the current precision
        if (st != FMM_OK)
            return st;
    }
    if (!vjp_only || t.p.precision == FMM_FP64) {
        StageTimer tm(t, s, 3);
        HIP_TRY(launch_far_mutual(t, s));
        tm.done();
    }
    if (!vjp_only) {
        StageTimer tm(t, s, 4);
        HIP_TRY(launch_near(t, a, s));
        tm.done();
    }
    t.has_forces = true;
    return FMM_OK;
}

static std::mutex g_scratch_mu;
static std::map<int, std::pair<double *, double *>> g_scratch;

static fmm_status stats_scratch(double **dev, double **host)
{
    int d = 0;
    HIP_TRY(hipGetDevice(&d));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(d);
    if (it == g_scratch.end()) {
        double *dp = nullptr, *hp = nullptr;
        HIP_TRY(hipMalloc((void **)&dp, (16 + 16 * 512) * sizeof(double)));
        HIP_TRY(hipHostMalloc((void **)&hp, 16 * sizeof(double), hipHostMallocDefault));
        it = g_scratch.emplace(d, std::make_pair(dp, hp)).first;
    }
    *dev = it->second.first;
    *host = it->second.second;
    return FMM_OK;
}

}  // namespace fmm

using namespace fmm;

extern "C" {

void fmm_default_params(fmm_params *p)
{
    if (!p)
        return;
    p->theta = 0.5;
    p->r_kern = 2.0;
    p->G = 1.0;
    p->leaf_size = 8;
    p->walk = FMM_WALK_PHANTOM;
    p->precision = FMM_FP64;
    p->expansion = FMM_EXPANSION_PHANTOM;
    p->tree = FMM_TREE_MEDIAN;
    p->reserved = 0;
    p->list_capacity = 0;
    p->device_bytes_limit = 0;
    p->dev_alloc = nullptr;
    p->dev_free = nullptr;
    p->alloc_ctx = nullptr;
}

const char *fmm_last_error(void) { return g_err.c_str(); }

fmm_status fmm_build_tree(const double *x, int64_t n, const fmm_params *p, void *stream,
                          fmm_tree **tree)
{
    return fmm_build_tree_weighted(x, nullptr, n, p, stream, tree);
}

fmm_status fmm_build_tree_weighted(const double *x, const double *m, int64_t n,
                                   const fmm_params *p, void *stream, fmm_tree **tree)
{
    if (!x || !tree)
        return fail(FMM_ERR_INVALID, "x and tree must not be NULL");
    if (n < 1 || n > (int64_t)INT32_MAX)
        return fail(FMM_ERR_INVALID, "n must lie in [1, 2^31-1] (got %lld)", (long long)n);
    fmm_status st = check_params(p);
    if (st != FMM_OK)
        return st;
    Tree *t = nullptr;
    if (*tree) {
        if (!tree_ok(*tree))
            return fail(FMM_ERR_STATE, "unknown or freed tree handle");
        t = reinterpret_cast<Tree *>(*tree);
        if (t->topo.n != n || t->topo.leaf_size != p->leaf_size)
            return fail(FMM_ERR_INVALID, "a reused tree must keep n and leaf_size");
        if (t->p.tree != p->tree)
            return fail(FMM_ERR_INVALID, "a reused tree must keep its tree shape");
        if (t->p.dev_alloc != p->dev_alloc || t->p.dev_free != p->dev_free ||
            t->p.alloc_ctx != p->alloc_ctx || t->p.device_bytes_limit != p->device_bytes_limit)
            return fail(FMM_ERR_INVALID, "a reused tree must keep its allocator and byte limit");
        if (t->p.list_capacity != p->list_capacity) {
            // the slots are sized for the old capacity: drop them with the lists
            fmm_status st = drop_slots(*t);
            if (st != FMM_OK)
                return st;
        }
        t->p = *p;
    } else {
        st = create_tree(n, *p, &t);
        if (st != FMM_OK)
            return st;
    }
    hipStream_t s = (hipStream_t)stream;
    StageTimer tm(*t, s, 0);
    hipError_t e = t->p.tree == FMM_TREE_COM ? launch_build_com(*t, x, m, s)
                                             : launch_build(*t, x, s);
    if (e == hipSuccess && t->topo.depth > COM_MAX_DEPTH) {
        // the walks' stacks hold a bounded number of levels
        const int d = t->topo.depth;
        t->has_tree = t->has_moments = t->has_lists = t->has_forces = false;
        if (!*tree)
            release(t);
        return fail(FMM_ERR_INVALID,
                    "the centre-of-mass tree has %d levels (at most %d are supported): the "
                    "particles are too strongly clustered for this tree shape",
                    d, COM_MAX_DEPTH);
    }
    if (e == hipSuccess && t->topo.depth > t->s2part_depth) {
        // a deeper centre-of-mass tree: grow the per-level s^2 partials
        e = hipStreamSynchronize(s);
        if (e == hipSuccess) {
            tree_free(*t, t->s2part);
            t->s2part = nullptr;
            t->s2part_depth = 0;
        }
        const int64_t d = t->topo.depth + 16;
        if (e == hipSuccess)
            e = tree_malloc(*t, (void **)&t->s2part, (size_t)d * ((n + 63) / 64) * sizeof(uint64_t));
        if (e == hipSuccess)
            t->s2part_depth = d;
    }
    if (e != hipSuccess) {
        if (!*tree)
            release(t);
        else
            t->has_tree = t->has_moments = t->has_lists = t->has_forces = false;
        return fail(e == hipErrorOutOfMemory ? FMM_ERR_ALLOC : FMM_ERR_HIP,
                    "tree build failed: %s", hipGetErrorString(e));
    }
    tm.done();
    t->has_tree = true;
    t->has_moments = t->has_lists = t->has_forces = false;
    *tree = reinterpret_cast<fmm_tree *>(t);
    return FMM_OK;
}

fmm_status fmm_moments(fmm_tree *tree, const double *x, const double *m, const double *h,
                       void *stream)
{
    if (!tree_ok(tree))
        return fail(FMM_ERR_STATE, "unknown or freed tree handle");
    if (!x || !m || !h)
        return fail(FMM_ERR_INVALID, "x, m and h must not be NULL");
    Tree &t = *reinterpret_cast<Tree *>(tree);
    if (!t.has_tree)
        return fail(FMM_ERR_STATE, "the tree has not been built");
    hipStream_t s = (hipStream_t)stream;
    StageTimer tm(t, s, 1);
    hipError_t e = launch_moments(t, x, m, h, s);
    if (e != hipSuccess)
        return fail(FMM_ERR_HIP, "moments launch failed: %s", hipGetErrorString(e));
    tm.done();
    t.has_moments = true;
    t.has_forces = false;
    return FMM_OK;
}

fmm_status fmm_forces(fmm_tree *tree, void *a, int32_t flags, void *stream)
{
    if (!tree_ok(tree))
        return fail(FMM_ERR_STATE, "unknown or freed tree handle");
    if (flags & ~(FMM_REWALK | FMM_VJP_ONLY))
        return fail(FMM_ERR_INVALID, "unknown flags 0x%x", (unsigned)flags);
    // FMM_VJP_ONLY: the state the reverse pass needs (lists; the far-field
    // expansions of an FP64 tree, which the reverse pass reads -- an FP32
    // tree's reverse pass forms its own FP64 ones), no forces
    const bool vjp_only = (flags & FMM_VJP_ONLY) != 0;
    if (!a && !vjp_only)
        return fail(FMM_ERR_INVALID, "a must not be NULL");
    Tree &t = *reinterpret_cast<Tree *>(tree);
    const bool far_needed = !vjp_only || t.p.precision == FMM_FP64;
    if (!t.has_moments)
        return fail(FMM_ERR_STATE, "fmm_moments must run before fmm_forces");
    hipStream_t s = (hipStream_t)stream;
    const bool walk = !t.has_lists || (flags & FMM_REWALK) || t.lists_policy != t.p.walk;
    if (t.p.walk == FMM_WALK_MUTUAL) {
        fmm_status st = forces_mutual(t, a, walk, vjp_only, s);
        if (st != FMM_OK || walk)
            return st;
        return check_data_after(t, s);
    }
    if (walk) {
        // the lists are replaced: none until the walk has succeeded
        t.has_lists = t.has_forces = false;
        if (!t.far_buf.p || t.slots_nl < t.topo.nleaves) {
            fmm_status st = ensure_slots(t, t.far_buf.p ? t.cap_far : 512,
                                         t.near_buf.p ? t.cap_near : 128);
            if (st != FMM_OK)
                return st;
        }
    }
    // Lists are evaluated whole, or split into pieces when the last walk
    // found lists longer than one piece, or, on a tree's first walk, when
    // that walk does (the sums are bit-identical either way; pieces only
    // balance the work).  Whole lists: walk, M2L, P2P, then
    // one readback of the list maxima.  Split lists: the list lengths are read
    // back first, then the pieces are laid out and evaluated.  If a slot
    // overflowed, the slots grow and it is done again.
    if (!walk) {
        if (t.split_lists && !t.pieces_valid) {
            fmm_status st = build_pieces(t, s, false);
            if (st != FMM_OK)
                return st;
        }
        if (far_needed) {
            StageTimer tm(t, s, 3);
            HIP_TRY(launch_far(t, s));
            tm.done();
        }
        if (!vjp_only) {
            StageTimer tm(t, s, 4);
            HIP_TRY(launch_near(t, a, s));
            tm.done();
        }
        return check_data_after(t, s);
    }
    for (int attempt = 0; attempt < 4; ++attempt) {
        t.pieces_valid = false;
        {
            StageTimer tm(t, s, 2);
            HIP_TRY(launch_walk(t, s));
            tm.done();
        }
        // the first walk of a tree has no earlier maxima to predict from: it
        // reads its own before evaluating, as a split walk does
        const bool split = t.split_lists || !t.lists_seen;
        if (split) {
            fmm_status st = ensure_piece_base(t);
            if (st != FMM_OK)
                return st;
            HIP_TRY(launch_piece_counts(t, s));
            HIP_TRY(read_piece_totals_async(t, s));
        } else {
            if (far_needed) {
                StageTimer tm(t, s, 3);
                HIP_TRY(launch_far(t, s));
                tm.done();
            }
            if (!vjp_only) {
                StageTimer tm(t, s, 4);
                HIP_TRY(launch_near(t, a, s));
                tm.done();
            }
        }
        HIP_TRY(hipMemcpyAsync(t.h_flags, t.walk_flags, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(read_err_async(t, s));
        HIP_TRY(hipMemcpyAsync(t.h_flags + 5, t.run_cnt + 2, 2 * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        note_long_runs(t);
        uint32_t errbits = err_bits(t);
        if (errbits) {
            t.has_lists = false;
            return bad_input(errbits);
        }
        const bool fallback = t.h_flags[2] != 0;
        if (fallback) {
            // some leaves overflowed the wide walk's stack: redo those exactly
            HIP_TRY(launch_walk_fallback(t, s));
            HIP_TRY(hipMemcpyAsync(t.h_flags, t.walk_flags, 4 * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        const int64_t mf = t.h_flags[0], mn = t.h_flags[1];
        if (t.p.list_capacity > 0 && (mf > t.cap_far || mn > t.cap_near))
            return fail(FMM_ERR_CAPACITY,
                        "a sink list needs %lld entries (far) / %lld (near); list_capacity is %lld",
                        (long long)mf, (long long)mn, (long long)t.p.list_capacity);
        if (mf <= t.cap_far && mn <= t.cap_near) {
            t.has_lists = true;
            t.has_transposed = false;
            t.lists_policy = t.p.walk;
            t.nsinks = t.topo.nleaves;
            t.n_far = t.n_near = -1;  // totals computed on demand
            t.max_far = (int32_t)mf;
            t.max_near = (int32_t)mn;
            const int nsub = (t.topo.leaf_size + 7) / 8;
            t.split_lists = mf > t.far_piece_entries || mn * nsub > t.near_piece_blocks;
            t.lists_seen = true;
            if (split || fallback) {
                // evaluate now: on the pieces of these lists (their totals were
                // read with the maxima unless the fallback changed the lists),
                // or whole lists again after the fallback completed them
                if (t.split_lists) {
                    fmm_status st = build_pieces(t, s, split && !fallback);
                    if (st != FMM_OK)
                        return st;
                }
                if (far_needed) {
                    StageTimer tm(t, s, 3);
                    HIP_TRY(launch_far(t, s));
                    tm.done();
                }
                if (!vjp_only) {
                    StageTimer tm(t, s, 4);
                    HIP_TRY(launch_near(t, a, s));
                    tm.done();
                }
            }
            t.has_forces = true;
            return FMM_OK;
        }
        fmm_status st = ensure_slots(t, std::max(t.cap_far, round_cap(mf)),
                                     std::max(t.cap_near, round_cap(mn)));
        if (st != FMM_OK)
            return st;
    }
    return fail(FMM_ERR_CAPACITY, "interaction lists did not fit after resizing");
}

fmm_status fmm_forces_vjp(fmm_tree *tree, const void *a_bar, void *x_bar, void *m_bar,
                          void *stream)
{
    if (!tree_ok(tree))
        return fail(FMM_ERR_STATE, "unknown or freed tree handle");
    if (!a_bar || !x_bar || !m_bar)
        return fail(FMM_ERR_INVALID, "a_bar, x_bar and m_bar must not be NULL");
    Tree &t = *reinterpret_cast<Tree *>(tree);
    if (!t.has_forces)
        return fail(FMM_ERR_STATE, "fmm_forces must run on this tree state before the VJP");
    if (!t.has_lists)
        return fail(FMM_ERR_STATE, "no interaction lists: call fmm_forces first");
    if (t.lists_policy == FMM_WALK_MUTUAL && !t.mw.Lown) {
        // the reverse pass of an FP32 tree recomputes the M2L sums in FP64
        void *p = nullptr;
        fmm_status st = mw_alloc(t, &p, (size_t)NLOC * t.topo.node_cap * sizeof(double));
        if (st != FMM_OK)
            return st;
        t.mw.Lown = (double *)p;
    }
    hipStream_t s = (hipStream_t)stream;
    StageTimer tm(t, s, 5);
    hipError_t e = launch_vjp(t, a_bar, x_bar, m_bar, s);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? FMM_ERR_ALLOC : FMM_ERR_HIP,
                    "reverse pass failed: %s", hipGetErrorString(e));
    tm.done();
    return FMM_OK;
}

fmm_status fmm_asymmetry_estimate(fmm_tree *tree, double m_leaf, double *out, void *stream)
{
    if (!tree_ok(tree))
        return fail(FMM_ERR_STATE, "unknown or freed tree handle");
    if (!out)
        return fail(FMM_ERR_INVALID, "out must not be NULL");
    if (!std::isfinite(m_leaf))
        return fail(FMM_ERR_INVALID, "m_leaf must be finite");
    Tree &t = *reinterpret_cast<Tree *>(tree);
    if (!t.has_forces || !t.has_lists)
        return fail(FMM_ERR_STATE, "no interaction lists for the current moments: call fmm_forces "
                                   "first");
    HIP_TRY(launch_asym(t, m_leaf, out, (hipStream_t)stream));  // out of memory -> FMM_ERR_ALLOC
    return FMM_OK;
}

fmm_status fmm_momentum_stats(const double *x, const double *v, const double *m, const void *a,
                              int32_t a_precision, int64_t n, fmm_stats *out, void *stream)
{
    if (!x || !m || !a || !out)
        return fail(FMM_ERR_INVALID, "x, m, a and out must not be NULL");
    if (n < 1)
        return fail(FMM_ERR_INVALID, "n must be positive");
    if (a_precision != FMM_FP64 && a_precision != FMM_FP32)
        return fail(FMM_ERR_INVALID, "unknown precision %d", a_precision);
    double *dev = nullptr, *host = nullptr;
    fmm_status st = stats_scratch(&dev, &host);
    if (st != FMM_OK)
        return st;
    HIP_TRY(launch_stats(x, v, m, a, a_precision == FMM_FP32, n, dev, nullptr, host,
                         (hipStream_t)stream));
    static_assert(sizeof(fmm_stats) == 16 * sizeof(double), "fmm_stats layout");
    std::memcpy(out, host, sizeof(fmm_stats));
    return FMM_OK;
}

fmm_status fmm_momentum_stats_async(const double *x, const double *v, const double *m,
                                    const void *a, int32_t a_precision, int64_t n,
                                    fmm_stats *out, void *stream)
{
    if (!x || !m || !a || !out)
        return fail(FMM_ERR_INVALID, "x, m, a and out must not be NULL");
    if (n < 1)
        return fail(FMM_ERR_INVALID, "n must be positive");
    if (a_precision != FMM_FP64 && a_precision != FMM_FP32)
        return fail(FMM_ERR_INVALID, "unknown precision %d", a_precision);
    double *dev = nullptr, *host = nullptr;
    fmm_status st = stats_scratch(&dev, &host);
    if (st != FMM_OK)
        return st;
    HIP_TRY(launch_stats(x, v, m, a, a_precision == FMM_FP32, n, dev, (double *)out, nullptr,
                         (hipStream_t)stream));
    return FMM_OK;
}

fmm_status fmm_momentum_stats_noalloc(const double *x, const double *v, const double *m,
                                      const void *a, int32_t a_precision, int64_t n,
                                      fmm_stats *out, void *stream)
{
    if (!x || !m || !a || !out)
        return fail(FMM_ERR_INVALID, "x, m, a and out must not be NULL");
    if (n < 1)
        return fail(FMM_ERR_INVALID, "n must be positive");
    if (n > NOALLOC_MAX_N)
        return fail(FMM_ERR_CAPACITY, "n = %lld exceeds the %lld particles the no-allocation "
                    "statistics accept", (long long)n, (long long)NOALLOC_MAX_N);
    if (a_precision != FMM_FP64 && a_precision != FMM_FP32)
        return fail(FMM_ERR_INVALID, "unknown precision %d", a_precision);
    double *scr = nullptr;
    HIP_TRY(stats_noalloc_scratch(&scr));
    HIP_TRY(launch_stats(x, v, m, a, a_precision == FMM_FP32, n, scr, (double *)out, nullptr,
                         (hipStream_t)stream));
    return FMM_OK;
}

fmm_status fmm_kick_drift(double *x, double *v, const void *a, int32_t a_precision, int64_t n,
                          double kick, double drift, void *stream)
{
    if (!x || !v || !a)
        return fail(FMM_ERR_INVALID, "x, v and a must not be NULL");
    if (n < 1)
        return fail(FMM_ERR_INVALID, "n must be positive");
    if (a_precision != FMM_FP64 && a_precision != FMM_FP32)
        return fail(FMM_ERR_INVALID, "unknown precision %d", a_precision);
    if (!std::isfinite(kick) || !std::isfinite(drift))
        return fail(FMM_ERR_INVALID, "kick and drift must be finite");
    HIP_TRY(launch_kick_drift(x, v, a, a_precision == FMM_FP32, n, kick, drift,
                              (hipStream_t)stream));
    return FMM_OK;
}

void fmm_tree_free(fmm_tree *tree)
{
    if (!tree_ok(tree))
        return;
    release(reinterpret_cast<Tree *>(tree));
}

fmm_status fmm_tree_info(const fmm_tree *tree, int64_t *info)
{
    if (!tree_ok(tree))
        return fail(FMM_ERR_STATE, "unknown or freed tree handle");
    if (!info)
        return fail(FMM_ERR_INVALID, "info must not be NULL");
    Tree &t = *const_cast<Tree *>(reinterpret_cast<const Tree *>(tree));
    if (t.has_lists && t.n_far < 0 && t.lists_policy == FMM_WALK_PHANTOM) {
        std::vector<int32_t> cf(t.nsinks), cn(t.nsinks);
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(cf.data(), t.far_cnt, cf.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(cn.data(), t.near_cnt, cn.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        t.n_far = t.n_near = 0;
        for (int k = 0; k < t.nsinks; ++k) {
            t.n_far += cf[k];
            t.n_near += cn[k];
        }
    }
    info[0] = t.topo.n;
    info[1] = t.topo.nnodes;
    info[2] = t.topo.nleaves;
    info[3] = t.topo.depth;
    info[4] = t.has_lists ? t.n_far : 0;
    info[5] = t.has_lists ? t.n_near : 0;
    info[6] = t.has_lists ? t.nsinks : 0;
    info[7] = t.has_lists ? 1 : 0;
    return FMM_OK;
}

fmm_status fmm_tree_device_bytes(const fmm_tree *tree, int64_t *bytes)
{
    if (!tree_ok(tree))
        return fail(FMM_ERR_STATE, "unknown or freed tree handle");
    if (!bytes)
        return fail(FMM_ERR_INVALID, "bytes must not be NULL");
    *bytes = reinterpret_cast<const Tree *>(tree)->held_bytes;
    return FMM_OK;
}

fmm_status fmm_tree_params(const fmm_tree *tree, fmm_params *p, int64_t *n)
{
    if (!tree_ok(tree))
        return fail(FMM_ERR_STATE, "unknown or freed tree handle");
    const Tree &t = *reinterpret_cast<const Tree *>(tree);
    if (p)
        *p = t.p;
    if (n)
        *n = t.topo.n;
    return FMM_OK;
}

fmm_status fmm_debug_export(const fmm_tree *tree, int32_t *perm, int32_t *first, int32_t *count,
                            int32_t *left, int32_t *right, int32_t *axis, double *rec,
                            int64_t *far_off, int32_t *far_src, int64_t *near_off,
                            int32_t *near_src, double *local)
{
    if (!tree_ok(tree))
        return fail(FMM_ERR_STATE, "unknown or freed tree handle");
    const Tree &t = *reinterpret_cast<const Tree *>(tree);
    const Topology &T = t.topo;
    const int64_t nn = T.nnodes;
    HIP_TRY(hipDeviceSynchronize());
    // the topology as the device holds it (the centre-of-mass tree has no
    // host copy)
    std::vector<int32_t> hl(nn), hnl(nn);
    HIP_TRY(hipMemcpy(hl.data(), t.left, nn * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hnl.data(), t.node_leaf, nn * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (perm)
        HIP_TRY(hipMemcpy(perm, t.perm, T.n * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (first)
        HIP_TRY(hipMemcpy(first, t.first, nn * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (count)
        HIP_TRY(hipMemcpy(count, t.count, nn * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (left)
        std::memcpy(left, hl.data(), nn * sizeof(int32_t));
    if (right)
        HIP_TRY(hipMemcpy(right, t.right, nn * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (axis) {
        HIP_TRY(hipMemcpy(axis, t.axis, nn * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int64_t v = 0; v < nn; ++v)
            if (hl[v] < 0)
                axis[v] = -1;
    }
    if (rec) {
        std::vector<double> a(NREC * nn), q(NREC * nn);
        HIP_TRY(hipMemcpy(a.data(), t.recA, a.size() * sizeof(double), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(q.data(), t.recQ, q.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int64_t v = 0; v < nn; ++v) {
            double *r = rec + 12 * v;
            r[0] = a[NREC * v + 3];
            r[1] = a[NREC * v + 0];
            r[2] = a[NREC * v + 1];
            r[3] = a[NREC * v + 2];
            r[4] = a[NREC * v + 4];
            r[5] = a[NREC * v + 5];
            for (int k = 0; k < 6; ++k)
                r[6 + k] = q[NREC * v + k];
        }
    }
    if (far_off || far_src || near_off || near_src) {
        if (!t.has_lists)
            return fail(FMM_ERR_STATE, "no interaction lists to export");
        const int ns = T.nleaves;
        std::vector<int32_t> cf(ns), cn(ns);
        if (t.lists_policy == FMM_WALK_PHANTOM)
            HIP_TRY(hipMemcpy(cf.data(), t.far_cnt, ns * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(cn.data(), t.near_cnt, ns * sizeof(int32_t), hipMemcpyDeviceToHost));
        // sinks are leaves: node-indexed CSR, entries in emission order
        auto export_lists = [&](const std::vector<int32_t> &cnt, const int32_t *dev, int64_t cap,
                                int64_t *off, int32_t *src) -> fmm_status {
            std::vector<int32_t> slots((size_t)ns * cap);
            if (src)
                HIP_TRY(hipMemcpy(slots.data(), dev, slots.size() * sizeof(int32_t),
                                  hipMemcpyDeviceToHost));
            int64_t o = 0;
            if (off)
                off[0] = 0;
            for (int64_t v = 0; v < nn; ++v) {
                int lf = hnl[v];
                if (lf >= 0) {
                    if (src)
                        std::memcpy(src + o, slots.data() + (size_t)lf * cap,
                                    cnt[lf] * sizeof(int32_t));
                    o += cnt[lf];
                }
                if (off)
                    off[v + 1] = o;
            }
            return FMM_OK;
        };
        fmm_status st = FMM_OK;
        if (t.lists_policy == FMM_WALK_PHANTOM) {
            st = export_lists(cf, t.far_src, t.cap_far, far_off, far_src);
            if (st != FMM_OK)
                return st;
        } else if (far_off || far_src) {
            // mutual walk: sorted (sink, source) keys with a CSR range per sink cell
            const MutualLists &M = t.mw;
            std::vector<int64_t> se(2 * nn);
            std::vector<uint64_t> keys(M.n_far);
            HIP_TRY(hipMemcpy(se.data(), M.fstart, nn * sizeof(int64_t), hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(se.data() + nn, M.fend, nn * sizeof(int64_t),
                              hipMemcpyDeviceToHost));
            if (M.n_far)
                HIP_TRY(hipMemcpy(keys.data(), M.far_sorted, keys.size() * sizeof(uint64_t),
                                  hipMemcpyDeviceToHost));
            const uint64_t mask = (1ull << mutual_key_bits(t)) - 1ull;
            int64_t o = 0;
            if (far_off)
                far_off[0] = 0;
            for (int64_t v = 0; v < nn; ++v) {
                for (int64_t k = se[v]; k < se[nn + v]; ++k, ++o)
                    if (far_src)
                        far_src[o] = (int32_t)(keys[k] & mask);
                if (far_off)
                    far_off[v + 1] = o;
            }
        }
        st = export_lists(cn, t.near_src, t.cap_near, near_off, near_src);
        if (st != FMM_OK)
            return st;
    }
    if (local) {
        std::vector<double> Lh(NLOC * nn);
        HIP_TRY(hipMemcpy(Lh.data(), t.L, Lh.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int64_t v = 0; v < nn; ++v)
            for (int k = 0; k < 19; ++k)
                local[19 * v + k] = (t.has_forces && hl[v] < 0) ? Lh[NLOC * v + k] : 0.0;
    }
    return FMM_OK;
}

fmm_status fmm_debug_import(fmm_tree *tree, const double *x, const double *m, const double *h,
                            const int32_t *perm, const int32_t *first, const int32_t *count,
                            const int32_t *left, const int32_t *right, const double *rec,
                            const int64_t *far_off, const int32_t *far_src,
                            const int64_t *near_off, const int32_t *near_src, void *stream)
{
    if (!tree_ok(tree))
        return fail(FMM_ERR_STATE, "unknown or freed tree handle");
    if (!x || !m || !h || !perm || !first || !count || !left || !right || !rec || !far_off ||
        !near_off)
        return fail(FMM_ERR_INVALID, "x, m, h, perm, topology, rec and the list offsets must "
                                     "not be NULL");
    Tree &t = *reinterpret_cast<Tree *>(tree);
    if (!t.has_tree)
        return fail(FMM_ERR_STATE, "the tree has not been built");
    if (t.p.tree != FMM_TREE_MEDIAN || t.p.walk != FMM_WALK_PHANTOM)
        return fail(FMM_ERR_INVALID, "import needs a median-split tree with the leaf <- cell walk");
    const Topology &T = t.topo;
    const int64_t n = T.n, nn = T.nnodes, nl = T.nleaves;
    // the imported tree must have this tree's shape (node ids in the same order)
    for (int64_t v = 0; v < nn; ++v)
        if (first[v] != T.first[v] || count[v] != T.count[v] || left[v] != T.left[v] ||
            right[v] != T.right[v])
            return fail(FMM_ERR_INVALID, "imported topology differs from the tree's at node %lld",
                        (long long)v);
    {
        std::vector<uint8_t> seen(n, 0);
        for (int64_t p = 0; p < n; ++p) {
            const int32_t i = perm[p];
            if (i < 0 || i >= n || seen[i])
                return fail(FMM_ERR_INVALID, "perm is not a permutation of [0, n)");
            seen[i] = 1;
        }
    }
    int64_t mf = 0, mnr = 0;
    for (int pass = 0; pass < 2; ++pass) {
        const int64_t *off = pass ? near_off : far_off;
        const int32_t *src = pass ? near_src : far_src;
        if (off[0] != 0)
            return fail(FMM_ERR_INVALID, "list offsets must start at 0");
        for (int64_t v = 0; v < nn; ++v) {
            const int64_t c = off[v + 1] - off[v];
            if (c < 0 || (c > 0 && (T.left[v] >= 0 || !src)))
                return fail(FMM_ERR_INVALID, "lists must be CSR over leaf sinks (node %lld)",
                            (long long)v);
            for (int64_t k = off[v]; k < off[v + 1]; ++k)
                if (src[k] < 0 || src[k] >= nn || (pass && T.left[src[k]] >= 0))
                    return fail(FMM_ERR_INVALID, "list entry %lld of node %lld is not a valid %s",
                                (long long)k, (long long)v, pass ? "leaf" : "cell");
            (pass ? mnr : mf) = std::max(pass ? mnr : mf, c);
        }
    }
    if (t.p.list_capacity > 0 && (mf > t.p.list_capacity || mnr > t.p.list_capacity))
        return fail(FMM_ERR_CAPACITY, "imported lists need %lld / %lld entries; list_capacity is "
                    "%lld", (long long)mf, (long long)mnr, (long long)t.p.list_capacity);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
    t.has_moments = t.has_lists = t.has_forces = false;
    t.pieces_valid = false;
    t.split_lists = false;
    fmm_status st = ensure_slots(t, std::max<int64_t>(mf, 1), std::max<int64_t>(mnr, 1));
    if (st != FMM_OK)
        return st;
    // host images of the slots, counts and records
    std::vector<int32_t> fs((size_t)nl * t.cap_far, 0), ns((size_t)nl * t.cap_near, 0);
    std::vector<int32_t> fc(nl), nc(nl);
    int64_t tf = 0, tn = 0;
    for (int64_t lf = 0; lf < nl; ++lf) {
        const int32_t v = T.leaf_node[lf];
        fc[lf] = (int32_t)(far_off[v + 1] - far_off[v]);
        nc[lf] = (int32_t)(near_off[v + 1] - near_off[v]);
        for (int32_t k = 0; k < fc[lf]; ++k)
            fs[(size_t)lf * t.cap_far + k] = far_src[far_off[v] + k];
        for (int32_t k = 0; k < nc[lf]; ++k)
            ns[(size_t)lf * t.cap_near + k] = near_src[near_off[v] + k];
        tf += fc[lf];
        tn += nc[lf];
    }
    void *rdev = nullptr;
    HIP_TRY(tree_malloc(t, &rdev, (size_t)nn * 12 * sizeof(double)));
    hipError_t e = hipMemcpy(rdev, rec, (size_t)nn * 12 * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(t.perm, perm, (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(t.far_src, fs.data(), fs.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(t.near_src, ns.data(), ns.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(t.far_cnt, fc.data(), fc.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(t.near_cnt, nc.data(), nc.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = launch_import(t, x, m, h, (const double *)rdev, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    tree_free(t, rdev);
    if (e != hipSuccess)
        return fail(FMM_ERR_HIP, "import failed: %s", hipGetErrorString(e));
    t.has_moments = true;
    t.has_lists = true;
    t.has_transposed = false;
    t.lists_policy = FMM_WALK_PHANTOM;
    t.nsinks = (int)nl;
    t.n_far = tf;
    t.n_near = tn;
    return FMM_OK;
}

fmm_status fmm_set_timing(fmm_tree *tree, int32_t on)
{
    if (!tree_ok(tree))
        return fail(FMM_ERR_STATE, "unknown or freed tree handle");
    Tree &t = *reinterpret_cast<Tree *>(tree);
    for (int k = 0; k < 8; ++k) {
        harvest(t, k);
        t.acc_ms[k] = 0.0;
        t.acc_n[k] = 0;
    }
    t.timing = on != 0;
    return FMM_OK;
}

fmm_status fmm_stage_times(const fmm_tree *tree, double *ms)
{
    if (!tree_ok(tree))
        return fail(FMM_ERR_STATE, "unknown or freed tree handle");
    if (!ms)
        return fail(FMM_ERR_INVALID, "ms must not be NULL");
    Tree &t = *const_cast<Tree *>(reinterpret_cast<const Tree *>(tree));
    double tot = 0.0;
    for (int k = 0; k < 7; ++k) {
        harvest(t, k);
        ms[k] = t.acc_n[k] ? t.acc_ms[k] / (double)t.acc_n[k] : 0.0;
        tot += ms[k];
    }
    ms[7] = tot;
    return FMM_OK;
}

}  // extern "C"
