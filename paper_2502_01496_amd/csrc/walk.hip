// Interaction lists on gfx950.
//
// Leaf <- cell walk of the paper (Sec. 4: partners are sought for leaf cells
// only, each with the one-sided opening criterion).  For a sink leaf a and a
// cell b, with r = c_a - c_b:
//   eq. (4)  opened if  s_b * s_b > theta^2 * r^2;
//   eq. (5)  opened if  r^2 < (s_a + s_b + R_kern * max(h_a, h_b))^2.
// A cell meeting neither is far (M2L); an opened leaf is near (direct sum);
// an opened internal cell is descended.
//
// The lists live in fixed per-leaf slots (capacities grown by the host when a
// count exceeds them), so one pass both counts and writes.
//
// Compiled with -ffp-contract=off so the criteria are evaluated with exactly
// the operations of their definition.
#include <algorithm>

#include "fmm_internal.h"

namespace fmm {

constexpr int WALK_STACK = 96;
// a DFS holds at most depth + 1 entries
static_assert(COM_MAX_DEPTH + 2 <= WALK_STACK, "narrow walk stack shorter than the deepest tree");
constexpr int WIDE_STACK = 1024;

// Cell b's centre, size s_b, h_max,b and child ids (left < 0: leaf), read
// from its one 64-byte record once per visit.
struct CellRec {
    double c0, c1, c2, sb, hb;
    int left, right;
};

__device__ __forceinline__ CellRec load_cell(const double *recA, int b)
{
    const double *rb = recA + (int64_t)NREC * b;
    const double2 a = *(const double2 *)rb;
    const double c2 = rb[2];
    const double2 q = *(const double2 *)(rb + 4);
    const int2 kids = *(const int2 *)(rb + REC_KIDS);
    return {a.x, a.y, c2, q.x, q.y, kids.x, kids.y};
}

__device__ __forceinline__ bool opened(double ca0, double ca1, double ca2, double sa, double ha,
                                       const CellRec &cb, double theta2, double r_kern)
{
    const double dx = ca0 - cb.c0, dy = ca1 - cb.c1, dz = ca2 - cb.c2;
    const double sb = cb.sb, hb = cb.hb;
    const double r2 = (dx * dx + dy * dy) + dz * dz;
    const bool open4 = sb * sb > theta2 * r2;
    const double tt = (sa + sb) + r_kern * (ha > hb ? ha : hb);
    const bool open5 = r2 < tt * tt;
    return open4 || open5;
}

// Group walk: one wavefront walks WG consecutive sink leaves (in pre-order,
// a compact group) together.  A stack entry carries a cell and the mask of
// the group's leaves for which it is pending (all of them had its parent
// opened); each step pops up to 64 entries, loads each cell's record once and
// applies the criteria for every pending leaf, writes the far / near entries
// of each leaf with ballot compaction, and pushes the children with the mask
// of the leaves that opened the cell.  Per leaf the decisions, and so the
// lists, are those of the single-leaf walk.  A full stack marks the group's
// leaves for the exact narrow-stack walk.
//
// A group still walking after `budget` steps stops and is queued for
// k_walk_heavy (its counts read -2 until then): the few groups whose leaves
// see most of the tree would otherwise hold one wavefront for thousands of
// dependent steps.
constexpr int WG = 4;
constexpr int WALK_WAVES = 1;  // one wavefront per workgroup

__global__ __launch_bounds__(64 * WALK_WAVES) void k_walk_group(
    const double *__restrict__ recA, const int32_t *__restrict__ leaf_node, int nleaves,
    double theta2, double r_kern, int32_t *far_src, int cap_far, int32_t *near_src,
    int cap_near, int32_t *far_cnt, int32_t *near_cnt, int32_t *stack_overflow, int stack_limit,
    int budget, int32_t *nheavy, int32_t *heavy)
{
    __shared__ int32_t stk[WALK_WAVES][WIDE_STACK];
    __shared__ uint8_t msk[WALK_WAVES][WIDE_STACK];
    const int w = threadIdx.x >> 6, lane = lane_id();
    const int g0 = __builtin_amdgcn_readfirstlane(
        (xcd_block(blockIdx.x, gridDim.x) * WALK_WAVES + w) * WG);
    if (g0 >= nleaves)
        return;
    const int ng = min(WG, nleaves - g0);
    const uint64_t lt = lanemask_lt();
    double ca0[WG], ca1[WG], ca2[WG], sa[WG], ha[WG];
#pragma unroll
    for (int g = 0; g < WG; ++g) {
        const double *ra = recA + (int64_t)NREC * leaf_node[g0 + min(g, ng - 1)];
        ca0[g] = ra[0];
        ca1[g] = ra[1];
        ca2[g] = ra[2];
        sa[g] = ra[4];
        ha[g] = ra[5];
    }
    int nf[WG], nn[WG];
#pragma unroll
    for (int g = 0; g < WG; ++g)
        nf[g] = nn[g] = 0;
    int sp = 1, steps = 0;
    bool ovf = false, hvy = false;
    if (lane == 0) {
        stk[w][0] = 0;
        msk[w][0] = (uint8_t)((1u << ng) - 1u);
    }
    while (sp > 0) {
        if (++steps > budget) {
            hvy = true;
            break;
        }
        const int take = sp < 64 ? sp : 64;
        const int base = sp - take;
        const bool act = lane < take;
        const int b = act ? stk[w][base + lane] : 0;
        const uint32_t m = act ? msk[w][base + lane] : 0u;
        sp = base;
        // the record is read once for all leaves of the group (idle lanes
        // read the root's)
        const CellRec cb = load_cell(recA, b);
        const int lb = cb.left, rgt = cb.right;
        uint32_t open = 0;
#pragma unroll
        for (int g = 0; g < WG; ++g) {
            const bool live = (m >> g) & 1u;
            const bool op =
                opened(ca0[g], ca1[g], ca2[g], sa[g], ha[g], cb, theta2, r_kern) && live;
            const bool far = live && !op;
            const bool nea = op && lb < 0;
            open |= (op ? 1u : 0u) << g;
            const uint64_t mf = __ballot(far), mn = __ballot(nea);
            if (far) {
                const int k = nf[g] + __popcll(mf & lt);
                if (k < cap_far)
                    far_src[(int64_t)(g0 + g) * cap_far + k] = b;
            }
            if (nea) {
                const int k = nn[g] + __popcll(mn & lt);
                if (k < cap_near)
                    near_src[(int64_t)(g0 + g) * cap_near + k] = b;
            }
            nf[g] += __popcll(mf);
            nn[g] += __popcll(mn);
        }
        const bool desc = open != 0u && lb >= 0;
        const uint64_t md = __ballot(desc);
        const int nd = __popcll(md);
        if (sp + 2 * nd > stack_limit) {
            ovf = true;
            break;
        }
        if (desc) {
            const int k = sp + 2 * __popcll(md & lt);
            stk[w][k] = rgt;
            msk[w][k] = (uint8_t)open;
            stk[w][k + 1] = lb;
            msk[w][k + 1] = (uint8_t)open;
        }
        sp += 2 * nd;
    }
    if (lane < ng) {
        int f = 0, q = 0;
#pragma unroll
        for (int g = 0; g < WG; ++g)
            if (g == lane) {
                f = nf[g];
                q = nn[g];
            }
        if (hvy) {
            far_cnt[g0 + lane] = -2;
            near_cnt[g0 + lane] = 0;
        } else if (ovf) {
            // marked for the narrow-stack walk; until then the leaf has no
            // list entries (the force kernels may run before that walk)
            far_cnt[g0 + lane] = -1;
            near_cnt[g0 + lane] = 0;
        } else {
            far_cnt[g0 + lane] = f;
            near_cnt[g0 + lane] = q;
        }
    }
    if (ovf && lane == 0)
        atomicOr(stack_overflow, 1);
    if (hvy && lane == 0)
        heavy[atomicAdd(nheavy, 1)] = g0 / WG;
}

// The queued groups, one workgroup of HEAVY_WAVES wavefronts each: the same
// walk with up to 64 HEAVY_WAVES stack entries per step, a shared LDS stack,
// and each step's far / near entries and pushes placed in stack order (the
// wavefronts' ballot counts scanned through LDS), so the lists come out in a
// fixed order.  A full stack (at most HEAVY_STACK entries, stack_limit) marks
// the group's leaves for the narrow walk.
constexpr int HEAVY_WAVES = 16;
constexpr int HEAVY_STACK = 1536 * HEAVY_WAVES;  // 120 KB of LDS with the masks

__global__ __launch_bounds__(64 * HEAVY_WAVES) void k_walk_heavy(
    const double *__restrict__ recA, const int32_t *__restrict__ leaf_node, int nleaves,
    double theta2, double r_kern, int32_t *far_src, int cap_far, int32_t *near_src,
    int cap_near, int32_t *far_cnt, int32_t *near_cnt, int32_t *stack_overflow,
    int stack_limit, const int32_t *nheavy, const int32_t *__restrict__ heavy)
{
    constexpr int NT = 64 * HEAVY_WAVES;
    __shared__ int32_t stk[HEAVY_STACK];
    __shared__ uint8_t msk[HEAVY_STACK];
    __shared__ int32_t wc[HEAVY_WAVES][2 * WG + 1];  // per wavefront: far, near per leaf; pushes
    __shared__ int32_t wpre[HEAVY_WAVES][2 * WG + 1];  // the same, summed over earlier wavefronts
    __shared__ int32_t wtot[2 * WG + 1];               // and over all of them
    const int t = threadIdx.x, w = t >> 6, lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const int nh = *nheavy;
    for (int h = blockIdx.x; h < nh; h += gridDim.x) {
        const int g0 = heavy[h] * WG;
        const int ng = min(WG, nleaves - g0);
        double ca0[WG], ca1[WG], ca2[WG], sa[WG], ha[WG];
#pragma unroll
        for (int g = 0; g < WG; ++g) {
            const double *ra = recA + (int64_t)NREC * leaf_node[g0 + min(g, ng - 1)];
            ca0[g] = ra[0];
            ca1[g] = ra[1];
            ca2[g] = ra[2];
            sa[g] = ra[4];
            ha[g] = ra[5];
        }
        int nf[WG], nn[WG];  // the same in every thread
#pragma unroll
        for (int g = 0; g < WG; ++g)
            nf[g] = nn[g] = 0;
        int sp = 1;
        bool ovf = false;
        if (t == 0) {
            stk[0] = 0;
            msk[0] = (uint8_t)((1u << ng) - 1u);
        }
        __syncthreads();
        while (sp > 0) {
            const int take = sp < NT ? sp : NT;
            const int base = sp - take;
            const bool act = t < take;
            const int b = act ? stk[base + t] : 0;
            const uint32_t m = act ? msk[base + t] : 0u;
            sp = base;
            const CellRec cb = load_cell(recA, b);
            const int lb = cb.left, rgt = cb.right;
            uint32_t open = 0;
            uint64_t mf[WG], mn[WG];
            bool far[WG], nea[WG];
#pragma unroll
            for (int g = 0; g < WG; ++g) {
                const bool live = (m >> g) & 1u;
                const bool op =
                    opened(ca0[g], ca1[g], ca2[g], sa[g], ha[g], cb, theta2, r_kern) && live;
                far[g] = live && !op;
                nea[g] = op && lb < 0;
                open |= (op ? 1u : 0u) << g;
                mf[g] = __ballot(far[g]);
                mn[g] = __ballot(nea[g]);
            }
            const bool desc = open != 0u && lb >= 0;
            const uint64_t md = __ballot(desc);
            if (lane == 0) {
#pragma unroll
                for (int g = 0; g < WG; ++g) {
                    wc[w][g] = __popcll(mf[g]);
                    wc[w][WG + g] = __popcll(mn[g]);
                }
                wc[w][2 * WG] = __popcll(md);
            }
            __syncthreads();  // the pops are read and the counts published
            if (t < 2 * WG + 1) {
                // column t: exclusive scan over the wavefronts, then the total
                int run = 0;
                for (int v = 0; v < HEAVY_WAVES; ++v) {
                    const int c = wc[v][t];
                    wpre[v][t] = run;
                    run += c;
                }
                wtot[t] = run;
            }
            __syncthreads();
            const int td = wtot[2 * WG], bd = wpre[w][2 * WG];
#pragma unroll
            for (int g = 0; g < WG; ++g) {
                if (far[g]) {
                    const int k = nf[g] + wpre[w][g] + __popcll(mf[g] & lt);
                    if (k < cap_far)
                        far_src[(int64_t)(g0 + g) * cap_far + k] = b;
                }
                if (nea[g]) {
                    const int k = nn[g] + wpre[w][WG + g] + __popcll(mn[g] & lt);
                    if (k < cap_near)
                        near_src[(int64_t)(g0 + g) * cap_near + k] = b;
                }
                nf[g] += wtot[g];
                nn[g] += wtot[WG + g];
            }
            if (sp + 2 * td > stack_limit) {
                ovf = true;
                break;
            }
            if (desc) {
                const int k = sp + 2 * (bd + __popcll(md & lt));
                stk[k] = rgt;
                msk[k] = (uint8_t)open;
                stk[k + 1] = lb;
                msk[k + 1] = (uint8_t)open;
            }
            sp += 2 * td;
            __syncthreads();  // the pushes are visible and wc may be reused
        }
        if (t < ng) {
            int f = 0, q = 0;
#pragma unroll
            for (int g = 0; g < WG; ++g)
                if (g == t) {
                    f = nf[g];
                    q = nn[g];
                }
            far_cnt[g0 + t] = ovf ? -1 : f;
            near_cnt[g0 + t] = ovf ? 0 : q;
        }
        if (ovf && t == 0)
            atomicOr(stack_overflow, 1);
        __syncthreads();  // the stack is reused by the next group
    }
}

// Fallback for leaves whose wide walk overflowed its stack (far_cnt == -1):
// 64 consecutive leaves per wave share one DFS stack whose entries carry the
// mask of lanes that opened the parent (depth-bounded), writing the same slots.
__global__ __launch_bounds__(256) void k_walk_p(
    const double *__restrict__ recA, const int32_t *__restrict__ leaf_node, int nleaves,
    double theta2, double r_kern, int32_t *far_src, int cap_far, int32_t *near_src,
    int cap_near, int32_t *far_cnt, int32_t *near_cnt, int32_t *maxcnt)
{
    __shared__ int32_t stk_node[4][WALK_STACK];
    __shared__ uint64_t stk_mask[4][WALK_STACK];
    const int w = threadIdx.x >> 6, lane = lane_id();
    const int leaf = blockIdx.x * 256 + threadIdx.x;
    const bool valid = leaf < nleaves && far_cnt[leaf] < 0;
    const int a = valid ? leaf_node[leaf] : 0;
    const double *ra = recA + (int64_t)NREC * a;
    const double ca0 = ra[0], ca1 = ra[1], ca2 = ra[2], sa = ra[4], ha = ra[5];
    int32_t *fo = far_src + (int64_t)(valid ? leaf : 0) * cap_far;
    int32_t *no = near_src + (int64_t)(valid ? leaf : 0) * cap_near;
    int nf = 0, nn = 0;
    const uint64_t vmask = __ballot(valid);
    if (vmask == 0ull)
        return;
    int sp = 1;
    if (lane == 0) {
        stk_node[w][0] = 0;
        stk_mask[w][0] = vmask;
    }
    while (sp > 0) {
        --sp;
        const int b = __builtin_amdgcn_readfirstlane(stk_node[w][sp]);
        const uint64_t mask = stk_mask[w][sp];
        const CellRec cb = load_cell(recA, b);
        const int lb = cb.left;
        const bool active = (mask >> lane) & 1ull;
        bool descend = false;
        if (active) {
            if (!opened(ca0, ca1, ca2, sa, ha, cb, theta2, r_kern)) {
                if (nf < cap_far)
                    fo[nf] = b;
                ++nf;
            } else if (lb < 0) {
                if (nn < cap_near)
                    no[nn] = b;
                ++nn;
            } else {
                descend = true;
            }
        }
        const uint64_t om = __ballot(descend);
        if (om != 0ull) {
            if (lane == 0) {
                stk_node[w][sp] = cb.right;
                stk_mask[w][sp] = om;
                stk_node[w][sp + 1] = lb;
                stk_mask[w][sp + 1] = om;
            }
            sp += 2;
        }
    }
    if (valid) {
        far_cnt[leaf] = nf;
        near_cnt[leaf] = nn;
    }
}

__global__ void k_walk_init(int32_t *maxcnt) {
    if (threadIdx.x < 4)
        maxcnt[threadIdx.x] = 0;
}

// Largest far and near list over all leaves: per-workgroup maxima, then one
// atomicMax per workgroup into maxcnt[0..1] (zeroed by k_walk_init; the
// overflow flag in maxcnt[2] is left as the walk set it).
constexpr int LIST_MAX_BLOCKS = 64;

__global__ __launch_bounds__(1024) void k_list_max(const int32_t *__restrict__ far_cnt,
                                                   const int32_t *__restrict__ near_cnt, int n,
                                                   int32_t *maxcnt)
{
    __shared__ int32_t sh[2][16];
    int mf = 0, mn = 0;
    for (int i = blockIdx.x * 1024 + threadIdx.x; i < n; i += gridDim.x * 1024) {
        mf = max(mf, far_cnt[i]);
        mn = max(mn, near_cnt[i]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        mf = max(mf, __shfl_xor(mf, off));
        mn = max(mn, __shfl_xor(mn, off));
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        sh[0][w] = mf;
        sh[1][w] = mn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 16; ++i) {
            mf = max(mf, sh[0][i]);
            mn = max(mn, sh[1][i]);
        }
        atomicMax(&maxcnt[0], mf);
        atomicMax(&maxcnt[1], mn);
    }
}

hipError_t launch_walk(Tree &t, hipStream_t s)
{
    const Topology &T = t.topo;
    const double theta2 = t.p.theta * t.p.theta;
    const int nl = T.nleaves;
    k_walk_init<<<1, 64, 0, s>>>(t.walk_flags);
    const int groups = (nl + WG - 1) / WG;
    k_walk_group<<<(groups + WALK_WAVES - 1) / WALK_WAVES, 64 * WALK_WAVES, 0, s>>>(
        t.recA, t.leaf_node, nl, theta2, t.p.r_kern, t.far_src, (int)t.cap_far,
        t.near_src, (int)t.cap_near, t.far_cnt, t.near_cnt, t.walk_flags + 2,
        std::min(std::max(t.wide_stack_limit, 2), WIDE_STACK), std::max(t.walk_budget, 1),
        t.walk_flags + 3, t.walk_heavy);
    k_walk_heavy<<<std::min(groups, 4096 / HEAVY_WAVES), 64 * HEAVY_WAVES, 0, s>>>(
        t.recA, t.leaf_node, nl, theta2, t.p.r_kern, t.far_src, (int)t.cap_far, t.near_src,
        (int)t.cap_near, t.far_cnt, t.near_cnt, t.walk_flags + 2,
        std::min(std::max(t.wide_stack_limit, 2), HEAVY_STACK), t.walk_flags + 3, t.walk_heavy);
    k_list_max<<<std::min(LIST_MAX_BLOCKS, (nl + 1023) / 1024), 1024, 0, s>>>(t.far_cnt, t.near_cnt,
                                                                           nl, t.walk_flags);
    return hipGetLastError();
}

hipError_t launch_walk_fallback(Tree &t, hipStream_t s)
{
    const Topology &T = t.topo;
    const double theta2 = t.p.theta * t.p.theta;
    const int nl = T.nleaves;
    k_walk_p<<<(nl + 255) / 256, 256, 0, s>>>(t.recA, t.leaf_node, nl, theta2,
                                               t.p.r_kern, t.far_src, (int)t.cap_far, t.near_src,
                                               (int)t.cap_near, t.far_cnt, t.near_cnt,
                                               t.walk_flags);
    k_list_max<<<std::min(LIST_MAX_BLOCKS, (nl + 1023) / 1024), 1024, 0, s>>>(t.far_cnt, t.near_cnt,
                                                                           nl, t.walk_flags);
    return hipGetLastError();
}

}  // namespace fmm
