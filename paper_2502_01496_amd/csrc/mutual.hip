// Mutual (symmetric) dual-tree walk on gfx950.
//
// Sec. 7 of the paper traces the momentum error of the leaf <- cell walk to
// interactions that are formed in one direction only, and names symmetric
// opening criteria as the remedy.  Here a pair of cells (A, B) is well
// separated iff
//   (s_A + s_B)^2 <= theta^2 r^2   and   r^2 >= (s_A + s_B + R_kern max(h_A, h_B))^2
// (the second condition is the negation of eq. (5)), with r = |c_A - c_B|.
// Starting from the pairs (left child, right child) of every internal cell,
// a pair that is well separated interacts through M2L in both directions;
// a pair of leaves that is not goes to the near field in both directions;
// otherwise the cell with the larger s (A on ties; never a leaf) is split and
// both halves are paired with the other cell.  Every leaf is also near to
// itself.  Every particle pair is then covered exactly once, by a far pair
// or a near pair of cells.
//
// GPU form: breadth-first expansion of the pair frontier, one launch per
// two levels of the recursion with a fixed grid (counts stay on the device), and
// wavefront-aggregated appends to the next frontier and to the far / near
// pair buffers.  The pairs are then sorted by the key (sink, source), which
// makes the lists independent of the order of the appends: far lists become
// CSR ranges of sink cells, near lists fill the per-leaf slots read by the
// near-field kernel.
//
// Compiled with -ffp-contract=off so the criterion is evaluated with exactly
// the operations of its definition.
#include <algorithm>

#include "fmm_internal.h"

namespace fmm {

constexpr int MW_GRID = 1024;  // workgroups of a frontier step (grid-stride)

// A cell's centre, s and h_max (the fields the criterion reads), its child
// ids (left < 0: leaf) and leaf index, all from its one 64-byte record.
struct MwCell {
    double c0, c1, c2, s, h;
    int left, right, leaf;
};

__device__ __forceinline__ MwCell load_mw(const double *recA, int v)
{
    const double *r = recA + (int64_t)NREC * v;
    const double2 a = *(const double2 *)r;
    const double2 q = *(const double2 *)(r + 4);
    const int4 t = *(const int4 *)(r + REC_KIDS);  // kids (slot 6), leaf index (slot 7)
    return {a.x, a.y, r[2], q.x, q.y, t.x, t.y, t.z};
}

__device__ __forceinline__ bool separated(const MwCell &A, const MwCell &B, double theta2,
                                          double r_kern)
{
    const double dx = A.c0 - B.c0, dy = A.c1 - B.c1, dz = A.c2 - B.c2;
    const double r2 = (dx * dx + dy * dy) + dz * dz;
    const double sa = A.s, sb = B.s, ha = A.h, hb = B.h;
    const double ss = sa + sb;
    const bool ok4 = theta2 * r2 >= ss * ss;
    const double tt = ss + r_kern * (ha > hb ? ha : hb);
    const bool ok5 = r2 >= tt * tt;
    return ok4 && ok5;
}

__global__ void k_mw_zero(unsigned long long *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        p[i] = 0ull;
}

// Seed (no atomics: the seeds are known): the (left, right) pair of every
// internal cell, and the self pair of every leaf (near count 1).
__global__ __launch_bounds__(256) void k_mw_init(
    const int32_t *__restrict__ left, const int32_t *__restrict__ right,
    const int32_t *__restrict__ int_nodes, int n_int, const int32_t *__restrict__ leaf_node,
    int nleaves, int lbits, int2 *tout, int64_t cap_task, uint64_t *nkeys, int64_t cap_n,
    int32_t *near_cnt, unsigned long long *cnt)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n_int && i < cap_task) {
        const int v = int_nodes[i];
        tout[i] = make_int2(left[v], right[v]);
    }
    if (i < nleaves) {
        near_cnt[i] = 1;
        if (i < cap_n)
            nkeys[i] = ((uint64_t)i << lbits) | (uint64_t)i;
    }
    if (i == 0) {
        cnt[MW_IT] = (unsigned long long)n_int;
        cnt[MW_NNEAR] = (unsigned long long)nleaves;
        cnt[MW_FLAGS] = (n_int > cap_task ? 1ull : 0ull) | (nleaves > cap_n ? 4ull : 0ull);
    }
}

// Block-wide exclusive offsets of three per-thread counts, with one atomic
// per counter per workgroup of 256 threads (same-address atomics from every
// wavefront would serialise in L2).
__device__ __forceinline__ void block_append3(const uint32_t (&v)[3],
                                              unsigned long long *const (&ctr)[3], uint64_t (&pos)[3])
{
    __shared__ uint32_t wsum[3][4];
    __shared__ unsigned long long gbase[3];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t inc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        inc[c] = v[c];
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc[c], off);
            if (lane >= off)
                inc[c] += o;
        }
    }
    if (lane == 63) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            wsum[c][w] = inc[c];
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int c = threadIdx.x;
        const uint32_t tot = wsum[c][0] + wsum[c][1] + wsum[c][2] + wsum[c][3];
        gbase[c] = tot ? atomicAdd(ctr[c], (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        uint32_t woff = 0;
        for (int k = 0; k < w; ++k)
            woff += wsum[c][k];
        pos[c] = gbase[c] + woff + inc[c] - v[c];
    }
    __syncthreads();  // wsum / gbase are reused by the next call
}

// Classification of a pair (A, B): 0 none, 1 far, 2 near, 3 split A, 4 split B;
// op: the two leaf indices (near) or the split cell's children (split).
__device__ __forceinline__ uint32_t mw_classify(const MwCell &A, const MwCell &B, double theta2,
                                                double r_kern, int2 &op)
{
    uint32_t c;
    if (separated(A, B, theta2, r_kern))
        c = 1;
    else if (A.left < 0 && B.left < 0)
        c = 2;
    else
        c = (B.left < 0 || (A.left >= 0 && A.s >= B.s)) ? 3 : 4;
    op = c == 2 ? make_int2(A.leaf, B.leaf)
                : (c == 3 ? make_int2(A.left, A.right) : make_int2(B.left, B.right));
    return c;
}

// Two levels of the pair recursion per launch: frontier cnt[MW_IT + it] ->
// cnt[MW_IT + it + 1].  A thread classifies its pair; if one cell of it is
// split, it classifies the two child pairs at once (the other cell's record
// is already loaded), so a pair leaves far / near output and at most four
// grandchild pairs for the next launch.  A workgroup takes MW_K x 256
// consecutive pairs per round and reserves the outputs of the whole round
// with one atomic per output buffer.
constexpr int MW_K = 2;

__global__ __launch_bounds__(256) void k_mw_step(
    const int2 *__restrict__ tin, int2 *tout, int it, int64_t cap_task,
    const double *__restrict__ recA, double theta2, double r_kern, int bits, int lbits,
    uint64_t *fkeys, int64_t cap_f, uint64_t *nkeys, int64_t cap_n, int32_t *near_cnt,
    unsigned long long *cnt)
{
    const int64_t nin = min((int64_t)cnt[MW_IT + it], cap_task);
    unsigned long long *const ctr[3] = {&cnt[MW_NFAR], &cnt[MW_NNEAR], &cnt[MW_IT + it + 1]};
    const int t = threadIdx.x;
    for (int64_t r0 = (int64_t)blockIdx.x * (256 * MW_K); r0 < nin;
         r0 += (int64_t)gridDim.x * (256 * MW_K)) {
        // per input pair k: the pair itself (slot 0) and, when it splits, its
        // two child pairs (slots 1, 2); pairs past the frontier's end re-read
        // its last pair and are classified 0
        int2 pr[MW_K][3], op[MW_K][3];
        uint32_t cd[MW_K][3];
        MwCell A[MW_K], B[MW_K];
#pragma unroll
        for (int k = 0; k < MW_K; ++k) {
            pr[k][0] = tin[min(r0 + k * 256 + t, nin - 1)];
            A[k] = load_mw(recA, pr[k][0].x);
            B[k] = load_mw(recA, pr[k][0].y);
        }
        MwCell C0[MW_K], C1[MW_K];
        bool sa[MW_K];
#pragma unroll
        for (int k = 0; k < MW_K; ++k) {
            cd[k][0] = r0 + k * 256 + t < nin ? mw_classify(A[k], B[k], theta2, r_kern, op[k][0])
                                              : 0u;
            cd[k][1] = cd[k][2] = 0u;
            sa[k] = cd[k][0] == 3;
            // children of the split cell (loads issued for both pairs together)
            const int c0 = cd[k][0] >= 3 ? op[k][0].x : pr[k][0].x;
            const int c1 = cd[k][0] >= 3 ? op[k][0].y : pr[k][0].x;
            C0[k] = load_mw(recA, c0);
            C1[k] = load_mw(recA, c1);
        }
#pragma unroll
        for (int k = 0; k < MW_K; ++k) {
            if (cd[k][0] >= 3) {
                const int o = sa[k] ? pr[k][0].y : pr[k][0].x;
                const MwCell &O = sa[k] ? B[k] : A[k];
                pr[k][1] = sa[k] ? make_int2(op[k][0].x, o) : make_int2(o, op[k][0].x);
                pr[k][2] = sa[k] ? make_int2(op[k][0].y, o) : make_int2(o, op[k][0].y);
                cd[k][1] = sa[k] ? mw_classify(C0[k], O, theta2, r_kern, op[k][1])
                                 : mw_classify(O, C0[k], theta2, r_kern, op[k][1]);
                cd[k][2] = sa[k] ? mw_classify(C1[k], O, theta2, r_kern, op[k][2])
                                 : mw_classify(O, C1[k], theta2, r_kern, op[k][2]);
            }
        }
        uint32_t num[3] = {0u, 0u, 0u};
#pragma unroll
        for (int k = 0; k < MW_K; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                num[0] += cd[k][j] == 1 ? 2u : 0u;
                num[1] += cd[k][j] == 2 ? 2u : 0u;
                num[2] += (j > 0 && cd[k][j] >= 3) ? 2u : 0u;
            }
        uint64_t pos[3];
        block_append3(num, ctr, pos);
        uint32_t ovf = 0;
#pragma unroll
        for (int k = 0; k < MW_K; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const uint32_t c = cd[k][j];
                const int a = pr[k][j].x, b = pr[k][j].y;
                // every reserved slot below a capacity is written, so a consumer
                // that clamps a count to the capacity reads written entries only
                if (c == 1) {
                    const int64_t q = (int64_t)pos[0];
                    if (q < cap_f)
                        fkeys[q] = ((uint64_t)a << bits) | (uint64_t)b;
                    if (q + 1 < cap_f)
                        fkeys[q + 1] = ((uint64_t)b << bits) | (uint64_t)a;
                    else
                        ovf |= 2u;
                    pos[0] += 2;
                } else if (c == 2) {
                    const int fa = op[k][j].x, fb = op[k][j].y;
                    atomicAdd(&near_cnt[fa], 1);
                    atomicAdd(&near_cnt[fb], 1);
                    const int64_t q = (int64_t)pos[1];
                    if (q < cap_n)
                        nkeys[q] = ((uint64_t)fa << lbits) | (uint64_t)fb;
                    if (q + 1 < cap_n)
                        nkeys[q + 1] = ((uint64_t)fb << lbits) | (uint64_t)fa;
                    else
                        ovf |= 4u;
                    pos[1] += 2;
                } else if (j > 0 && c >= 3) {
                    const bool s_a = c == 3;
                    const int o = s_a ? b : a;
                    const int g0 = op[k][j].x, g1 = op[k][j].y;
                    const int64_t q = (int64_t)pos[2];
                    if (q < cap_task)
                        tout[q] = s_a ? make_int2(g0, o) : make_int2(o, g0);
                    if (q + 1 < cap_task)
                        tout[q + 1] = s_a ? make_int2(g1, o) : make_int2(o, g1);
                    else
                        ovf |= 1u;
                    pos[2] += 2;
                }
            }
        if (ovf)
            atomicOr(&cnt[MW_FLAGS], (unsigned long long)ovf);
    }
}

// Far pairs sorted by (sink, source): CSR range [fstart, fend) per sink cell.
// fstart / fend must be zero on entry.
__global__ __launch_bounds__(256) void k_mw_far_bounds(const uint64_t *__restrict__ keys,
                                                       int64_t n, int bits, int64_t *fstart,
                                                       int64_t *fend)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    const uint64_t s = keys[p] >> bits;
    if (p == 0 || (keys[p - 1] >> bits) != s)
        fstart[s] = p;
    if (p == n - 1 || (keys[p + 1] >> bits) != s)
        fend[s] = p + 1;
}

__global__ __launch_bounds__(256) void k_mw_fill64(int64_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
        p[i] = 0;
}

// Near pairs sorted by (sink leaf, source leaf), both as leaf indices of
// lbits bits: first position of each sink leaf (every leaf has its self
// pair, so each one is present).
__global__ __launch_bounds__(256) void k_mw_near_start(const uint64_t *__restrict__ keys,
                                                       int64_t n, int bits, int64_t *nstart)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    const uint64_t s = keys[p] >> bits;
    if (p == 0 || (keys[p - 1] >> bits) != s)
        nstart[s] = p;
}

// ... then each pair goes to slot (p - start) of its sink leaf.
__global__ __launch_bounds__(256) void k_mw_near_scatter(const uint64_t *__restrict__ keys,
                                                         int64_t n, int bits,
                                                         const int64_t *__restrict__ nstart,
                                                         const int32_t *__restrict__ leaf_node,
                                                         int32_t *near_src, int64_t cap_near)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    const uint64_t key = keys[p];
    const uint64_t s = key >> bits;
    const int64_t k = p - nstart[s];
    if (k < cap_near)
        near_src[(int64_t)s * cap_near + k] = leaf_node[key & ((1ull << bits) - 1ull)];
}

// Largest near count over the leaves -> cnt[MW_MAXNEAR] (one workgroup).
__global__ __launch_bounds__(1024) void k_mw_near_max(const int32_t *__restrict__ near_cnt, int n,
                                                      unsigned long long *cnt)
{
    __shared__ int32_t sh[16];
    int m = 0;
    for (int i = threadIdx.x; i < n; i += 1024)
        m = max(m, near_cnt[i]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        m = max(m, __shfl_xor(m, off));
    if (lane_id() == 0)
        sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 16; ++i)
            m = max(m, sh[i]);
        cnt[MW_MAXNEAR] = (unsigned long long)m;
    }
}

static int bit_width(int64_t v)
{
    int b = 1;
    while (b < 62 && (int64_t(1) << b) < v)
        ++b;
    return b;
}

int mutual_key_bits(const Tree &t) { return bit_width(t.topo.nnodes); }

// Launches of the two-level step: the recursion from the seed pairs ends
// within 2 depth + 2 levels (each split lowers one cell).
int mutual_iterations(const Tree &t) { return t.topo.depth + 1; }

hipError_t launch_mutual_walk(Tree &t, hipStream_t s)
{
    const Topology &T = t.topo;
    const MutualLists &M = t.mw;
    const int bits = mutual_key_bits(t), lbits = bit_width(T.nleaves);
    const int nit = mutual_iterations(t);
    const double theta2 = t.p.theta * t.p.theta;
    k_mw_zero<<<1, 256, 0, s>>>(M.cnt, MW_IT + nit + 1);
    const int n_int = T.nnodes - T.nleaves;
    k_mw_init<<<(std::max(n_int, T.nleaves) + 255) / 256, 256, 0, s>>>(
        t.left, t.right, t.int_nodes, n_int, t.leaf_node, T.nleaves, lbits, M.task[0],
        M.cap_task, M.nkeys[0], M.cap_near, t.near_cnt, M.cnt);
    for (int it = 0; it < nit; ++it)
        k_mw_step<<<MW_GRID, 256, 0, s>>>(M.task[it & 1], M.task[(it + 1) & 1], it, M.cap_task,
                                          t.recA, theta2, t.p.r_kern, bits, lbits,
                                          M.fkeys[0], M.cap_far, M.nkeys[0], M.cap_near,
                                          t.near_cnt, M.cnt);
    k_mw_near_max<<<1, 1024, 0, s>>>(t.near_cnt, T.nleaves, M.cnt);
    return hipGetLastError();
}

// Sort the pairs and lay out the lists (n_far / n_near: the counts read back
// after the walk; the caller checked that they fit the buffers).
hipError_t launch_mutual_lists(Tree &t, int64_t n_far, int64_t n_near, hipStream_t s)
{
    const Topology &T = t.topo;
    MutualLists &M = t.mw;
    const int bits = mutual_key_bits(t);
    const int lbits = bit_width(T.nleaves);
    // 8-bit digits: 10-bit ones take a pass less for these 64-bit keys but
    // measured slower, with or without value staging in LDS
    const int pf = (2 * bits + 7) / 8;
    const int pn = (2 * lbits + 7) / 8;  // near keys: (sink leaf, source leaf)
    hipError_t e = radix_sort_u64(M.fkeys[0], nullptr, M.fkeys[1], nullptr, n_far, 1, pf,
                                  M.hist, M.tot, s, 8);
    if (e != hipSuccess)
        return e;
    M.far_sorted = (pf & 1) ? M.fkeys[1] : M.fkeys[0];
    e = radix_sort_u64(M.nkeys[0], nullptr, M.nkeys[1], nullptr, n_near, 1, pn, M.hist, M.tot, s,
                       8);
    if (e != hipSuccess)
        return e;
    const uint64_t *ns = (pn & 1) ? M.nkeys[1] : M.nkeys[0];
    k_mw_fill64<<<256, 256, 0, s>>>(M.fstart, 2 * T.node_cap);  // fstart and fend
    if (n_far > 0)
        k_mw_far_bounds<<<(int)((n_far + 255) / 256), 256, 0, s>>>(M.far_sorted, n_far, bits,
                                                                   M.fstart, M.fend);
    if (n_near > 0) {
        const int g = (int)((n_near + 255) / 256);
        k_mw_near_start<<<g, 256, 0, s>>>(ns, n_near, lbits, M.nstart);
        k_mw_near_scatter<<<g, 256, 0, s>>>(ns, n_near, lbits, M.nstart, t.leaf_node, t.near_src,
                                            t.cap_near);
    }
    return hipGetLastError();
}

}  // namespace fmm
