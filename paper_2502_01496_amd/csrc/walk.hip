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
// One wavefront walks 64 consecutive sink leaves together: it shares one DFS
// stack whose entries carry the 64-bit mask of lanes that opened the parent,
// so every node record is a wave-uniform load and the per-lane visit order is
// the serial DFS order (lists come out in ascending tree order).  A count pass
// sizes the CSR; after a scan, a fill pass writes the node ids.
//
// Compiled with -ffp-contract=off so the criteria are evaluated with exactly
// the operations of their definition.
#include "fmm_internal.h"

namespace fmm {

constexpr int WALK_STACK = 96;

template <bool FILL>
__global__ __launch_bounds__(256) void k_walk_p(
    const double *__restrict__ recA, const int32_t *__restrict__ left,
    const int32_t *__restrict__ right, const int32_t *__restrict__ leaf_node, int nleaves,
    double theta2, double r_kern, int32_t *far_cnt, int32_t *near_cnt,
    const int64_t *__restrict__ far_off, const int64_t *__restrict__ near_off, int32_t *far_src,
    int32_t *near_src)
{
    __shared__ int32_t stk_node[4][WALK_STACK];
    __shared__ uint64_t stk_mask[4][WALK_STACK];
    const int w = threadIdx.x >> 6, lane = lane_id();
    const int leaf = blockIdx.x * 256 + threadIdx.x;
    const bool valid = leaf < nleaves;
    const int a = valid ? leaf_node[leaf] : 0;
    const double *ra = recA + (int64_t)NREC * a;
    const double ca0 = ra[0], ca1 = ra[1], ca2 = ra[2], sa = ra[4], ha = ra[5];
    int64_t fo = 0, no = 0;
    if (FILL && valid) {
        fo = far_off[leaf];
        no = near_off[leaf];
    }
    int nf = 0, nn = 0;
    uint64_t vmask = __ballot(valid);
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
        const double *rb = recA + (int64_t)NREC * b;
        const double cb0 = rb[0], cb1 = rb[1], cb2 = rb[2], sb = rb[4], hb = rb[5];
        const int lb = left[b];
        const bool leafb = lb < 0;
        const bool active = (mask >> lane) & 1ull;
        bool descend = false;
        if (active) {
            double dx = ca0 - cb0, dy = ca1 - cb1, dz = ca2 - cb2;
            double r2 = (dx * dx + dy * dy) + dz * dz;
            bool open4 = sb * sb > theta2 * r2;
            double tt = (sa + sb) + r_kern * (ha > hb ? ha : hb);
            bool open5 = r2 < tt * tt;
            if (!(open4 || open5)) {
                if (FILL)
                    far_src[fo + nf] = b;
                ++nf;
            } else if (leafb) {
                if (FILL)
                    near_src[no + nn] = b;
                ++nn;
            } else {
                descend = true;
            }
        }
        const uint64_t om = __ballot(descend);
        if (om != 0ull) {
            if (lane == 0) {
                stk_node[w][sp] = right[b];
                stk_mask[w][sp] = om;
                stk_node[w][sp + 1] = lb;
                stk_mask[w][sp + 1] = om;
            }
            sp += 2;
        }
    }
    if (!FILL && valid) {
        far_cnt[leaf] = nf;
        near_cnt[leaf] = nn;
    }
}

// ---------------------------------------------------------------- offsets
// Exclusive scans of the far and near counts (int32 -> int64 offsets, with the
// total at [nsinks]): per-tile sums, one scan of the tile sums, tile rescans.
constexpr int SCAN_TILE = 4096;

__device__ __forceinline__ int64_t block_excl_scan_i64(int64_t v, int64_t *sh, int64_t &total)
{
    int t = threadIdx.x, lane = lane_id(), w = t >> 6, nw = blockDim.x >> 6;
    int64_t inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int64_t o = __shfl_up(inc, off);
        if (lane >= off)
            inc += o;
    }
    if (lane == 63)
        sh[w] = inc;
    __syncthreads();
    int64_t wb = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        int64_t s = sh[i];
        wb += i < w ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return wb + inc - v;
}

__global__ __launch_bounds__(256) void k_scan_tiles(const int32_t *cf, const int32_t *cn, int ns,
                                                    int64_t *tsum, int ntiles)
{
    __shared__ int64_t sh[8];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t sf = 0, sn = 0;
    for (int k = threadIdx.x; k < SCAN_TILE; k += 256) {
        int64_t i = base + k;
        if (i < ns) {
            sf += cf[i];
            sn += cn[i];
        }
    }
    int64_t tf, tn;
    block_excl_scan_i64(sf, sh, tf);
    block_excl_scan_i64(sn, sh, tn);
    if (threadIdx.x == 0) {
        tsum[blockIdx.x] = tf;
        tsum[ntiles + blockIdx.x] = tn;
    }
}

__global__ __launch_bounds__(1024) void k_scan_tile_sums(int64_t *tsum, int ntiles, int64_t *totals)
{
    __shared__ int64_t sh[16];
    for (int q = 0; q < 2; ++q) {
        int64_t run = 0;
        for (int c0 = 0; c0 < ntiles; c0 += 1024) {
            int i = c0 + threadIdx.x;
            int64_t v = i < ntiles ? tsum[q * ntiles + i] : 0;
            int64_t total;
            int64_t ex = block_excl_scan_i64(v, sh, total);
            if (i < ntiles)
                tsum[q * ntiles + i] = run + ex;
            run += total;
        }
        if (threadIdx.x == 0)
            totals[q] = run;
    }
}

__global__ __launch_bounds__(256) void k_scan_write(const int32_t *cf, const int32_t *cn, int ns,
                                                    const int64_t *tsum, int ntiles,
                                                    int64_t *far_off, int64_t *near_off,
                                                    const int64_t *totals)
{
    constexpr int PER = SCAN_TILE / 256;
    __shared__ int64_t sh[8];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * PER;
    int32_t vf[PER], vn[PER];
    int64_t sf = 0, sn = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        int64_t i = base + k;
        vf[k] = i < ns ? cf[i] : 0;
        vn[k] = i < ns ? cn[i] : 0;
        sf += vf[k];
        sn += vn[k];
    }
    int64_t tf, tn;
    int64_t ef = block_excl_scan_i64(sf, sh, tf) + tsum[blockIdx.x];
    int64_t en = block_excl_scan_i64(sn, sh, tn) + tsum[ntiles + blockIdx.x];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        int64_t i = base + k;
        if (i < ns) {
            far_off[i] = ef;
            near_off[i] = en;
        }
        ef += vf[k];
        en += vn[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        far_off[ns] = totals[0];
        near_off[ns] = totals[1];
    }
}

hipError_t launch_walk_count(Tree &t, hipStream_t s)
{
    const Topology &T = t.topo;
    const double theta2 = t.p.theta * t.p.theta;
    int nl = T.nleaves;
    k_walk_p<false><<<(nl + 255) / 256, 256, 0, s>>>(t.recA, t.left, t.right, t.leaf_node, nl,
                                                     theta2, t.p.r_kern, t.far_cnt, t.near_cnt,
                                                     nullptr, nullptr, nullptr, nullptr);
    int ntiles = (nl + SCAN_TILE - 1) / SCAN_TILE;
    k_scan_tiles<<<ntiles, 256, 0, s>>>(t.far_cnt, t.near_cnt, nl, t.scan_tmp, ntiles);
    k_scan_tile_sums<<<1, 1024, 0, s>>>(t.scan_tmp, ntiles, t.totals);
    k_scan_write<<<ntiles, 256, 0, s>>>(t.far_cnt, t.near_cnt, nl, t.scan_tmp, ntiles, t.far_off,
                                        t.near_off, t.totals);
    return hipGetLastError();
}

hipError_t launch_walk_fill(Tree &t, hipStream_t s)
{
    const Topology &T = t.topo;
    const double theta2 = t.p.theta * t.p.theta;
    int nl = T.nleaves;
    k_walk_p<true><<<(nl + 255) / 256, 256, 0, s>>>(t.recA, t.left, t.right, t.leaf_node, nl,
                                                    theta2, t.p.r_kern, nullptr, nullptr,
                                                    t.far_off, t.near_off, t.far_src, t.near_src);
    return hipGetLastError();
}

}  // namespace fmm
