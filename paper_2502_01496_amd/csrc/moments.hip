// Cell properties on gfx950 (Sec. 2 of the paper: mass, centre of mass, size
// s, h_max; quadrupole eq. (7)).
//
//   k_gather     caller-order x, m, h -> tree-order (x, y, z, m), h and
//                (1/h, 1/h^3, 4 h^2, h); flags bad inputs in the call's own
//                check word (cleared first by k_clear_word); clears the s^2
//                maxima.
//   k_leaf_moments  one thread per leaf: M, sum(m x) left to right, c = S / M,
//                h_max and the quadrupole about c.
//   k_combine_level one launch per tree level, deepest first: parents from
//                their two children -- M = M_L + M_R, c = (M_L c_L + M_R c_R) / M,
//                Q by the parallel-axis shift, h_max = max.
//   k_sub_moments / k_top_moments  the same two steps for the median-split
//                tree in two launches: one workgroup per subtree of at most
//                SUBTREE_MAX particles (its leaves, then its levels through
//                LDS), then one workgroup for the cells above the subtrees
//                when they fit LDS (per-level launches otherwise); the
//                centre-of-mass tree takes k_leaf_moments + k_combine_level.
//   k_node_s2    s^2 = max over the node's particles of |x - c|^2, exactly:
//                one thread per particle walks root -> leaf; lanes on the same
//                node reduce with a segmented wave max, then one u64 atomicMax
//                on the bit pattern (order-free for non-negative doubles).
//   k_node_final s = sqrt(s^2), the child ids and leaf index in the record's
//                topology slots, and the FP32 mirrors.
//
// Compiled with -ffp-contract=off: M, c, s and h_max are bit-identical to the
// serial definition (same operations, same order).
#include "fmm_internal.h"

namespace fmm {

// The moments call's data-check word starts at zero on every call (a kernel,
// not a memset, so that the call can be captured in a graph).
__global__ void k_clear_word(uint32_t *w) { *w = 0u; }

__global__ void k_gather(const double *__restrict__ x, const double *__restrict__ m,
                         const double *__restrict__ h, int64_t n, const int32_t *__restrict__ perm,
                         double4 *pm, double *hs, double4 *ph, uint32_t *err, int nnodes,
                         uint64_t *s2bits, int32_t *upcnt, int want_fp32, float4 *pfh)
{
    int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t bad = 0;
    for (int64_t p = gid; p < n; p += stride) {
        int64_t i = perm[p];
        double xx = x[3 * i], yy = x[3 * i + 1], zz = x[3 * i + 2], mm = m[i], hh = h[i];
        if (!(isfinite(xx) && isfinite(yy) && isfinite(zz)))
            bad |= 1u;
        if (!(mm > 0.0 && isfinite(mm)))
            bad |= 2u;
        if (!(hh > 0.0 && isfinite(hh)))
            bad |= 4u;
        pm[p] = make_double4(xx, yy, zz, mm);
        hs[p] = hh;
        double hi = 1.0 / hh;
        ph[p] = make_double4(hi, hi * hi * hi, 4.0 * hh * hh, hh);
        if (want_fp32)
            pfh[p] = make_float4((float)hi, (float)(hi * hi * hi), (float)(4.0 * hh * hh), 0.0f);
    }
    for (int64_t v = gid; v < nnodes; v += stride) {
        s2bits[v] = 0ull;
        upcnt[v] = 0;
    }
    if (gid == 0) {  // null source record at index n (far away, no mass, no smoothing)
        pm[n] = make_double4(1e30, 1e30, 1e30, 0.0);
        ph[n] = make_double4(0.0, 0.0, 0.0, 0.0);
    }
    // OR-reduce the error bits over the wave, one atomic per wave
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        bad |= (uint32_t)__shfl_xor((int)bad, off);
    if (lane_id() == 0 && bad)
        atomicOr(err, bad);
}

__device__ __forceinline__ void quad_add(double *Q, double w, double y0, double y1, double y2)
{
    double yy = y0 * y0 + y1 * y1 + y2 * y2;
    Q[0] += w * (3.0 * y0 * y0 - yy);
    Q[1] += w * (3.0 * y0 * y1);
    Q[2] += w * (3.0 * y0 * y2);
    Q[3] += w * (3.0 * y1 * y1 - yy);
    Q[4] += w * (3.0 * y1 * y2);
    Q[5] += w * (3.0 * y2 * y2 - yy);
}

// P2M of leaf v (node id): M, c, h_max and the quadrupole about c, written to
// its records; the values are also returned for a caller that combines them.
__device__ __forceinline__ void leaf_p2m(const double4 *__restrict__ pm,
                                         const double *__restrict__ hs, int v,
                                         const int32_t *__restrict__ first,
                                         const int32_t *__restrict__ count, double *recA,
                                         double *recQ, int want_fp32, float4 *pf, double *outA,
                                         double *outQ)
{
    int64_t f = first[v];
    int c = count[v];
    // particles are read U at a time, all loads in flight together (indices
    // past the leaf re-read its last particle and are not summed); sums run
    // in particle order.  A leaf of at most U particles stays in registers
    // for the second pass.
    constexpr int U = 8;
    double4 q[U];
    double M = 0.0, S0 = 0.0, S1 = 0.0, S2 = 0.0, hm = 0.0;
    for (int k0 = 0; k0 < c; k0 += U) {
        double hh[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int64_t i = f + min(k0 + j, c - 1);
            q[j] = pm[i];
            hh[j] = hs[i];
        }
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (k0 + j < c) {
                M += q[j].w;
                S0 += q[j].w * q[j].x;
                S1 += q[j].w * q[j].y;
                S2 += q[j].w * q[j].z;
                hm = hh[j] > hm ? hh[j] : hm;
            }
    }
    double c0 = S0 / M, c1 = S1 / M, c2 = S2 / M;
    double Q[6] = {0, 0, 0, 0, 0, 0};
    for (int k0 = 0; k0 < c; k0 += U) {
        if (c > U) {
#pragma unroll
            for (int j = 0; j < U; ++j)
                q[j] = pm[f + min(k0 + j, c - 1)];
        }
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (k0 + j < c) {
                double y0 = q[j].x - c0, y1 = q[j].y - c1, y2 = q[j].z - c2;
                quad_add(Q, q[j].w, y0, y1, y2);
                if (want_fp32)
                    pf[f + k0 + j] = make_float4((float)y0, (float)y1, (float)y2, (float)q[j].w);
            }
    }
    double *ra = recA + (int64_t)NREC * v;
    *(double4 *)ra = make_double4(c0, c1, c2, M);
    ra[5] = hm;
    double *rq = recQ + (int64_t)NREC * v;
    for (int k = 0; k < 6; ++k)
        rq[k] = Q[k];
    outA[0] = c0;
    outA[1] = c1;
    outA[2] = c2;
    outA[3] = M;
    outA[4] = hm;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        outQ[k] = Q[k];
}

// P2M at the leaves: one thread per leaf.
__global__ __launch_bounds__(256) void k_leaf_moments(
    const double4 *__restrict__ pm, const double *__restrict__ hs,
    const int32_t *__restrict__ leaf_node, int nleaves, const int32_t *__restrict__ first,
    const int32_t *__restrict__ count, double *recA, double *recQ, int want_fp32, float4 *pf)
{
    int lf = blockIdx.x * blockDim.x + threadIdx.x;
    if (lf >= nleaves)
        return;
    double a[5], q[6];
    leaf_p2m(pm, hs, leaf_node[lf], first, count, recA, recQ, want_fp32, pf, a, q);
}

// M2M for the internal nodes of one level (children were done by the
// previous launch): M = M_L + M_R, c = (M_L c_L + M_R c_R) / M, quadrupole by
// the parallel-axis shift of both children, h_max = max of the children.
// Parent from its two children: al / ar = (c0, c1, c2, M, h_max), ql / qr the
// quadrupoles; the parent's record is written to pa (5 values) and pq.
__device__ __forceinline__ void combine2(const double *al, const double *ql, const double *ar,
                                         const double *qr, double *pa, double *pq)
{
    const double Ml = al[3], Mr = ar[3];
    const double cl[3] = {al[0], al[1], al[2]}, cr[3] = {ar[0], ar[1], ar[2]};
    const double Mp = Ml + Mr;
    double cp[3];
    for (int d = 0; d < 3; ++d)
        cp[d] = (Ml * cl[d] + Mr * cr[d]) / Mp;
    double Qp[6] = {0, 0, 0, 0, 0, 0};
    for (int j = 0; j < 6; ++j)
        Qp[j] += ql[j];
    quad_add(Qp, Ml, cl[0] - cp[0], cl[1] - cp[1], cl[2] - cp[2]);
    for (int j = 0; j < 6; ++j)
        Qp[j] += qr[j];
    quad_add(Qp, Mr, cr[0] - cp[0], cr[1] - cp[1], cr[2] - cp[2]);
    const double hl = al[4], hr = ar[4];
    pa[0] = cp[0];
    pa[1] = cp[1];
    pa[2] = cp[2];
    pa[3] = Mp;
    pa[4] = hl > hr ? hl : hr;
    for (int j = 0; j < 6; ++j)
        pq[j] = Qp[j];
}

__device__ __forceinline__ void store_rec(double *recA, double *recQ, int p, const double *a,
                                          const double *q)
{
    double *ra = recA + (int64_t)NREC * p;
    *(double4 *)ra = make_double4(a[0], a[1], a[2], a[3]);
    ra[5] = a[4];
    double *rq = recQ + (int64_t)NREC * p;
    for (int j = 0; j < 6; ++j)
        rq[j] = q[j];
}

__global__ __launch_bounds__(256) void k_combine_level(const int32_t *__restrict__ nodes, int cnt,
                                                       const int32_t *__restrict__ left,
                                                       const int32_t *__restrict__ right,
                                                       double *recA, double *recQ)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cnt)
        return;
    const int p = nodes[k];
    const int l = left[p], r = right[p];
    const double *ral = recA + (int64_t)NREC * l, *rar = recA + (int64_t)NREC * r;
    const double4 A = *(const double4 *)ral, B = *(const double4 *)rar;
    const double al[5] = {A.x, A.y, A.z, A.w, ral[5]}, ar[5] = {B.x, B.y, B.z, B.w, rar[5]};
    double ql[6], qr[6];
    for (int j = 0; j < 6; ++j) {
        ql[j] = recQ[(int64_t)NREC * l + j];
        qr[j] = recQ[(int64_t)NREC * r + j];
    }
    double pa[5], pq[6];
    combine2(al, ql, ar, qr, pa, pq);
    store_rec(recA, recQ, p, pa, pq);
}

// All moments of one LDS subtree (cells of at most SUBTREE_MAX particles)
// per workgroup: P2M of its leaves, then its internal cells level by level,
// deepest first, the children read from LDS (a subtree's cells are the
// pre-order ids [r, r + size), at most SM_MAXNODES of them).  The same
// operations in the same order as k_leaf_moments and k_combine_level.
__global__ __launch_bounds__(256) void k_sub_moments(
    const double4 *__restrict__ pm, const double *__restrict__ hs,
    const int32_t *__restrict__ leaf_node, const int32_t *__restrict__ first,
    const int32_t *__restrict__ count, const int32_t *__restrict__ sub_root,
    const int32_t *__restrict__ sm_leaf, const int32_t *__restrict__ sm_lvl,
    const int2 *__restrict__ sm_nodes, double *recA, double *recQ, int want_fp32, float4 *pf)
{
    __shared__ double sA[SM_MAXNODES][5];
    __shared__ double sQ[SM_MAXNODES][6];
    const int s = blockIdx.x, t = threadIdx.x;
    const int r = sub_root[s];
    const int lf0 = sm_leaf[2 * s], lf1 = sm_leaf[2 * s + 1];
    for (int lf = lf0 + t; lf < lf1; lf += 256) {
        const int v = leaf_node[lf];
        leaf_p2m(pm, hs, v, first, count, recA, recQ, want_fp32, pf, sA[v - r], sQ[v - r]);
    }
    const int32_t *g = sm_lvl + s * (SM_MAXL + 1);
    for (int k = 0; k < SM_MAXL; ++k) {
        const int g0 = g[k], g1 = g[k + 1];
        if (g0 == g1)
            continue;
        __syncthreads();
        for (int i = g0 + t; i < g1; i += 256) {
            const int2 e = sm_nodes[i];
            const int p = e.x, l = p + 1, rr = e.y;  // pre-order: left child = p + 1
            combine2(sA[l - r], sQ[l - r], sA[rr - r], sQ[rr - r], sA[p - r], sQ[p - r]);
            store_rec(recA, recQ, p, sA[p - r], sQ[p - r]);
        }
    }
}

// The cells above the LDS subtrees in one workgroup: the subtree roots'
// records (from k_sub_moments) are loaded into LDS slots [0, nroots), then
// the cells are combined level by level, deepest first, cell k of the task
// list into slot nroots + k (the same operations as k_combine_level).
__global__ __launch_bounds__(1024) void k_top_moments(const int32_t *__restrict__ slot_node,
                                                      int nroots, const int32_t *__restrict__ task,
                                                      const int32_t *__restrict__ grp, int ngrp,
                                                      double *recA, double *recQ)
{
    __shared__ double sA[SM_MAXNODES][5];
    __shared__ double sQ[SM_MAXNODES][6];
    const int t = threadIdx.x;
    for (int i = t; i < nroots; i += 1024) {
        const int v = slot_node[i];
        const double *ra = recA + (int64_t)NREC * v;
        sA[i][0] = ra[0];
        sA[i][1] = ra[1];
        sA[i][2] = ra[2];
        sA[i][3] = ra[3];
        sA[i][4] = ra[5];
        for (int j = 0; j < 6; ++j)
            sQ[i][j] = recQ[(int64_t)NREC * v + j];
    }
    for (int g = 0; g < ngrp; ++g) {
        __syncthreads();
        const int k1 = grp[g + 1];
        for (int k = grp[g] + t; k < k1; k += 1024) {
            const int p = task[3 * k], ls = task[3 * k + 1], rs = task[3 * k + 2];
            combine2(sA[ls], sQ[ls], sA[rs], sQ[rs], sA[nroots + k], sQ[nroots + k]);
            store_rec(recA, recQ, p, sA[nroots + k], sQ[nroots + k]);
        }
    }
}

// Exact s^2 per node, phase 1: one thread per particle walks root -> leaf.
// At each level, a wavefront whose 64 particles all lie in one node writes
// its maximum to part[level][wave]; otherwise the lanes of each node reduce
// with a segmented max and one atomicMax per node run (few lanes per node, so
// little contention).  Nodes are numbered in depth-first pre-order, so an
// internal node's left child is v + 1: the centre, both child ids and the
// left child's particle range are loaded together, one round trip per level.
__global__ __launch_bounds__(256) void k_node_s2(const double4 *__restrict__ pm, int64_t n,
                                                 const double *__restrict__ recA,
                                                 const int32_t *__restrict__ first,
                                                 const int32_t *__restrict__ count,
                                                 const int32_t *__restrict__ left,
                                                 const int32_t *__restrict__ right, int nnodes,
                                                 uint64_t *s2bits, uint64_t *part, int64_t nwaves)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t wave = p >> 6;
    const int lane = lane_id();
    bool done = p >= n;
    double4 xp = done ? make_double4(0, 0, 0, 0) : pm[p];
    int v = 0;
    for (int lvl = 0; __ballot(!done) != 0ull; ++lvl) {
        const int key = done ? -1 : v;
        uint64_t val = 0ull;
        int l = -1, rgt = -1;
        int64_t bnd = 0;
        if (!done) {
            const double *ra = recA + (int64_t)NREC * v;
            l = left[v];
            rgt = right[v];
            const int vn = min(v + 1, nnodes - 1);  // read only when v is internal
            bnd = (int64_t)first[vn] + count[vn];
            double dx = xp.x - ra[0], dy = xp.y - ra[1], dz = xp.z - ra[2];
            double d2 = (dx * dx + dy * dy) + dz * dz;
            val = (uint64_t)__double_as_longlong(d2);
        }
        const int k0 = __shfl(key, 0);
        const bool uniform = __ballot(key == k0 && key >= 0) == ~0ull;
        if (uniform) {
            // one node for the whole wavefront: a butterfly max
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const uint64_t ov = __shfl_xor(val, off);
                val = ov > val ? ov : val;
            }
            if (lane == 63)
                part[(int64_t)lvl * nwaves + wave] = val;
        } else {
            // segmented inclusive max over runs of equal key (runs are contiguous)
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                uint64_t ov = __shfl_up(val, off);
                int ok = __shfl_up(key, off);
                if (lane >= off && ok == key)
                    val = ov > val ? ov : val;
            }
            int nk = __shfl_down(key, 1);
            bool tail = (lane == 63) || (nk != key);
            if (!done && tail)
                atomicMax((unsigned long long *)&s2bits[v], (unsigned long long)val);
        }
        if (!done) {
            if (l < 0)
                done = true;
            else
                v = p < bnd ? l : rgt;
        }
    }
}

// Leaves of a count-median cell of c particles: cells are halved (the left
// half takes ceil) while they hold more than L particles.  At depth k the
// sizes are floor(c / 2^k) or one more (c mod 2^k of them); every cell above
// the first depth K at which ceil(c / 2^K) <= L splits, and at depth K - 1
// those holding more than L particles split once more.
__device__ __forceinline__ int med_leaves(int c, int L)
{
    if (c <= L)
        return 1;
    const int a = 31 - __clz(c), b = 31 - __clz(L);
    const int k = ((uint64_t)L << (a - b)) >= (uint64_t)c ? a - b : a - b + 1;  // K >= 1
    const int km = k - 1;
    const int q = c >> km, r = c & ((1 << km) - 1);
    return (1 << km) + (q + 1 > L ? r : 0) + (q > L ? (1 << km) - r : 0);
}

// k_node_s2 for the count-median tree: its pre-order ids follow from the
// split rule (the right child of v is v + 2 leaves(left child)), so a
// particle's path needs no memory reads, and the centres of S2_BATCH levels
// are loaded together.  Same reductions and outputs as k_node_s2.
constexpr int S2_BATCH = 4;

__global__ __launch_bounds__(256) void k_node_s2_med(const double4 *__restrict__ pm, int64_t n,
                                                     const double *__restrict__ recA, int leaf_size,
                                                     uint64_t *s2bits, uint64_t *part,
                                                     int64_t nwaves)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t wave = p >> 6;
    const int lane = lane_id();
    bool alive = p < n;
    const double4 xp = alive ? pm[p] : make_double4(0, 0, 0, 0);
    int v = 0, f = 0, c = (int)n;
    for (int lvl = 0; __ballot(alive) != 0ull; lvl += S2_BATCH) {
        int vb[S2_BATCH];
        bool ab[S2_BATCH];
#pragma unroll
        for (int j = 0; j < S2_BATCH; ++j) {
            ab[j] = alive;
            vb[j] = v;
            if (alive) {
                if (c > leaf_size) {
                    const int nl = (c + 1) >> 1;
                    if (p < f + nl) {
                        v += 1;
                        c = nl;
                    } else {
                        v += 2 * med_leaves(nl, leaf_size);
                        f += nl;
                        c -= nl;
                    }
                } else {
                    alive = false;
                }
            }
        }
        double cx[S2_BATCH], cy[S2_BATCH], cz[S2_BATCH];
#pragma unroll
        for (int j = 0; j < S2_BATCH; ++j) {
            const double *ra = recA + (int64_t)NREC * (ab[j] ? vb[j] : 0);
            cx[j] = ra[0];
            cy[j] = ra[1];
            cz[j] = ra[2];
        }
#pragma unroll
        for (int j = 0; j < S2_BATCH; ++j) {
            const int key = ab[j] ? vb[j] : -1;
            uint64_t val = 0ull;
            if (ab[j]) {
                const double dx = xp.x - cx[j], dy = xp.y - cy[j], dz = xp.z - cz[j];
                const double d2 = (dx * dx + dy * dy) + dz * dz;
                val = (uint64_t)__double_as_longlong(d2);
            }
            const int k0 = __shfl(key, 0);
            const bool uniform = __ballot(key == k0 && key >= 0) == ~0ull;
            if (uniform) {
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    const uint64_t ov = __shfl_xor(val, off);
                    val = ov > val ? ov : val;
                }
                if (lane == 63)
                    part[(int64_t)(lvl + j) * nwaves + wave] = val;
            } else if (__ballot(key >= 0) != 0ull) {
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const uint64_t ov = __shfl_up(val, off);
                    const int ok = __shfl_up(key, off);
                    if (lane >= off && ok == key)
                        val = ov > val ? ov : val;
                }
                const int nk = __shfl_down(key, 1);
                const bool tail = (lane == 63) || (nk != key);
                if (key >= 0 && tail)
                    atomicMax((unsigned long long *)&s2bits[key], (unsigned long long)val);
            }
        }
    }
}

// Phase 2: one wavefront per node of at least 64 particles folds the partial
// maxima of the wavefronts lying entirely inside it.
__global__ __launch_bounds__(256) void k_node_s2_fold(const int32_t *__restrict__ big,
                                                      int nbig,
                                                      const int32_t *__restrict__ first,
                                                      const int32_t *__restrict__ count,
                                                      const int32_t *__restrict__ level,
                                                      const uint64_t *__restrict__ part,
                                                      int64_t nwaves, uint64_t *s2bits)
{
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= nbig)
        return;
    const int v = big[k];
    const int64_t w0 = ((int64_t)first[v] + 63) >> 6;
    const int64_t w1 = ((int64_t)first[v] + count[v]) >> 6;
    const uint64_t *pl = part + (int64_t)level[v] * nwaves;
    uint64_t m = 0ull;
    // eight loads in flight per lane; indices past w1 re-read entry w0, which
    // belongs to the node and so leaves the maximum unchanged
    constexpr int U = 8;
    for (int64_t wb = w0 + lane_id(); wb < w1; wb += 64 * U) {
        uint64_t x[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int64_t q = wb + 64 * j;
            x[j] = pl[q < w1 ? q : w0];
        }
#pragma unroll
        for (int j = 0; j < U; ++j)
            m = x[j] > m ? x[j] : m;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        uint64_t o = __shfl_xor(m, off);
        m = o > m ? o : m;
    }
    if (lane_id() == 0 && w1 > w0)
        atomicMax((unsigned long long *)&s2bits[v], (unsigned long long)m);
}

__global__ void k_node_final(int nnodes, const uint64_t *__restrict__ s2bits,
                             const int32_t *__restrict__ left, const int32_t *__restrict__ right,
                             const int32_t *__restrict__ node_leaf, double *recA,
                             const double *__restrict__ recQ, int want_fp32, float *recF)
{
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nnodes; v += gridDim.x * blockDim.x) {
        double s2 = __longlong_as_double((long long)s2bits[v]);
        recA[(int64_t)NREC * v + 4] = sqrt(s2);
        const uint64_t kids = (uint64_t)(uint32_t)left[v] | ((uint64_t)(uint32_t)right[v] << 32);
        recA[(int64_t)NREC * v + REC_KIDS] = __longlong_as_double((long long)kids);
        recA[(int64_t)NREC * v + REC_LEAF] =
            __longlong_as_double((long long)(uint64_t)(uint32_t)node_leaf[v]);
        if (want_fp32) {
            float *rf = recF + (int64_t)NREC * v;
            rf[0] = (float)recA[(int64_t)NREC * v + 3];
            for (int k = 0; k < 6; ++k)
                rf[1 + k] = (float)recQ[(int64_t)NREC * v + k];
            rf[7] = 0.0f;
        }
    }
}

// Imported cell records (host layout of fmm_debug_import, 12 doubles per
// node: M, c[3], s, h_max, Q[6]) into the device records, with the child ids
// and leaf index from the topology and the FP32 mirror.
__global__ void k_import_records(int nnodes, const double *__restrict__ rec12,
                                 const int32_t *__restrict__ left,
                                 const int32_t *__restrict__ right,
                                 const int32_t *__restrict__ node_leaf, double *recA, double *recQ,
                                 int want_fp32, float *recF)
{
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nnodes; v += gridDim.x * blockDim.x) {
        const double *r = rec12 + 12 * (int64_t)v;
        double *ra = recA + (int64_t)NREC * v;
        double *rq = recQ + (int64_t)NREC * v;
        ra[0] = r[1];
        ra[1] = r[2];
        ra[2] = r[3];
        ra[3] = r[0];
        ra[4] = r[4];
        ra[5] = r[5];
        const uint64_t kids = (uint64_t)(uint32_t)left[v] | ((uint64_t)(uint32_t)right[v] << 32);
        ra[REC_KIDS] = __longlong_as_double((long long)kids);
        ra[REC_LEAF] = __longlong_as_double((long long)(uint64_t)(uint32_t)node_leaf[v]);
        for (int k = 0; k < 6; ++k)
            rq[k] = r[6 + k];
        rq[6] = rq[7] = 0.0;
        if (want_fp32) {
            float *rf = recF + (int64_t)NREC * v;
            rf[0] = (float)r[0];
            for (int k = 0; k < 6; ++k)
                rf[1 + k] = (float)r[6 + k];
            rf[7] = 0.0f;
        }
    }
}

// FP32 form: particle offsets from the (imported) centre of mass of their
// leaf, one thread per leaf.
__global__ void k_import_offsets(int nleaves, const int32_t *__restrict__ leaf_node,
                                 const int32_t *__restrict__ first,
                                 const int32_t *__restrict__ count,
                                 const double *__restrict__ recA, const double4 *__restrict__ pm,
                                 float4 *pf)
{
    const int lf = blockIdx.x * blockDim.x + threadIdx.x;
    if (lf >= nleaves)
        return;
    const int v = leaf_node[lf];
    const double *c = recA + (int64_t)NREC * v;
    for (int64_t p = first[v]; p < (int64_t)first[v] + count[v]; ++p) {
        const double4 q = pm[p];
        pf[p] = make_float4((float)(q.x - c[0]), (float)(q.y - c[1]), (float)(q.z - c[2]),
                            (float)q.w);
    }
}

// fmm_debug_import: tree-order particles from the imported permutation (with
// the data checks of a moments call), then the imported cell records.
hipError_t launch_import(Tree &t, const double *x, const double *m, const double *h,
                         const double *rec12, hipStream_t s)
{
    const Topology &T = t.topo;
    const int64_t n = T.n;
    const int64_t work = n > T.nnodes ? n : T.nnodes;
    const int gs = (int)std::min<int64_t>((work + 255) / 256, 4096);
    const int want32 = t.p.precision == FMM_FP32;
    k_clear_word<<<1, 1, 0, s>>>(t.err + 1);
    k_gather<<<gs, 256, 0, s>>>(x, m, h, n, t.perm, t.pm, t.hs, t.ph, t.err + 1, T.nnodes,
                                t.s2bits, t.upcnt, want32, t.pfh);
    k_import_records<<<(T.nnodes + 255) / 256, 256, 0, s>>>(T.nnodes, rec12, t.left, t.right,
                                                           t.node_leaf, t.recA, t.recQ, want32,
                                                           t.recF);
    if (want32)
        k_import_offsets<<<(T.nleaves + 255) / 256, 256, 0, s>>>(T.nleaves, t.leaf_node, t.first,
                                                                 t.count, t.recA, t.pm, t.pf);
    return hipGetLastError();
}

hipError_t launch_moments(Tree &t, const double *x, const double *m, const double *h,
                          hipStream_t s)
{
    const Topology &T = t.topo;
    int64_t n = T.n;
    int64_t work = n > T.nnodes ? n : T.nnodes;
    int gs = (int)std::min<int64_t>((work + 255) / 256, 4096);
    int want32 = t.p.precision == FMM_FP32;
    k_clear_word<<<1, 1, 0, s>>>(t.err + 1);
    k_gather<<<gs, 256, 0, s>>>(x, m, h, n, t.perm, t.pm, t.hs, t.ph, t.err + 1, T.nnodes, t.s2bits,
                                t.upcnt, want32, t.pfh);
    if (!T.com && T.sub_moments) {
        // the subtrees in one launch, then the cells above them level by level
        k_sub_moments<<<(int)T.sub_root.size(), 256, 0, s>>>(
            t.pm, t.hs, t.leaf_node, t.first, t.count, t.sub_root, t.sm_leaf, t.sm_lvl,
            (const int2 *)t.sm_nodes, t.recA, t.recQ, want32, t.pf);
        if (T.top_fused) {
            if (!T.top_nodes.empty())
                k_top_moments<<<1, 1024, 0, s>>>(t.top_slot_node, (int)T.sub_root.size(),
                                                 t.top_task, t.top_grp,
                                                 (int)T.top_grp.size() - 1, t.recA, t.recQ);
        } else {
            for (int l = T.depth - 2; l >= 0; --l) {
                int o = T.top_lvl_off[l], cnt = T.top_lvl_off[l + 1] - o;
                if (cnt > 0)
                    k_combine_level<<<(cnt + 255) / 256, 256, 0, s>>>(
                        t.top_nodes + o, cnt, t.left, t.right, t.recA, t.recQ);
            }
        }
    } else {
        k_leaf_moments<<<(T.nleaves + 255) / 256, 256, 0, s>>>(
            t.pm, t.hs, t.leaf_node, T.nleaves, t.first, t.count, t.recA, t.recQ, want32, t.pf);
        for (int l = T.depth - 2; l >= 0; --l) {
            int o = T.lvl_int_off[l], cnt = T.lvl_int_off[l + 1] - o;
            if (cnt > 0)
                k_combine_level<<<(cnt + 255) / 256, 256, 0, s>>>(t.int_nodes + o, cnt, t.left,
                                                                  t.right, t.recA, t.recQ);
        }
    }
    const int64_t nwaves = (n + 63) / 64;
    if (T.com)
        k_node_s2<<<(int)((n + 255) / 256), 256, 0, s>>>(t.pm, n, t.recA, t.first, t.count,
                                                         t.left, t.right, T.nnodes, t.s2bits,
                                                         t.s2part, nwaves);
    else
        k_node_s2_med<<<(int)((n + 255) / 256), 256, 0, s>>>(t.pm, n, t.recA, T.leaf_size,
                                                             t.s2bits, t.s2part, nwaves);
    const int nbig = T.nbig;
    if (nbig > 0)
        k_node_s2_fold<<<(nbig + 3) / 4, 256, 0, s>>>(t.big_nodes, nbig, t.first, t.count,
                                                      t.level, t.s2part, nwaves, t.s2bits);
    k_node_final<<<(T.nnodes + 255) / 256, 256, 0, s>>>(T.nnodes, t.s2bits, t.left, t.right,
                                                       t.node_leaf, t.recA, t.recQ,
                                                       want32, t.recF);
    return hipGetLastError();
}

}  // namespace fmm
