// Asymmetric cell pairs of the interaction lists and the total-force
// estimates of Sec. 4, eq. (33), and Sec. 6, eq. (46), on gfx950.
//
// A pair "sink a receives the field of source b" is asymmetric when the
// reverse pair (b receiving a) is absent from the lists.  For a cell v with
// N_v >= 2 leaves, v1 is its lightest leaf (smallest mass; among equal masses
// the one farthest from c_v) and l_v = |c_v1 - c_v|:
//   T(v) = M_v1 l_v^3 / (M_v - M_v1) (1 - M_v1 / (M_v - M_v1)),
//   U(v) = s_v^3 (N_v - 2) / (N_v - 1)^2,
// both zero for a leaf.  Each asymmetric pair adds
//   eq. (33): 4 M_a M_b / r^5 (T(a) + T(b)),
//   eq. (46): 4 M_l^2 N_a N_b / r^5 (U(a) + U(b)),   r = |c_a - c_b|.
// Sums: per lane in list order, a fixed butterfly per sink, then one
// workgroup over the sinks in a fixed order (deterministic, no atomics).
#include "fmm_internal.h"

namespace fmm {

constexpr int ASYM_FOLD = 1024;

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off);
    return v;
}

// Per node: T, U and N.  One wavefront per node; the leaves of the node's
// subtree are consecutive in leaf order (pre-order ids, left child first),
// from the leftmost to the rightmost descendant.
__global__ __launch_bounds__(256) void k_asym_node(const double *__restrict__ recA,
                                                   const int32_t *__restrict__ left,
                                                   const int32_t *__restrict__ right,
                                                   const int32_t *__restrict__ node_leaf,
                                                   const int32_t *__restrict__ leaf_node,
                                                   int nnodes, double *tun)
{
    const int v = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (v >= nnodes)
        return;
    const int lane = lane_id();
    int lo = v, hi = v;
    while (left[lo] >= 0)
        lo = left[lo];
    while (right[hi] >= 0)
        hi = right[hi];
    const int l0 = node_leaf[lo], l1 = node_leaf[hi];
    const int nlv = l1 - l0 + 1;
    double *o = tun + 3 * (int64_t)v;
    if (nlv < 2) {
        if (lane == 0) {
            o[0] = 0.0;
            o[1] = 0.0;
            o[2] = (double)nlv;
        }
        return;
    }
    double m1 = __builtin_huge_val();
    for (int k = l0 + lane; k <= l1; k += 64)
        m1 = fmin(m1, recA[(int64_t)NREC * leaf_node[k] + 3]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        m1 = fmin(m1, __shfl_xor(m1, off));
    const double *rv = recA + (int64_t)NREC * v;
    const double cx = rv[0], cy = rv[1], cz = rv[2];
    double d2 = -1.0;
    for (int k = l0 + lane; k <= l1; k += 64) {
        const double *ru = recA + (int64_t)NREC * leaf_node[k];
        if (ru[3] == m1) {
            const double dx = ru[0] - cx, dy = ru[1] - cy, dz = ru[2] - cz;
            d2 = fmax(d2, dx * dx + dy * dy + dz * dz);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        d2 = fmax(d2, __shfl_xor(d2, off));
    if (lane == 0) {
        const double l = sqrt(d2);
        const double rest = rv[3] - m1;
        const double N = (double)nlv, s = rv[4];
        o[0] = m1 * l * l * l / rest * (1.0 - m1 / rest);
        o[1] = s * s * s * (N - 2.0) / ((N - 1.0) * (N - 1.0));
        o[2] = N;
    }
}

// M_l of eq. (46): the given value, or the mean leaf mass (root mass over
// the number of leaves) when it is not positive.
__device__ __forceinline__ double leaf_mass(double m_leaf, const double *__restrict__ recA,
                                            int nleaves)
{
    return m_leaf > 0.0 ? m_leaf : recA[3] / (double)nleaves;
}

// One pair's terms, added to the four per-lane sums.
__device__ __forceinline__ void asym_add(const double *__restrict__ recA,
                                         const double *__restrict__ tun, int a, int b,
                                         double m_leaf, double (&acc)[4])
{
    const double *ra = recA + (int64_t)NREC * a, *rb = recA + (int64_t)NREC * b;
    const double *ta = tun + 3 * (int64_t)a, *tb = tun + 3 * (int64_t)b;
    const double dx = ra[0] - rb[0], dy = ra[1] - rb[1], dz = ra[2] - rb[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double r5 = r2 * r2 * sqrt(r2);
    acc[0] += 4.0 * ra[3] * rb[3] / r5 * (ta[0] + tb[0]);
    acc[1] += 4.0 * m_leaf * m_leaf * ta[2] * tb[2] / r5 * (ta[1] + tb[1]);
    acc[2] += 1.0;
    acc[3] += (ta[2] >= 2.0 || tb[2] >= 2.0) ? 1.0 : 0.0;
}

// Leaf <- cell lists: one wavefront per sink leaf, lanes over its far list.
// The reverse pair exists only if the source b is itself a leaf whose far
// list holds a, i.e. b appears among the sinks of a in the transposed lists
// (ascending: binary search).
__global__ __launch_bounds__(256) void k_asym_pairs_leaf(
    const double *__restrict__ recA, const double *__restrict__ tun,
    const int32_t *__restrict__ left, const int32_t *__restrict__ leaf_node,
    const int32_t *__restrict__ node_leaf, int nleaves, const int32_t *__restrict__ far_cnt,
    const int32_t *__restrict__ far_src, int cap_far, const int64_t *__restrict__ toff,
    const uint32_t *__restrict__ tsrc, double m_leaf_in, double *part)
{
    const int g = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (g >= nleaves)
        return;
    const double m_leaf = leaf_mass(m_leaf_in, recA, nleaves);
    const int lane = lane_id();
    const int a = leaf_node[g];
    const int nk = max(0, min(far_cnt[g], cap_far));
    const int32_t *fl = far_src + (int64_t)g * cap_far;
    const int64_t t0 = toff[a], t1 = toff[a + 1];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = lane; k < nk; k += 64) {
        const int b = fl[k];
        bool rev = false;
        if (left[b] < 0) {
            // the transposed far lists hold sink leaf indices, ascending
            const int bl = node_leaf[b];
            int64_t lo = t0, hi = t1;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if ((int)tsrc[mid] < bl)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            rev = lo < t1 && (int)tsrc[lo] == bl;
        }
        if (!rev)
            asym_add(recA, tun, a, b, m_leaf, acc);
    }
    double *o = part + 4 * (int64_t)g;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double t = wave_sum_d(acc[q]);
        if (lane == 0)
            o[q] = t;
    }
}

// Mutual lists: one wavefront per sink cell over its range of the sorted
// (sink, source) keys; the reverse pair is looked up in the source's range.
__global__ __launch_bounds__(256) void k_asym_pairs_mutual(
    const double *__restrict__ recA, const double *__restrict__ tun, int nnodes,
    const int64_t *__restrict__ fstart, const int64_t *__restrict__ fend,
    const uint64_t *__restrict__ keys, int bits, int nleaves, double m_leaf_in, double *part)
{
    const int a = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (a >= nnodes)
        return;
    const double m_leaf = leaf_mass(m_leaf_in, recA, nleaves);
    const int lane = lane_id();
    const uint64_t mask = (1ull << bits) - 1ull;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t k = fstart[a] + lane; k < fend[a]; k += 64) {
        const int b = (int)(keys[k] & mask);
        const uint64_t want = ((uint64_t)b << bits) | (uint64_t)a;
        int64_t lo = fstart[b], hi = fend[b];
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < want)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (!(lo < fend[b] && keys[lo] == want))
            asym_add(recA, tun, a, b, m_leaf, acc);
    }
    double *o = part + 4 * (int64_t)a;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double t = wave_sum_d(acc[q]);
        if (lane == 0)
            o[q] = t;
    }
}

// The per-sink sums in a fixed order: thread t takes sinks t, t + 1024, ...,
// then a tree over the threads.
__global__ __launch_bounds__(ASYM_FOLD) void k_asym_fold(const double *__restrict__ part, int nsinks,
                                                         double *out)
{
    __shared__ double sh[4][ASYM_FOLD];
    const int t = threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int g = t; g < nsinks; g += ASYM_FOLD)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc[q] += part[4 * (int64_t)g + q];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        sh[q][t] = acc[q];
    __syncthreads();
    for (int w = ASYM_FOLD / 2; w >= 1; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                sh[q][t] += sh[q][t + w];
        __syncthreads();
    }
    if (t < 4)
        out[t] = sh[t][0];
}

hipError_t launch_asym(Tree &t, double m_leaf, double *out, hipStream_t s)
{
    const Topology &T = t.topo;
    const int nn = T.nnodes, nl = T.nleaves;
    hipError_t e = hipSuccess;
    if (!t.asym) {
        // T, U, N per node; four sums per sink (nodes >= leaves); four totals
        const size_t nc = (size_t)T.node_cap;
        e = tree_malloc(t, (void **)&t.asym, (3 * nc + 4 * nc + 4) * sizeof(double));
        if (e == hipSuccess && !t.h_asym)
            e = hipHostMalloc((void **)&t.h_asym, 4 * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) {
            tree_free(t, t.asym);
            t.asym = nullptr;
            return e;
        }
    }
    double *tun = t.asym, *part = t.asym + 3 * (size_t)T.node_cap,
           *dout = part + 4 * (size_t)T.node_cap;
    const bool mutual = t.lists_policy == FMM_WALK_MUTUAL;
    if (!mutual) {
        e = ensure_transposed(t, s);
        if (e != hipSuccess)
            return e;
    }
    k_asym_node<<<(nn + 3) / 4, 256, 0, s>>>(t.recA, t.left, t.right, t.node_leaf, t.leaf_node,
                                             nn, tun);
    int nsinks;
    if (mutual) {
        nsinks = nn;
        k_asym_pairs_mutual<<<(nn + 3) / 4, 256, 0, s>>>(t.recA, tun, nn, t.mw.fstart, t.mw.fend,
                                                         t.mw.far_sorted, mutual_key_bits(t),
                                                         nl, m_leaf, part);
    } else {
        nsinks = nl;
        k_asym_pairs_leaf<<<(nl + 3) / 4, 256, 0, s>>>(
            t.recA, tun, t.left, t.leaf_node, t.node_leaf, nl, t.far_cnt, t.far_src,
            (int)t.cap_far, t.farT.off, t.farT.src, m_leaf, part);
    }
    k_asym_fold<<<1, ASYM_FOLD, 0, s>>>(part, nsinks, dout);
    e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(t.h_asym, dout, 4 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        for (int q = 0; q < 4; ++q)
            out[q] = t.h_asym[q];
    return e;
}

void release_asym(Tree &t)
{
    tree_free(t, t.asym);
    if (t.h_asym)
        (void)hipHostFree(t.h_asym);
    t.asym = nullptr;
    t.h_asym = nullptr;
}

}  // namespace fmm
