// kd-tree cut through the centre of mass (FMM_TREE_COM) on gfx950.
//
// Sec. 2 describes the tree as cut recursively through each cell's centre of
// mass across its longest axis, down to cells of at most leaf_size
// particles.  Positions are quantised on a grid of 2^32 steps over the
// largest extent of the global bounding box and masses to integer weights
// (w = floor(m / m_max 2^24) in [1, 2^24]); per cell the axis is the longest
// of the quantised bounding box (ties -> lowest) and a particle goes left iff
// q_d sum(w) < sum(w q_d).  All of it is integer arithmetic, so the partition
// does not depend on how the sums are split over threads.  A cell whose
// particles share one grid point is halved in tree order.
//
// The shape depends on the data, so the build is level-synchronous over the
// cells still to be cut ("active"), each cut in chunks of COM_CHUNK
// particles:
//   stats (per chunk: quantised box, sum w, sum w q) -> split (per cell:
//   fold its chunks, axis and cut) -> count (per chunk: particles going
//   left) -> offsets (per cell: exclusive bases of its chunks) -> scatter
//   (per chunk: stable partition into a copy) -> copy back -> children (per
//   cell: two new cells) -> next (one workgroup: the next level's active
//   cells and chunks).
// One readback per level gives the host the next launch sizes.  Cells are
// numbered breadth-first while building and renumbered to DFS pre-order
// (subtree sizes bottom-up, ids top-down), the numbering every later stage
// expects.
#include "fmm_internal.h"

namespace fmm {

constexpr int CB = 256;  // threads per chunk workgroup

// BFS node table rows
enum { NF = 0, NC = 1, NP = 2, NLV = 3, NAX = 4, NL = 5, NR = 6, NIR = 7 };
// renumbering rows
enum { RSUB = 0, RLEAF = 1, RPRE = 2, RLOFS = 3 };

__device__ __forceinline__ void add128(uint64_t &lo, uint64_t &hi, uint64_t blo, uint64_t bhi)
{
    const uint64_t s = lo + blo;
    hi += bhi + (s < lo ? 1ull : 0ull);
    lo = s;
}

// q_d sum(w) < sum(w q_d), both sides exact 128-bit integers
__device__ __forceinline__ bool left_of_cut(uint32_t qd, uint64_t sw, uint64_t lo, uint64_t hi)
{
    const uint64_t plo = (uint64_t)qd * sw;
    const uint64_t phi = __umul64hi((uint64_t)qd, sw);
    return phi < hi || (phi == hi && plo < lo);
}

__global__ void k_com_zero(int64_t *ctl)
{
    if (threadIdx.x < 8)
        ctl[threadIdx.x] = 0;
}

// Largest positive mass (NaN and non-positive masses ignored), as ordered
// bits in ctl[3].
__global__ __launch_bounds__(256) void k_com_mmax(const double *__restrict__ m, int64_t n,
                                                  int64_t *ctl)
{
    uint64_t best = 0ull;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = m[i];
        if (v > 0.0) {
            const uint64_t b = ordbits(v);
            best = b > best ? b : best;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint64_t o = __shfl_xor((unsigned long long)best, off);
        best = o > best ? o : best;
    }
    if (lane_id() == 0 && best)
        atomicMax((unsigned long long *)&ctl[3], (unsigned long long)best);
}

// Tree order = Morton order; quantised coordinates and weights.
__global__ __launch_bounds__(256) void k_com_init(const double *__restrict__ x,
                                                  const double *__restrict__ m, int64_t n,
                                                  const uint64_t *__restrict__ bbox,
                                                  const int64_t *__restrict__ ctl,
                                                  const uint32_t *__restrict__ order,
                                                  int32_t *perm, uint32_t *q)
{
    double lo[3], ext = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = from_ordbits(bbox[d]);
        const double e = from_ordbits(bbox[3 + d]) - lo[d];
        if (e > ext)
            ext = e;
    }
    if (ext == 0.0)
        ext = 1.0;
    const double scale = 4294967296.0 / ext;
    const uint64_t mb = (uint64_t)ctl[3];
    const double mmax = mb ? from_ordbits(mb) : 0.0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = order[p];
        perm[p] = (int32_t)i;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double v = floor((x[3 * i + d] - lo[d]) * scale);
            q[d * n + p] = v >= 4294967295.0 ? 4294967295u : (v >= 0.0 ? (uint32_t)v : 0u);
        }
        uint32_t w = 1u;
        if (m && mmax > 0.0) {
            const double v = floor(m[i] / mmax * 16777216.0);
            w = v >= 1.0 ? (v <= 16777216.0 ? (uint32_t)v : 16777216u) : 1u;
        }
        q[3 * n + p] = w;
    }
}

// The root cell and, when it is to be cut, its chunks.
__global__ __launch_bounds__(256) void k_com_root(int64_t n, int leaf_size, int32_t *node,
                                                  int64_t cap, int32_t *act, int64_t *choff,
                                                  int32_t *chk, int64_t cap_c, int32_t *big,
                                                  int64_t *ctl)
{
    const int t = threadIdx.x;
    const bool cut = n > leaf_size;
    const int64_t nch = cut ? (n + COM_CHUNK - 1) / COM_CHUNK : 0;
    if (t == 0) {
        node[NF * cap] = 0;
        node[NC * cap] = (int32_t)n;
        node[NP * cap] = -1;
        node[NLV * cap] = 0;
        node[NAX * cap] = -1;
        node[NL * cap] = -1;
        node[NR * cap] = -1;
        node[NIR * cap] = -1;
        if (cut) {
            act[0] = 0;
            choff[0] = 0;
            choff[1] = nch;
        }
        ctl[0] = cut ? 1 : 0;
        ctl[1] = nch;
        ctl[2] = n >= 64 ? 1 : 0;
        if (n >= 64)
            big[0] = 0;
    }
    for (int64_t c = t; c < nch; c += blockDim.x) {
        chk[c] = 0;
        chk[cap_c + c] = (int32_t)(c * COM_CHUNK);
        chk[2 * cap_c + c] = (int32_t)std::min<int64_t>(n, (c + 1) * COM_CHUNK);
    }
}

// Per chunk: quantised box, sum w and sum w q_d (d = 0..2, 128-bit).
__global__ __launch_bounds__(CB) void k_com_stats(const uint32_t *__restrict__ q, int64_t n,
                                                  const int32_t *__restrict__ chk, int64_t cap_c,
                                                  uint64_t *cpart)
{
    __shared__ uint64_t sh[CB / 64][13];
    const int c = blockIdx.x;
    const int start = chk[cap_c + c], end = chk[2 * cap_c + c];
    uint32_t mn[3] = {~0u, ~0u, ~0u}, mx[3] = {0u, 0u, 0u};
    uint64_t sw = 0ull, lo[3] = {0ull, 0ull, 0ull}, hi[3] = {0ull, 0ull, 0ull};
    for (int p = start + threadIdx.x; p < end; p += CB) {
        const uint64_t w = q[3 * n + p];
        sw += w;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const uint32_t v = q[d * n + p];
            mn[d] = v < mn[d] ? v : mn[d];
            mx[d] = v > mx[d] ? v : mx[d];
            add128(lo[d], hi[d], w * (uint64_t)v, 0ull);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sw += __shfl_xor((unsigned long long)sw, off);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const uint32_t a = (uint32_t)__shfl_xor((int)mn[d], off);
            const uint32_t b = (uint32_t)__shfl_xor((int)mx[d], off);
            mn[d] = a < mn[d] ? a : mn[d];
            mx[d] = b > mx[d] ? b : mx[d];
            const uint64_t ol = __shfl_xor((unsigned long long)lo[d], off);
            const uint64_t oh = __shfl_xor((unsigned long long)hi[d], off);
            add128(lo[d], hi[d], ol, oh);
        }
    }
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0) {
        for (int d = 0; d < 3; ++d) {
            sh[wv][d] = mn[d];
            sh[wv][3 + d] = mx[d];
            sh[wv][7 + 2 * d] = lo[d];
            sh[wv][8 + 2 * d] = hi[d];
        }
        sh[wv][6] = sw;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t r[13];
        for (int k = 0; k < 13; ++k)
            r[k] = sh[0][k];
        for (int w = 1; w < CB / 64; ++w) {
            for (int d = 0; d < 3; ++d) {
                r[d] = sh[w][d] < r[d] ? sh[w][d] : r[d];
                r[3 + d] = sh[w][3 + d] > r[3 + d] ? sh[w][3 + d] : r[3 + d];
                add128(r[7 + 2 * d], r[8 + 2 * d], sh[w][7 + 2 * d], sh[w][8 + 2 * d]);
            }
            r[6] += sh[w][6];
        }
        uint64_t *o = cpart + 16 * (int64_t)c;
        for (int k = 0; k < 13; ++k)
            o[k] = r[k];
    }
}

// Per active cell: fold its chunks; axis, degenerate flag and the cut.
// split[4a] = axis | degenerate << 8, then sum w, sum w q_axis (lo, hi).
__global__ __launch_bounds__(256) void k_com_split(int64_t A, const int64_t *__restrict__ choff,
                                                  const uint64_t *__restrict__ cpart,
                                                  uint64_t *split)
{
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= A)
        return;
    uint64_t mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0ull, 0ull, 0ull};
    uint64_t sw = 0ull, lo[3] = {0ull, 0ull, 0ull}, hi[3] = {0ull, 0ull, 0ull};
    for (int64_t c = choff[a]; c < choff[a + 1]; ++c) {
        const uint64_t *r = cpart + 16 * c;
        for (int d = 0; d < 3; ++d) {
            mn[d] = r[d] < mn[d] ? r[d] : mn[d];
            mx[d] = r[3 + d] > mx[d] ? r[3 + d] : mx[d];
            add128(lo[d], hi[d], r[7 + 2 * d], r[8 + 2 * d]);
        }
        sw += r[6];
    }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
        if (mx[d] - mn[d] > mx[ax] - mn[ax])
            ax = d;
    const uint64_t degenerate = mx[ax] == mn[ax] ? 1ull : 0ull;
    split[4 * a] = (uint64_t)ax | (degenerate << 8);
    split[4 * a + 1] = sw;
    split[4 * a + 2] = lo[ax];
    split[4 * a + 3] = hi[ax];
}

__device__ __forceinline__ bool goes_left(const uint32_t *__restrict__ q, int64_t n, int p,
                                          int first, int count, const uint64_t *sp)
{
    const int ax = (int)(sp[0] & 0xffull);
    if (sp[0] >> 8)
        return p - first < (count + 1) / 2;  // one grid point: halve in tree order
    return left_of_cut(q[ax * n + p], sp[1], sp[2], sp[3]);
}

// Per chunk: particles going left.
__global__ __launch_bounds__(CB) void k_com_count(const uint32_t *__restrict__ q, int64_t n,
                                                  const int32_t *__restrict__ chk, int64_t cap_c,
                                                  const int32_t *__restrict__ act,
                                                  const int32_t *__restrict__ node, int64_t cap,
                                                  const uint64_t *__restrict__ split,
                                                  int32_t *cleft)
{
    __shared__ int sh[CB / 64];
    const int c = blockIdx.x;
    const int a = chk[c], start = chk[cap_c + c], end = chk[2 * cap_c + c];
    const int v = act[a];
    const int f = node[NF * cap + v], cnt = node[NC * cap + v];
    const uint64_t *sp = split + 4 * (int64_t)a;
    int k = 0;
    for (int p = start + threadIdx.x; p < end; p += CB)
        k += goes_left(q, n, p, f, cnt, sp) ? 1 : 0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        k += __shfl_xor(k, off);
    if (lane_id() == 0)
        sh[threadIdx.x >> 6] = k;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < CB / 64; ++w)
            tot += sh[w];
        cleft[c] = tot;
    }
}

// Per active cell, over its chunks in order: cleft becomes the exclusive base
// of the chunk's left particles, cbase that of its right particles; nl = the
// cell's left count.
__global__ __launch_bounds__(256) void k_com_offsets(int64_t A, const int64_t *__restrict__ choff,
                                                    const int32_t *__restrict__ chk,
                                                    int64_t cap_c, int32_t *cleft,
                                                    int32_t *cbase, int32_t *nl)
{
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= A)
        return;
    int rl = 0, rr = 0;
    for (int64_t c = choff[a]; c < choff[a + 1]; ++c) {
        const int len = chk[2 * cap_c + c] - chk[cap_c + c];
        const int l = cleft[c];
        cleft[c] = rl;
        cbase[c] = rr;
        rl += l;
        rr += len - l;
    }
    nl[a] = rl;
}

// Per chunk: stable partition into the copy, 256 particles per round in
// order (a round's lanes hold consecutive particles).
__global__ __launch_bounds__(CB) void k_com_scatter(
    const uint32_t *__restrict__ q, const int32_t *__restrict__ perm, int64_t n,
    const int32_t *__restrict__ chk, int64_t cap_c, const int32_t *__restrict__ act,
    const int32_t *__restrict__ node, int64_t cap, const uint64_t *__restrict__ split,
    const int32_t *__restrict__ cleft, const int32_t *__restrict__ cbase,
    const int32_t *__restrict__ nl, uint32_t *q_tmp, int32_t *perm_tmp)
{
    __shared__ int wl[CB / 64];
    const int c = blockIdx.x;
    const int a = chk[c], start = chk[cap_c + c], end = chk[2 * cap_c + c];
    const int v = act[a];
    const int f = node[NF * cap + v], cnt = node[NC * cap + v];
    const uint64_t *sp = split + 4 * (int64_t)a;
    int bl = f + cleft[c], br = f + nl[a] + cbase[c];
    const int wv = threadIdx.x >> 6;
    const uint64_t lt = lanemask_lt();
    for (int r0 = start; r0 < end; r0 += CB) {
        const int p = r0 + threadIdx.x;
        const bool valid = p < end;
        const bool left = valid && goes_left(q, n, p, f, cnt, sp);
        const uint64_t bal = __ballot(left);
        if (lane_id() == 0)
            wl[wv] = __popcll(bal);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < CB / 64; ++w) {
            before += w < wv ? wl[w] : 0;
            total += wl[w];
        }
        const int rank_l = before + __popcll(bal & lt);
        if (valid) {
            const int dst = left ? bl + rank_l : br + (threadIdx.x - rank_l);
#pragma unroll
            for (int d = 0; d < 4; ++d)
                q_tmp[d * n + dst] = q[d * n + p];
            perm_tmp[dst] = perm[p];
        }
        const int nvalid = min(CB, end - r0);
        bl += total;
        br += nvalid - total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(CB) void k_com_copyback(const int32_t *__restrict__ chk,
                                                     int64_t cap_c,
                                                     const uint32_t *__restrict__ q_tmp,
                                                     const int32_t *__restrict__ perm_tmp,
                                                     int64_t n, uint32_t *q, int32_t *perm)
{
    const int c = blockIdx.x;
    const int start = chk[cap_c + c], end = chk[2 * cap_c + c];
    for (int p = start + threadIdx.x; p < end; p += CB) {
#pragma unroll
        for (int d = 0; d < 4; ++d)
            q[d * n + p] = q_tmp[d * n + p];
        perm[p] = perm_tmp[p];
    }
}

// Per active cell a: children NN + 2a (left) and NN + 2a + 1 (right).
__global__ __launch_bounds__(256) void k_com_children(int64_t A, const int32_t *__restrict__ act,
                                                     const int32_t *__restrict__ nl,
                                                     const uint64_t *__restrict__ split,
                                                     int32_t *node, int64_t cap, int NN,
                                                     int level, int int_off)
{
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= A)
        return;
    const int v = act[a];
    const int f = node[NF * cap + v], c = node[NC * cap + v];
    const int l = NN + 2 * (int)a, r = l + 1;
    const int nleft = nl[a];
    const int fs[2] = {f, f + nleft}, cs[2] = {nleft, c - nleft}, ids[2] = {l, r};
    for (int k = 0; k < 2; ++k) {
        const int u = ids[k];
        node[NF * cap + u] = fs[k];
        node[NC * cap + u] = cs[k];
        node[NP * cap + u] = v;
        node[NLV * cap + u] = level + 1;
        node[NAX * cap + u] = -1;
        node[NL * cap + u] = -1;
        node[NR * cap + u] = -1;
        node[NIR * cap + u] = -1;
    }
    node[NL * cap + v] = l;
    node[NR * cap + v] = r;
    node[NAX * cap + v] = (int)(split[4 * a] & 0xffull);
    node[NIR * cap + v] = int_off + (int)a;
}

// One workgroup: over the children [NN, NN + m), the next level's active cells
// (count > leaf_size) with their chunks, and the children of >= 64 particles
// appended to the list of large cells.  ctl[0], ctl[1] = next A, C;
// ctl[2] += large cells.
constexpr int NEXT_T = 1024;

__device__ __forceinline__ int block_excl_scan(int v, int *sh, int &total)
{
    // inclusive scan within waves, then over the wave sums
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off)
            x += y;
    }
    if (lane == 63)
        sh[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int w = 0; w < NEXT_T / 64; ++w) {
            const int t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[NEXT_T / 64] = run;
    }
    __syncthreads();
    const int ex = sh[wv] + x - v;
    total = sh[NEXT_T / 64];
    __syncthreads();
    return ex;
}

__global__ __launch_bounds__(NEXT_T) void k_com_next(int NN, int m, int leaf_size,
                                                    const int32_t *__restrict__ node, int64_t cap,
                                                    int32_t *act, int64_t *choff, int32_t *chk,
                                                    int64_t cap_c, int32_t *big, int64_t *ctl)
{
    __shared__ int sh[NEXT_T / 64 + 1];
    int base_a = 0, base_b = (int)ctl[2];
    int64_t base_c = 0;
    for (int k0 = 0; k0 < m; k0 += NEXT_T) {
        const int k = k0 + threadIdx.x;
        const int u = NN + k;
        const int cnt = k < m ? node[NC * cap + u] : 0;
        const int isact = k < m && cnt > leaf_size ? 1 : 0;
        const int nch = isact ? (cnt + COM_CHUNK - 1) / COM_CHUNK : 0;
        const int isbig = k < m && cnt >= 64 ? 1 : 0;
        int ta, tc, tb;
        const int pa = block_excl_scan(isact, sh, ta);
        const int pc = block_excl_scan(nch, sh, tc);
        const int pb = block_excl_scan(isbig, sh, tb);
        if (isact) {
            const int ai = base_a + pa;
            const int64_t c0 = base_c + pc;
            act[ai] = u;
            choff[ai] = c0;
            const int f = node[NF * cap + u];
            for (int j = 0; j < nch; ++j) {
                chk[c0 + j] = ai;
                chk[cap_c + c0 + j] = f + j * COM_CHUNK;
                chk[2 * cap_c + c0 + j] = f + min(cnt, (j + 1) * COM_CHUNK);
            }
        }
        if (isbig)
            big[base_b + pb] = u;
        base_a += ta;
        base_c += tc;
        base_b += tb;
    }
    if (threadIdx.x == 0) {
        choff[base_a] = base_c;
        ctl[0] = base_a;
        ctl[1] = base_c;
        ctl[2] = base_b;
    }
}

// Renumbering.  Bottom-up, one level at a time: subtree node and leaf counts.
__global__ __launch_bounds__(256) void k_com_sizes(int b, int e, const int32_t *__restrict__ node,
                                                  int64_t cap, int32_t *ren)
{
    const int v = b + blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= e)
        return;
    const int l = node[NL * cap + v], r = node[NR * cap + v];
    if (l < 0) {
        ren[RSUB * cap + v] = 1;
        ren[RLEAF * cap + v] = 1;
    } else {
        ren[RSUB * cap + v] = 1 + ren[RSUB * cap + l] + ren[RSUB * cap + r];
        ren[RLEAF * cap + v] = ren[RLEAF * cap + l] + ren[RLEAF * cap + r];
    }
    if (v == 0) {  // the root opens the top-down pass
        ren[RPRE * cap] = 0;
        ren[RLOFS * cap] = 0;
    }
}

// Top-down, one level at a time: pre-order ids and leaf offsets of the
// children (left subtree first).
__global__ __launch_bounds__(256) void k_com_pre(int b, int e, const int32_t *__restrict__ node,
                                                int64_t cap, int32_t *ren)
{
    const int v = b + blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= e)
        return;
    const int l = node[NL * cap + v], r = node[NR * cap + v];
    if (l < 0)
        return;
    const int pv = ren[RPRE * cap + v], ov = ren[RLOFS * cap + v];
    ren[RPRE * cap + l] = pv + 1;
    ren[RPRE * cap + r] = pv + 1 + ren[RSUB * cap + l];
    ren[RLOFS * cap + l] = ov;
    ren[RLOFS * cap + r] = ov + ren[RLEAF * cap + l];
}

// Per BFS node: the topology arrays at its pre-order id.
__global__ __launch_bounds__(256) void k_com_emit(int NN, const int32_t *__restrict__ node,
                                                 int64_t cap, const int32_t *__restrict__ ren,
                                                 int32_t *first, int32_t *count, int32_t *left,
                                                 int32_t *right, int32_t *parent, int32_t *level,
                                                 int32_t *axis, int32_t *node_leaf,
                                                 int32_t *leaf_node, int32_t *int_nodes)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= NN)
        return;
    const int P = ren[RPRE * cap + v];
    const int l = node[NL * cap + v], r = node[NR * cap + v], pa = node[NP * cap + v];
    first[P] = node[NF * cap + v];
    count[P] = node[NC * cap + v];
    left[P] = l >= 0 ? ren[RPRE * cap + l] : -1;
    right[P] = r >= 0 ? ren[RPRE * cap + r] : -1;
    parent[P] = pa >= 0 ? ren[RPRE * cap + pa] : -1;
    level[P] = node[NLV * cap + v];
    axis[P] = node[NAX * cap + v];
    if (l < 0) {
        const int lf = ren[RLOFS * cap + v];
        node_leaf[P] = lf;
        leaf_node[lf] = P;
    } else {
        node_leaf[P] = -1;
        int_nodes[node[NIR * cap + v]] = P;
    }
}

__global__ __launch_bounds__(256) void k_com_bigmap(int nbig, const int32_t *__restrict__ bigbfs,
                                                   const int32_t *__restrict__ ren, int64_t cap,
                                                   int32_t *big_nodes)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nbig)
        big_nodes[k] = ren[RPRE * cap + bigbfs[k]];
}

static hipError_t read_ctl(Tree &t, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(t.cw.h_ctl, t.cw.ctl, 8 * sizeof(int64_t),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    return e;
}

hipError_t launch_build_com(Tree &t, const double *x, const double *m, hipStream_t s)
{
    Topology &T = t.topo;
    Tree::ComWork &W = t.cw;
    const int64_t n = T.n, cap = T.node_cap, cap_c = W.cap_c;
    hipError_t e = launch_morton_order(t, x, s);
    if (e != hipSuccess)
        return e;
    const int gs = (int)std::min<int64_t>((n + 255) / 256, 2048);
    k_com_zero<<<1, 64, 0, s>>>(W.ctl);
    if (m)
        k_com_mmax<<<gs, 256, 0, s>>>(m, n, W.ctl);
    k_com_init<<<gs, 256, 0, s>>>(x, m, n, t.bbox, W.ctl, t.vals0, t.perm, W.q);
    k_com_root<<<1, 256, 0, s>>>(n, T.leaf_size, W.node, cap, W.act[0], W.act_choff[0], W.chk[0],
                                 cap_c, W.big, W.ctl);
    if ((e = read_ctl(t, s)) != hipSuccess)
        return e;
    int64_t A = W.h_ctl[0], C = W.h_ctl[1];
    int NN = 1, level = 0, int_off = 0, cur = 0;
    W.lev_off.assign({0, 1});
    T.lvl_int_off.assign(1, 0);
    while (A > 0) {
        if (A > W.cap_a || C > cap_c || NN + 2 * A > cap)
            return hipErrorInvalidValue;  // impossible by the capacity bounds
        const int ga = (int)((A + 255) / 256);
        k_com_stats<<<(int)C, CB, 0, s>>>(W.q, n, W.chk[cur], cap_c, W.cpart);
        k_com_split<<<ga, 256, 0, s>>>(A, W.act_choff[cur], W.cpart, W.split);
        k_com_count<<<(int)C, CB, 0, s>>>(W.q, n, W.chk[cur], cap_c, W.act[cur], W.node, cap,
                                          W.split, W.cleft);
        k_com_offsets<<<ga, 256, 0, s>>>(A, W.act_choff[cur], W.chk[cur], cap_c, W.cleft,
                                         W.cbase, W.nl);
        k_com_scatter<<<(int)C, CB, 0, s>>>(W.q, t.perm, n, W.chk[cur], cap_c, W.act[cur],
                                            W.node, cap, W.split, W.cleft, W.cbase, W.nl,
                                            W.q_tmp, W.perm_tmp);
        k_com_copyback<<<(int)C, CB, 0, s>>>(W.chk[cur], cap_c, W.q_tmp, W.perm_tmp, n, W.q,
                                             t.perm);
        k_com_children<<<ga, 256, 0, s>>>(A, W.act[cur], W.nl, W.split, W.node, cap, NN, level,
                                          int_off);
        k_com_next<<<1, NEXT_T, 0, s>>>(NN, (int)(2 * A), T.leaf_size, W.node, cap,
                                        W.act[cur ^ 1], W.act_choff[cur ^ 1], W.chk[cur ^ 1],
                                        cap_c, W.big, W.ctl);
        if ((e = read_ctl(t, s)) != hipSuccess)
            return e;
        int_off += (int)A;
        T.lvl_int_off.push_back(int_off);
        NN += (int)(2 * A);
        W.lev_off.push_back(NN);
        ++level;
        A = W.h_ctl[0];
        C = W.h_ctl[1];
        cur ^= 1;
    }
    const int depth = level + 1;
    T.lvl_int_off.push_back(int_off);  // the deepest level holds leaves only
    const int nbig = (int)W.h_ctl[2];
    for (int l = depth - 1; l >= 0; --l) {
        const int b = W.lev_off[l], en = W.lev_off[l + 1];
        k_com_sizes<<<(en - b + 255) / 256, 256, 0, s>>>(b, en, W.node, cap, W.ren);
    }
    for (int l = 0; l + 1 < depth; ++l) {
        const int b = W.lev_off[l], en = W.lev_off[l + 1];
        k_com_pre<<<(en - b + 255) / 256, 256, 0, s>>>(b, en, W.node, cap, W.ren);
    }
    k_com_emit<<<(NN + 255) / 256, 256, 0, s>>>(NN, W.node, cap, W.ren, t.first, t.count, t.left,
                                               t.right, t.parent, t.level, t.axis, t.node_leaf,
                                               t.leaf_node, t.int_nodes);
    if (nbig > 0)
        k_com_bigmap<<<(nbig + 255) / 256, 256, 0, s>>>(nbig, W.big, W.ren, cap, t.big_nodes);
    T.nnodes = NN;
    T.nleaves = NN - int_off;
    T.depth = depth;
    T.nbig = nbig;
    return hipGetLastError();
}

}  // namespace fmm
