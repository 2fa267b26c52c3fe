// kd-tree build on gfx950.
//
// The paper's tree (Sec. 2) cuts every cell along its longest axis until a
// cell holds at most a few particles.  The cut used here is the count median
// of the longest axis of the cell's particle bounding box, ties broken by
// (coordinate, Morton rank); both halves keep ascending Morton rank.
//
// Steps (all on the caller's stream):
//   1. global bounding box (ordered-bit atomics, order-free);
//   2. 63-bit Morton keys of positions quantised to 2^21 per axis;
//   3. stable LSD radix sort by key -> Morton rank order (by halves, see
//      sort_by_halves; a tree whose earlier builds met long runs of equal
//      high halves sorts all eight digits instead);
//   4. three stable radix sorts by ordered coordinate bits, from rank order,
//      giving per axis the particles sorted by (x_d, rank);
//   5. for cells larger than SUBTREE_MAX, one level at a time: the median of
//      the longest axis is the middle entry of that axis's sorted segment, so
//      the split is a stable partition of the four lists (three axis lists +
//      the rank list); an entry's side follows from comparing its key
//      (coordinate bits, rank) with that of the last left entry;
//   6. every cell of at most SUBTREE_MAX particles is finished by one
//      workgroup in LDS (all levels below it), which writes the final order.
//
// Compiled with -ffp-contract=off: the quantisation and the split-axis test
// are single IEEE operations in the same order as the definition.
#include "fmm_internal.h"

namespace fmm {

// ---------------------------------------------------------------- bbox / keys
__global__ void k_bbox_init(uint64_t *bbox, uint32_t *err)
{
    int t = threadIdx.x;
    if (t < 3) {
        bbox[t] = ~0ull;
        bbox[3 + t] = 0ull;
    }
    if (t == 0)
        err[0] = 0u;
}

__global__ __launch_bounds__(256) void k_bbox(const double *__restrict__ x, int64_t n,
                                              uint64_t *bbox, uint32_t *err)
{
    __shared__ uint64_t sh[4][7];
    uint64_t mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0ull, 0ull, 0ull};
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double v = x[3 * i + d];
            bad |= !isfinite(v);
            uint64_t k = ordbits(v);
            mn[d] = k < mn[d] ? k : mn[d];
            mx[d] = k > mx[d] ? k : mx[d];
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            uint64_t a = __shfl_xor(mn[d], off);
            uint64_t b = __shfl_xor(mx[d], off);
            mn[d] = a < mn[d] ? a : mn[d];
            mx[d] = b > mx[d] ? b : mx[d];
        }
    const int w = threadIdx.x >> 6;
    uint64_t anybad = __ballot(bad);
    if (lane_id() == 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            sh[w][d] = mn[d];
            sh[w][3 + d] = mx[d];
        }
        sh[w][6] = anybad ? 1ull : 0ull;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        const int k = threadIdx.x;
        uint64_t r = sh[0][k];
        for (int i = 1; i < 4; ++i) {
            uint64_t o = sh[i][k];
            r = (k < 3) ? (o < r ? o : r) : (o > r ? o : r);
        }
        if (k < 3)
            atomicMin((unsigned long long *)&bbox[k], (unsigned long long)r);
        else if (k < 6)
            atomicMax((unsigned long long *)&bbox[k], (unsigned long long)r);
        else if (r)
            atomicOr(err, 1u);
    }
}

__device__ __forceinline__ uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__global__ void k_morton(const double *__restrict__ x, int64_t n, const uint64_t *bbox,
                         uint64_t *keys, uint32_t *vals)
{
    double lo[3], ext = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = from_ordbits(bbox[d]);
        double e = from_ordbits(bbox[3 + d]) - lo[d];
        if (e > ext)
            ext = e;
    }
    if (ext == 0.0)
        ext = 1.0;
    double scale = 2097152.0 / ext;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = 0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double t = floor((x[3 * i + d] - lo[d]) * scale);
            uint64_t q = t >= 2097151.0 ? 2097151ull : (t >= 0.0 ? (uint64_t)t : 0ull);
            k |= spread3(q) << d;
        }
        keys[i] = k;
        vals[i] = (uint32_t)i;
    }
}

// Coordinates in Morton-rank order, and the three axis keys (ordered bits,
// value = rank) for the per-axis sorts; the rank list starts as the identity.
__global__ void k_rank_gather(const double *__restrict__ x, int64_t n, const uint32_t *order,
                              int32_t *r2o, double *xr, uint64_t *keys, uint32_t *vals,
                              uint32_t *ranklist)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = order[r];
        r2o[r] = (int32_t)i;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double v = x[3 * i + d];
            xr[d * n + r] = v;
            keys[d * n + r] = ordbits(v);
            vals[d * n + r] = (uint32_t)r;
        }
        ranklist[r] = (uint32_t)r;
    }
}

// ---------------------------------------------------------------- radix sort
// Stable LSD radix sort of B independent (key u64, value u32) arrays of
// length n laid out back to back.  Per 8-bit pass: per-tile digit histograms,
// a scan per (digit, array) over the tiles that also stores the digit's
// total, then a stable scatter that adds the digit bases (a scan of the 256
// totals in LDS, so no tile updates a shared counter).  Inside a tile the 16
// waves take consecutive sixteenths; a wave ranks its 64 keys of a round with
// ballot-based digit matching, so rank order = input order.
__global__ void k_rs_zero(uint32_t *p, int64_t cnt)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

template <typename K, int BITS>
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const K *__restrict__ keys, int64_t n,
                                                        int shift, uint32_t *hist, int nblk)
{
    constexpr int NB = 1 << BITS;  // digits (at most RS_THREADS)
    __shared__ uint32_t h[NB];
    int b = blockIdx.y, blk = blockIdx.x, t = threadIdx.x;
    if (t < NB)
        h[t] = 0u;
    __syncthreads();
    const K *k = keys + (int64_t)b * n;
    int64_t base = (int64_t)blk * RS_TILE;
    // all loads first (indices past the end re-read key n - 1, not counted)
    K kr[RS_ROUNDS];
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r)
        kr[r] = k[min(base + r * RS_THREADS + t, n - 1)];
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r)
        if (base + r * RS_THREADS + t < n)
            atomicAdd(&h[(uint32_t)(kr[r] >> shift) & (NB - 1u)], 1u);
    __syncthreads();
    if (t < NB)
        hist[((int64_t)b * NB + t) * nblk + blk] = h[t];
}

// Exclusive scan across one block of up to 256 threads (values <= 2^32).
__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t *sh, uint32_t &total)
{
    int t = threadIdx.x, lane = lane_id(), w = t >> 6, nw = blockDim.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(inc, off);
        if (lane >= off)
            inc += o;
    }
    if (lane == 63)
        sh[w] = inc;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        uint32_t s = sh[i];
        wbase += i < w ? s : 0u;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return wbase + inc - v;
}

// Row (digit d of array b) of the tile histograms -> offsets of the tiles
// within the digit's output run; the row total goes to tot.
__global__ __launch_bounds__(RS_SCAN_THREADS) void k_rs_scan(uint32_t *hist, uint32_t *tot,
                                                             int nblk)
{
    __shared__ uint32_t sh[8];
    const int nb = gridDim.x;  // digits
    int d = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
    uint32_t *row = hist + ((int64_t)b * nb + d) * nblk;
    uint32_t run = 0;
    for (int c0 = 0; c0 < nblk; c0 += RS_SCAN_THREADS) {
        int i = c0 + t;
        uint32_t v = i < nblk ? row[i] : 0u;
        uint32_t total;
        uint32_t ex = block_excl_scan_u32(v, sh, total);
        if (i < nblk)
            row[i] = run + ex;
        run += total;
    }
    if (t == 0)
        tot[b * nb + d] = run;
}

template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid)
{
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < BITS; ++bit) {
        bool on = (d >> bit) & 1u;
        uint64_t bb = __ballot(valid && on);
        m &= on ? bb : ~bb;
    }
    return m;
}

// Stable scatter of one tile: rank the keys by digit (per wave, ballot
// matching; waves in order), place the tile digit-sorted in LDS, then write
// each digit's run to its global position with consecutive threads on
// consecutive addresses.  VALS = false: keys only (no values loaded, staged
// in LDS or written).
template <typename K, int BITS, bool VALS>
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(
    const K *__restrict__ kin, const uint32_t *__restrict__ vin, K *kout, uint32_t *vout,
    int64_t n, int shift, const uint32_t *__restrict__ hist, const uint32_t *__restrict__ tot,
    int nblk)
{
    constexpr int NB = 1 << BITS;  // digits, one per thread of the first NB threads
    constexpr uint32_t DM = NB - 1u;
    __shared__ K skey[RS_TILE];
    __shared__ uint32_t sval[VALS ? RS_TILE : 1];
    __shared__ uint16_t wrun[RS_WAVES][NB];
    __shared__ uint32_t loff[NB];
    __shared__ uint32_t gofs[NB];
    __shared__ uint32_t wtot[NB / 64], wtot2[NB / 64];
    const int b = blockIdx.y, blk = blockIdx.x, t = threadIdx.x, w = t >> 6, lane = lane_id();
    for (int i = t; i < RS_WAVES * NB; i += RS_THREADS)
        (&wrun[0][0])[i] = 0;
    __syncthreads();
    const K *k = kin + (int64_t)b * n;
    const uint32_t *v = VALS ? vin + (int64_t)b * n : nullptr;
    const int64_t tile0 = (int64_t)blk * RS_TILE;
    const int nv = (int)min((int64_t)RS_TILE, n - tile0);
    const int wbase = w * (RS_TILE / RS_WAVES);
    K key[RS_ROUNDS];
    uint32_t val[RS_ROUNDS];
    uint32_t rank[RS_ROUNDS];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int i = wbase + r * 64 + lane;
        key[r] = i < nv ? k[tile0 + i] : K(0);
        val[r] = (VALS && i < nv) ? v[tile0 + i] : 0u;
    }
    // this tile's offsets within the digit runs and the digit totals, loaded
    // while the keys are in flight
    const uint32_t gofs_t = t < NB ? hist[((int64_t)b * NB + t) * nblk + blk] : 0u;
    const uint32_t dtot = t < NB ? tot[b * NB + t] : 0u;
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const bool valid = wbase + r * 64 + lane < nv;
        const uint32_t d = valid ? (uint32_t)(key[r] >> shift) & DM : 0u;
        const uint64_t peers = match_digit<BITS>(d, valid);
        const uint32_t cur = wrun[w][d];
        rank[r] = cur + (uint32_t)__popcll(peers & lt);
        if (valid && (peers & lt) == 0ull)
            wrun[w][d] = (uint16_t)(cur + (uint32_t)__popcll(peers));
    }
    __syncthreads();
    // per digit: offsets of the waves, then the tile-local digit offsets
    uint32_t cnt = 0;
    if (t < NB) {
#pragma unroll
        for (int i = 0; i < RS_WAVES; ++i) {
            const uint32_t c = wrun[i][t];
            wrun[i][t] = (uint16_t)cnt;
            cnt += c;
        }
        // exclusive scans over the digits: tile-local offsets (of cnt) and
        // the digit bases (of the totals)
        uint32_t inc = cnt, inc2 = dtot;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off), o2 = __shfl_up(inc2, off);
            if (lane >= off) {
                inc += o;
                inc2 += o2;
            }
        }
        if (lane == 63) {
            wtot[w] = inc;
            wtot2[w] = inc2;
        }
        loff[t] = inc - cnt;
        gofs[t] = gofs_t + (inc2 - dtot);
    }
    __syncthreads();
    if (t < NB) {
        uint32_t add = 0, add2 = 0;
        for (int i = 0; i < w; ++i) {
            add += wtot[i];
            add2 += wtot2[i];
        }
        loff[t] += add;
        gofs[t] += add2;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        if (wbase + r * 64 + lane < nv) {
            const uint32_t d = (uint32_t)(key[r] >> shift) & DM;
            const uint32_t lp = loff[d] + wrun[w][d] + rank[r];
            skey[lp] = key[r];
            if constexpr (VALS)
                sval[lp] = val[r];
        }
    }
    __syncthreads();
    K *ko = kout + (int64_t)b * n;
    uint32_t *vo = VALS ? vout + (int64_t)b * n : nullptr;
    for (int j = t; j < nv; j += RS_THREADS) {
        const K kk = skey[j];
        const uint32_t d = (uint32_t)(kk >> shift) & DM;
        const int64_t gp = (int64_t)gofs[d] + (j - (int)loff[d]);
        ko[gp] = kk;
        if constexpr (VALS)
            vo[gp] = sval[j];
    }
}

// Sort B arrays of n (key, value) pairs by the low BITS * passes key bits
// (v0 == v1 == nullptr: keys only), BITS = 8 or 10 bits per pass.  The result
// ends in (k0, v0) after an even number of passes, in (k1, v1) after an odd
// one.  hist needs B * 2^BITS * ceil(n / RS_TILE) words, tot
// passes * B * 2^BITS.
template <typename K, int BITS>
static hipError_t radix_sort(K *k0, uint32_t *v0, K *k1, uint32_t *v1, int64_t n, int B,
                             int passes, uint32_t *hist, uint32_t *tot, hipStream_t s)
{
    constexpr int NB = 1 << BITS;
    int nblk = (int)((n + RS_TILE - 1) / RS_TILE);
    if (nblk == 0)
        return hipSuccess;
    for (int pass = 0; pass < passes; ++pass) {
        int shift = BITS * pass;
        K *ki = (pass & 1) ? k1 : k0, *ko = (pass & 1) ? k0 : k1;
        uint32_t *vi = (pass & 1) ? v1 : v0, *vo = (pass & 1) ? v0 : v1;
        uint32_t *tp = tot + (int64_t)pass * B * NB;
        dim3 g(nblk, B);
        k_rs_hist<K, BITS><<<g, RS_THREADS, 0, s>>>(ki, n, shift, hist, nblk);
        k_rs_scan<<<dim3(NB, B), RS_SCAN_THREADS, 0, s>>>(hist, tp, nblk);
        if (vi)
            k_rs_scatter<K, BITS, true><<<g, RS_THREADS, 0, s>>>(ki, vi, ko, vo, n, shift, hist,
                                                                 tp, nblk);
        else
            k_rs_scatter<K, BITS, false><<<g, RS_THREADS, 0, s>>>(ki, vi, ko, vo, n, shift, hist,
                                                                  tp, nblk);
    }
    return hipGetLastError();
}

hipError_t radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n,
                          int B, int passes, uint32_t *hist, uint32_t *tot, hipStream_t s,
                          int digit_bits)
{
    return digit_bits == 10
               ? radix_sort<uint64_t, 10>(k0, v0, k1, v1, n, B, passes, hist, tot, s)
               : radix_sort<uint64_t, 8>(k0, v0, k1, v1, n, B, passes, hist, tot, s);
}

// 32-bit keys: half the key traffic of the 64-bit sort.
hipError_t radix_sort_u32(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n,
                          int B, int passes, uint32_t *hist, uint32_t *tot, hipStream_t s,
                          int digit_bits)
{
    return digit_bits == 10
               ? radix_sort<uint32_t, 10>(k0, v0, k1, v1, n, B, passes, hist, tot, s)
               : radix_sort<uint32_t, 8>(k0, v0, k1, v1, n, B, passes, hist, tot, s);
}

// Passes and digit width for keys of `bits` bits: 10-bit digits where they
// take fewer passes than 8-bit ones.
void radix_plan(int bits, int &passes, int &digit_bits)
{
    const int p8 = (bits + 7) / 8, p10 = (bits + 9) / 10;
    digit_bits = p10 < p8 ? 10 : 8;
    passes = p10 < p8 ? p10 : p8;
}

// ---------------------------------------------------------------- (key, value) by halves
// Order by (key, value), the values being the input positions (so this is a
// stable sort by key): four LSD passes over the high 32 key bits, then the
// runs of equal high halves are put in (low half, value) order.  Runs of at
// most RUN_SHORT entries are ranked by one thread per entry; the (rare)
// longer ones by one workgroup each.  For the sorts of the build (Morton keys
// and ordered coordinate bits of spread-out particles) nearly every run has
// one entry, so this replaces the four low passes by one light pass.
constexpr int RUN_SHORT = 64;

__device__ __forceinline__ uint32_t hi32(uint64_t k) { return (uint32_t)(k >> 32); }

// A block stages its 256 entries with RUN_SHORT + 1 more on each side in
// LDS (coalesced loads), so that finding a run's ends and ranking inside it
// read LDS only.
constexpr int RUN_BLOCK = 256;
constexpr int RUN_HALO = RUN_SHORT + 1;

__global__ __launch_bounds__(RUN_BLOCK) void k_run_fix(const uint64_t *__restrict__ kin,
                                                       const uint32_t *__restrict__ vin,
                                                       uint64_t *kout, uint32_t *vout, int64_t n,
                                                       uint32_t *long_cnt, int64_t *long_list,
                                                       int64_t long_cap, uint32_t *err)
{
    __shared__ uint64_t sk[RUN_BLOCK + 2 * RUN_HALO];
    __shared__ uint32_t sv[RUN_BLOCK + 2 * RUN_HALO];
    const int b = blockIdx.y, t = threadIdx.x;
    const uint64_t *k = kin + (int64_t)b * n;
    const uint32_t *v = vin + (int64_t)b * n;
    uint64_t *ko = kout + (int64_t)b * n;
    uint32_t *vo = vout + (int64_t)b * n;
    for (int64_t base = (int64_t)blockIdx.x * RUN_BLOCK; base < n;
         base += (int64_t)gridDim.x * RUN_BLOCK) {
        // window [base - RUN_HALO, base + RUN_BLOCK + RUN_HALO) of the array
        for (int i = t; i < RUN_BLOCK + 2 * RUN_HALO; i += RUN_BLOCK) {
            const int64_t g = base - RUN_HALO + i;
            if (g >= 0 && g < n) {
                sk[i] = k[g];
                sv[i] = v[g];
            }
        }
        __syncthreads();
        const int64_t p = base + t;
        if (p < n) {
            const int i = t + RUN_HALO;  // window index of p
            const uint64_t kp = sk[i];
            const uint32_t vp = sv[i];
            const uint32_t hp = hi32(kp);
            const bool prev_same = p > 0 && hi32(sk[i - 1]) == hp;
            const bool next_same = p + 1 < n && hi32(sk[i + 1]) == hp;
            if (!prev_same && !next_same) {
                // a run of one entry (nearly all of them)
                ko[p] = kp;
                vo[p] = vp;
            } else {
                // window indices: ia - 1 >= i - RUN_SHORT - 1 >= 0 and
                // ie <= i + RUN_SHORT + 1 < RUN_BLOCK + 2 RUN_HALO
                int64_t a = p;
                int ia = i;
                while (a > 0 && p - a < RUN_SHORT && hi32(sk[ia - 1]) == hp) {
                    --a;
                    --ia;
                }
                bool lng = a > 0 && hi32(sk[ia - 1]) == hp;
                int64_t e = p + 1;
                int ie = i + 1;
                while (!lng && e < n && e - p <= RUN_SHORT && hi32(sk[ie]) == hp) {
                    ++e;
                    ++ie;
                }
                lng = lng || (e < n && hi32(sk[ie]) == hp) || e - a > RUN_SHORT;
                if (lng) {
                    if (!prev_same) {
                        const uint32_t slot = atomicAdd(long_cnt, 1u);
                        if ((int64_t)slot < long_cap)
                            long_list[slot] = ((int64_t)b << 40) | p;
                        else
                            atomicOr(err, 8u);
                    }
                } else {
                    const uint32_t lp = (uint32_t)kp;
                    int r = 0;
                    for (int q = ia; q < ie; ++q) {
                        const uint32_t lq = (uint32_t)sk[q], vq = sv[q];
                        r += (lq < lp || (lq == lp && vq < vp)) ? 1 : 0;
                    }
                    ko[a + r] = kp;
                    vo[a + r] = vp;
                }
            }
        }
        __syncthreads();
    }
}

// One workgroup per long run: find its end, then a stable LSD radix sort of
// the low key half in four 8-bit passes, ping-ponging between the run's
// segments of the input and output arrays.  The values of a run are already
// ascending (the high-half passes are stable and the values are the input
// positions), so the stable sort by the low half leaves it in (low half,
// value) order.
__global__ __launch_bounds__(RS_THREADS) void k_run_long(uint64_t *kin, uint32_t *vin,
                                                         uint64_t *kout, uint32_t *vout, int64_t n,
                                                         uint32_t *long_cnt,
                                                         const int64_t *__restrict__ long_list,
                                                         int64_t long_cap)
{
    __shared__ uint32_t hist[256];
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[RS_WAVES][256];
    __shared__ uint32_t ctot[256];
    __shared__ int64_t end_sh;
    const int t = threadIdx.x, w = t >> 6, lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const int64_t nl = min((int64_t)*long_cnt, long_cap);
    for (int64_t r = blockIdx.x; r < nl; r += gridDim.x) {
        const int64_t code = long_list[r];
        const int b = (int)(code >> 40);
        const int64_t a = code & ((1ll << 40) - 1);
        uint64_t *K[2] = {kin + (int64_t)b * n, kout + (int64_t)b * n};
        uint32_t *V[2] = {vin + (int64_t)b * n, vout + (int64_t)b * n};
        const uint32_t hp = hi32(K[0][a]);
        // end of the run: first position with another high half (or n)
        if (t == 0)
            end_sh = n;
        __syncthreads();
        for (int64_t c0 = a; c0 < n; c0 += RS_THREADS) {
            const int64_t q = c0 + t;
            if (q < n && hi32(K[0][q]) != hp)
                atomicMin((unsigned long long *)&end_sh, (unsigned long long)q);
            __syncthreads();
            const bool found = end_sh < n;
            __syncthreads();
            if (found)
                break;
        }
        const int64_t L = end_sh - a;
        if (t == 0)
            atomicAdd(&long_cnt[1], (uint32_t)L);  // entries in long runs, for the host
        for (int pass = 0; pass < 4; ++pass) {
            const int src = pass & 1, dst = src ^ 1;
            const uint64_t *ks = K[src] + a;
            const uint32_t *vs = V[src] + a;
            uint64_t *kd = K[dst] + a;
            uint32_t *vd = V[dst] + a;
            const int sh = 8 * pass;
            auto digit = [&](int64_t i) -> uint32_t { return ((uint32_t)ks[i] >> sh) & 255u; };
            if (t < 256)
                hist[t] = 0u;
            __syncthreads();
            for (int64_t i = t; i < L; i += RS_THREADS)
                atomicAdd(&hist[digit(i)], 1u);
            __syncthreads();
            if (t == 0) {
                uint32_t run = 0;
                for (int d = 0; d < 256; ++d) {
                    base[d] = run;
                    run += hist[d];
                }
            }
            __syncthreads();
            for (int64_t c0 = 0; c0 < L; c0 += RS_THREADS) {
                const int64_t i = c0 + t;
                const bool valid = i < L;
                const uint32_t d = valid ? digit(i) : 0u;
                for (int j = t; j < RS_WAVES * 256; j += RS_THREADS)
                    (&wcnt[0][0])[j] = 0u;
                __syncthreads();
                const uint64_t peers = match_digit<8>(d, valid);
                const uint32_t rk = (uint32_t)__popcll(peers & lt);
                if (valid && (peers & lt) == 0ull)
                    wcnt[w][d] = (uint32_t)__popcll(peers);
                __syncthreads();
                if (t < 256) {
                    uint32_t run = 0;
                    for (int ww = 0; ww < RS_WAVES; ++ww) {
                        const uint32_t c = wcnt[ww][t];
                        wcnt[ww][t] = run;
                        run += c;
                    }
                    ctot[t] = run;
                }
                __syncthreads();
                if (valid) {
                    const int64_t pos = (int64_t)base[d] + wcnt[w][d] + rk;
                    kd[pos] = ks[i];
                    vd[pos] = vs[i];
                }
                __syncthreads();
                if (t < 256)
                    base[t] += ctot[t];
                __syncthreads();
            }
        }
        // four passes end in the input arrays: copy the run to the output
        for (int64_t i = t; i < L; i += RS_THREADS) {
            K[1][a + i] = K[0][a + i];
            V[1][a + i] = V[0][a + i];
        }
        __syncthreads();
    }
}

// Sort B arrays of (key, position) pairs held in (k0, v0); the result lands
// in (k1, v1).  work: B * (n / (RUN_SHORT + 1) + 1) int64 for the long-run
// list; long_cnt[0] counts the long runs, long_cnt[1] their entries.
hipError_t sort_by_halves(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n,
                          int B, uint32_t *hist, uint32_t *tot, uint32_t *long_cnt,
                          int64_t *long_list, uint32_t *err, hipStream_t s)
{
    const int nblk = (int)((n + RS_TILE - 1) / RS_TILE);
    if (nblk == 0)
        return hipSuccess;
    const int64_t long_cap = (int64_t)B * (n / (RUN_SHORT + 1) + 1);
    k_rs_zero<<<1, 64, 0, s>>>(long_cnt, 2);
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 32 + 8 * pass;
        uint64_t *ki = (pass & 1) ? k1 : k0, *ko = (pass & 1) ? k0 : k1;
        uint32_t *vi = (pass & 1) ? v1 : v0, *vo = (pass & 1) ? v0 : v1;
        uint32_t *tp = tot + (int64_t)pass * B * 256;
        dim3 g(nblk, B);
        k_rs_hist<uint64_t, 8><<<g, RS_THREADS, 0, s>>>(ki, n, shift, hist, nblk);
        k_rs_scan<<<dim3(256, B), RS_SCAN_THREADS, 0, s>>>(hist, tp, nblk);
        k_rs_scatter<uint64_t, 8, true><<<g, RS_THREADS, 0, s>>>(ki, vi, ko, vo, n, shift, hist,
                                                               tp, nblk);
    }
    const int gf = (int)std::min<int64_t>((n + 255) / 256, 4096);
    k_run_fix<<<dim3(gf, B), 256, 0, s>>>(k0, v0, k1, v1, n, long_cnt, long_list, long_cap, err);
    k_run_long<<<256, RS_THREADS, 0, s>>>(k0, v0, k1, v1, n, long_cnt, long_list, long_cap);
    return hipGetLastError();
}

// ---------------------------------------------------------------- level kernels
// Longest axis of a node from its three sorted lists (first = min, last = max).
__device__ __forceinline__ int node_axis(const uint32_t *L, int64_t n, const double *xr,
                                         int64_t f, int64_t c)
{
    int ax = 0;
    double best = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double lo = xr[d * n + L[d * n + f]];
        double hi = xr[d * n + L[d * n + f + c - 1]];
        double e = hi - lo;
        if (d == 0 || e > best) {
            best = e;
            ax = d;
        }
    }
    return ax;
}

// The split of a cell: the left child takes the first ceil(c/2) entries of
// the longest axis's list, i.e. the particles whose key (ordered coordinate
// bits, Morton rank) is at most the key of entry ceil(c/2) - 1.
struct Split {
    int64_t f, nl;
    int ax;
    uint64_t ob;  // ordered coordinate bits of the last left entry
    uint32_t rm;  // its Morton rank
};

__device__ __forceinline__ Split node_split(const uint32_t *L, int64_t n, const double *xr,
                                            int64_t f, int64_t c)
{
    Split S;
    S.f = f;
    S.nl = (c + 1) / 2;
    S.ax = node_axis(L, n, xr, f, c);
    S.rm = L[S.ax * n + f + S.nl - 1];
    S.ob = ordbits(xr[S.ax * n + S.rm]);
    return S;
}

// Side of the entry at position p of list d (rank r): 1 = left child.
__device__ __forceinline__ uint32_t goes_left(const Split &S, const double *xr, int64_t n, int d,
                                              int64_t p, uint32_t r)
{
    if (d == S.ax)
        return p - S.f < S.nl ? 1u : 0u;
    const uint64_t o = ordbits(xr[S.ax * n + r]);
    return (o < S.ob || (o == S.ob && r <= S.rm)) ? 1u : 0u;
}

// Sides of a chunk of one list (also stored per position for the scatter)
// and the chunk's left count.  A chunk holds at most LVL_CHUNK entries, PER
// per thread: the entries are loaded before the split is found and the
// coordinates gathered all at once, so a thread waits for two memory round
// trips rather than two per entry.
__global__ __launch_bounds__(LVL_THREADS) void k_lvl_count(
    const uint32_t *__restrict__ L, int64_t n, const double *__restrict__ xr,
    const int32_t *blk_node, const int32_t *blk_start, const int32_t *blk_end,
    const int32_t *first, const int32_t *count, int32_t *axis_out, uint8_t *side, int32_t *cnt,
    int stride)
{
    constexpr int PER = LVL_CHUNK / LVL_THREADS;
    __shared__ uint32_t sh[8];
    const int b = blockIdx.x, d = blockIdx.y, t = threadIdx.x;
    const int v = blk_node[b];
    const int64_t s0 = blk_start[b], e0 = blk_end[b];
    const uint32_t *Ld = L + d * n;
    // loads past the chunk's end re-read its last entry (a chunk is never
    // empty) and are discarded, so that every load is issued unconditionally
    uint32_t r[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k)
        r[k] = Ld[min(s0 + t + k * LVL_THREADS, e0 - 1)];
    const Split S = node_split(L, n, xr, first[v], count[v]);
    if (d == 0 && t == 0 && s0 == S.f)
        axis_out[v] = S.ax;
    uint32_t g[PER];
    if (d == S.ax) {
#pragma unroll
        for (int k = 0; k < PER; ++k)
            g[k] = s0 + t + k * LVL_THREADS - S.f < S.nl ? 1u : 0u;
    } else {
        uint64_t o[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k)
            o[k] = ordbits(xr[S.ax * n + r[k]]);
#pragma unroll
        for (int k = 0; k < PER; ++k)
            g[k] = (o[k] < S.ob || (o[k] == S.ob && r[k] <= S.rm)) ? 1u : 0u;
    }
    uint8_t *sd = side + d * n;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t p = s0 + t + k * LVL_THREADS;
        if (p < e0) {
            sd[p] = (uint8_t)g[k];
            c += g[k];
        }
    }
    uint32_t total;
    block_excl_scan_u32(c, sh, total);
    if (t == 0)
        cnt[d * stride + b] = (int32_t)total;
}

// Sides by Morton rank at one level: each cell's longest-axis list gives
// them by position (its first ceil(c/2) entries go left), and the other
// lists of the cell then look their entries' sides up by rank (one byte per
// particle instead of a gathered coordinate).  For trees of LVL_BYRANK_MIN
// particles or more, whose coordinate arrays miss in L2; smaller ones gather
// the coordinates and save the extra launch per level.
constexpr int64_t LVL_BYRANK_MIN = int64_t(1) << 20;
__global__ __launch_bounds__(LVL_THREADS) void k_lvl_side(
    const uint32_t *__restrict__ L, int64_t n, const double *__restrict__ xr,
    const int32_t *blk_node, const int32_t *blk_start, const int32_t *blk_end,
    const int32_t *first, const int32_t *count, int32_t *axis_out, uint8_t *byrank)
{
    constexpr int PER = LVL_CHUNK / LVL_THREADS;
    const int b = blockIdx.x, t = threadIdx.x;
    const int v = blk_node[b];
    const int64_t s0 = blk_start[b], e0 = blk_end[b];
    const int64_t f = first[v], c = count[v], nl = (c + 1) / 2;
    const int ax = node_axis(L, n, xr, f, c);
    if (t == 0 && s0 == f)
        axis_out[v] = ax;
    const uint32_t *La = L + ax * n;
    uint32_t r[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k)
        r[k] = La[min(s0 + t + k * LVL_THREADS, e0 - 1)];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t p = s0 + t + k * LVL_THREADS;
        if (p < e0)
            byrank[r[k]] = p - f < nl ? 1 : 0;
    }
}

// Sides of a chunk of one list from the sides by rank (stored per position
// for the scatter) and the chunk's left count.
__global__ __launch_bounds__(LVL_THREADS) void k_lvl_count_byrank(
    const uint32_t *__restrict__ L, int64_t n, const int32_t *blk_node,
    const int32_t *blk_start, const int32_t *blk_end, const int32_t *first,
    const int32_t *count, const int32_t *__restrict__ axis, const uint8_t *__restrict__ byrank,
    uint8_t *side, int32_t *cnt, int stride)
{
    constexpr int PER = LVL_CHUNK / LVL_THREADS;
    __shared__ uint32_t sh[8];
    const int b = blockIdx.x, d = blockIdx.y, t = threadIdx.x;
    const int v = blk_node[b];
    const int64_t s0 = blk_start[b], e0 = blk_end[b];
    const int64_t f = first[v], nl = (count[v] + 1) / 2;
    const int ax = axis[v];
    uint32_t g[PER];
    if (d == ax) {
#pragma unroll
        for (int k = 0; k < PER; ++k)
            g[k] = s0 + t + k * LVL_THREADS - f < nl ? 1u : 0u;
    } else {
        const uint32_t *Ld = L + d * n;
        uint32_t r[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k)
            r[k] = Ld[min(s0 + t + k * LVL_THREADS, e0 - 1)];
#pragma unroll
        for (int k = 0; k < PER; ++k)
            g[k] = byrank[r[k]];
    }
    uint8_t *sd = side + d * n;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t p = s0 + t + k * LVL_THREADS;
        if (p < e0) {
            sd[p] = (uint8_t)g[k];
            c += g[k];
        }
    }
    uint32_t total;
    block_excl_scan_u32(c, sh, total);
    if (t == 0)
        cnt[d * stride + b] = (int32_t)total;
}

// Stable partition of one chunk of one list: the chunk is staged in LDS,
// each thread ranks PER consecutive entries, the chunk's left and right runs
// are assembled in LDS and written out as two contiguous runs.
__global__ __launch_bounds__(LVL_THREADS) void k_lvl_scatter(
    const uint32_t *__restrict__ Lsrc, uint32_t *Ldst, int64_t n, const uint8_t *__restrict__ side,
    const int32_t *blk_node, const int32_t *blk_start, const int32_t *blk_end,
    const int32_t *blk_first, const int32_t *first, const int32_t *count, const int32_t *cnt,
    int stride)
{
    constexpr int PER = LVL_CHUNK / LVL_THREADS;
    __shared__ uint32_t sh[8];
    __shared__ uint32_t sv[LVL_CHUNK];
    __shared__ uint32_t so[LVL_CHUNK];
    __shared__ uint8_t sf[LVL_CHUNK];
    const int b = blockIdx.x, d = blockIdx.y, t = threadIdx.x;
    const int v = blk_node[b];
    const int64_t f = first[v], nl = (count[v] + 1) / 2;
    const int64_t s = blk_start[b];
    const int len = (int)(blk_end[b] - s);
    const uint32_t *Ls = Lsrc + d * n + s;
    const uint8_t *sd = side + d * n + s;
    uint32_t *Ld = Ldst + d * n;
    uint32_t part = 0;
    {
        uint32_t lv[PER];
        uint8_t lf[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = min(t + k * LVL_THREADS, len - 1);  // len >= 1
            lv[k] = Ls[i];
            lf[k] = sd[i];
        }
        // left entries of the node before this chunk: the counts of the
        // node's earlier chunks, loaded while the chunk is in flight
        for (int j = blk_first[b] + t; j < b; j += LVL_THREADS)
            part += (uint32_t)cnt[d * stride + j];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = t + k * LVL_THREADS;
            if (i < len) {
                sv[i] = lv[k];
                sf[i] = lf[k];
            }
        }
    }
    __syncthreads();
    uint32_t fl[PER];
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = t * PER + k;
        fl[k] = i < len ? sf[i] : 0u;
        mine += fl[k];
    }
    uint32_t nleft;
    uint32_t lx = block_excl_scan_u32(mine, sh, nleft);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = t * PER + k;
        if (i < len) {
            const uint32_t pos = fl[k] ? lx : nleft + (uint32_t)i - lx;
            so[pos] = sv[i];
            lx += fl[k];
        }
    }
    __syncthreads();
    // then the two runs
    uint32_t before;
    block_excl_scan_u32(part, sh, before);
    const int64_t nb = (int64_t)before;
    const int64_t lbase = f + nb, rbase = f + nl + (s - f - nb);
    for (int i = t; i < len; i += LVL_THREADS)
        Ld[i < (int)nleft ? lbase + i : rbase + (i - (int)nleft)] = so[i];
}

// ---------------------------------------------------------------- LDS subtrees
// Exclusive scan of 64-bit packed counters across the block.
__device__ __forceinline__ uint64_t block_excl_scan_u64(uint64_t v, uint64_t *sh)
{
    int t = threadIdx.x, lane = lane_id(), w = t >> 6, nw = blockDim.x >> 6;
    uint64_t inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint64_t o = __shfl_up(inc, off);
        if (lane >= off)
            inc += o;
    }
    if (lane == 63)
        sh[w] = inc;
    __syncthreads();
    uint64_t wb = 0;
    for (int i = 0; i < nw; ++i)
        wb += i < w ? sh[i] : 0ull;
    __syncthreads();
    return wb + inc - v;
}

__device__ __forceinline__ int find_seg(const int16_t *sf, const int16_t *sn, int nseg, int p)
{
    int lo = 0, hi = nseg - 1, k = -1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        if (sf[mid] <= p) {
            k = mid;
            lo = mid + 1;
        } else {
            hi = mid - 1;
        }
    }
    if (k >= 0 && p < sf[k] + sn[k])
        return k;
    return -1;
}

__global__ __launch_bounds__(SUBTREE_THREADS) void k_subtree(
    const uint32_t *__restrict__ Lall, int64_t n, const double *__restrict__ xr,
    const int32_t *__restrict__ r2o, const int32_t *__restrict__ sub_root,
    const int32_t *__restrict__ first, const int32_t *__restrict__ count,
    const int32_t *__restrict__ left, const int32_t *__restrict__ right,
    const int32_t *__restrict__ level, int leaf_size, int32_t *perm, int32_t *axis_out)
{
    constexpr int PER = SUBTREE_MAX / SUBTREE_THREADS;  // 4 positions per thread
    __shared__ uint32_t rk[SUBTREE_MAX];
    __shared__ uint16_t lst[2][3][SUBTREE_MAX];
    __shared__ uint8_t flg[SUBTREE_MAX];
    __shared__ int16_t sf[2][SUBTREE_MAXSEG], sn[2][SUBTREE_MAXSEG];
    __shared__ int32_t snode[2][SUBTREE_MAXSEG];
    __shared__ uint8_t sax[SUBTREE_MAXSEG];
    __shared__ uint64_t segE[SUBTREE_MAXSEG];
    __shared__ uint32_t emit_ofs[SUBTREE_MAXSEG];
    __shared__ uint64_t shs[16];
    __shared__ int nseg_sh[2];

    const int t = threadIdx.x;
    const int root = sub_root[blockIdx.x];
    const int64_t f0 = first[root];
    const int n0 = count[root];
    const uint32_t *L = Lall + (int64_t)(level[root] & 1) * 4 * n;

    for (int p = t; p < n0; p += SUBTREE_THREADS)
        rk[p] = L[3 * n + f0 + p];
    __syncthreads();
    for (int d = 0; d < 3; ++d)
        for (int p = t; p < n0; p += SUBTREE_THREADS) {
            uint32_t r = L[d * n + f0 + p];
            int lo = 0, hi = n0;  // lower_bound in the ascending rank list
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (rk[mid] < r)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            lst[0][d][p] = (uint16_t)lo;
        }
    if (t == 0) {
        sf[0][0] = 0;
        sn[0][0] = (int16_t)n0;
        snode[0][0] = root;
        nseg_sh[0] = n0 > leaf_size ? 1 : 0;
    }
    __syncthreads();

    int cur = 0;
    int nseg = nseg_sh[0];
    while (nseg > 0) {
        const int nxt = cur ^ 1;
        // A. split axis per segment and the number of children that split again
        uint32_t my_emit[2] = {0u, 0u};
        for (int q = 0; q < 2; ++q) {
            int k = t * 2 + q;
            if (k < nseg) {
                int fk = sf[cur][k], nk = sn[cur][k];
                int ax = 0;
                double best = 0.0;
                for (int d = 0; d < 3; ++d) {
                    double lo = xr[d * n + rk[lst[cur][d][fk]]];
                    double hi = xr[d * n + rk[lst[cur][d][fk + nk - 1]]];
                    double e = hi - lo;
                    if (d == 0 || e > best) {
                        best = e;
                        ax = d;
                    }
                }
                sax[k] = (uint8_t)ax;
                axis_out[snode[cur][k]] = ax;
                int nl = (nk + 1) >> 1;
                my_emit[q] = (uint32_t)(nl > leaf_size) + (uint32_t)(nk - nl > leaf_size);
            }
        }
        {
            uint32_t tot2;
            uint32_t ex = block_excl_scan_u32(my_emit[0] + my_emit[1], (uint32_t *)shs, tot2);
            if (t * 2 < nseg)
                emit_ofs[t * 2] = ex;
            if (t * 2 + 1 < nseg)
                emit_ofs[t * 2 + 1] = ex + my_emit[0];
            if (t == 0)
                nseg_sh[nxt] = (int)tot2;
        }
        __syncthreads();
        // B. side flags, by local id, from the split axis's list
        for (int p = t; p < n0; p += SUBTREE_THREADS) {
            int k = find_seg(sf[cur], sn[cur], nseg, p);
            if (k >= 0) {
                int fk = sf[cur][k], nk = sn[cur][k];
                flg[lst[cur][sax[k]][p]] = (uint8_t)(p - fk < ((nk + 1) >> 1));
            }
        }
        __syncthreads();
        // C. packed exclusive scan of the flags of the three lists
        int segk[PER];
        uint64_t pk[PER];
        uint64_t mine = 0;
        const int pbase = t * PER;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int p = pbase + j;
            segk[j] = p < n0 ? find_seg(sf[cur], sn[cur], nseg, p) : -1;
            uint64_t v = 0;
            if (segk[j] >= 0) {
                v = (uint64_t)flg[lst[cur][0][p]] | ((uint64_t)flg[lst[cur][1][p]] << 21) |
                    ((uint64_t)flg[lst[cur][2][p]] << 42);
            }
            pk[j] = v;
            mine += v;
        }
        uint64_t ex = block_excl_scan_u64(mine, shs);
        uint64_t E[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            E[j] = ex;
            ex += pk[j];
            int p = pbase + j;
            if (segk[j] >= 0 && p == sf[cur][segk[j]])
                segE[segk[j]] = E[j];
        }
        __syncthreads();
        // D. stable partition into the other buffer; unsplit positions copy through
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int p = pbase + j;
            if (p >= n0)
                continue;
            int k = segk[j];
            if (k < 0) {
                for (int d = 0; d < 3; ++d)
                    lst[nxt][d][p] = lst[cur][d][p];
                continue;
            }
            int fk = sf[cur][k], nk = sn[cur][k], nl = (nk + 1) >> 1;
            uint64_t rel = E[j] - segE[k];
            for (int d = 0; d < 3; ++d) {
                int nb = (int)((rel >> (21 * d)) & 0x1fffffull);
                int fl = (int)((pk[j] >> (21 * d)) & 1ull);
                int pos = fl ? fk + nb : fk + nl + (p - fk - nb);
                lst[nxt][d][pos] = lst[cur][d][p];
            }
        }
        // next segments, in position order
        for (int k = t; k < nseg; k += SUBTREE_THREADS) {
            int fk = sf[cur][k], nk = sn[cur][k], nl = (nk + 1) >> 1;
            int node = snode[cur][k];
            uint32_t o = emit_ofs[k];
            if (nl > leaf_size) {
                sf[nxt][o] = (int16_t)fk;
                sn[nxt][o] = (int16_t)nl;
                snode[nxt][o] = left[node];
                ++o;
            }
            if (nk - nl > leaf_size) {
                sf[nxt][o] = (int16_t)(fk + nl);
                sn[nxt][o] = (int16_t)(nk - nl);
                snode[nxt][o] = right[node];
            }
        }
        __syncthreads();
        cur = nxt;
        nseg = nseg_sh[cur];
    }

    // leaves: members in ascending local id (= ascending Morton rank).  The
    // leaf holding position p follows from the split rule alone (the left
    // child takes the first ceil(c / 2) positions; a cell of more than
    // leaf_size particles splits), so it is found without memory reads.
    for (int p = t; p < n0; p += SUBTREE_THREADS) {
        int lf = 0, ln = n0;
        while (ln > leaf_size) {
            const int nl = (ln + 1) >> 1;
            if (p < lf + nl) {
                ln = nl;
            } else {
                lf += nl;
                ln -= nl;
            }
        }
        uint16_t me = lst[cur][0][p];
        int rank = 0;
        for (int q = 0; q < ln; ++q)
            rank += lst[cur][0][lf + q] < me;
        perm[f0 + lf + rank] = r2o[rk[me]];
    }
}

// ---------------------------------------------------------------- driver
// Bounding box (with the non-finite check) and the Morton order: sorted keys
// in keys0, caller indices in ascending Morton rank in vals0.
hipError_t launch_morton_order(Tree &t, const double *x, hipStream_t s)
{
    const int64_t n = t.topo.n;
    const int gs = (int)std::min<int64_t>((n + 255) / 256, 2048);
    k_bbox_init<<<1, 64, 0, s>>>(t.bbox, t.err);
    k_bbox<<<(int)std::min<int64_t>((n + 255) / 256, 256), 256, 0, s>>>(x, n, t.bbox, t.err);
    // Morton keys in (keys1, vals1) -> sorted into (keys0, vals0)
    k_morton<<<gs, 256, 0, s>>>(x, n, t.bbox, t.keys1, t.vals1);
    if (t.morton_full) {
        // concentrated data with distant outliers: most keys share their high
        // half, so the run fix would sort long runs one workgroup each; all
        // eight digits device-wide give the same (key, position) order
        hipError_t e = radix_sort_u64(t.keys1, t.vals1, t.keys0, t.vals0, n, 1, 8, t.rs_hist,
                                      t.rs_tot, s, 8);
        if (e == hipSuccess)
            e = hipMemcpyAsync(t.keys0, t.keys1, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(t.vals0, t.vals1, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        return e;
    }
    return sort_by_halves(t.keys1, t.vals1, t.keys0, t.vals0, n, 1, t.rs_hist, t.rs_tot,
                          t.run_cnt + 2, t.run_list, t.err, s);
}

hipError_t launch_build(Tree &t, const double *x, hipStream_t s)
{
    const Topology &T = t.topo;
    const int64_t n = T.n;
    const int gs = (int)std::min<int64_t>((n + 255) / 256, 2048);
    hipError_t e = launch_morton_order(t, x, s);
    if (e != hipSuccess)
        return e;
    // lists buffer 0: axis lists 0..2 and the rank list 3
    uint32_t *L0 = t.lists, *L1 = t.lists + 4 * n;
    k_rank_gather<<<gs, 256, 0, s>>>(x, n, t.vals0, t.r2o, t.xr, t.keys1, t.vals1, L0 + 3 * n);
    // the three axis arrays (keys1, vals1) -> sorted into (keys0, vals0); the
    // values are the Morton ranks, copied into list buffer 0.
    e = sort_by_halves(t.keys1, t.vals1, t.keys0, t.vals0, n, 3, t.rs_hist, t.rs_tot, t.run_cnt,
                       t.run_list, t.err, s);
    if (e != hipSuccess)
        return e;
    e = hipMemcpyAsync(L0, t.vals0, sizeof(uint32_t) * 3 * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess)
        return e;
    for (int l = 0; l < T.nlevels_up; ++l) {
        int b0 = T.lvl_blk_off[l], nb = T.lvl_blk_off[l + 1] - b0;
        const uint32_t *Ls = (l & 1) ? L1 : L0;
        uint32_t *Ld = (l & 1) ? L0 : L1;
        if (n >= LVL_BYRANK_MIN) {
            uint8_t *byrank = t.side + 4 * n;
            k_lvl_side<<<nb, LVL_THREADS, 0, s>>>(Ls, n, t.xr, t.blk_node + b0,
                                                  t.blk_start + b0, t.blk_end + b0, t.first,
                                                  t.count, t.axis, byrank);
            k_lvl_count_byrank<<<dim3(nb, 4), LVL_THREADS, 0, s>>>(
                Ls, n, t.blk_node + b0, t.blk_start + b0, t.blk_end + b0, t.first, t.count,
                t.axis, byrank, t.side, t.lvl_cnt, T.max_lvl_blocks);
        } else {
            k_lvl_count<<<dim3(nb, 4), LVL_THREADS, 0, s>>>(
                Ls, n, t.xr, t.blk_node + b0, t.blk_start + b0, t.blk_end + b0, t.first,
                t.count, t.axis, t.side, t.lvl_cnt, T.max_lvl_blocks);
        }
        k_lvl_scatter<<<dim3(nb, 4), LVL_THREADS, 0, s>>>(
            Ls, Ld, n, t.side, t.blk_node + b0, t.blk_start + b0, t.blk_end + b0,
            t.blk_first + b0, t.first, t.count, t.lvl_cnt, T.max_lvl_blocks);
    }
    int nsub = (int)T.sub_root.size();
    k_subtree<<<nsub, SUBTREE_THREADS, 0, s>>>(t.lists, n, t.xr, t.r2o, t.sub_root, t.first,
                                               t.count, t.left, t.right, t.level, T.leaf_size,
                                               t.perm, t.axis);
    return hipGetLastError();
}

}  // namespace fmm
