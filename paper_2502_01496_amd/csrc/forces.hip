// Far and near field on gfx950.
//
// M2L (eq. (6) of the paper and its first two r-derivatives): for a sink cell
// and a source cell with mass M, quadrupole Q about its centre of mass, and
// r = c_sink - c_source, the local expansion is L = (a, grad a, grad grad a)
// at c_sink.  With g_n = (-1)^n (2n-1)!! r^-(2n+1) (so d/dr_i g_n = g_{n+1} r_i),
// q = Q r, qq = r.q and
//   a0 = M g1 + g3 qq / 6,  a1 = M g2 + g4 qq / 6,  a2 = M g3 + g5 qq / 6,
//   b2 = g2 / 3, b3 = g3 / 3, b4 = g4 / 3:
//   L1_i   = a0 r_i + b2 q_i                                   (= eq. (6))
//   L2_ij  = a1 r_i r_j + a0 d_ij + b3 (r_i q_j + q_i r_j) + b2 Q_ij
//   L3_ijk = a2 r_i r_j r_k + a1 (d_ij r_k + d_ik r_j + d_jk r_i)
//            + b4 (r_i r_j q_k + r_i r_k q_j + r_j r_k q_i)
//            + b3 (d_ij q_k + d_ik q_j + d_jk q_i) + b3 (r_i Q_jk + r_j Q_ik + r_k Q_ij)
// The second expansion form (eqs. (25)-(26) with p = 3: combined order of the
// source and sink offsets at most 2) keeps L1 and replaces L2, L3 by the
// derivatives of the monopole field alone:
//   L2_ij  = A1 r_i r_j + A0 d_ij,  L3_ijk = A2 r_i r_j r_k + A1 (d_ij r_k + d_ik r_j + d_jk r_i),
//   A0 = M g1, A1 = M g2, A2 = M g3 (highest power of 1/r: 4, against 6).
// L2P (eq. (8)): a(y) = L1 + L2 y + 1/2 L3 : y y, y = x - c_sink.
// Near field (Sec. 3, eqs. (12)-(15), M4 kernel, R_kern = 2): particle i gets
//   -m_j * 1/2 [g(r, h_i) + g(r, h_j)] * (x_i - x_j) from every j != i of its
// near cells, with g = phi'/r:
//   q < 1:      h^-3 (4/3 - 6/5 q^2 + 1/2 q^3)
//   1 <= q < 2: h^-3 (8/3 - 3 q + 6/5 q^2 - 1/6 q^3) - 1/(15 r^3)
//   q >= 2:     1/r^3.
//
// Storage: symmetric rank-2 (xx,xy,xz,yy,yz,zz); rank-3
// (xxx,xxy,xxz,xyy,xyz,xzz,yyy,yyz,yzz,zzz).
#include <type_traits>

#include "fmm_internal.h"

namespace fmm {

template <typename T>
__device__ __forceinline__ T rsqrt_t(T x);
template <>
__device__ __forceinline__ double rsqrt_t<double>(double x) { return rsqrt(x); }
template <>
__device__ __forceinline__ float rsqrt_t<float>(float x) { return rsqrtf(x); }

// Second expansion form: L1 as eq. (6), L2 and L3 from the monopole only.
template <typename T>
__device__ __forceinline__ void m2l_acc_dehnen(T rx, T ry, T rz, T M, const T *Q, T *L)
{
    const T r2 = rx * rx + ry * ry + rz * rz;
    const T u = rsqrt_t<T>(r2);
    const T u2 = u * u;
    const T g1 = -u * u2;
    const T g2 = T(-3) * g1 * u2;
    const T g3 = T(-5) * g2 * u2;
    const T Qxx = Q[0], Qxy = Q[1], Qxz = Q[2], Qyy = Q[3], Qyz = Q[4], Qzz = Q[5];
    const T qx = Qxx * rx + Qxy * ry + Qxz * rz;
    const T qy = Qxy * rx + Qyy * ry + Qyz * rz;
    const T qz = Qxz * rx + Qyz * ry + Qzz * rz;
    const T qq = qx * rx + qy * ry + qz * rz;
    const T sixth = T(1) / T(6), third = T(1) / T(3);
    const T a0 = M * g1 + g3 * qq * sixth;
    const T b2 = g2 * third;
    const T A0 = M * g1, A1 = M * g2, A2 = M * g3;
    L[0] += a0 * rx + b2 * qx;
    L[1] += a0 * ry + b2 * qy;
    L[2] += a0 * rz + b2 * qz;
    const T A1x = A1 * rx, A1y = A1 * ry, A1z = A1 * rz;
    L[3] += A1x * rx + A0;
    L[4] += A1x * ry;
    L[5] += A1x * rz;
    L[6] += A1y * ry + A0;
    L[7] += A1y * rz;
    L[8] += A1z * rz + A0;
    const T A2x = A2 * rx, A2y = A2 * ry, A2z = A2 * rz;
    L[9] += A2x * rx * rx + T(3) * A1x;
    L[10] += A2x * rx * ry + A1y;
    L[11] += A2x * rx * rz + A1z;
    L[12] += A2x * ry * ry + A1x;
    L[13] += A2x * ry * rz;
    L[14] += A2x * rz * rz + A1x;
    L[15] += A2y * ry * ry + T(3) * A1y;
    L[16] += A2y * ry * rz + A1z;
    L[17] += A2y * rz * rz + A1y;
    L[18] += A2z * rz * rz + T(3) * A1z;
}

// One source -> sink M2L, accumulated into L[19]; FORM is FMM_EXPANSION_*.
template <typename T, int FORM>
__device__ __forceinline__ void m2l_acc(T rx, T ry, T rz, T M, const T *Q, T *L)
{
    if constexpr (FORM == FMM_EXPANSION_DEHNEN) {
        m2l_acc_dehnen<T>(rx, ry, rz, M, Q, L);
        return;
    }
    const T r2 = rx * rx + ry * ry + rz * rz;
    const T u = rsqrt_t<T>(r2);
    const T u2 = u * u;
    const T g1 = -u * u2;
    const T g2 = T(-3) * g1 * u2;
    const T g3 = T(-5) * g2 * u2;
    const T g4 = T(-7) * g3 * u2;
    const T g5 = T(-9) * g4 * u2;
    const T Qxx = Q[0], Qxy = Q[1], Qxz = Q[2], Qyy = Q[3], Qyz = Q[4], Qzz = Q[5];
    const T qx = Qxx * rx + Qxy * ry + Qxz * rz;
    const T qy = Qxy * rx + Qyy * ry + Qyz * rz;
    const T qz = Qxz * rx + Qyz * ry + Qzz * rz;
    const T qq = qx * rx + qy * ry + qz * rz;
    const T sixth = T(1) / T(6), third = T(1) / T(3);
    const T a0 = M * g1 + g3 * qq * sixth;
    const T a1 = M * g2 + g4 * qq * sixth;
    const T a2 = M * g3 + g5 * qq * sixth;
    const T b2 = g2 * third, b3 = g3 * third, b4 = g4 * third;
    // L1
    L[0] += a0 * rx + b2 * qx;
    L[1] += a0 * ry + b2 * qy;
    L[2] += a0 * rz + b2 * qz;
    // L2
    L[3] += a1 * rx * rx + a0 + b3 * (T(2) * rx * qx) + b2 * Qxx;
    L[4] += a1 * rx * ry + b3 * (rx * qy + qx * ry) + b2 * Qxy;
    L[5] += a1 * rx * rz + b3 * (rx * qz + qx * rz) + b2 * Qxz;
    L[6] += a1 * ry * ry + a0 + b3 * (T(2) * ry * qy) + b2 * Qyy;
    L[7] += a1 * ry * rz + b3 * (ry * qz + qy * rz) + b2 * Qyz;
    L[8] += a1 * rz * rz + a0 + b3 * (T(2) * rz * qz) + b2 * Qzz;
    // L3: the delta terms are folded per component
    const T a2x = a2 * rx, a2y = a2 * ry, a2z = a2 * rz;
    // xxx: rrr = x^3; dr = 3x; rrq = 3 x^2 qx; dq = 3 qx; rQ = 3 x Qxx
    L[9] += a2x * rx * rx + a1 * T(3) * rx + b4 * (T(3) * rx * rx * qx) + b3 * (T(3) * qx) +
            b3 * (T(3) * rx * Qxx);
    // xxy: dr = y; rrq = x^2 qy + 2 x y qx; dq = qy; rQ = 2 x Qxy + y Qxx
    L[10] += a2x * rx * ry + a1 * ry + b4 * (rx * rx * qy + T(2) * rx * ry * qx) + b3 * qy +
             b3 * (T(2) * rx * Qxy + ry * Qxx);
    // xxz
    L[11] += a2x * rx * rz + a1 * rz + b4 * (rx * rx * qz + T(2) * rx * rz * qx) + b3 * qz +
             b3 * (T(2) * rx * Qxz + rz * Qxx);
    // xyy: dr = x; rrq = y^2 qx + 2 x y qy; dq = qx; rQ = x Qyy + 2 y Qxy
    L[12] += a2x * ry * ry + a1 * rx + b4 * (ry * ry * qx + T(2) * rx * ry * qy) + b3 * qx +
             b3 * (rx * Qyy + T(2) * ry * Qxy);
    // xyz: dr = 0; rrq = xy qz + xz qy + yz qx; dq = 0; rQ = x Qyz + y Qxz + z Qxy
    L[13] += a2x * ry * rz + b4 * (rx * ry * qz + rx * rz * qy + ry * rz * qx) +
             b3 * (rx * Qyz + ry * Qxz + rz * Qxy);
    // xzz
    L[14] += a2x * rz * rz + a1 * rx + b4 * (rz * rz * qx + T(2) * rx * rz * qz) + b3 * qx +
             b3 * (rx * Qzz + T(2) * rz * Qxz);
    // yyy
    L[15] += a2y * ry * ry + a1 * T(3) * ry + b4 * (T(3) * ry * ry * qy) + b3 * (T(3) * qy) +
             b3 * (T(3) * ry * Qyy);
    // yyz
    L[16] += a2y * ry * rz + a1 * rz + b4 * (ry * ry * qz + T(2) * ry * rz * qy) + b3 * qz +
             b3 * (T(2) * ry * Qyz + rz * Qyy);
    // yzz
    L[17] += a2y * rz * rz + a1 * ry + b4 * (rz * rz * qy + T(2) * ry * rz * qz) + b3 * qy +
             b3 * (ry * Qzz + T(2) * rz * Qyz);
    // zzz
    L[18] += a2z * rz * rz + a1 * T(3) * rz + b4 * (T(3) * rz * rz * qz) + b3 * (T(3) * qz) +
             b3 * (T(3) * rz * Qzz);
}

// ---------------------------------------------------------------- list pieces
// Pieces per leaf for a list of min(cnt, cap) entries of `mult` work units
// each: ceil(work / per), at least one.
__global__ void k_piece_count(const int32_t *__restrict__ cnt, int cap, int nleaves, int mult,
                              int64_t per, int32_t *np)
{
    const int lf = blockIdx.x * blockDim.x + threadIdx.x;
    if (lf >= nleaves)
        return;
    const int64_t wk = (int64_t)max(0, min(cnt[lf], cap)) * mult;
    np[lf] = (int32_t)max<int64_t>(1, (wk + per - 1) / per);
}

__global__ void k_piece_fill(const int64_t *__restrict__ off, const int32_t *__restrict__ np,
                             int nleaves, int2 *list)
{
    const int lf = blockIdx.x * blockDim.x + threadIdx.x;
    if (lf >= nleaves)
        return;
    const int64_t extra = off[nleaves] - nleaves;
    for (int k = 0; k < np[lf]; ++k)
        list[piece_pos(off, extra, lf, k)] = make_int2(lf, k);
}

// Folding the partial sums of a split leaf's pieces, in piece order: one
// thread per extra list entry, the one holding piece 1 of its leaf folds it.
template <typename T>
__global__ __launch_bounds__(256) void k_m2l_fold(const int32_t *__restrict__ leaf_node,
                                                  const int64_t *__restrict__ off,
                                                  const int2 *__restrict__ list, int extra,
                                                  const T *__restrict__ part, T *Lout)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= extra || list[e].y != 1)
        return;
    const int lf = list[e].x;
    T L[19];
#pragma unroll
    for (int k = 0; k < 19; ++k)
        L[k] = T(0);
    const int np = (int)(off[lf + 1] - off[lf]);
    for (int q = 0; q < np; ++q) {
        const T *pp = part + (int64_t)NLOC * piece_pos(off, extra, lf, q);
#pragma unroll
        for (int k = 0; k < 19; ++k)
            L[k] += pp[k];
    }
    T *o = Lout + (int64_t)NLOC * leaf_node[lf];
#pragma unroll
    for (int k = 0; k < 19; ++k)
        o[k] = L[k];
    o[19] = T(0);
}

// ---------------------------------------------------------------- M2L at the leaves
// One source of the leaf M2L: FP64 records, or the FP32 form (r formed in
// FP64 and rounded, M and Q from the FP32 mirror of the records, FP32
// accumulation).
template <int FORM>
__device__ __forceinline__ void m2l_leaf_src(const double *__restrict__ recA,
                                             const double *__restrict__ recQ, const float *,
                                             int b, double c0, double c1, double c2, double *L)
{
    const double4 cb = *(const double4 *)(recA + (int64_t)NREC * b);
    const double *qb = recQ + (int64_t)NREC * b;
    const double2 q01 = *(const double2 *)qb, q23 = *(const double2 *)(qb + 2),
                  q45 = *(const double2 *)(qb + 4);
    const double Q[6] = {q01.x, q01.y, q23.x, q23.y, q45.x, q45.y};
    m2l_acc<double, FORM>(c0 - cb.x, c1 - cb.y, c2 - cb.z, cb.w, Q, L);
}
template <int FORM>
__device__ __forceinline__ void m2l_leaf_src(const double *__restrict__ recA, const double *,
                                             const float *__restrict__ recF, int b, double c0,
                                             double c1, double c2, float *L)
{
    const double4 cb = *(const double4 *)(recA + (int64_t)NREC * b);
    const float4 f0 = *(const float4 *)(recF + (int64_t)NREC * b);
    const float4 f1 = *(const float4 *)(recF + (int64_t)NREC * b + 4);
    const float Q[6] = {f0.y, f0.z, f0.w, f1.x, f1.y, f1.z};
    m2l_acc<float, FORM>((float)(c0 - cb.x), (float)(c1 - cb.y), (float)(c2 - cb.z), f0.x, Q, L);
}

// The FP32 form with the load of the source record apart from the
// arithmetic, so that the next source's record can be in flight while the
// current one is evaluated.
struct M2lSrc32 {
    double4 cb;
    float4 f0, f1;
};
__device__ __forceinline__ void m2l_src_load(const double *__restrict__ recA,
                                             const float *__restrict__ recF, int b, M2lSrc32 &S)
{
    S.cb = *(const double4 *)(recA + (int64_t)NREC * b);
    S.f0 = *(const float4 *)(recF + (int64_t)NREC * b);
    S.f1 = *(const float4 *)(recF + (int64_t)NREC * b + 4);
}
template <int FORM>
__device__ __forceinline__ void m2l_src_eval(const M2lSrc32 &S, double c0, double c1, double c2,
                                             float *L)
{
    const float Q[6] = {S.f0.y, S.f0.z, S.f0.w, S.f1.x, S.f1.y, S.f1.z};
    m2l_acc<float, FORM>((float)(c0 - S.cb.x), (float)(c1 - S.cb.y), (float)(c2 - S.cb.z), S.f0.x,
                         Q, L);
}

// M2L of eq. (6) at the sink leaves.  8 lanes per unit, 8 units per wave
// (consecutive leaves, whose far lists largely coincide, so the wave's loads
// of a source record often share an address); lanes stride the far list,
// and a butterfly sum over the unit's lanes ends each
// piece of `per` list entries; piece sums add up in piece order, starting
// from zero (fixed order: deterministic).  A unit is a leaf (pieces == nullptr: all its pieces in
// turn, total to Lout) or one entry of the piece list: the only piece of its
// leaf (total to Lout) or one piece of a split list (its sum to part, added
// by k_m2l_fold), with bit-identical totals either way.
constexpr int M2L_LANES = 8;  // lanes per unit

template <typename T, int FORM>
__global__ __launch_bounds__(256) void k_m2l_leaf(
    const double *__restrict__ recA, const double *__restrict__ recQ,
    const float *__restrict__ recF, const int32_t *__restrict__ leaf_node, int nunits,
    const int32_t *__restrict__ far_cnt, const int32_t *__restrict__ far_src, int cap_far,
    T *Lout, const int2 *__restrict__ pieces, int per, T *part)
{
    const int g = (xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x) / M2L_LANES;
    const int sub = threadIdx.x & (M2L_LANES - 1);
    const bool valid = g < nunits;
    const int2 pc = pieces && valid ? pieces[g] : make_int2(valid ? g : 0, 0);
    const int lf = pc.x;
    const int v = valid ? leaf_node[lf] : 0;
    const double *rv = recA + (int64_t)NREC * v;
    const double c0 = rv[0], c1 = rv[1], c2 = rv[2];
    const int nfull = valid ? max(0, min(far_cnt[lf], cap_far)) : 0;
    const int lo = pieces ? pc.y * per : 0;
    const int hi = pieces ? min(nfull, lo + per) : nfull;
    const int32_t *fl = far_src + (int64_t)lf * cap_far;
    const bool split = pieces && nfull > per;
    T *o = split ? part + (int64_t)NLOC * g : Lout + (int64_t)NLOC * v;
    if (valid && sub == 0) {
#pragma unroll
        for (int k = 0; k < NLOC; ++k)
            o[k] = T(0);
    }
    for (int p0 = lo; p0 < hi; p0 += per) {
        const int p1 = min(hi, p0 + per);
        T L[19];
#pragma unroll
        for (int k = 0; k < 19; ++k)
            L[k] = T(0);
        if constexpr (std::is_same<T, float>::value) {
            // FP32: the next source's record and the index after it are in
            // flight while the current source is evaluated (the FP64 form
            // keeps one wavefront more per SIMD without them, which pays more)
            M2lSrc32 cur;
            int bn = 0;
            if (p0 + sub < p1) {
                m2l_src_load(recA, recF, fl[p0 + sub], cur);
                if (p0 + sub + M2L_LANES < p1)
                    bn = fl[p0 + sub + M2L_LANES];
            }
            for (int k = p0 + sub; k < p1; k += M2L_LANES) {
                M2lSrc32 nxt;
                if (k + M2L_LANES < p1) {
                    m2l_src_load(recA, recF, bn, nxt);
                    if (k + 2 * M2L_LANES < p1)
                        bn = fl[k + 2 * M2L_LANES];
                }
                m2l_src_eval<FORM>(cur, c0, c1, c2, L);
                cur = nxt;
            }
        } else {
            // the next source's index is loaded one interaction ahead
            int bn = p0 + sub < p1 ? fl[p0 + sub] : 0;
            for (int k = p0 + sub; k < p1; k += M2L_LANES) {
                const int b = bn;
                if (k + M2L_LANES < p1)
                    bn = fl[k + M2L_LANES];
                m2l_leaf_src<FORM>(recA, recQ, recF, b, c0, c1, c2, L);
            }
        }
#pragma unroll
        for (int off = M2L_LANES / 2; off >= 1; off >>= 1)
#pragma unroll
            for (int k = 0; k < 19; ++k)
                L[k] += __shfl_xor(L[k], off);
        // the piece sums add up in the output itself (no registers held for a
        // running total), in piece order: 0 + L_0 + L_1 + ...
        if (valid && sub == 0) {
#pragma unroll
            for (int k = 0; k < 19; ++k)
                o[k] = o[k] + L[k];
        }
    }
}

// ---------------------------------------------------------------- P2P + L2P, FP64
__device__ __forceinline__ double m4g_f64(double q, double hinv3, double u3)
{
    // both pieces are evaluated and selected (no divergent branches)
    const double p1 = hinv3 * (4.0 / 3.0 + q * q * (-1.2 + 0.5 * q));
    const double p2 = hinv3 * (8.0 / 3.0 + q * (-3.0 + q * (1.2 - q * (1.0 / 6.0)))) -
                      u3 * (1.0 / 15.0);
    const double g = __builtin_unpredictable(q < 2.0) ? p2 : u3;
    return __builtin_unpredictable(q < 1.0) ? p1 : g;
}

// m / r^3 for finite r2 > 0: the hardware reciprocal square root y refined
// once with the series (1 - e)^(-1/2) = 1 + e/2 + 3/8 e^2 + O(e^3),
// e = 1 - r2 y^2, then cubed.
__device__ __forceinline__ double m_over_r3(double r2, double m)
{
    const double y = __builtin_amdgcn_rsq(r2);
    const double e = fma(-(r2 * y), y, 1.0);
    const double u = fma(y * e, fma(e, 0.375, 0.5), y);
    return m * ((u * u) * u);
}

// Reduce-scatter of 24 per-lane values over the 64 lanes of a wavefront.
// Each xor step halves the set of values a lane keeps (it sends the other
// half to its partner); after the steps over lane bits 5..1 a lane holds the
// partial sum of one value, and a last butterfly step finishes it.  Value
// index held by lane l: 12 b5 + 6 b4 + 3 b3 + (2 b2 + b1), valid when
// (2 b2 + b1) < 3.
template <typename T>
__device__ __forceinline__ T xchg_keep(T keep, T send, int off)
{
    return keep + __shfl_xor(send, off);
}

// Value index a lane holds after reduce_scatter24 (-1: none).
__device__ __forceinline__ int rs24_index(int lane)
{
    const int sub = 2 * ((lane >> 2) & 1) + ((lane >> 1) & 1);
    return sub < 3 ? 12 * ((lane >> 5) & 1) + 6 * ((lane >> 4) & 1) + 3 * ((lane >> 3) & 1) + sub
                   : -1;
}

template <typename T>
__device__ __forceinline__ T reduce_scatter24(const T *v, int lane)
{
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
    T a[12];
#pragma unroll
    for (int k = 0; k < 12; ++k)
        a[k] = xchg_keep<T>(b5 ? v[12 + k] : v[k], b5 ? v[k] : v[12 + k], 32);
    T b[6];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        b[k] = xchg_keep<T>(b4 ? a[6 + k] : a[k], b4 ? a[k] : a[6 + k], 16);
    T cc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        cc[k] = xchg_keep<T>(b3 ? b[3 + k] : b[k], b3 ? b[k] : b[3 + k], 8);
    const T d0 = xchg_keep<T>(b2 ? cc[2] : cc[0], b2 ? cc[0] : cc[2], 4);
    const T d1 = xchg_keep<T>(b2 ? T(0) : cc[1], b2 ? cc[1] : T(0), 4);
    T e = xchg_keep<T>(b1 ? d1 : d0, b1 ? d0 : d1, 2);
    e += __shfl_xor(e, 1);
    return e;
}

// Near field.  One wavefront per sink leaf; P2P_NS sink particles per pass
// are wave-uniform, and a step takes 8 source blocks (a near leaf gives
// ceil(leaf_size / 8) blocks of at most 8 particles): lane = 8 g + t holds
// particle t of the g-th block, loaded once per pass.  The block ranges of
// a chunk of the near list are staged in LDS (empty blocks dropped), and the
// next step's sources load while the current step computes.  Missing
// sources are the null record (far away, zero mass, zero smoothing length),
// which adds exactly zero.
//
// Every pair is first tested against the softening support of eqs. (14)-(15),
// with the largest 4 h^2 of the pass's sinks standing in for the sink's own:
// r^2 < max(H4, 4 h_j^2).  Pairs outside it are Newtonian for certain and
// take the form m / r^3 in the step.  Pairs inside are appended to their
// sink's queue in LDS (the source's tree position) and evaluated with the M4
// kernel, which is exact on both sides of the support, 64 at a time, so that
// the softened form runs with every lane busy instead of stalling a whole
// step whenever one of its pairs may be softened (a queue is drained each
// time it has gathered 64 pairs, and at the end of the pass).  The order of
// all additions depends on the lists only, so results are bitwise
// reproducible.
// The per-lane sums are reduce-scattered so that the lane holding component
// c of sink s adds L2P and writes G * a.
// One wavefront per workgroup: the leaves' near lists differ in length, and a
// workgroup's slots are only freed when its last wavefront ends.
constexpr int P2P_WAVES = 1;
constexpr int P2P_WG = 64 * P2P_WAVES;
constexpr int P2P_NS = 8;        // sinks per pass
constexpr int P2P_QCAP = 128;    // softened pairs a sink's queue holds (a step adds <= 64)
constexpr int P2P_BLOCKS = 256;  // source blocks staged in LDS per chunk

// Stage the non-empty blocks of list entries [c0, c0 + nc) (entry k: block
// k % nsub of near leaf k / nsub) in list order; returns their number.
__device__ __forceinline__ int stage_blocks_in_order(const int32_t *__restrict__ nl, int c0, int nc,
                                                     int nsub, const int32_t *__restrict__ first,
                                                     const int32_t *__restrict__ count, int lane,
                                                     int2 *R)
{
    int ne = 0;
    for (int k0 = 0; k0 < nc; k0 += 64) {
        const int k = k0 + lane;
        int2 r = make_int2(0, 0);
        if (k < nc) {
            const int e = (c0 + k) / nsub, u = (c0 + k) - e * nsub;
            const int bn = nl[e];
            r = make_int2(first[bn] + 8 * u, max(0, min(8, count[bn] - 8 * u)));
        }
        const bool keep = r.y > 0;
        const uint64_t mk = __ballot(keep);
        if (keep)
            R[ne + __popcll(mk & lanemask_lt())] = r;
        ne += __popcll(mk);
    }
    if (lane < 8)
        R[ne + lane] = make_int2(0, 0);  // eight empty blocks after the last one
    return ne;
}

// Source particle of a lane in block rg (the null record past its end).
__device__ __forceinline__ int64_t block_src(int2 rg, int slot, int64_t nnull)
{
    return slot < rg.y ? (int64_t)rg.x + slot : nnull;
}

// The softened pairs of sink q: cnt <= 64 entries of its queue from position
// head, one per lane, with the mean of the two M4 kernels.
template <int NS>
__device__ __forceinline__ void p2p_drain_f64(const double4 *__restrict__ pm,
                                              const double4 *__restrict__ ph,
                                              const int32_t *Q, int head, int cnt, int lane,
                                              int64_t nnull, double sx, double sy, double sz,
                                              double shi, double sh3, double &ax, double &ay,
                                              double &az)
{
    const int64_t j = lane < cnt ? (int64_t)Q[(head + lane) & (P2P_QCAP - 1)] : nnull;
    const double4 xj = pm[j];
    const double4 hj = ph[j];
    const double dx = sx - xj.x, dy = sy - xj.y, dz = sz - xj.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double u = r2 > 0.0 ? rsqrt_pos(r2) : 0.0;
    const double r = r2 * u;
    const double u3 = u * u * u;
    const double gi = m4g_f64(r * shi, sh3, u3);
    const double gj = m4g_f64(r * hj.x, hj.y, u3);
    const double fm = 0.5 * xj.w * (gi + gj);
    ax -= fm * dx;
    ay -= fm * dy;
    az -= fm * dz;
}

__global__ __launch_bounds__(P2P_WG) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_p2p_src_f64(
    const double4 *__restrict__ pm, const double4 *__restrict__ ph,
    const int32_t *__restrict__ first, const int32_t *__restrict__ count,
    const int32_t *__restrict__ leaf_node, int nleaves, const int32_t *__restrict__ near_cnt,
    const int32_t *__restrict__ near_src, int cap_near, int nsub, const double *__restrict__ Lloc,
    const double *__restrict__ recA, const int32_t *__restrict__ perm, double G, double r_kern,
    int64_t nnull, double *aout, const int2 *__restrict__ pieces, int per, double *part,
    int part_stride)
{
    constexpr int NS = P2P_NS;
    __shared__ int2 rng[P2P_WAVES][P2P_BLOCKS + 8];
    __shared__ int32_t que[P2P_WAVES][NS][P2P_QCAP];
    __shared__ double2 shh[P2P_WAVES][NS];  // 1/h, 1/h^3 of the pass's sinks
    (void)r_kern;
    const int w = threadIdx.x >> 6;
    const int unit =
        __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * P2P_WAVES + w);
    if (unit >= nleaves)
        return;
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const int grp = lane >> 3, slot = lane & 7;
    const int2 pc = pieces ? pieces[unit] : make_int2(unit, 0);
    const int leaf = pc.x;
    const int v = leaf_node[leaf];
    const int64_t f = first[v];
    const int c = count[v];
    const int nbf = max(0, min(near_cnt[leaf], cap_near)) * nsub;
    const int b_lo = pieces ? pc.y * per : 0;
    const int b_hi = pieces ? min(nbf, b_lo + per) : nbf;
    const int32_t *nl = near_src + (int64_t)leaf * cap_near;
    const double *rv = recA + (int64_t)NREC * v;
    const double *Lv = Lloc + (int64_t)NLOC * v;
    int2 *R = rng[w];
    for (int sb = 0; sb < c; sb += NS) {
        double sx[NS], sy[NS], sz[NS], H4 = 0.0;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int64_t is = f + min(sb + q, c - 1);
            const double4 x4 = pm[is];
            sx[q] = x4.x;
            sy[q] = x4.y;
            sz[q] = x4.z;
            const double h4q = ph[is].z;
            H4 = h4q > H4 ? h4q : H4;
        }
        if (lane < NS) {
            const double4 h4 = ph[f + min(sb + lane, c - 1)];
            shh[w][lane] = make_double2(h4.x, h4.y);
        }
        // pieces of `per` source blocks: each ends with its queues drained
        // and its per-lane sums reduce-scattered, and the piece sums add up
        // in piece order (the same sums, bit for bit, whether a wavefront
        // takes all of a leaf's pieces or one piece each)
        double tot = 0.0;
        double acc[3 * NS];
        int tail[NS];  // queue fill counts; entries [tail & ~63, tail) are pending
        auto drain = [&](int q, int head, int cnt) {
            const double2 hs = shh[w][q];
            p2p_drain_f64<NS>(pm, ph, que[w][q], head, cnt, lane, nnull, sx[q], sy[q], sz[q],
                              hs.x, hs.y, acc[3 * q], acc[3 * q + 1], acc[3 * q + 2]);
        };
        for (int p0 = b_lo; p0 < b_hi; p0 += per) {
        const int nb = min(b_hi, p0 + per);
#pragma unroll
        for (int q = 0; q < 3 * NS; ++q)
            acc[q] = 0.0;
#pragma unroll
        for (int q = 0; q < NS; ++q)
            tail[q] = 0;
        for (int c0 = p0; c0 < nb; c0 += P2P_BLOCKS) {
            const int nc = min(nb - c0, P2P_BLOCKS);
            const int ne = __builtin_amdgcn_readfirstlane(
                stage_blocks_in_order(nl, c0, nc, nsub, first, count, lane, R));
            __builtin_amdgcn_wave_barrier();
            for (int kb = 0; kb < ne; kb += 8) {
                // (the latency of these loads is covered by the other
                // wavefronts of the SIMD: no registers are held for a prefetch)
                const int32_t j = (int32_t)block_src(R[kb + grp], slot, nnull);
                const double4 xj = pm[j];
                const double hj4 = ph[j].z;
                const double hmax4 = hj4 > H4 ? hj4 : H4;
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    const double dx = sx[q] - xj.x, dy = sy[q] - xj.y, dz = sz[q] - xj.z;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    // (every lane is active here: the softened mask is the
                    // complement of the Newtonian one)
                    const bool newt = !(r2 < hmax4);
                    const uint64_t bal = ~__ballot(newt);
                    const double fm = newt ? m_over_r3(r2, xj.w) : 0.0;
                    acc[3 * q] -= fm * dx;
                    acc[3 * q + 1] -= fm * dy;
                    acc[3 * q + 2] -= fm * dz;
                    if (bal) {
                        // possibly softened pairs leave the step for the sink's queue
                        const int t0 = tail[q];
                        if (!newt)
                            que[w][q][(t0 + __popcll(bal & lt)) & (P2P_QCAP - 1)] = j;
                        tail[q] = t0 + __popcll(bal);
                        // a queue that has gathered another 64 pairs is evaluated
                        if ((tail[q] >> 6) != (t0 >> 6)) {
                            __builtin_amdgcn_wave_barrier();
                            drain(q, t0 & ~63, 64);
                        }
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int q = 0; q < NS; ++q)
            if (tail[q] & 63)
                drain(q, tail[q] & ~63, tail[q] & 63);
        __builtin_amdgcn_wave_barrier();
        tot += reduce_scatter24<double>(acc, lane);
        }
        const int idx = rs24_index(lane);
        const int q = idx / 3, comp = idx - 3 * (idx / 3);
        if (pieces && nbf > per) {
            if (idx >= 0 && (lane & 1) == 0 && sb + q < c)
                part[(int64_t)unit * part_stride + 3 * (sb + q) + comp] = tot;
        } else if (idx >= 0 && (lane & 1) == 0 && sb + q < c) {
            // component comp of eq. (8) at sink q
            double sxq = sx[0], syq = sy[0], szq = sz[0];
#pragma unroll
            for (int r = 1; r < NS; ++r)
                if (q == r) {
                    sxq = sx[r];
                    syq = sy[r];
                    szq = sz[r];
                }
            double Lr[19];
#pragma unroll
            for (int k = 0; k < 19; ++k)
                Lr[k] = Lv[k];
            double fx, fy, fz;
            l2p<double>(Lr, sxq - rv[0], syq - rv[1], szq - rv[2], fx, fy, fz);
            const double far_c = comp == 0 ? fx : (comp == 1 ? fy : fz);
            const int64_t o = 3 * (int64_t)perm[f + sb + q] + comp;
            aout[o] = G * (far_c + tot);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------- FP32 form
__device__ __forceinline__ float m4g_f32(float q, float hinv3, float u3)
{
    // both pieces are evaluated and selected (no divergent branches)
    const float p1 = hinv3 * (4.0f / 3.0f + q * q * (-1.2f + 0.5f * q));
    const float p2 = hinv3 * (8.0f / 3.0f + q * (-3.0f + q * (1.2f - q * (1.0f / 6.0f)))) -
                     u3 * (1.0f / 15.0f);
    const float g = __builtin_unpredictable(q < 2.0f) ? p2 : u3;
    return __builtin_unpredictable(q < 1.0f) ? p1 : g;
}

// FP32 near field with leaf-relative offsets: for a sink in leaf a and a
// source in leaf b, x_i - x_j = (c_a - c_b) + (y_i - y_j) with c_a - c_b formed
// in FP64 and rounded once per leaf pair, and y = x - c_leaf stored in FP32.
// Eight sinks per pass (wave-uniform), source per lane, FP32 accumulation;
// pf[p] = (y, m), pfh[p] = (1/h, 1/h^3, 4 h^2, 0), all rounded from FP64.
// A step whose pairs all lie outside both softening supports of eqs.
// (14)-(15) takes the Newtonian form; otherwise the whole step takes the M4
// form (exact on both sides of the support).  In FP32 the M4 form costs
// little more than the Newtonian one, so, unlike the FP64 kernel, no pair is
// deferred: instead the blocks of a chunk of the near list whose leaves lie
// within CLOSE_FRAC of the bound of eq. (5),
//   |c_a - c_b| < CLOSE_FRAC ((s_a + s_b) + R_kern max(h_a, h_b)),
// are staged first (each group in list order), so that the softened pairs
// gather in few steps.  The order of all additions depends on the lists
// only.  Long lists are cut into pieces of `per` blocks as in the FP64
// kernel.
__device__ __forceinline__ float rsq_pos_f(float x) { return __builtin_amdgcn_rsqf(x); }

constexpr int P2P_RANGES_F32 = 256;    // blocks staged in LDS per chunk
constexpr double CLOSE_FRAC2 = 0.49;   // CLOSE_FRAC = 0.7, squared

// Position of a block in the partitioned chunk; front / back are the
// wave-uniform fill positions (front grows from 0, back shrinks from nc).
__device__ __forceinline__ int close_first_slot(bool act, bool close, int &front, int &back)
{
    const uint64_t lt = lanemask_lt();
    const uint64_t mc = __ballot(act && close), mf = __ballot(act && !close);
    const int nf = __popcll(mf);
    const int pos = close ? front + __popcll(mc & lt) : back - nf + __popcll(mf & lt);
    front += __popcll(mc);
    back -= nf;
    return pos;
}

// Staged position of step block k (close blocks, then the far ones after the
// gap left by dropped empty blocks).
__device__ __forceinline__ int skip_gap(int k, int front, int gap)
{
    return k < front ? k : k + gap;
}

__global__ __launch_bounds__(P2P_WG) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_p2p_src_f32(
    const float4 *__restrict__ pf, const float4 *__restrict__ pfh,
    const int32_t *__restrict__ first,
    const int32_t *__restrict__ count, const int32_t *__restrict__ leaf_node, int nleaves,
    const int32_t *__restrict__ near_cnt, const int32_t *__restrict__ near_src, int cap_near,
    int nsub, const float *__restrict__ Lloc, const double *__restrict__ recA,
    const int32_t *__restrict__ perm, float G, double r_kern, float *aout,
    const int2 *__restrict__ pieces, int per, float *part, int part_stride)
{
    constexpr int NS = P2P_NS;
    constexpr int NR = P2P_RANGES_F32;
    __shared__ int2 rng[P2P_WAVES][NR + 8];
    __shared__ float4 dcs[P2P_WAVES][NR + 8];
    const int w = threadIdx.x >> 6;
    const int unit =
        __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * P2P_WAVES + w);
    if (unit >= nleaves)
        return;
    const int lane = lane_id();
    const int grp = lane >> 3, slot = lane & 7;
    const int2 pc = pieces ? pieces[unit] : make_int2(unit, 0);
    const int leaf = pc.x;
    const int v = leaf_node[leaf];
    const int64_t f = first[v];
    const int c = count[v];
    const int nbf = max(0, min(near_cnt[leaf], cap_near)) * nsub;
    const int b_lo = pieces ? pc.y * per : 0;
    const int b_hi = pieces ? min(nbf, b_lo + per) : nbf;
    const int32_t *nl = near_src + (int64_t)leaf * cap_near;
    const double *rv = recA + (int64_t)NREC * v;
    const double ca0 = rv[0], ca1 = rv[1], ca2 = rv[2];
    const float *Lv = Lloc + (int64_t)NLOC * v;
    int2 *R = rng[w];
    float4 *D = dcs[w];
    for (int sb = 0; sb < c; sb += NS) {
        float sx[NS], sy[NS], sz[NS], shi[NS], sh3[NS], sh4[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int64_t is = f + min(sb + q, c - 1);
            const float4 y4 = pf[is];
            const float4 h4 = pfh[is];
            sx[q] = y4.x;
            sy[q] = y4.y;
            sz[q] = y4.z;
            shi[q] = h4.x;
            sh3[q] = h4.y;
            sh4[q] = h4.z;
        }
        float tot = 0.0f;
        for (int p0 = b_lo; p0 < b_hi; p0 += per) {
        const int nb = min(b_hi, p0 + per);
        float acc[3 * NS];
#pragma unroll
        for (int q = 0; q < 3 * NS; ++q)
            acc[q] = 0.0f;
        for (int c0 = p0; c0 < nb; c0 += NR) {
            const int nc = min(nb - c0, NR);
            // stage the source blocks of this chunk: their particle range and
            // the leaf-centre difference c_a - c_b, formed in FP64 and rounded
            // to FP32; close leaves first, empty blocks dropped, eight empty
            // blocks after the last one
            int front = 0, back = nc;
            for (int k0 = 0; k0 < nc; k0 += 64) {
                const int k = k0 + lane;
                int2 r = make_int2(0, 0);
                float4 d = make_float4(0.f, 0.f, 0.f, 0.f);
                bool close = false;
                if (k < nc) {
                    const int e = (c0 + k) / nsub, u = (c0 + k) - e * nsub;
                    const int bn = nl[e];
                    r = make_int2(first[bn] + 8 * u, max(0, min(8, count[bn] - 8 * u)));
                    const double *rb = recA + (int64_t)NREC * bn;
                    const double dx = ca0 - rb[0], dy = ca1 - rb[1], dz = ca2 - rb[2];
                    d = make_float4((float)dx, (float)dy, (float)dz, 0.f);
                    const double t5 = (rv[4] + rb[4]) + r_kern * fmax(rv[5], rb[5]);
                    close = dx * dx + dy * dy + dz * dz < CLOSE_FRAC2 * t5 * t5;
                }
                const bool keep = r.y > 0;
                const int pos = close_first_slot(keep, close, front, back);
                if (keep) {
                    R[pos] = r;
                    D[pos] = d;
                }
            }
            front = __builtin_amdgcn_readfirstlane(front);
            const int gap = __builtin_amdgcn_readfirstlane(back - front), ne = nc - gap;
            if (lane < 8) {
                R[nc + lane] = make_int2(0, 0);
                D[nc + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
            __builtin_amdgcn_wave_barrier();
            for (int kb = 0; kb < ne; kb += 8) {
                const int kk = skip_gap(kb + grp, front, gap);
                const int2 rg = R[kk];
                const float4 dc = D[kk];
                // a missing source reads particle 0 (an empty block's start
                // may be one past the last particle) and is then replaced by
                // a far, massless one
                const bool valid = slot < rg.y;
                const int64_t j = valid ? (int64_t)rg.x + slot : 0;
                float4 yj = pf[j];
                float4 hj = pfh[j];
                if (!valid) {
                    yj = make_float4(1e30f, 1e30f, 1e30f, 0.0f);
                    hj.z = 0.0f;
                }
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    const float dx = dc.x + (sx[q] - yj.x), dy = dc.y + (sy[q] - yj.y),
                                dz = dc.z + (sz[q] - yj.z);
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    float fm;
                    if ((__ballot(r2 < hj.z) | __ballot(r2 < sh4[q])) == 0ull) {
                        const float u = rsq_pos_f(r2);
                        fm = yj.w * (u * u * u);
                    } else {
                        const float u = r2 > 0.0f ? rsq_pos_f(r2) : 0.0f;
                        const float r = r2 * u;
                        const float u3 = u * u * u;
                        const float gi = m4g_f32(r * shi[q], sh3[q], u3);
                        const float gj = m4g_f32(r * hj.x, hj.y, u3);
                        fm = yj.w * 0.5f * (gi + gj);
                    }
                    acc[3 * q] -= fm * dx;
                    acc[3 * q + 1] -= fm * dy;
                    acc[3 * q + 2] -= fm * dz;
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        tot += reduce_scatter24<float>(acc, lane);
        }
        const int idx = rs24_index(lane);
        const int q = idx / 3, comp = idx - 3 * (idx / 3);
        if (pieces && nbf > per) {
            if (idx >= 0 && (lane & 1) == 0 && sb + q < c)
                part[(int64_t)unit * part_stride + 3 * (sb + q) + comp] = tot;
        } else if (idx >= 0 && (lane & 1) == 0 && sb + q < c) {
            float sxq = sx[0], syq = sy[0], szq = sz[0];
#pragma unroll
            for (int r = 1; r < NS; ++r)
                if (q == r) {
                    sxq = sx[r];
                    syq = sy[r];
                    szq = sz[r];
                }
            float Lr[19];
#pragma unroll
            for (int k = 0; k < 19; ++k)
                Lr[k] = Lv[k];
            float fx, fy, fz;
            l2p<float>(Lr, sxq, syq, szq, fx, fy, fz);
            const float far_c = comp == 0 ? fx : (comp == 1 ? fy : fz);
            const int64_t o = 3 * (int64_t)perm[f + sb + q] + comp;
            aout[o] = G * (far_c + tot);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------- mutual walk
// Far field of the mutual walk: M2L into every sink cell over its CSR range
// of the sorted (sink, source) keys, then L2L down to the leaves.
template <int FORM>
__device__ __forceinline__ void m2l_node_src(const double *recA, const double *recQ,
                                             const float *, int b, double c0, double c1,
                                             double c2, double *L)
{
    const double4 cb = *(const double4 *)(recA + (int64_t)NREC * b);
    const double *qb = recQ + (int64_t)NREC * b;
    const double2 q01 = *(const double2 *)qb, q23 = *(const double2 *)(qb + 2),
                  q45 = *(const double2 *)(qb + 4);
    const double Q[6] = {q01.x, q01.y, q23.x, q23.y, q45.x, q45.y};
    m2l_acc<double, FORM>(c0 - cb.x, c1 - cb.y, c2 - cb.z, cb.w, Q, L);
}
template <int FORM>
__device__ __forceinline__ void m2l_node_src(const double *recA, const double *,
                                             const float *recF, int b, double c0, double c1,
                                             double c2, float *L)
{
    const double4 cb = *(const double4 *)(recA + (int64_t)NREC * b);
    const float4 f0 = *(const float4 *)(recF + (int64_t)NREC * b);
    const float4 f1 = *(const float4 *)(recF + (int64_t)NREC * b + 4);
    const float Q[6] = {f0.y, f0.z, f0.w, f1.x, f1.y, f1.z};
    m2l_acc<float, FORM>((float)(c0 - cb.x), (float)(c1 - cb.y), (float)(c2 - cb.z), f0.x, Q, L);
}

// 16 lanes per sink cell (all cells; zero where the range is empty).
template <typename T, int FORM>
__global__ __launch_bounds__(256) void k_m2l_node(const double *__restrict__ recA,
                                                  const double *__restrict__ recQ,
                                                  const float *__restrict__ recF, int nnodes,
                                                  const int64_t *__restrict__ fstart,
                                                  const int64_t *__restrict__ fend,
                                                  const uint64_t *__restrict__ keys,
                                                  uint64_t mask, T *Lown)
{
    const int v = (blockIdx.x * 256 + threadIdx.x) >> 4;
    const int sub = threadIdx.x & 15;
    const bool valid = v < nnodes;
    const double *rv = recA + (int64_t)NREC * (valid ? v : 0);
    const double c0 = rv[0], c1 = rv[1], c2 = rv[2];
    T L[19];
#pragma unroll
    for (int k = 0; k < 19; ++k)
        L[k] = T(0);
    const int64_t e0 = valid ? fstart[v] : 0, e1 = valid ? fend[v] : 0;
    for (int64_t k = e0 + sub; k < e1; k += 16)
        m2l_node_src<FORM>(recA, recQ, recF, (int)(keys[k] & mask), c0, c1, c2, L);
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1)
#pragma unroll
        for (int k = 0; k < 19; ++k)
            L[k] += __shfl_xor(L[k], off);
    if (valid && sub == 0) {
        T *o = Lown + (int64_t)NLOC * v;
#pragma unroll
        for (int k = 0; k < 19; ++k)
            o[k] = L[k];
        o[19] = T(0);
    }
}

// One thread per listed cell: descend from the root (pre-order ids: a cell
// lies in the left subtree of v iff its id is below right[v]), at each step
// shifting the parent's total expansion to the child's centre of mass and
// adding the child's own M2L sum.  The forces need the leaves' totals (for
// L2P); the reverse pass also lists the internal cells.
template <typename T>
__global__ __launch_bounds__(256) void k_l2l_chain(const double *__restrict__ recA,
                                                   const int32_t *__restrict__ left,
                                                   const int32_t *__restrict__ right,
                                                   const int32_t *__restrict__ nodes, int count,
                                                   const T *__restrict__ Lown, T *Lout)
{
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= count)
        return;
    const int u = nodes[g];
    T L[19];
#pragma unroll
    for (int k = 0; k < 19; ++k)
        L[k] = Lown[k];
    double p0 = recA[0], p1 = recA[1], p2 = recA[2];
    // the next cell on the path and its centre and own sum are loaded while
    // the current shift computes
    int ch = 0;
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    T lo[19];
    if (u != 0) {
        ch = u < right[0] ? left[0] : right[0];
        const double *rc = recA + (int64_t)NREC * ch;
        q0 = rc[0];
        q1 = rc[1];
        q2 = rc[2];
#pragma unroll
        for (int k = 0; k < 19; ++k)
            lo[k] = Lown[(int64_t)NLOC * ch + k];
    }
    while (ch != 0) {
        int nx = 0;
        double n0 = 0.0, n1 = 0.0, n2 = 0.0;
        T ln[19];
        if (ch != u) {
            nx = u < right[ch] ? left[ch] : right[ch];
            const double *rc = recA + (int64_t)NREC * nx;
            n0 = rc[0];
            n1 = rc[1];
            n2 = rc[2];
#pragma unroll
            for (int k = 0; k < 19; ++k)
                ln[k] = Lown[(int64_t)NLOC * nx + k];
        }
        l2l_shift<T>(L, (T)(q0 - p0), (T)(q1 - p1), (T)(q2 - p2));
#pragma unroll
        for (int k = 0; k < 19; ++k)
            L[k] = lo[k] + L[k];
        p0 = q0;
        p1 = q1;
        p2 = q2;
        ch = nx;
        q0 = n0;
        q1 = n1;
        q2 = n2;
#pragma unroll
        for (int k = 0; k < 19; ++k)
            lo[k] = ln[k];
    }
    T *o = Lout + (int64_t)NLOC * u;
#pragma unroll
    for (int k = 0; k < 19; ++k)
        o[k] = L[k];
    o[19] = T(0);
}

template <int FORM>
static void far_mutual(Tree &t, bool fp64, hipStream_t s)
{
    const Topology &T = t.topo;
    const MutualLists &M = t.mw;
    const uint64_t mask = (1ull << mutual_key_bits(t)) - 1ull;
    const int gm = (int)(((int64_t)T.nnodes * 16 + 255) / 256);
    const int gl = (T.nleaves + 255) / 256;
    if (fp64) {
        k_m2l_node<double, FORM><<<gm, 256, 0, s>>>(t.recA, t.recQ, t.recF, T.nnodes, M.fstart,
                                                    M.fend, M.far_sorted, mask, M.Lown);
        k_l2l_chain<double><<<gl, 256, 0, s>>>(t.recA, t.left, t.right, t.leaf_node, T.nleaves,
                                               M.Lown, t.L);
    } else {
        k_m2l_node<float, FORM><<<gm, 256, 0, s>>>(t.recA, t.recQ, t.recF, T.nnodes, M.fstart,
                                                   M.fend, M.far_sorted, mask, M.Lownf);
        k_l2l_chain<float><<<gl, 256, 0, s>>>(t.recA, t.left, t.right, t.leaf_node, T.nleaves,
                                              M.Lownf, t.Lf);
    }
}

static hipError_t far_mutual_form(Tree &t, bool fp64, hipStream_t s)
{
    if (t.p.expansion == FMM_EXPANSION_DEHNEN)
        far_mutual<FMM_EXPANSION_DEHNEN>(t, fp64, s);
    else
        far_mutual<FMM_EXPANSION_PHANTOM>(t, fp64, s);
    return hipGetLastError();
}

hipError_t launch_far_mutual(Tree &t, hipStream_t s)
{
    return far_mutual_form(t, t.p.precision == FMM_FP64, s);
}

// FP64 totals of the internal cells from the FP64 M2L sums (mutual walk).
hipError_t launch_l2l_internal(Tree &t, hipStream_t s)
{
    const Topology &T = t.topo;
    const int n_int = T.nnodes - T.nleaves;
    if (n_int > 0)
        k_l2l_chain<double><<<(n_int + 255) / 256, 256, 0, s>>>(t.recA, t.left, t.right,
                                                               t.int_nodes, n_int, t.mw.Lown, t.L);
    return hipGetLastError();
}

template <int FORM>
static void far_leaf(Tree &t, bool fp64, hipStream_t s)
{
    const int nl = t.topo.nleaves;
    const bool pc = use_pieces(t);
    const int nu = pc ? (int)t.pfar.n : nl;
    const int g = (int)(((int64_t)nu * M2L_LANES + 255) / 256);
    const int2 *pl = pc ? t.pfar.list : nullptr;
    const int per = (int)t.far_piece_entries;
    const int extra = pc ? nu - nl : 0;
    if (fp64) {
        k_m2l_leaf<double, FORM><<<g, 256, 0, s>>>(t.recA, t.recQ, t.recF, t.leaf_node, nu,
                                                   t.far_cnt, t.far_src, (int)t.cap_far, t.L, pl,
                                                   per, (double *)t.pfar.part);
        if (extra > 0)
            k_m2l_fold<double><<<(extra + 255) / 256, 256, 0, s>>>(
                t.leaf_node, t.pfar.off, t.pfar.list, extra, (const double *)t.pfar.part, t.L);
    } else {
        k_m2l_leaf<float, FORM><<<g, 256, 0, s>>>(t.recA, t.recQ, t.recF, t.leaf_node, nu,
                                                  t.far_cnt, t.far_src, (int)t.cap_far, t.Lf, pl,
                                                  per, (float *)t.pfar.part);
        if (extra > 0)
            k_m2l_fold<float><<<(extra + 255) / 256, 256, 0, s>>>(
                t.leaf_node, t.pfar.off, t.pfar.list, extra, (const float *)t.pfar.part, t.Lf);
    }
}

static hipError_t far_leaves(Tree &t, bool fp64, hipStream_t s)
{
    if (t.p.expansion == FMM_EXPANSION_DEHNEN)
        far_leaf<FMM_EXPANSION_DEHNEN>(t, fp64, s);
    else
        far_leaf<FMM_EXPANSION_PHANTOM>(t, fp64, s);
    return hipGetLastError();
}

hipError_t launch_far(Tree &t, hipStream_t s)
{
    return far_leaves(t, t.p.precision == FMM_FP64, s);
}

hipError_t launch_far_f64(Tree &t, hipStream_t s)
{
    return t.lists_policy == FMM_WALK_MUTUAL ? far_mutual_form(t, true, s) : far_leaves(t, true, s);
}

// The near field of leaves whose lists were split: each leaf's piece sums
// in piece order, then L2P (eq. (8)) and the output, exactly as the kernels
// finish an unsplit leaf.  One wavefront per extra list entry; the one
// holding piece 1 of its leaf folds it, lanes over the leaf's 3 x count
// values.
template <typename T>
__global__ __launch_bounds__(256) void k_p2p_fold(
    const int32_t *__restrict__ leaf_node, const int2 *__restrict__ list, int extra,
    const int32_t *__restrict__ first, const int32_t *__restrict__ count,
    const int64_t *__restrict__ off, const T *__restrict__ part, int stride,
    const T *__restrict__ Lloc, const double *__restrict__ recA, const double4 *__restrict__ pm,
    const float4 *__restrict__ pf, const int32_t *__restrict__ perm, T G, T *aout)
{
    const int e = (blockIdx.x * 256 + threadIdx.x) >> 6;
    if (e >= extra || list[e].y != 1)
        return;
    const int lf = list[e].x;
    const int lane = lane_id();
    const int v = leaf_node[lf];
    const int64_t f = first[v];
    const int c = count[v];
    const int np = (int)(off[lf + 1] - off[lf]);
    const double *rv = recA + (int64_t)NREC * v;
    const T *Lv = Lloc + (int64_t)NLOC * v;
    for (int i3 = lane; i3 < 3 * c; i3 += 64) {
        T tot = T(0);
        for (int q = 0; q < np; ++q)
            tot += part[piece_pos(off, extra, lf, q) * stride + i3];
        const int i = i3 / 3, comp = i3 - 3 * (i3 / 3);
        T Lr[19];
#pragma unroll
        for (int k = 0; k < 19; ++k)
            Lr[k] = Lv[k];
        T fx, fy, fz;
        if constexpr (sizeof(T) == 8) {
            const double4 x4 = pm[f + i];
            l2p<double>(Lr, x4.x - rv[0], x4.y - rv[1], x4.z - rv[2], fx, fy, fz);
        } else {
            const float4 y4 = pf[f + i];
            l2p<float>(Lr, y4.x, y4.y, y4.z, fx, fy, fz);
        }
        const T far_c = comp == 0 ? fx : (comp == 1 ? fy : fz);
        aout[3 * (int64_t)perm[f + i] + comp] = G * (far_c + tot);
    }
}

hipError_t launch_near(Tree &t, void *a, hipStream_t s)
{
    const Topology &T = t.topo;
    const int nl = T.nleaves;
    const int nsub = (T.leaf_size + 7) / 8;
    const bool pc = use_pieces(t);
    const int nu = pc ? (int)t.pnear.n : nl;
    const int2 *pl = pc ? t.pnear.list : nullptr;
    const int per = (int)t.near_piece_blocks;
    const int stride = 3 * T.leaf_size;
    const int extra = pc ? nu - nl : 0;
    if (t.p.precision == FMM_FP64) {
        k_p2p_src_f64<<<(nu + P2P_WAVES - 1) / P2P_WAVES, P2P_WG, 0, s>>>(
            t.pm, t.ph, t.first, t.count, t.leaf_node, nu, t.near_cnt, t.near_src,
            (int)t.cap_near, nsub, t.L, t.recA, t.perm, t.p.G, t.p.r_kern, T.n, (double *)a, pl,
            per, (double *)t.pnear.part, stride);
        if (extra > 0)
            k_p2p_fold<double><<<(extra + 3) / 4, 256, 0, s>>>(
                t.leaf_node, t.pnear.list, extra, t.first, t.count, t.pnear.off,
                (const double *)t.pnear.part, stride, t.L, t.recA, t.pm, t.pf, t.perm, t.p.G,
                (double *)a);
    } else {
        k_p2p_src_f32<<<(nu + P2P_WAVES - 1) / P2P_WAVES, P2P_WG, 0, s>>>(
            t.pf, t.pfh, t.first, t.count, t.leaf_node, nu, t.near_cnt, t.near_src,
            (int)t.cap_near, nsub, t.Lf, t.recA, t.perm, (float)t.p.G, t.p.r_kern, (float *)a, pl,
            per, (float *)t.pnear.part, stride);
        if (extra > 0)
            k_p2p_fold<float><<<(extra + 3) / 4, 256, 0, s>>>(
                t.leaf_node, t.pnear.list, extra, t.first, t.count, t.pnear.off,
                (const float *)t.pnear.part, stride, t.Lf, t.recA, t.pm, t.pf, t.perm,
                (float)t.p.G, (float *)a);
    }
    return hipGetLastError();
}

// Pieces per leaf of the current lists and their offsets (device; the totals
// sit at off[nleaves]).
hipError_t launch_piece_counts(Tree &t, hipStream_t s)
{
    const int nl = t.topo.nleaves;
    const int nsub = (t.topo.leaf_size + 7) / 8;
    const int g = (nl + 255) / 256;
    k_piece_count<<<g, 256, 0, s>>>(t.near_cnt, (int)t.cap_near, nl, nsub, t.near_piece_blocks,
                                    t.pnear.np);
    k_piece_count<<<g, 256, 0, s>>>(t.far_cnt, (int)t.cap_far, nl, 1, t.far_piece_entries,
                                    t.pfar.np);
    hipError_t e = launch_count_scan(t.pnear.np, INT32_MAX, nl, t.pnear.tsum, t.pnear.off, s);
    if (e == hipSuccess)
        e = launch_count_scan(t.pfar.np, INT32_MAX, nl, t.pfar.tsum, t.pfar.off, s);
    return e;
}

hipError_t launch_piece_fill(Tree &t, hipStream_t s)
{
    const int nl = t.topo.nleaves;
    const int g = (nl + 255) / 256;
    k_piece_fill<<<g, 256, 0, s>>>(t.pnear.off, t.pnear.np, nl, t.pnear.list);
    k_piece_fill<<<g, 256, 0, s>>>(t.pfar.off, t.pfar.np, nl, t.pfar.list);
    return hipGetLastError();
}

hipError_t launch_piece_table(const int64_t *off, const int32_t *np, int nleaves, int2 *list,
                              hipStream_t s)
{
    if (nleaves > 0)
        k_piece_fill<<<(nleaves + 255) / 256, 256, 0, s>>>(off, np, nleaves, list);
    return hipGetLastError();
}

}  // namespace fmm
