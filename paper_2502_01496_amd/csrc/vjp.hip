// Vector-Jacobian product of the FMM accelerations on gfx950, with the tree
// membership and the interaction lists held fixed (the cell moments do
// depend on x and m).
//
// With abar' = G abar, the accelerations are
//   a_i = L2P(L_a, x_i - c_a) - sum_{b in near(a)} sum_{j in b} m_j G_ij (x_i - x_j),
//   L_a = sum_{b in far(a)} K(c_a - c_b; M_b, Q_b)                (eqs. (6)-(8))
// and the reverse pass is:
//   1. L2P^T per leaf: Lbar_a = sum_i d<abar'_i, L2P>/dL, xbar_i += (L2 + L3 y_i)^T abar'_i,
//      cbar_a -= the same sum over the leaf;
//   2. M2L^T, sink side per leaf over its far list (cbar_a += rbar) and source
//      side per cell over the transposed far list (Mbar_b, Qbar_b, cbar_b -= rbar);
//      the adjoint of one M2L term is the reverse-mode derivative of the
//      forward factorisation (a0, a1, a2, b2, b3, b4, q) and needs g_1..g_6;
//   3. P2P^T: per pair dbar = -m_j [G_ij abar'_i + (G'_ij / r)(d . abar'_i) d],
//      xbar_i += dbar (sink side, near lists), xbar_j -= dbar and
//      mbar_j -= G_ij (d . abar'_i) (source side, transposed near lists);
//   4. moments: for every cell n holding particle j, with y = x_j - c_n,
//      xbar_j += m_j / M_n cbar_n + m_j (6 Qf y - 2 tr(Qf) y),
//      mbar_j += Mbar_n + cbar_n . y / M_n + 3 y^T Qf y - |y|^2 tr(Qf),
//      (Qf: the symmetric matrix whose stored entries give Qbar; the dependence
//      of Q on c cancels because sum m y = 0), evaluated by one thread per
//      particle walking root -> leaf.
// With the lists of the mutual walk (Sec. 7), L_a is the sum over the cells
// v on the leaf's root path of v's own M2L sum shifted down by L2L, and the
// far pairs are symmetric: step 2 then first carries Lbar up the tree level
// by level (the adjoint of the shifts, whose centre derivatives go to the
// child and are taken from the parent), and does the sink and source sides
// of every cell in one pass over its own pairs (section 2c below).
// Every accumulator has exactly one owning thread (no floating-point
// atomics), so the result is bitwise reproducible.  The arithmetic is FP64.
#include "fmm_internal.h"

namespace fmm {

// Index of the stored entry of a symmetric 3x3 tensor (xx, xy, xz, yy, yz, zz)
// and of a symmetric 3x3x3 tensor (xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz,
// yzz, zzz).  Written without recursion so that, with unrolled loops, every
// index folds to a constant and the tensors stay in registers.
__device__ __forceinline__ constexpr int sym2(int i, int j)
{
    const int a = i < j ? i : j, b = i < j ? j : i;
    return a == 0 ? b : (a == 1 ? 2 + b : 5);
}

__device__ __forceinline__ constexpr int sym3(int i, int j, int k)
{
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    const int a = lo < k ? lo : k;
    const int c = hi > k ? hi : k;
    const int b = i + j + k - a - c;
    return a == 0 ? (b == 0 ? c : (b == 1 ? 2 + c : 5)) : (a == 1 ? (b == 1 ? 5 + c : 8) : 9);
}

__device__ __forceinline__ constexpr double mult3(int i, int j, int k)
{
    return (i == j && j == k) ? 1.0 : ((i == j || j == k || i == k) ? 3.0 : 6.0);
}

// ---------------------------------------------------------------- M2L adjoint
// Adjoint of the second expansion form: L1 = a0 r + b2 q (a0 = M g1 + g3 qq / 6,
// b2 = g2 / 3), L2 = A1 r r + A0 d, L3 = A2 r r r + A1 (d r + d r + d r).
__device__ __forceinline__ void m2l_vjp_dehnen(const double r[3], double M, const double *Qs,
                                               const double *Lb, double rb[3], double &Mb,
                                               double Qb[6])
{
    const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double u = rsqrt_pos(r2);  // r2 > 0: far pairs are separated
    const double u2 = u * u;
    const double g1 = -u * u2, g2 = -3.0 * g1 * u2, g3 = -5.0 * g2 * u2, g4 = -7.0 * g3 * u2;
    double Qf[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Qf[i][j] = Qs[sym2(i, j)];
    double q[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        q[i] = Qf[i][0] * r[0] + Qf[i][1] * r[1] + Qf[i][2] * r[2];
    const double qq = q[0] * r[0] + q[1] * r[1] + q[2] * r[2];
    constexpr double k3 = 1.0 / 3.0, k6 = 1.0 / 6.0;
    const double qq6 = qq * k6;
    const double a0 = M * g1 + g3 * qq6, b2 = g2 * k3;
    const double A1 = M * g2, A2 = M * g3;
    const double A[3] = {Lb[0], Lb[1], Lb[2]};
    double B[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            B[i][j] = Lb[3 + sym2(i, j)] * (i == j ? 1.0 : 0.5);
    double T[3][3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                T[i][j][k] = Lb[9 + sym3(i, j, k)] * (1.0 / mult3(i, j, k));
    double Br[3], tr1[3], Trr[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        Br[m] = B[m][0] * r[0] + B[m][1] * r[1] + B[m][2] * r[2];
        tr1[m] = T[0][0][m] + T[1][1][m] + T[2][2][m];
        double s_rr = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                s_rr += T[i][j][m] * r[i] * r[j];
        Trr[m] = s_rr;
    }
    const double Ar = A[0] * r[0] + A[1] * r[1] + A[2] * r[2];
    const double Aq = A[0] * q[0] + A[1] * q[1] + A[2] * q[2];
    const double trB = B[0][0] + B[1][1] + B[2][2];
    const double Brr = Br[0] * r[0] + Br[1] * r[1] + Br[2] * r[2];
    const double tr1r = tr1[0] * r[0] + tr1[1] * r[1] + tr1[2] * r[2];
    const double Trrr = Trr[0] * r[0] + Trr[1] * r[1] + Trr[2] * r[2];
    // cotangents of a0, b2 (L1) and A0, A1, A2 (L2, L3)
    const double a0b = Ar, b2b = Aq;
    const double A0b = trB, A1b = Brr + 3.0 * tr1r, A2b = Trrr;
    double qb[3];
    Mb += (a0b + A0b) * g1 + A1b * g2 + A2b * g3;
    const double qqb = a0b * g3 * k6;
    const double gb1 = (a0b + A0b) * M;
    const double gb2 = A1b * M + b2b * k3;
    const double gb3 = A2b * M + a0b * qq6;
    const double sg = gb1 * g2 + gb2 * g3 + gb3 * g4;
#pragma unroll
    for (int m = 0; m < 3; ++m)
        qb[m] = b2 * A[m] + qqb * r[m];
#pragma unroll
    for (int m = 0; m < 3; ++m)
        rb[m] += a0 * A[m] + 2.0 * A1 * Br[m] + 3.0 * A2 * Trr[m] + 3.0 * A1 * tr1[m] +
                 qqb * q[m] + (qb[0] * Qf[0][m] + qb[1] * Qf[1][m] + qb[2] * Qf[2][m]) + sg * r[m];
    // stored quadrupole entries, through q = Qf r only
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            Qb[sym2(i, j)] += i == j ? qb[i] * r[i] : qb[i] * r[j] + qb[j] * r[i];
}

// Given the stored cotangent Lb[19] of one M2L term K(r; M, Q), accumulate
// d<Lb, K>/dr into rb, d/dM into Mb and d/dQ (stored entries) into Qb.
// FORM = FMM_EXPANSION_DEHNEN: K's second and third orders come from the
// monopole alone (A0 = M g1, A1 = M g2, A2 = M g3 in place of a0, a1, a2 and
// no b3, b4 terms), so the quadrupole is reached through L1 only.
template <int FORM>
__device__ __forceinline__ void m2l_vjp(const double r[3], double M, const double *Qs,
                                        const double *Lb, double rb[3], double &Mb, double Qb[6])
{
    if constexpr (FORM == FMM_EXPANSION_DEHNEN) {
        m2l_vjp_dehnen(r, M, Qs, Lb, rb, Mb, Qb);
        return;
    }
    const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double u = rsqrt_pos(r2);  // r2 > 0: far pairs are separated
    const double u2 = u * u;
    const double g1 = -u * u2, g2 = -3.0 * g1 * u2, g3 = -5.0 * g2 * u2, g4 = -7.0 * g3 * u2,
                 g5 = -9.0 * g4 * u2, g6 = -11.0 * g5 * u2;
    double Qf[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Qf[i][j] = Qs[sym2(i, j)];
    double q[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        q[i] = Qf[i][0] * r[0] + Qf[i][1] * r[1] + Qf[i][2] * r[2];
    const double qq = q[0] * r[0] + q[1] * r[1] + q[2] * r[2];
    // divisions by the constants 3 and 6 are taken as products with their
    // rounded reciprocals (no FP64 divide in the loop)
    constexpr double k3 = 1.0 / 3.0, k6 = 1.0 / 6.0;
    const double qq6 = qq * k6;
    const double a0 = M * g1 + g3 * qq6, a1 = M * g2 + g4 * qq6, a2 = M * g3 + g5 * qq6;
    const double b2 = g2 * k3, b3 = g3 * k3, b4 = g4 * k3;
    // full symmetric cotangent tensors
    const double A[3] = {Lb[0], Lb[1], Lb[2]};
    double B[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            B[i][j] = Lb[3 + sym2(i, j)] * (i == j ? 1.0 : 0.5);
    double T[3][3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                T[i][j][k] = Lb[9 + sym3(i, j, k)] * (1.0 / mult3(i, j, k));
    // contractions
    double Br[3], Bq[3], tr1[3], Trr[3], Trq[3], TQ[3], Tr[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        Br[m] = B[m][0] * r[0] + B[m][1] * r[1] + B[m][2] * r[2];
        Bq[m] = B[m][0] * q[0] + B[m][1] * q[1] + B[m][2] * q[2];
        tr1[m] = T[0][0][m] + T[1][1][m] + T[2][2][m];
        double s_rr = 0.0, s_rq = 0.0, s_Q = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                s_rr += T[i][j][m] * r[i] * r[j];
                s_rq += T[i][j][m] * r[i] * q[j];
                s_Q += T[m][i][j] * Qf[i][j];
            }
        Trr[m] = s_rr;
        Trq[m] = s_rq;
        TQ[m] = s_Q;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            Tr[m][k] = T[0][m][k] * r[0] + T[1][m][k] * r[1] + T[2][m][k] * r[2];
    }
    const double Ar = A[0] * r[0] + A[1] * r[1] + A[2] * r[2];
    const double Aq = A[0] * q[0] + A[1] * q[1] + A[2] * q[2];
    const double trB = B[0][0] + B[1][1] + B[2][2];
    const double Brr = Br[0] * r[0] + Br[1] * r[1] + Br[2] * r[2];
    const double Brq = Bq[0] * r[0] + Bq[1] * r[1] + Bq[2] * r[2];
    double BQ = 0.0, TrQ = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            BQ += B[i][j] * Qf[i][j];
            TrQ += Tr[i][j] * Qf[i][j];
        }
    const double tr1r = tr1[0] * r[0] + tr1[1] * r[1] + tr1[2] * r[2];
    const double tr1q = tr1[0] * q[0] + tr1[1] * q[1] + tr1[2] * q[2];
    const double Trrr = Trr[0] * r[0] + Trr[1] * r[1] + Trr[2] * r[2];
    const double Trrq = Trr[0] * q[0] + Trr[1] * q[1] + Trr[2] * q[2];
    // cotangents of the scalar coefficients
    const double a0b = Ar + trB;
    const double a1b = Brr + 3.0 * tr1r;
    const double a2b = Trrr;
    const double b2b = Aq + BQ;
    const double b3b = 2.0 * Brq + 3.0 * tr1q + 3.0 * TrQ;
    const double b4b = 3.0 * Trrq;
    // explicit dependence on r, q, Q
    double rbl[3], qb[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        rbl[m] = a0 * A[m] + 2.0 * a1 * Br[m] + 2.0 * b3 * Bq[m] + 3.0 * a2 * Trr[m] +
                 3.0 * a1 * tr1[m] + 6.0 * b4 * Trq[m] + 3.0 * b3 * TQ[m];
        qb[m] = b2 * A[m] + 2.0 * b3 * Br[m] + 3.0 * b4 * Trr[m] + 3.0 * b3 * tr1[m];
    }
    // through the coefficients
    Mb += a0b * g1 + a1b * g2 + a2b * g3;
    const double qqb = (a0b * g3 + a1b * g4 + a2b * g5) * k6;
    const double gb1 = a0b * M;
    const double gb2 = a1b * M + b2b * k3;
    const double gb3 = a2b * M + a0b * qq6 + b3b * k3;
    const double gb4 = a1b * qq6 + b4b * k3;
    const double gb5 = a2b * qq6;
    const double sg = gb1 * g2 + gb2 * g3 + gb3 * g4 + gb4 * g5 + gb5 * g6;
#pragma unroll
    for (int m = 0; m < 3; ++m)
        qb[m] += qqb * r[m];
#pragma unroll
    for (int m = 0; m < 3; ++m)
        rb[m] += rbl[m] + qqb * q[m] + (qb[0] * Qf[0][m] + qb[1] * Qf[1][m] + qb[2] * Qf[2][m]) +
                 sg * r[m];
    // stored quadrupole entries: explicit symmetric part + q = Qf r
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const double ex = b2 * B[i][j] + 3.0 * b3 * Tr[i][j];
            if (i == j)
                Qb[sym2(i, j)] += ex + qb[i] * r[i];
            else
                Qb[sym2(i, j)] += 2.0 * ex + qb[i] * r[j] + qb[j] * r[i];
        }
}

// ---------------------------------------------------------------- L2P adjoint
// Stored-coefficient cotangent of a = L2P(L, y) for the cotangent ab.
__device__ __forceinline__ void l2p_vjp_L(double a0, double a1, double a2, double y0, double y1,
                                          double y2, double *Lb)
{
    Lb[0] += a0;
    Lb[1] += a1;
    Lb[2] += a2;
    Lb[3] += a0 * y0;
    Lb[4] += a0 * y1 + a1 * y0;
    Lb[5] += a0 * y2 + a2 * y0;
    Lb[6] += a1 * y1;
    Lb[7] += a1 * y2 + a2 * y1;
    Lb[8] += a2 * y2;
    Lb[9] += 0.5 * a0 * y0 * y0;
    Lb[10] += a0 * y0 * y1 + 0.5 * a1 * y0 * y0;
    Lb[11] += a0 * y0 * y2 + 0.5 * a2 * y0 * y0;
    Lb[12] += 0.5 * a0 * y1 * y1 + a1 * y0 * y1;
    Lb[13] += a0 * y1 * y2 + a1 * y0 * y2 + a2 * y0 * y1;
    Lb[14] += 0.5 * a0 * y2 * y2 + a2 * y0 * y2;
    Lb[15] += 0.5 * a1 * y1 * y1;
    Lb[16] += a1 * y1 * y2 + 0.5 * a2 * y1 * y1;
    Lb[17] += 0.5 * a1 * y2 * y2 + a2 * y1 * y2;
    Lb[18] += 0.5 * a2 * y2 * y2;
}

// (L2 + L3 y)^T ab
__device__ __forceinline__ void l2p_vjp_y(const double *L, double a0, double a1, double a2,
                                          double y0, double y1, double y2, double &b0, double &b1,
                                          double &b2)
{
    const double t00 = L[3] + L[9] * y0 + L[10] * y1 + L[11] * y2;
    const double t01 = L[4] + L[10] * y0 + L[12] * y1 + L[13] * y2;
    const double t02 = L[5] + L[11] * y0 + L[13] * y1 + L[14] * y2;
    const double t11 = L[6] + L[12] * y0 + L[15] * y1 + L[16] * y2;
    const double t12 = L[7] + L[13] * y0 + L[16] * y1 + L[17] * y2;
    const double t22 = L[8] + L[14] * y0 + L[17] * y1 + L[18] * y2;
    b0 = a0 * t00 + a1 * t01 + a2 * t02;
    b1 = a0 * t01 + a1 * t11 + a2 * t12;
    b2 = a0 * t02 + a1 * t12 + a2 * t22;
}

// ---------------------------------------------------------------- pair kernel
__device__ __forceinline__ double m4g(double q, double hinv3, double u3)
{
    const double p1 = hinv3 * (4.0 / 3.0 + q * q * (-1.2 + 0.5 * q));
    const double p2 = hinv3 * (8.0 / 3.0 + q * (-3.0 + q * (1.2 - q * (1.0 / 6.0)))) -
                      u3 * (1.0 / 15.0);
    return q < 1.0 ? p1 : (q < 2.0 ? p2 : u3);
}

// (dg/dr) / r for the M4 kernel: h^-5 (-12/5 + 3/2 q) for q < 1,
// h^-5 (-3/q + 12/5 - q/2 + 1/(5 q^5)) for 1 <= q < 2, -3 / r^5 beyond.
__device__ __forceinline__ double m4dgr(double q, double hinv, double hinv3, double h, double u)
{
    const double h5 = hinv3 * hinv * hinv;
    const double iq = h * u;  // 1 / q
    const double iq2 = iq * iq;
    const double p1 = h5 * (-2.4 + 1.5 * q);
    const double p2 = h5 * (-3.0 * iq + 2.4 - 0.5 * q + 0.2 * iq2 * iq2 * iq);
    const double u2 = u * u;
    return q < 1.0 ? p1 : (q < 2.0 ? p2 : -3.0 * u2 * u2 * u);
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double xk(double keep, double send, int off)
{
    return keep + __shfl_xor(send, off);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off);
    return v;
}

// ---------------------------------------------------------------- kernels
template <typename TA>
__global__ void k_vjp_prep(const TA *__restrict__ abar, int64_t n, const int32_t *__restrict__ perm,
                           double G, double *abt)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = perm[p];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            abt[3 * p + d] = G * (double)abar[3 * i + d];
    }
    if (blockIdx.x == 0 && threadIdx.x < 3)  // null record: no adjoint
        abt[3 * n + threadIdx.x] = 0.0;
}

// 1. L2P^T: one thread per leaf.
__global__ __launch_bounds__(256) void k_vjp_l2p(const double4 *__restrict__ pm,
                                                 const double *__restrict__ abt,
                                                 const int32_t *__restrict__ leaf_node, int nleaves,
                                                 const int32_t *__restrict__ first,
                                                 const int32_t *__restrict__ count,
                                                 const double *__restrict__ recA,
                                                 const double *__restrict__ Lloc, double *Lbar,
                                                 double *Lleaf, double *xbt, double *nadj)
{
    const int lf = blockIdx.x * blockDim.x + threadIdx.x;
    if (lf >= nleaves)
        return;
    const int v = leaf_node[lf];
    const int64_t f = first[v];
    const int c = count[v];
    const double *rv = recA + (int64_t)NREC * v;
    const double *Lv = Lloc + (int64_t)NLOC * v;
    double L[19], Lb[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) {
        L[k] = Lv[k];
        Lb[k] = 0.0;
    }
    double cb0 = 0.0, cb1 = 0.0, cb2 = 0.0;
    for (int k = 0; k < c; ++k) {
        const int64_t p = f + k;
        const double4 x = pm[p];
        const double y0 = x.x - rv[0], y1 = x.y - rv[1], y2 = x.z - rv[2];
        const double a0 = abt[3 * p], a1 = abt[3 * p + 1], a2 = abt[3 * p + 2];
        l2p_vjp_L(a0, a1, a2, y0, y1, y2, Lb);
        double b0, b1, b2;
        l2p_vjp_y(L, a0, a1, a2, y0, y1, y2, b0, b1, b2);
        xbt[3 * p] = b0;
        xbt[3 * p + 1] = b1;
        xbt[3 * p + 2] = b2;
        cb0 -= b0;
        cb1 -= b1;
        cb2 -= b2;
    }
    double *o = Lbar + (int64_t)NLOC * v;
#pragma unroll
    for (int k = 0; k < 19; ++k)
        o[k] = Lb[k];
    // the same by leaf index with the leaf's centre: the record the M2L^T
    // source side reads once per far pair (consecutive sinks of a transposed
    // list are adjacent records)
    double *ol = Lleaf + (int64_t)LLEAF * lf;
#pragma unroll
    for (int k = 0; k < 19; ++k)
        ol[k] = Lb[k];
    ol[19] = rv[0];
    ol[20] = rv[1];
    ol[21] = rv[2];
    ol[22] = 0.0;
    ol[23] = 0.0;
    double *na = nadj + 16 * (int64_t)v;
    na[0] = cb0;
    na[1] = cb1;
    na[2] = cb2;
}

// 2a. M2L^T, sink side: 16 lanes per leaf over its far list, cbar_sink += rbar.
constexpr int M2LT_LANES = 16;  // lanes per sink leaf (8 and 4 measured no different)

template <int FORM>
__global__ __launch_bounds__(256) void k_vjp_m2l_sink(
    const double *__restrict__ recA, const double *__restrict__ recQ,
    const int32_t *__restrict__ leaf_node, int nleaves, const int32_t *__restrict__ far_cnt,
    const int32_t *__restrict__ far_src, int cap_far, const double *__restrict__ Lbar, double *nadj)
{
    const int g = (xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x) / M2LT_LANES;
    const int sub = threadIdx.x & (M2LT_LANES - 1);
    const bool valid = g < nleaves;
    const int v = valid ? leaf_node[g] : 0;
    const double *rv = recA + (int64_t)NREC * v;
    double Lb[19];
#pragma unroll
    for (int k = 0; k < 19; ++k)
        Lb[k] = Lbar[(int64_t)NLOC * v + k];
    double rb[3] = {0.0, 0.0, 0.0};
    const int nk = valid ? max(0, min(far_cnt[g], cap_far)) : 0;
    const int32_t *fl = far_src + (int64_t)(valid ? g : 0) * cap_far;
    for (int k = sub; k < nk; k += M2LT_LANES) {
        const int b = fl[k];
        const double *rbp = recA + (int64_t)NREC * b;
        const double r[3] = {rv[0] - rbp[0], rv[1] - rbp[1], rv[2] - rbp[2]};
        double Mb = 0.0, Qb[6] = {0, 0, 0, 0, 0, 0};
        m2l_vjp<FORM>(r, rbp[3], recQ + (int64_t)NREC * b, Lb, rb, Mb, Qb);
    }
#pragma unroll
    for (int off = M2LT_LANES / 2; off >= 1; off >>= 1)
#pragma unroll
        for (int d = 0; d < 3; ++d)
            rb[d] += __shfl_xor(rb[d], off);
    if (valid && sub == 0) {
        double *na = nadj + 16 * (int64_t)v;
        na[0] += rb[0];
        na[1] += rb[1];
        na[2] += rb[2];
    }
}

// 2b. M2L^T, source side.  The sinks that took a cell as far field are
// processed in pieces of M2LT_PIECE pairs (a cell high in the tree is far
// field for a large part of the leaves, so one wavefront per cell would leave
// a few wavefronts with most of the work): one wavefront per piece writes the
// piece's sums, then one thread per cell adds its pieces in order
// (deterministic).  Per cell: Mbar, Qbar and cbar_src (zero if none), and
// cbar_sink of internal cells zeroed.
constexpr int M2LT_PIECE = 256;

__global__ void k_piece_count(const int64_t *__restrict__ toff, int nnodes, int32_t *pc)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nnodes; b += gridDim.x * blockDim.x)
        pc[b] = (int32_t)((toff[b + 1] - toff[b] + M2LT_PIECE - 1) / M2LT_PIECE);
}

__global__ void k_piece_fill(const int64_t *__restrict__ poff, int nnodes, int32_t *pnode)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nnodes; b += gridDim.x * blockDim.x)
        for (int64_t j = poff[b]; j < poff[b + 1]; ++j)
            pnode[j] = b;
}

constexpr int VJPM_WAVES = 1;  // wavefronts (pieces) per workgroup

template <int FORM>
__global__ __launch_bounds__(64 * VJPM_WAVES)
    __attribute__((amdgpu_waves_per_eu(3, 8))) void k_vjp_m2l_src_piece(
    const double *__restrict__ recA, const double *__restrict__ recQ,
    const int64_t *__restrict__ toff, const uint32_t *__restrict__ tsrc,
    const double *__restrict__ Lleaf, const int32_t *__restrict__ pnode,
    const int64_t *__restrict__ poff, int64_t npieces, double *part)
{
    // consecutive pieces (neighbouring source cells, which share most of
    // their sinks) run behind the same L2
    const int64_t pc =
        (int64_t)xcd_block(blockIdx.x, gridDim.x) * VJPM_WAVES + (threadIdx.x >> 6);
    if (pc >= npieces)
        return;
    const int lane = lane_id();
    const int b = pnode[pc];
    const int64_t e0 = toff[b] + (pc - poff[b]) * M2LT_PIECE;
    const int64_t e1 = min(e0 + M2LT_PIECE, toff[b + 1]);
    const double *rbp = recA + (int64_t)NREC * b;
    const double cb0 = rbp[0], cb1 = rbp[1], cb2 = rbp[2], M = rbp[3];
    const double *Qs = recQ + (int64_t)NREC * b;
    double acc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k)
        acc[k] = 0.0;
    for (int64_t e = e0 + lane; e < e1; e += 64) {
        // the sink leaf's L-bar and centre, one 192-byte record
        const double2 *lr = (const double2 *)(Lleaf + (int64_t)LLEAF * (int)tsrc[e]);
        double Lb[20];
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const double2 q = lr[k];
            Lb[2 * k] = q.x;
            Lb[2 * k + 1] = q.y;
        }
        const double2 c12 = lr[10];
        const double r[3] = {Lb[19] - cb0, c12.x - cb1, c12.y - cb2};
        double rb[3] = {0.0, 0.0, 0.0}, Mb = 0.0, Qb[6] = {0, 0, 0, 0, 0, 0};
        m2l_vjp<FORM>(r, M, Qs, Lb, rb, Mb, Qb);
        acc[0] += Mb;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            acc[1 + k] += Qb[k];
        acc[7] -= rb[0];
        acc[8] -= rb[1];
        acc[9] -= rb[2];
    }
#pragma unroll
    for (int k = 0; k < 10; ++k)
        acc[k] = wave_sum(acc[k]);
    if (lane == 0) {
        double *pp = part + 10 * pc;
#pragma unroll
        for (int k = 0; k < 10; ++k)
            pp[k] = acc[k];
    }
}

__global__ __launch_bounds__(256) void k_vjp_m2l_src_fold(const int32_t *__restrict__ left,
                                                          int nnodes,
                                                          const int64_t *__restrict__ poff,
                                                          const double *__restrict__ part,
                                                          double *nadj)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nnodes)
        return;
    double acc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k)
        acc[k] = 0.0;
    for (int64_t pc = poff[b]; pc < poff[b + 1]; ++pc)
#pragma unroll
        for (int k = 0; k < 10; ++k)
            acc[k] += part[10 * pc + k];
    double *na = nadj + 16 * (int64_t)b;
    na[3] = acc[7];
    na[4] = acc[8];
    na[5] = acc[9];
    na[6] = acc[0];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        na[7 + k] = acc[1 + k];
    if (left[b] >= 0)
        na[0] = na[1] = na[2] = 0.0;
}

// 2c. Mutual walk.  There the far field of a leaf is the sum, over the cells
// v on its root path, of the M2L sum into v shifted down to the leaf (L2L),
// so the reverse pass first carries Lbar up the tree: per level (deepest
// first), each internal cell v with children a, b takes
//   Lbar_v = S(d_a)^T Lbar_a + S(d_b)^T Lbar_b,   d_ch = c_ch - c_v,
// where S(d) is the L2L shift; the derivative of <Lbar_ch, S(d) L_v> in d
// (L_v: the forward total of v) is added to cbar_ch and taken from cbar_v.
// Lbar_v is then also the cotangent of v's own M2L sum.
__global__ __launch_bounds__(256) void k_vjp_l2l_level(const int32_t *__restrict__ nodes, int cnt,
                                                       const int32_t *__restrict__ left,
                                                       const int32_t *__restrict__ right,
                                                       const double *__restrict__ recA,
                                                       const double *__restrict__ Ltot,
                                                       double *Lbar, double *nadj)
{
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= cnt)
        return;
    const int v = nodes[g];
    const double *rv = recA + (int64_t)NREC * v;
    const double *Lf = Ltot + (int64_t)NLOC * v;
    double L[19], Lb[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) {
        L[k] = Lf[k];
        Lb[k] = 0.0;
    }
    double ds0 = 0.0, ds1 = 0.0, ds2 = 0.0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int ch = side == 0 ? left[v] : right[v];
        const double *rc = recA + (int64_t)NREC * ch;
        const double d0 = rc[0] - rv[0], d1 = rc[1] - rv[1], d2 = rc[2] - rv[2];
        const double *B = Lbar + (int64_t)NLOC * ch;
        const double B0 = B[0], B1 = B[1], B2 = B[2];
        // first order: L1' = L2P(L, d)
        l2p_vjp_L(B0, B1, B2, d0, d1, d2, Lb);
        double e0, e1, e2;
        l2p_vjp_y(L, B0, B1, B2, d0, d1, d2, e0, e1, e2);
        // second order: L2' = L2 + L3 d (stored xx, xy, xz, yy, yz, zz)
        const double B3 = B[3], B4 = B[4], B5 = B[5], B6 = B[6], B7 = B[7], B8 = B[8];
        e0 += B3 * L[9] + B4 * L[10] + B5 * L[11] + B6 * L[12] + B7 * L[13] + B8 * L[14];
        e1 += B3 * L[10] + B4 * L[12] + B5 * L[13] + B6 * L[15] + B7 * L[16] + B8 * L[17];
        e2 += B3 * L[11] + B4 * L[13] + B5 * L[14] + B6 * L[16] + B7 * L[17] + B8 * L[18];
#pragma unroll
        for (int k = 3; k < 9; ++k)
            Lb[k] += B[k];
        Lb[9] += B3 * d0;
        Lb[10] += B3 * d1 + B4 * d0;
        Lb[11] += B3 * d2 + B5 * d0;
        Lb[12] += B4 * d1 + B6 * d0;
        Lb[13] += B4 * d2 + B5 * d1 + B7 * d0;
        Lb[14] += B5 * d2 + B8 * d0;
        Lb[15] += B6 * d1;
        Lb[16] += B6 * d2 + B7 * d1;
        Lb[17] += B7 * d2 + B8 * d1;
        Lb[18] += B8 * d2;
        // third order: L3' = L3
#pragma unroll
        for (int k = 9; k < 19; ++k)
            Lb[k] += B[k];
        double *nc = nadj + 16 * (int64_t)ch;
        nc[0] += e0;
        nc[1] += e1;
        nc[2] += e2;
        ds0 += e0;
        ds1 += e1;
        ds2 += e2;
    }
    double *o = Lbar + (int64_t)NLOC * v;
#pragma unroll
    for (int k = 0; k < 19; ++k)
        o[k] = Lb[k];
    double *na = nadj + 16 * (int64_t)v;
    na[0] = -ds0;
    na[1] = -ds1;
    na[2] = -ds2;
}

// M2L^T of the mutual pairs: the pair list is symmetric (v takes b iff b
// takes v), so the cells that took v as source are v's own partners and one
// pass over the CSR range of v does both sides: cbar_v += rbar of (v <- b)
// with Lbar_v, and Mbar_v, Qbar_v, cbar_v -= rbar of (b <- v) with Lbar_b.
// 16 lanes per cell, all cells.
template <int FORM>
__global__ __launch_bounds__(256) void k_vjp_m2l_mutual(
    const double *__restrict__ recA, const double *__restrict__ recQ, int nnodes,
    const int64_t *__restrict__ fstart, const int64_t *__restrict__ fend,
    const uint64_t *__restrict__ keys, uint64_t mask, const double *__restrict__ Lbar,
    double *nadj)
{
    const int v = (blockIdx.x * 256 + threadIdx.x) >> 4;
    const int sub = threadIdx.x & 15;
    const bool valid = v < nnodes;
    const int vv = valid ? v : 0;
    const double *rv = recA + (int64_t)NREC * vv;
    const double *Qv = recQ + (int64_t)NREC * vv;
    const double Mv = rv[3];
    double Lb[19];
#pragma unroll
    for (int k = 0; k < 19; ++k)
        Lb[k] = Lbar[(int64_t)NLOC * vv + k];
    double rs[3] = {0.0, 0.0, 0.0}, rt[3] = {0.0, 0.0, 0.0}, Mb = 0.0,
           Qb[6] = {0, 0, 0, 0, 0, 0};
    const int64_t e0 = valid ? fstart[v] : 0, e1 = valid ? fend[v] : 0;
    for (int64_t k = e0 + sub; k < e1; k += 16) {
        const int b = (int)(keys[k] & mask);
        const double *rb = recA + (int64_t)NREC * b;
        const double r[3] = {rv[0] - rb[0], rv[1] - rb[1], rv[2] - rb[2]};
        double Mx = 0.0, Qx[6] = {0, 0, 0, 0, 0, 0};
        m2l_vjp<FORM>(r, rb[3], recQ + (int64_t)NREC * b, Lb, rs, Mx, Qx);
        const double q[3] = {-r[0], -r[1], -r[2]};
        m2l_vjp<FORM>(q, Mv, Qv, Lbar + (int64_t)NLOC * b, rt, Mb, Qb);
    }
    double acc[13] = {rs[0], rs[1], rs[2], rt[0], rt[1], rt[2], Mb,
                      Qb[0], Qb[1], Qb[2], Qb[3], Qb[4], Qb[5]};
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1)
#pragma unroll
        for (int k = 0; k < 13; ++k)
            acc[k] += __shfl_xor(acc[k], off);
    if (valid && sub == 0) {
        double *na = nadj + 16 * (int64_t)v;
        na[0] += acc[0];
        na[1] += acc[1];
        na[2] += acc[2];
        na[3] = -acc[3];
        na[4] = -acc[4];
        na[5] = -acc[5];
#pragma unroll
        for (int k = 6; k < 13; ++k)
            na[k] = acc[k];
    }
}

// 3. P2P^T: the near pairs of eqs. (12)-(15) in reverse.  For a pair (i, j)
// with d = x_i - x_j, G_ij the mean of the two M4 kernels (r^-3 beyond both
// supports) and D_ij = (dG_ij / dr) / r, the adjoint of
// a_i = -sum_j m_j G_ij d gives
//   sink side:   xbar_i -= sum_j m_j (G_ij abar_i + D_ij (d . abar_i) d),
//   source side: xbar_j += m_j sum_i (G_ij abar_i + D_ij (d . abar_i) d),
//                mbar_j  = -sum_i G_ij (d . abar_i),
// the source side over the sink leaves whose near list holds j's leaf (the
// transposed lists).  Both kernels take the forward near field's layout: a
// lane per particle of a staged block (8 blocks a step), VJP_NS particles of
// the wavefront's own leaf per pass (wave-uniform), block ranges staged in
// LDS in list order.  A pair with r^2 < max(H4, 4 h^2) -- H4 the largest
// 4 h^2 of the pass's uniform particles, 4 h^2 the lane's own -- may be
// softened: it goes to its uniform particle's queue in LDS and is evaluated
// with the M4 kernels, 64 at a time; every other pair is Newtonian for
// certain (G = r^-3, D = -3 r^-5).  Two particles at one point have
// G = (g_i(0) + g_j(0)) / 2 and d = 0; a particle paired with itself adds
// nothing.  Long lists are cut into pieces of `per` blocks (pieces != null:
// a unit is one entry of the piece list, and a split leaf's piece sums go to
// part, folded in piece order); the order of all additions depends on the
// lists only.
constexpr int VJP_NS = 8;        // uniform particles per pass
constexpr int VJP_QCAP = 128;    // softened pairs a queue holds (a step adds <= 64)
// One unit (leaf or piece) per wavefront and one wavefront per workgroup: the
// units' lists differ in length, and a workgroup's slots are only freed when
// its last wavefront ends.
constexpr int VJP_WAVES = 1;
constexpr int VJP_WG = 64 * VJP_WAVES;
constexpr int VJP_BLOCKS = 256;  // blocks staged in LDS per chunk

// Stage the non-empty blocks of list entries [c0, c0 + nc) (entry k: block
// k % nsub of leaf lst[k / nsub]) in list order, then eight empty blocks;
// returns the number of staged blocks.
template <typename IX>
__device__ __forceinline__ int stage_list_blocks(const IX *__restrict__ lst, int c0, int nc,
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
            const int bn = (int)lst[e];
            r = make_int2(first[bn] + 8 * u, max(0, min(8, count[bn] - 8 * u)));
        }
        const bool keep = r.y > 0;
        const uint64_t mk = __ballot(keep);
        if (keep)
            R[ne + __popcll(mk & lanemask_lt())] = r;
        ne += __popcll(mk);
    }
    if (lane < 8)
        R[ne + lane] = make_int2(0, 0);
    return ne;
}

// Particle index of this lane in a staged block; missing particles read the
// null record at index nnull (far away, zero mass, zero smoothing length,
// zero adjoint), so their pairs add exactly zero.
__device__ __forceinline__ int64_t block_particle(int2 rg, int slot, int64_t nnull)
{
    return slot < rg.y ? (int64_t)rg.x + slot : nnull;
}

// G_ij and D_ij of a pair that may be softened: each side's M4 kernel
// (eq. (13) and its derivative) at q = r / h, and their mean.
__device__ __forceinline__ void pair_gd_soft(double r2, double4 ha, double4 hb, bool self,
                                             double &Gp, double &Dp)
{
    const double u = r2 > 0.0 ? rsqrt_pos(r2) : 0.0;
    const double r = r2 * u;
    const double u3 = u * u * u;
    const double qa = r * ha.x, qb = r * hb.x;
    const double g = 0.5 * (m4g(qa, ha.y, u3) + m4g(qb, hb.y, u3));
    Gp = self ? 0.0 : g;
    Dp = 0.5 * (m4dgr(qa, ha.x, ha.y, ha.w, u) + m4dgr(qb, hb.x, hb.y, hb.w, u));
}

// Reduce-scatter of 32 per-lane values over the wavefront: after xor steps
// over lane bits 5..1 (each keeps half of its values and sends the other
// half to its partner) and a last butterfly step, lanes 2v and 2v + 1 hold
// the sum of value v.
__device__ __forceinline__ double reduce_scatter32(const double *v, int lane)
{
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
    double a[16], b[8], c[4], d[2];
#pragma unroll
    for (int k = 0; k < 16; ++k)
        a[k] = xk(b5 ? v[16 + k] : v[k], b5 ? v[k] : v[16 + k], 32);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        b[k] = xk(b4 ? a[8 + k] : a[k], b4 ? a[k] : a[8 + k], 16);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        c[k] = xk(b3 ? b[4 + k] : b[k], b3 ? b[k] : b[4 + k], 8);
#pragma unroll
    for (int k = 0; k < 2; ++k)
        d[k] = xk(b2 ? c[2 + k] : c[k], b2 ? c[k] : c[2 + k], 4);
    double e = xk(b1 ? d[1] : d[0], b1 ? d[0] : d[1], 2);
    e += __shfl_xor(e, 1);
    return e;
}

// 3a. Sink side.  Per sink q the lanes sum S = sum_j m_j G_ij and
// V = sum_j m_j D_ij (d . abar_i) d; a piece adds -(abar_i S + V) to xbar_i
// (abar_i is wave-uniform, so the G term needs no per-pair product).  The
// queues that a step fills past a multiple of 64 are evaluated after the
// step, when its source data are no longer held.
__global__ __launch_bounds__(VJP_WG) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_vjp_p2p_sink(
    const double4 *__restrict__ pm, const double4 *__restrict__ ph,
    const double *__restrict__ abt, const int32_t *__restrict__ first,
    const int32_t *__restrict__ count, const int32_t *__restrict__ leaf_node, int nunits,
    const int32_t *__restrict__ near_cnt, const int32_t *__restrict__ near_src, int cap_near,
    int nsub, int64_t nnull, double *xbt, const int2 *__restrict__ pieces, int per, double *part,
    int part_stride)
{
    constexpr int NS = VJP_NS;
    __shared__ int2 rng[VJP_WAVES][VJP_BLOCKS + 8];
    __shared__ int32_t que[VJP_WAVES][NS][VJP_QCAP];
    __shared__ double4 shx[VJP_WAVES][NS];  // positions of the pass's sinks
    __shared__ double4 sha[VJP_WAVES][NS];  // abar of the pass's sinks
    __shared__ double4 sh3[VJP_WAVES][NS];  // -3 abar (the Newtonian D = -3 r^-5 folded in)
    __shared__ double4 shh[VJP_WAVES][NS];  // h data of the pass's sinks
    const int w = threadIdx.x >> 6;
    const int unit =
        __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * VJP_WAVES + w);
    if (unit >= nunits)
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
    const bool split = pieces && nbf > per;
    const int32_t *nl = near_src + (int64_t)leaf * cap_near;
    int2 *R = rng[w];
    // value 4 q + k of the reduce-scatter (lanes 8 q + 2 k, + 1): k = 0 S, k = 1..3 V_k
    const int qv = lane >> 3, kv = (lane >> 1) & 3;
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
            const int64_t is = f + min(sb + lane, c - 1);
            shx[w][lane] = pm[is];
            shh[w][lane] = ph[is];
            const double a0 = abt[3 * is], a1 = abt[3 * is + 1], a2 = abt[3 * is + 2];
            sha[w][lane] = make_double4(a0, a1, a2, 0.0);
            sh3[w][lane] = make_double4(-3.0 * a0, -3.0 * a1, -3.0 * a2, 0.0);
        }
        __builtin_amdgcn_wave_barrier();
        double tot = 0.0;
        double acc[4 * NS];
        int tail[NS];  // queue fill counts; entries [tail & ~63, tail) are pending
        // softened pairs of sink q: cnt <= 64 queue entries from position head
        auto drain = [&](int q, int head, int cnt) {
            const int64_t j =
                lane < cnt ? (int64_t)que[w][q][(head + lane) & (VJP_QCAP - 1)] : nnull;
            const double4 xj = pm[j];
            const double4 hj = ph[j];
            const double4 xs = shx[w][q];
            const double dx = xs.x - xj.x, dy = xs.y - xj.y, dz = xs.z - xj.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            double Gp, Dp;
            pair_gd_soft(r2, shh[w][q], hj, j == f + min(sb + q, c - 1), Gp, Dp);
            const double4 a = sha[w][q];
            const double t = xj.w * Dp * (dx * a.x + dy * a.y + dz * a.z);
            acc[4 * q] += xj.w * Gp;
            acc[4 * q + 1] += t * dx;
            acc[4 * q + 2] += t * dy;
            acc[4 * q + 3] += t * dz;
        };
        for (int p0 = b_lo; p0 < b_hi; p0 += per) {
            const int nb = min(b_hi, p0 + per);
#pragma unroll
            for (int q = 0; q < 4 * NS; ++q)
                acc[q] = 0.0;
#pragma unroll
            for (int q = 0; q < NS; ++q)
                tail[q] = 0;
            for (int c0 = p0; c0 < nb; c0 += VJP_BLOCKS) {
                const int nc = min(nb - c0, VJP_BLOCKS);
                const int ne = __builtin_amdgcn_readfirstlane(
                    stage_list_blocks(nl, c0, nc, nsub, first, count, lane, R));
                __builtin_amdgcn_wave_barrier();
                for (int kb = 0; kb < ne; kb += 8) {
                    uint32_t full = 0u;  // queues that passed a multiple of 64 in this step
                    {
                        const int32_t j = (int32_t)block_particle(R[kb + grp], slot, nnull);
                        const double4 xj = pm[j];
                        const double hj4 = ph[j].z;
                        const double hmax4 = hj4 > H4 ? hj4 : H4;
#pragma unroll
                        for (int q = 0; q < NS; ++q) {
                            const double dx = sx[q] - xj.x, dy = sy[q] - xj.y, dz = sz[q] - xj.z;
                            const double r2 = dx * dx + dy * dy + dz * dz;
                            // (every lane is active here: the softened mask is
                            // the complement of the Newtonian one)
                            const bool newt = !(r2 < hmax4);
                            const uint64_t bal = ~__ballot(newt);
                            if (newt) {
                                const double u = rsqrt_pos(r2);
                                const double u2 = u * u;
                                const double mg = xj.w * (u2 * u);
                                const double4 a = sh3[w][q];
                                const double t = (mg * u2) * (dx * a.x + dy * a.y + dz * a.z);
                                acc[4 * q] += mg;
                                acc[4 * q + 1] += t * dx;
                                acc[4 * q + 2] += t * dy;
                                acc[4 * q + 3] += t * dz;
                            }
                            if (bal) {
                                // possibly softened pairs leave the step for the sink's queue
                                const int t0 = tail[q];
                                if (!newt)
                                    que[w][q][(t0 + __popcll(bal & lt)) & (VJP_QCAP - 1)] = j;
                                tail[q] = t0 + __popcll(bal);
                                if ((tail[q] >> 6) != (t0 >> 6))
                                    full |= 1u << q;
                            }
                        }
                    }
                    if (full) {
                        __builtin_amdgcn_wave_barrier();
#pragma unroll
                        for (int q = 0; q < NS; ++q)
                            if (full & (1u << q))
                                drain(q, ((tail[q] >> 6) - 1) << 6, 64);
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
#pragma unroll
            for (int q = 0; q < NS; ++q)
                if (tail[q] & 63)
                    drain(q, tail[q] & ~63, tail[q] & 63);
            __builtin_amdgcn_wave_barrier();
            const double e = reduce_scatter32(acc, lane);
            const double S = __shfl(e, lane & ~7);
            const double4 a = sha[w][qv];
            const double ak = kv == 1 ? a.x : (kv == 2 ? a.y : a.z);
            tot += -fma(ak, S, e);
        }
        if (kv >= 1 && (lane & 1) == 0 && sb + qv < c) {
            if (split)
                part[(int64_t)unit * part_stride + 3 * (sb + qv) + (kv - 1)] = tot;
            else
                xbt[3 * (f + sb + qv) + (kv - 1)] += tot;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// 3b. Source side: the wavefront's own leaf holds the sources (uniform), the
// lanes the particles of the sink leaves of its transposed list.  Per source
// q the lanes sum X = sum_i (G_ij abar_i + D_ij (d . abar_i) d) and
// Y = sum_i G_ij (d . abar_i); a piece adds m_j X to xbar_j and -Y to mbar_j.
__global__ __launch_bounds__(VJP_WG) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_vjp_p2p_src(
    const double4 *__restrict__ pm, const double4 *__restrict__ ph,
    const double *__restrict__ abt, const int32_t *__restrict__ first,
    const int32_t *__restrict__ count, const int32_t *__restrict__ leaf_node, int nunits,
    const int64_t *__restrict__ toff, const uint32_t *__restrict__ tsrc, int nsub, int64_t nnull,
    double *xbt, double *mbt, const int2 *__restrict__ pieces, int per, double *part,
    int part_stride)
{
    constexpr int NS = VJP_NS;
    __shared__ int2 rng[VJP_WAVES][VJP_BLOCKS + 8];
    __shared__ int32_t que[VJP_WAVES][NS][VJP_QCAP];
    __shared__ double4 shx[VJP_WAVES][NS];  // positions of the pass's sources
    __shared__ double4 shh[VJP_WAVES][NS];  // h data of the pass's sources
    const int w = threadIdx.x >> 6;
    const int unit =
        __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * VJP_WAVES + w);
    if (unit >= nunits)
        return;
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const int grp = lane >> 3, slot = lane & 7;
    const int2 pc = pieces ? pieces[unit] : make_int2(unit, 0);
    const int leaf = pc.x;
    const int v = leaf_node[leaf];
    const int64_t f = first[v];
    const int c = count[v];
    const int64_t e0 = toff[v];
    const int nbf = (int)(toff[v + 1] - e0) * nsub;
    const int b_lo = pieces ? pc.y * per : 0;
    const int b_hi = pieces ? min(nbf, b_lo + per) : nbf;
    const bool split = pieces && nbf > per;
    const uint32_t *tl = tsrc + e0;
    int2 *R = rng[w];
    // value 4 q + k of the reduce-scatter (lanes 8 q + 2 k, + 1): k = 0..2 X_k, k = 3 Y
    const int qv = lane >> 3, kv = (lane >> 1) & 3;
    for (int sb = 0; sb < c; sb += NS) {
        double sx[NS], sy[NS], sz[NS], H4 = 0.0;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int64_t js = f + min(sb + q, c - 1);
            const double4 x4 = pm[js];
            sx[q] = x4.x;
            sy[q] = x4.y;
            sz[q] = x4.z;
            const double h4q = ph[js].z;
            H4 = h4q > H4 ? h4q : H4;
        }
        if (lane < NS) {
            const int64_t js = f + min(sb + lane, c - 1);
            shx[w][lane] = pm[js];
            shh[w][lane] = ph[js];
        }
        __builtin_amdgcn_wave_barrier();
        double tot = 0.0;
        double acc[4 * NS];
        int tail[NS];
        // softened pairs of source q: cnt <= 64 queued sink particles from head
        auto drain = [&](int q, int head, int cnt) {
            const int64_t i =
                lane < cnt ? (int64_t)que[w][q][(head + lane) & (VJP_QCAP - 1)] : nnull;
            const double4 xi = pm[i];
            const double4 hi = ph[i];
            const double a0 = abt[3 * i], a1 = abt[3 * i + 1], a2 = abt[3 * i + 2];
            const double4 xs = shx[w][q];
            const double dx = xi.x - xs.x, dy = xi.y - xs.y, dz = xi.z - xs.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            double Gp, Dp;
            pair_gd_soft(r2, hi, shh[w][q], i == f + min(sb + q, c - 1), Gp, Dp);
            const double da = dx * a0 + dy * a1 + dz * a2;
            const double t = Dp * da;
            acc[4 * q] += Gp * a0 + t * dx;
            acc[4 * q + 1] += Gp * a1 + t * dy;
            acc[4 * q + 2] += Gp * a2 + t * dz;
            acc[4 * q + 3] += Gp * da;
        };
        for (int p0 = b_lo; p0 < b_hi; p0 += per) {
            const int nb = min(b_hi, p0 + per);
#pragma unroll
            for (int q = 0; q < 4 * NS; ++q)
                acc[q] = 0.0;
#pragma unroll
            for (int q = 0; q < NS; ++q)
                tail[q] = 0;
            for (int c0 = p0; c0 < nb; c0 += VJP_BLOCKS) {
                const int nc = min(nb - c0, VJP_BLOCKS);
                const int ne = __builtin_amdgcn_readfirstlane(
                    stage_list_blocks(tl, c0, nc, nsub, first, count, lane, R));
                __builtin_amdgcn_wave_barrier();
                for (int kb = 0; kb < ne; kb += 8) {
                    uint32_t full = 0u;
                    {
                        const int32_t i = (int32_t)block_particle(R[kb + grp], slot, nnull);
                        const double4 xi = pm[i];
                        const double hi4 = ph[i].z;
                        const double a0 = abt[3 * (int64_t)i], a1 = abt[3 * (int64_t)i + 1],
                                     a2 = abt[3 * (int64_t)i + 2];
                        const double hmax4 = hi4 > H4 ? hi4 : H4;
#pragma unroll
                        for (int q = 0; q < NS; ++q) {
                            const double dx = xi.x - sx[q], dy = xi.y - sy[q], dz = xi.z - sz[q];
                            const double r2 = dx * dx + dy * dy + dz * dz;
                            const bool newt = !(r2 < hmax4);
                            const uint64_t bal = ~__ballot(newt);
                            if (newt) {
                                const double u = rsqrt_pos(r2);
                                const double u2 = u * u;
                                const double Gp = u2 * u;
                                const double da = dx * a0 + dy * a1 + dz * a2;
                                const double t = (-3.0 * (Gp * u2)) * da;
                                acc[4 * q] += Gp * a0 + t * dx;
                                acc[4 * q + 1] += Gp * a1 + t * dy;
                                acc[4 * q + 2] += Gp * a2 + t * dz;
                                acc[4 * q + 3] += Gp * da;
                            }
                            if (bal) {
                                const int t0 = tail[q];
                                if (!newt)
                                    que[w][q][(t0 + __popcll(bal & lt)) & (VJP_QCAP - 1)] = i;
                                tail[q] = t0 + __popcll(bal);
                                if ((tail[q] >> 6) != (t0 >> 6))
                                    full |= 1u << q;
                            }
                        }
                    }
                    if (full) {
                        __builtin_amdgcn_wave_barrier();
#pragma unroll
                        for (int q = 0; q < NS; ++q)
                            if (full & (1u << q))
                                drain(q, ((tail[q] >> 6) - 1) << 6, 64);
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
#pragma unroll
            for (int q = 0; q < NS; ++q)
                if (tail[q] & 63)
                    drain(q, tail[q] & ~63, tail[q] & 63);
            __builtin_amdgcn_wave_barrier();
            const double e = reduce_scatter32(acc, lane);
            const double mq = shx[w][qv].w;
            tot += kv < 3 ? mq * e : -e;
        }
        if ((lane & 1) == 0 && sb + qv < c) {
            const int64_t jj = f + sb + qv;
            if (split)
                part[(int64_t)unit * part_stride + 4 * (sb + qv) + kv] = tot;
            else if (kv < 3)
                xbt[3 * jj + kv] += tot;
            else
                mbt[jj] = tot;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// The near field's pieces of split leaves, folded in piece order: `vals`
// values per particle (3: xbar, sink side; 4: xbar and mbar, source side).
// One wavefront per extra entry of the piece list; the one holding piece 1
// of its leaf folds it.
__global__ __launch_bounds__(256) void k_vjp_p2p_fold(
    const int32_t *__restrict__ leaf_node, const int2 *__restrict__ list, int extra,
    const int32_t *__restrict__ first, const int32_t *__restrict__ count,
    const int64_t *__restrict__ off, const double *__restrict__ part, int stride, int vals,
    double *xbt, double *mbt)
{
    const int e = (blockIdx.x * 256 + threadIdx.x) >> 6;
    if (e >= extra || list[e].y != 1)
        return;
    const int lf = list[e].x;
    const int v = leaf_node[lf];
    const int64_t f = first[v];
    const int c = count[v];
    const int np = (int)(off[lf + 1] - off[lf]);
    for (int iv = lane_id(); iv < vals * c; iv += 64) {
        double tot = 0.0;
        for (int q = 0; q < np; ++q)
            tot += part[piece_pos(off, extra, lf, q) * stride + iv];
        const int i = iv / vals, k = iv - vals * (iv / vals);
        if (k < 3)
            xbt[3 * (f + i) + k] += tot;
        else
            mbt[f + i] = tot;
    }
}

// 4. Moments adjoint and output: one thread per particle walks root -> leaf.
// Cells are numbered in depth-first pre-order (an internal cell's left child
// is v + 1), so each level's loads -- the cell, its child ids and the left
// child's particle range -- are issued together.
template <typename TO>
__global__ __launch_bounds__(256) void k_vjp_moments(
    const double4 *__restrict__ pm, int64_t n, const double *__restrict__ recA,
    const double *__restrict__ nadj, const int32_t *__restrict__ first,
    const int32_t *__restrict__ count, const int32_t *__restrict__ left,
    const int32_t *__restrict__ right, int nnodes, const double *__restrict__ xbt,
    const double *__restrict__ mbt, const int32_t *__restrict__ perm, TO *xbar, TO *mbar)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    const double4 x = pm[p];
    double gx = xbt[3 * p], gy = xbt[3 * p + 1], gz = xbt[3 * p + 2], gm = mbt[p];
    int v = 0;
    while (true) {
        const double *ra = recA + (int64_t)NREC * v;
        const double *na = nadj + 16 * (int64_t)v;
        const int l = left[v], rgt = right[v];
        const int vn = min(v + 1, nnodes - 1);  // used only when v is internal
        const int64_t bnd = (int64_t)first[vn] + count[vn];
        const double M = ra[3];
        const double y0 = x.x - ra[0], y1 = x.y - ra[1], y2 = x.z - ra[2];
        const double c0 = na[0] + na[3], c1 = na[1] + na[4], c2 = na[2] + na[5];
        // Qf: stored cotangent -> symmetric matrix (off-diagonals halved)
        const double qxx = na[7], qxy = 0.5 * na[8], qxz = 0.5 * na[9], qyy = na[10],
                     qyz = 0.5 * na[11], qzz = na[12];
        const double tr = qxx + qyy + qzz;
        const double Qy0 = qxx * y0 + qxy * y1 + qxz * y2;
        const double Qy1 = qxy * y0 + qyy * y1 + qyz * y2;
        const double Qy2 = qxz * y0 + qyz * y1 + qzz * y2;
        const double wm = x.w / M;
        gx += wm * c0 + x.w * (6.0 * Qy0 - 2.0 * tr * y0);
        gy += wm * c1 + x.w * (6.0 * Qy1 - 2.0 * tr * y1);
        gz += wm * c2 + x.w * (6.0 * Qy2 - 2.0 * tr * y2);
        gm += na[6] + (c0 * y0 + c1 * y1 + c2 * y2) / M +
              3.0 * (y0 * Qy0 + y1 * Qy1 + y2 * Qy2) - (y0 * y0 + y1 * y1 + y2 * y2) * tr;
        if (l < 0)
            break;
        v = p < bnd ? l : rgt;
    }
    const int64_t i = perm[p];
    xbar[3 * i] = (TO)gx;
    xbar[3 * i + 1] = (TO)gy;
    xbar[3 * i + 2] = (TO)gz;
    mbar[i] = (TO)gm;
}

// ---------------------------------------------------------------- transposition
constexpr int SCAN_TILE = 4096;

__device__ __forceinline__ int64_t block_scan_i64(int64_t v, int64_t *sh, int64_t &total)
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

// exclusive scan of min(cnt, cap) over nl leaves -> off[0..nl]
__global__ __launch_bounds__(256) void k_cnt_tiles(const int32_t *cnt, int cap, int nl,
                                                   int64_t *tsum)
{
    __shared__ int64_t sh[8];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t sacc = 0;
    for (int k = threadIdx.x; k < SCAN_TILE; k += 256) {
        const int64_t i = base + k;
        if (i < nl)
            sacc += max(0, min(cnt[i], cap));
    }
    int64_t tot;
    block_scan_i64(sacc, sh, tot);
    if (threadIdx.x == 0)
        tsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_cnt_tile_scan(int64_t *tsum, int ntiles, int64_t *total)
{
    __shared__ int64_t sh[16];
    int64_t run = 0;
    for (int c0 = 0; c0 < ntiles; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const int64_t v = i < ntiles ? tsum[i] : 0;
        int64_t tot;
        const int64_t ex = block_scan_i64(v, sh, tot);
        if (i < ntiles)
            tsum[i] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0)
        *total = run;
}

__global__ __launch_bounds__(256) void k_cnt_write(const int32_t *cnt, int cap, int nl,
                                                   const int64_t *tsum, const int64_t *total,
                                                   int64_t *off)
{
    constexpr int PER = SCAN_TILE / 256;
    __shared__ int64_t sh[8];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * PER;
    int32_t v[PER];
    int64_t sacc = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = base + k;
        v[k] = i < nl ? max(0, min(cnt[i], cap)) : 0;
        sacc += v[k];
    }
    int64_t tot;
    int64_t e = block_scan_i64(sacc, sh, tot) + tsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = base + k;
        if (i < nl)
            off[i] = e;
        e += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        off[nl] = *total;
}

hipError_t launch_count_scan(const int32_t *cnt, int cap, int n, int64_t *tsum, int64_t *off,
                             hipStream_t s)
{
    const int ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    int64_t *total = tsum + ntiles;
    k_cnt_tiles<<<ntiles, 256, 0, s>>>(cnt, cap, n, tsum);
    k_cnt_tile_scan<<<1, 1024, 0, s>>>(tsum, ntiles, total);
    k_cnt_write<<<ntiles, 256, 0, s>>>(cnt, cap, n, tsum, total, off);
    return hipGetLastError();
}

int64_t count_scan_workspace(int n) { return n / SCAN_TILE + 2; }

// (target, sink) pairs in sink-major order: key = target node, value = the
// sink leaf's node id (node_values) or its leaf index
__global__ void k_pairs_write(const int32_t *__restrict__ cnt, const int32_t *__restrict__ slots,
                              int cap, int nl, const int32_t *__restrict__ leaf_node,
                              int node_values, const int64_t *__restrict__ off, uint32_t *keys,
                              uint32_t *vals)
{
    const int lf = blockIdx.x;
    const int c = max(0, min(cnt[lf], cap));
    const int64_t o = off[lf];
    const uint32_t sink = node_values ? (uint32_t)leaf_node[lf] : (uint32_t)lf;
    for (int k = threadIdx.x; k < c; k += blockDim.x) {
        keys[o + k] = (uint32_t)slots[(int64_t)lf * cap + k];
        vals[o + k] = sink;
    }
}

// CSR offsets over targets from the sorted keys: off[b] = first index with key >= b
__global__ void k_lower_bound(const uint32_t *__restrict__ keys, int64_t np, int nnodes,
                              int64_t *off)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= nnodes;
         b += gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = np;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < (uint32_t)b)
                lo = mid + 1;
            else
                hi = mid;
        }
        off[b] = lo;
    }
}

template <typename P>
static hipError_t valloc(Tree &t, P **out, size_t elems)
{
    void *p = nullptr;
    hipError_t e = tree_malloc(t, &p, elems * sizeof(P));
    if (e != hipSuccess)
        return e;
    t.vjp_owned.push_back({p, std::max<size_t>(elems * sizeof(P), 256)});
    *out = (P *)p;
    return hipSuccess;
}

// Free a list of device buffers of the reverse pass and clear the pointers.
static void vfree(Tree &t, std::initializer_list<void **> ptrs)
{
    for (void **pp : ptrs) {
        tree_free(t, *pp);
        *pp = nullptr;
    }
}

static hipError_t ensure_vjp_base(Tree &t)
{
    if (t.abt)
        return hipSuccess;
    const Topology &T = t.topo;
    const int64_t n = T.n, nc = T.node_cap;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = valloc(t, &t.abt, 3 * (n + 1));  // + null record
    if (e == hipSuccess) e = valloc(t, &t.xbt, 3 * n);
    if (e == hipSuccess) e = valloc(t, &t.mbt, n);
    if (e == hipSuccess) e = valloc(t, &t.Lbar, NLOC * nc);
    if (e == hipSuccess) e = valloc(t, &t.Lleaf, LLEAF * (int64_t)T.leaf_cap);
    if (e == hipSuccess) e = valloc(t, &t.nadj, 16 * nc);
    if (e == hipSuccess) e = valloc(t, &t.pair_off, T.leaf_cap + 1);
    if (e == hipSuccess) e = valloc(t, &t.vscan, T.leaf_cap / SCAN_TILE + 2);
    if (e == hipSuccess) e = valloc(t, &t.farT.off, nc + 1);
    if (e == hipSuccess) e = valloc(t, &t.pcnt, nc);
    if (e == hipSuccess) e = valloc(t, &t.poff, nc + 1);
    if (e == hipSuccess) e = valloc(t, &t.pscan, nc / SCAN_TILE + 2);
    if (e == hipSuccess) e = valloc(t, &t.nearT.off, nc + 1);
    if (e == hipSuccess && !t.h_pairs)
        e = hipHostMalloc((void **)&t.h_pairs, 4 * sizeof(int64_t), hipHostMallocDefault);
    if (e != hipSuccess) {
        // all or nothing: return what this call took
        for (auto &b : t.vjp_owned)
            tree_free(t, b.p);
        t.vjp_owned.clear();
        t.abt = t.xbt = t.mbt = t.Lbar = t.Lleaf = t.nadj = nullptr;
        t.pair_off = t.vscan = t.farT.off = t.poff = t.pscan = t.nearT.off = nullptr;
        t.pcnt = nullptr;
    }
    return e;
}

// Bits of a node index (the keys of the transposition sort).
static int key_bits(int nnodes)
{
    int bits = 1;
    while ((1ll << bits) <= nnodes)
        ++bits;
    return bits;
}

// Build one transposed list (sink-major pairs -> target-major CSR, stable).
static hipError_t transpose_lists(Tree &t, const int32_t *cnt, const int32_t *slots, int64_t cap,
                                  bool node_values, Tree::Transposed &out, hipStream_t s)
{
    const Topology &T = t.topo;
    const int nl = T.nleaves;
    const int ntiles = (nl + SCAN_TILE - 1) / SCAN_TILE;
    int64_t *total = t.vscan + ntiles;
    k_cnt_tiles<<<ntiles, 256, 0, s>>>(cnt, (int)cap, nl, t.vscan);
    k_cnt_tile_scan<<<1, 1024, 0, s>>>(t.vscan, ntiles, total);
    k_cnt_write<<<ntiles, 256, 0, s>>>(cnt, (int)cap, nl, t.vscan, total, t.pair_off);
    hipError_t e = hipMemcpyAsync(t.h_pairs, total, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return e;
    const int64_t np = t.h_pairs[0];
    if (np > t.vjp_pair_cap || !t.vv0) {
        // (re)allocate the pair sort buffers
        e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return e;
        vfree(t, {(void **)&t.vk0, (void **)&t.vk1, (void **)&t.vv0, (void **)&t.vv1,
                  (void **)&t.vhist, (void **)&t.vtot});
        t.vjp_pair_cap = 0;
        const int64_t cp = np + np / 4 + 1024;
        const int64_t nblk = (cp + RS_TILE - 1) / RS_TILE;
        e = tree_malloc(t, (void **)&t.vk0, cp * sizeof(uint32_t));
        if (e == hipSuccess) e = tree_malloc(t, (void **)&t.vk1, cp * sizeof(uint32_t));
        if (e == hipSuccess) e = tree_malloc(t, (void **)&t.vv0, cp * sizeof(uint32_t));
        if (e == hipSuccess) e = tree_malloc(t, (void **)&t.vv1, cp * sizeof(uint32_t));
        if (e == hipSuccess)
            e = tree_malloc(t, (void **)&t.vhist, RS_MAX_DIGITS * nblk * sizeof(uint32_t));
        if (e == hipSuccess)
            e = tree_malloc(t, (void **)&t.vtot, 8 * RS_MAX_DIGITS * sizeof(uint32_t));
        if (e != hipSuccess) {
            vfree(t, {(void **)&t.vk0, (void **)&t.vk1, (void **)&t.vv0, (void **)&t.vv1,
                      (void **)&t.vhist, (void **)&t.vtot});
            return e;
        }
        t.vjp_pair_cap = cp;
    }
    if (nl > 0)
        k_pairs_write<<<nl, 64, 0, s>>>(cnt, slots, (int)cap, nl, t.leaf_node, node_values ? 1 : 0,
                                        t.pair_off, t.vk0, t.vv0);
    int passes, dbits;
    radix_plan(key_bits(T.nnodes), passes, dbits);
    e = radix_sort_u32(t.vk0, t.vv0, t.vk1, t.vv1, np, 1, passes, t.vhist, t.vtot, s, dbits);
    if (e != hipSuccess)
        return e;
    uint32_t *ks = (passes & 1) ? t.vk1 : t.vk0;
    uint32_t *&vs = (passes & 1) ? t.vv1 : t.vv0;
    k_lower_bound<<<(T.nnodes + 256) / 256, 256, 0, s>>>(ks, np, T.nnodes, out.off);
    out.npairs = np;
    if (t.vjp_pair_cap - np > np / 2 + 1024) {
        // the sort buffers were sized for the other (longer) transposition:
        // keep a list-sized buffer and copy the sorted values into it
        if (out.src && out.src_cap < np) {
            (void)hipStreamSynchronize(s);
            vfree(t, {(void **)&out.src});
            out.src_cap = 0;
        }
        if (!out.src) {
            e = tree_malloc(t, (void **)&out.src, std::max<int64_t>(np, 1) * sizeof(uint32_t));
            if (e != hipSuccess)
                return e;
            out.src_cap = std::max<int64_t>(np, 1);
        }
        if (np > 0)
            e = hipMemcpyAsync(out.src, vs, np * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        return e;
    }
    // the sorted values become the transposed list without a copy: out takes
    // the sort's value buffer, which takes out's previous buffer in exchange
    // (or a new one when that is too small for the next sort)
    uint32_t *prev = out.src;
    const int64_t prev_cap = out.src_cap;
    out.src = vs;
    out.src_cap = t.vjp_pair_cap;
    if (prev && prev_cap >= t.vjp_pair_cap) {
        vs = prev;
    } else {
        vs = nullptr;
        if (prev) {
            (void)hipStreamSynchronize(s);
            vfree(t, {(void **)&prev});
        }
        e = tree_malloc(t, (void **)&vs, t.vjp_pair_cap * sizeof(uint32_t));
    }
    return e;
}

// Pieces of the transposed far lists for the source side of M2L^T.
static hipError_t build_m2lt_pieces(Tree &t, hipStream_t s)
{
    const int nn = t.topo.nnodes;
    const int ntiles = (nn + SCAN_TILE - 1) / SCAN_TILE;
    int64_t *total = t.pscan + ntiles;
    const int g = (nn + 255) / 256;
    k_piece_count<<<g, 256, 0, s>>>(t.farT.off, nn, t.pcnt);
    k_cnt_tiles<<<ntiles, 256, 0, s>>>(t.pcnt, INT32_MAX, nn, t.pscan);
    k_cnt_tile_scan<<<1, 1024, 0, s>>>(t.pscan, ntiles, total);
    k_cnt_write<<<ntiles, 256, 0, s>>>(t.pcnt, INT32_MAX, nn, t.pscan, total, t.poff);
    hipError_t e = hipMemcpyAsync(t.h_pairs + 1, total, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return e;
    const int64_t np = t.h_pairs[1];
    if (np > t.piece_cap) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return e;
        vfree(t, {(void **)&t.pnode, (void **)&t.ppart});
        t.piece_cap = 0;
        const int64_t cp = np + np / 4 + 256;
        e = tree_malloc(t, (void **)&t.pnode, cp * sizeof(int32_t));
        if (e == hipSuccess)
            e = tree_malloc(t, (void **)&t.ppart, 10 * cp * sizeof(double));
        if (e != hipSuccess) {
            vfree(t, {(void **)&t.pnode, (void **)&t.ppart});
            return e;
        }
        t.piece_cap = cp;
    }
    t.npieces = np;
    k_piece_fill<<<g, 256, 0, s>>>(t.poff, nn, t.pnode);
    return hipGetLastError();
}

// Pieces of the transposed near lists (the source side of P2P^T), cut as
// the forward lists are: ceil(blocks / per) per leaf, at least one.
__global__ void k_tpiece_count(const int32_t *__restrict__ leaf_node, int nleaves,
                               const int64_t *__restrict__ toff, int nsub, int64_t per,
                               int32_t *np)
{
    const int lf = blockIdx.x * blockDim.x + threadIdx.x;
    if (lf >= nleaves)
        return;
    const int v = leaf_node[lf];
    const int64_t wk = (toff[v + 1] - toff[v]) * nsub;
    np[lf] = (int32_t)max<int64_t>(1, (wk + per - 1) / per);
}

static hipError_t build_p2pt_pieces(Tree &t, hipStream_t s)
{
    Tree::Pieces &P = t.pnearT;
    const Topology &T = t.topo;
    const int nl = T.nleaves;
    const int nsub = (T.leaf_size + 7) / 8;
    hipError_t e = hipSuccess;
    if (!P.np) {
        const int64_t lc = T.leaf_cap;
        e = tree_malloc(t, (void **)&P.np, lc * sizeof(int32_t));
        if (e == hipSuccess)
            e = tree_malloc(t, (void **)&P.off, (lc + 1) * sizeof(int64_t));
        if (e == hipSuccess)
            e = tree_malloc(t, (void **)&P.tsum, count_scan_workspace((int)lc) * sizeof(int64_t));
        if (e != hipSuccess) {
            vfree(t, {(void **)&P.np, (void **)&P.off, (void **)&P.tsum});
            return e;
        }
    }
    P.n = 0;
    k_tpiece_count<<<(nl + 255) / 256, 256, 0, s>>>(t.leaf_node, nl, t.nearT.off, nsub,
                                                     t.vjp_src_piece_blocks, P.np);
    e = launch_count_scan(P.np, INT32_MAX, nl, P.tsum, P.off, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(t.h_pairs + 2, P.off + nl, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return e;
    const int64_t np = t.h_pairs[2];
    if (np > nl && np > P.cap) {
        vfree(t, {(void **)&P.list, &P.part});
        P.cap = 0;
        const int64_t cp = np + np / 4 + 64;
        e = tree_malloc(t, (void **)&P.list, cp * sizeof(int2));
        if (e == hipSuccess)
            e = tree_malloc(t, &P.part, cp * 4 * (size_t)T.leaf_size * sizeof(double));
        if (e != hipSuccess) {
            vfree(t, {(void **)&P.list, &P.part});
            return e;
        }
        P.cap = cp;
    }
    P.part_stride = 4 * (size_t)T.leaf_size * sizeof(double);
    P.n = np;
    return np > nl ? launch_piece_table(P.off, P.np, nl, P.list, s) : hipSuccess;
}

// M2L^T, sink side per leaf and source side in pieces.
template <int FORM>
static void vjp_m2l(Tree &t, hipStream_t s)
{
    const int nl = t.topo.nleaves;
    k_vjp_m2l_sink<FORM><<<(int)(((int64_t)nl * M2LT_LANES + 255) / 256), 256, 0, s>>>(
        t.recA, t.recQ, t.leaf_node, nl, t.far_cnt, t.far_src, (int)t.cap_far, t.Lbar, t.nadj);
    if (t.npieces > 0)
        k_vjp_m2l_src_piece<FORM>
            <<<(int)((t.npieces + VJPM_WAVES - 1) / VJPM_WAVES), 64 * VJPM_WAVES, 0, s>>>(
            t.recA, t.recQ, t.farT.off, t.farT.src, t.Lleaf, t.pnode, t.poff, t.npieces, t.ppart);
}

// Mutual walk: forward totals of the internal cells, L2L^T level by level
// (deepest first), then M2L^T of the symmetric pairs.
static hipError_t vjp_mutual_far(Tree &t, hipStream_t s)
{
    const Topology &T = t.topo;
    hipError_t e = launch_l2l_internal(t, s);
    if (e != hipSuccess)
        return e;
    for (int l = T.depth - 2; l >= 0; --l) {
        const int o = T.lvl_int_off[l], cnt = T.lvl_int_off[l + 1] - o;
        if (cnt > 0)
            k_vjp_l2l_level<<<(cnt + 255) / 256, 256, 0, s>>>(t.int_nodes + o, cnt, t.left,
                                                              t.right, t.recA, t.L, t.Lbar,
                                                              t.nadj);
    }
    const MutualLists &M = t.mw;
    const uint64_t mask = (1ull << mutual_key_bits(t)) - 1ull;
    const int g = (int)(((int64_t)T.nnodes * 16 + 255) / 256);
    if (t.p.expansion == FMM_EXPANSION_DEHNEN)
        k_vjp_m2l_mutual<FMM_EXPANSION_DEHNEN><<<g, 256, 0, s>>>(
            t.recA, t.recQ, T.nnodes, M.fstart, M.fend, M.far_sorted, mask, t.Lbar, t.nadj);
    else
        k_vjp_m2l_mutual<FMM_EXPANSION_PHANTOM><<<g, 256, 0, s>>>(
            t.recA, t.recQ, T.nnodes, M.fstart, M.fend, M.far_sorted, mask, t.Lbar, t.nadj);
    return hipGetLastError();
}

// The mutual walk's far pairs are symmetric and need no transposition (its
// near lists are symmetric too, but the source side of P2P^T reads the CSR
// form).
hipError_t ensure_transposed(Tree &t, hipStream_t s)
{
    hipError_t e = ensure_vjp_base(t);
    if (e != hipSuccess || t.has_transposed)
        return e;
    if (t.lists_policy != FMM_WALK_MUTUAL) {
        e = transpose_lists(t, t.far_cnt, t.far_src, t.cap_far, false, t.farT, s);
        if (e == hipSuccess)
            e = build_m2lt_pieces(t, s);
    }
    if (e == hipSuccess)
        e = transpose_lists(t, t.near_cnt, t.near_src, t.cap_near, true, t.nearT, s);
    if (e == hipSuccess)
        e = build_p2pt_pieces(t, s);
    if (e == hipSuccess)
        t.has_transposed = true;
    return e;
}

hipError_t launch_vjp(Tree &t, const void *abar, void *xbar, void *mbar, hipStream_t s)
{
    const Topology &T = t.topo;
    const int64_t n = T.n;
    const int nl = T.nleaves;
    hipError_t e = ensure_transposed(t, s);
    if (e != hipSuccess)
        return e;
    const bool fp32 = t.p.precision == FMM_FP32;
    if (fp32) {
        // the reverse pass runs in FP64: form the FP64 local expansions
        e = launch_far_f64(t, s);
        if (e != hipSuccess)
            return e;
    }
    const int gs = (int)std::min<int64_t>((n + 255) / 256, 4096);
    if (fp32)
        k_vjp_prep<float><<<gs, 256, 0, s>>>((const float *)abar, n, t.perm, t.p.G, t.abt);
    else
        k_vjp_prep<double><<<gs, 256, 0, s>>>((const double *)abar, n, t.perm, t.p.G, t.abt);
    k_vjp_l2p<<<(nl + 255) / 256, 256, 0, s>>>(t.pm, t.abt, t.leaf_node, nl, t.first, t.count,
                                               t.recA, t.L, t.Lbar, t.Lleaf, t.xbt, t.nadj);
    if (t.lists_policy == FMM_WALK_MUTUAL) {
        e = vjp_mutual_far(t, s);
        if (e != hipSuccess)
            return e;
    } else {
        if (t.p.expansion == FMM_EXPANSION_DEHNEN)
            vjp_m2l<FMM_EXPANSION_DEHNEN>(t, s);
        else
            vjp_m2l<FMM_EXPANSION_PHANTOM>(t, s);
        k_vjp_m2l_src_fold<<<(T.nnodes + 255) / 256, 256, 0, s>>>(t.left, T.nnodes, t.poff,
                                                                  t.ppart, t.nadj);
    }
    const int nsub = (T.leaf_size + 7) / 8;
    const int per = (int)t.near_piece_blocks;
    {
        // sink side: the forward near lists, in their pieces when split
        const bool pc = use_pieces(t);
        const int nu = pc ? (int)t.pnear.n : nl;
        const int stride = 3 * T.leaf_size;
        k_vjp_p2p_sink<<<(nu + VJP_WAVES - 1) / VJP_WAVES, VJP_WG, 0, s>>>(
            t.pm, t.ph, t.abt, t.first, t.count, t.leaf_node, nu, t.near_cnt, t.near_src,
            (int)t.cap_near, nsub, n, t.xbt, pc ? t.pnear.list : nullptr, per,
            (double *)t.pnear.part, stride);
        if (pc && nu > nl)
            k_vjp_p2p_fold<<<(nu - nl + 3) / 4, 256, 0, s>>>(
                t.leaf_node, t.pnear.list, nu - nl, t.first, t.count, t.pnear.off,
                (const double *)t.pnear.part, stride, 3, t.xbt, t.mbt);
    }
    {
        // source side: the transposed near lists, in their own pieces
        const bool pc = t.pnearT.n > nl;
        const int nu = pc ? (int)t.pnearT.n : nl;
        const int stride = 4 * T.leaf_size;
        k_vjp_p2p_src<<<(nu + VJP_WAVES - 1) / VJP_WAVES, VJP_WG, 0, s>>>(
            t.pm, t.ph, t.abt, t.first, t.count, t.leaf_node, nu, t.nearT.off, t.nearT.src, nsub,
            n, t.xbt, t.mbt, pc ? t.pnearT.list : nullptr, (int)t.vjp_src_piece_blocks,
            (double *)t.pnearT.part, stride);
        if (pc)
            k_vjp_p2p_fold<<<(nu - nl + 3) / 4, 256, 0, s>>>(
                t.leaf_node, t.pnearT.list, nu - nl, t.first, t.count, t.pnearT.off,
                (const double *)t.pnearT.part, stride, 4, t.xbt, t.mbt);
    }
    if (fp32)
        k_vjp_moments<float><<<(int)((n + 255) / 256), 256, 0, s>>>(
            t.pm, n, t.recA, t.nadj, t.first, t.count, t.left, t.right, T.nnodes, t.xbt, t.mbt,
            t.perm,
            (float *)xbar, (float *)mbar);
    else
        k_vjp_moments<double><<<(int)((n + 255) / 256), 256, 0, s>>>(
            t.pm, n, t.recA, t.nadj, t.first, t.count, t.left, t.right, T.nnodes, t.xbt, t.mbt,
            t.perm,
            (double *)xbar, (double *)mbar);
    return hipGetLastError();
}

void release_vjp(Tree &t)
{
    for (auto &b : t.vjp_owned)
        tree_free(t, b.p);
    t.vjp_owned.clear();
    vfree(t, {(void **)&t.vk0, (void **)&t.vk1, (void **)&t.vv0, (void **)&t.vv1,
              (void **)&t.vhist, (void **)&t.vtot, (void **)&t.farT.src, (void **)&t.nearT.src,
              (void **)&t.pnode, (void **)&t.ppart, (void **)&t.pnearT.np, (void **)&t.pnearT.off,
              (void **)&t.pnearT.tsum, (void **)&t.pnearT.list, &t.pnearT.part});
    t.pnearT.cap = t.pnearT.n = 0;
    t.vjp_pair_cap = t.farT.src_cap = t.nearT.src_cap = 0;
    if (t.h_pairs)
        (void)hipHostFree(t.h_pairs);
    t.h_pairs = nullptr;
}

}  // namespace fmm
