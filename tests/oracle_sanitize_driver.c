/*
 * Drives every entry point of the CPU oracle on small seeded inputs, with
 * every buffer allocated at its exact size, so that a build with
 * -fsanitize=address,undefined reports any out-of-bounds access, use of
 * freed memory, leak, signed overflow or other undefined behaviour in the
 * oracle.  Test infrastructure: built and run by tests/test_oracle_sanitize.py.
 * Exits 0 when every case ran; the sanitizers abort on the first error.
 */
#include "../oracle/fmm_oracle.c"

#include <stdio.h>

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

static double urand(void)
{
    /* splitmix64 */
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static void *xmalloc(size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static void run_case(int64_t n, int32_t leaf, double theta, int clumped, int tied)
{
    double *x = xmalloc(3 * n * sizeof(double)), *m = xmalloc(n * sizeof(double));
    double *h = xmalloc(n * sizeof(double)), *v = xmalloc(3 * n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            double u = urand();
            x[3 * i + d] = clumped ? 0.5 + 0.01 * (u - 0.5) * (i % 3 == 0 ? 100.0 : 1.0) : u;
            if (tied && i % 4 == 1)
                x[3 * i + d] = x[3 * (i - 1) + d];
            v[3 * i + d] = urand() - 0.5;
        }
        m[i] = 0.5 + urand();
        h[i] = 0.01 + 0.05 * urand();
    }
    double *a = xmalloc(3 * n * sizeof(double)), *ad = xmalloc(3 * n * sizeof(double));
    double *xb = xmalloc(3 * n * sizeof(double)), *mb = xmalloc(n * sizeof(double));
    orc_direct(n, x, m, h, 1.0, ad);
    orc_direct_vjp(n, x, m, h, 1.0, ad, xb, mb);
    int64_t sinks[2] = {0, n - 1};
    double as[6];
    orc_direct_sinks(n, x, m, h, 1.0, n > 1 ? 2 : 1, sinks, as);
    uint64_t *key = xmalloc(n * sizeof(uint64_t));
    int32_t *order = xmalloc(n * sizeof(int32_t));
    orc_morton(n, x, key, order);
    for (int shape = 0; shape < 2; ++shape) {
        const int64_t cap = 2 * n;
        int32_t *perm = xmalloc(n * sizeof(int32_t));
        int32_t *first = xmalloc(cap * sizeof(int32_t)), *count = xmalloc(cap * sizeof(int32_t));
        int32_t *left = xmalloc(cap * sizeof(int32_t)), *right = xmalloc(cap * sizeof(int32_t));
        int32_t *axis = xmalloc(cap * sizeof(int32_t));
        int32_t nn = shape == 0 ? orc_build_tree(n, x, leaf, perm, first, count, left, right, axis)
                                : orc_build_tree_com(n, x, m, leaf, perm, first, count, left,
                                                     right, axis);
        double *M = xmalloc(nn * sizeof(double)), *c = xmalloc(3 * nn * sizeof(double));
        double *s = xmalloc(nn * sizeof(double)), *hm = xmalloc(nn * sizeof(double));
        double *Q = xmalloc(6 * nn * sizeof(double));
        orc_moments(n, x, m, h, perm, nn, first, count, left, right, M, c, s, hm, Q);
        for (int policy = 0; policy < 2; ++policy) {
            int32_t *fo = xmalloc((nn + 1) * sizeof(int32_t));
            int32_t *no = xmalloc((nn + 1) * sizeof(int32_t));
            int64_t tot[2];
            orc_walk(policy, nn, left, right, c, s, hm, theta, 2.0, fo, NULL, no, NULL, tot);
            int32_t *fs = xmalloc(tot[0] * sizeof(int32_t)), *ns = xmalloc(tot[1] * sizeof(int32_t));
            orc_walk(policy, nn, left, right, c, s, hm, theta, 2.0, fo, fs, no, ns, tot);
            double *L = xmalloc(19 * nn * sizeof(double));
            for (int form = 0; form < 2; ++form) {
                orc_far_field(policy, form, nn, left, right, M, c, Q, fo, fs, L);
                orc_near_and_l2p(n, x, m, h, perm, nn, first, count, left, c, L, no, ns, 1.0, a);
            }
            double st[16], est[4];
            orc_stats(n, x, v, m, a, st);
            orc_stats(n, x, NULL, m, a, st);
            orc_asym_estimate(nn, left, right, M, c, s, fo, fs, 0.0, est);
            free(fs);
            free(ns);
            free(fo);
            free(no);
            free(L);
        }
        if (shape == 0) {
            int32_t nl = 0;
            for (int32_t u = 0; u < nn; ++u)
                nl += left[u] < 0;
            int32_t *lv = xmalloc(nl * sizeof(int32_t));
            int64_t *cnt = xmalloc(2 * (size_t)nl * sizeof(int64_t));
            for (int32_t u = 0, k = 0; u < nn; ++u)
                if (left[u] < 0)
                    lv[k++] = u;
            orc_fmm_leaves(n, x, m, h, perm, nn, first, count, left, right, M, c, s, hm, Q, theta,
                           2.0, 1.0, 0, nl, lv, a, cnt);
            free(lv);
            free(cnt);
        }
        double Mp, cp[3], Qp[6], Lm[19], y[3] = {0.01, -0.02, 0.03}, ap[3], Ls[19];
        orc_p2m(n, x, m, &Mp, cp, Qp);
        double rv[3] = {3.0, -1.0, 2.0};
        orc_m2l(0, rv, Mp, Qp, Lm);
        orc_m2l(1, rv, Mp, Qp, Lm);
        orc_l2p(Lm, y, ap);
        orc_l2l(Lm, y, Ls);
        (void)orc_m4_g(0.5, 0.3);
        (void)orc_m4_dg_over_r(0.5, 0.3);
        free(perm);
        free(first);
        free(count);
        free(left);
        free(right);
        free(axis);
        free(M);
        free(c);
        free(s);
        free(hm);
        free(Q);
    }
    free(key);
    free(order);
    free(x);
    free(m);
    free(h);
    free(v);
    free(a);
    free(ad);
    free(xb);
    free(mb);
}

int main(void)
{
    const int64_t ns[] = {1, 2, 7, 9, 64, 301};
    const int32_t leaves[] = {1, 3, 8, 10};
    const double thetas[] = {0.0, 0.5, 1.0};
    int cases = 0;
    for (size_t i = 0; i < sizeof ns / sizeof ns[0]; ++i)
        for (size_t j = 0; j < sizeof leaves / sizeof leaves[0]; ++j)
            for (size_t k = 0; k < sizeof thetas / sizeof thetas[0]; ++k) {
                run_case(ns[i], leaves[j], thetas[k], (int)((i + j + k) % 2), (int)((i + k) % 2));
                ++cases;
            }
    printf("sanitized oracle: %d cases\n", cases);
    return 0;
}
