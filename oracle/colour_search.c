/*
 * Oracle: exhaustive search for the torus colouring c(x) = sum_j sigma_j x_j
 * mod n_c (Sec. 3, eq. coloring-formula).  TEST INFRASTRUCTURE ONLY: loaded
 * by the tests through ctypes, never by the product library.
 *
 * A colouring is valid at distance d when any two distinct sites whose
 * periodic L1 (graph) distance is at most d get different colours, wrap-around
 * included.  Search order: n_c = 2, 3, ... ; for each n_c, sigma runs over
 * [0, n_c)^nD in lexicographic order with sigma_1 most significant; the first
 * valid sigma is returned.
 *
 * Validity is decided by brute force over displacements: for every integer
 * displacement delta with 0 < |delta|_1 <= d that moves to a different site,
 * and every way each coordinate can wrap (x_j + delta_j crosses the boundary
 * or not), the colour difference sum_j sigma_j (delta_j - L_j w_j) must be
 * nonzero mod n_c.  w_j takes the two values floor(delta_j / L_j) and
 * floor((delta_j + L_j - 1) / L_j), the only wrap counts a start coordinate in
 * [0, L_j) can produce.
 */
#include <stdint.h>
#include <stdlib.h>

#define MAXD 4

static int floordiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

/* All colour-difference vectors a = delta - L*w that must not vanish mod n_c. */
static int build_forbidden(const int *L, int nD, int d, int *out /* [cap][MAXD] */, int cap)
{
    int cnt = 0;
    int lo[MAXD], delta[MAXD];
    for (int j = 0; j < nD; ++j) lo[j] = -d;
    for (int j = 0; j < nD; ++j) delta[j] = lo[j];
    for (;;) {
        int l1 = 0, same = 1;
        for (int j = 0; j < nD; ++j) {
            l1 += abs(delta[j]);
            if (((delta[j] % L[j]) + L[j]) % L[j] != 0) same = 0;
        }
        if (l1 >= 1 && l1 <= d && !same) {
            int w0[MAXD], nw[MAXD];
            for (int j = 0; j < nD; ++j) {
                w0[j] = floordiv(delta[j], L[j]);
                nw[j] = (floordiv(delta[j] + L[j] - 1, L[j]) != w0[j]) ? 2 : 1;
            }
            int total = 1;
            for (int j = 0; j < nD; ++j) total *= nw[j];
            for (int p = 0; p < total; ++p) {
                int q = p;
                if (cnt >= cap) return -1;
                for (int j = 0; j < nD; ++j) {
                    int w = w0[j] + (q % nw[j]);
                    q /= nw[j];
                    out[cnt * MAXD + j] = delta[j] - L[j] * w;
                }
                for (int j = nD; j < MAXD; ++j) out[cnt * MAXD + j] = 0;
                ++cnt;
            }
        }
        int j = nD - 1;
        while (j >= 0 && delta[j] == d) { delta[j] = -d; --j; }
        if (j < 0) break;
        ++delta[j];
    }
    return cnt;
}

/* Colour differences whose last nonzero coordinate is `level` are tested as
 * soon as sigma_1..sigma_level are fixed (a prefix that fails them fails for
 * every completion, so pruning it keeps the lexicographic first-valid order). */
static int valid_level(const int *sigma, int level, int nc, const int *forb,
                       const int *last, int nf)
{
    for (int f = 0; f < nf; ++f) {
        if (last[f] != level) continue;
        long s = 0;
        for (int j = 0; j <= level; ++j) s += (long)sigma[j] * forb[f * MAXD + j];
        if (((s % nc) + nc) % nc == 0) return 0;
    }
    return 1;
}

static int search_rec(int *s, int level, int nD, int nc, const int *forb,
                      const int *last, int nf)
{
    for (s[level] = 0; s[level] < nc; ++s[level]) {
        if (!valid_level(s, level, nc, forb, last, nf)) continue;
        if (level == nD - 1) return 1;
        if (search_rec(s, level + 1, nD, nc, forb, last, nf)) return 1;
    }
    return 0;
}

/* Returns 0 and fills n_c, sigma on success; -1 if no n_c <= max_nc works. */
int oracle_colour_search(const int32_t *dims, int32_t nD, int32_t d, int32_t max_nc,
                         int32_t *n_c, int32_t *sigma)
{
    int L[MAXD];
    if (nD < 1 || nD > MAXD || d < 1) return -2;
    for (int j = 0; j < nD; ++j) L[j] = dims[j];
    int cap = 1 << 20;
    int *forb = (int *)malloc(sizeof(int) * MAXD * cap);
    int nf = build_forbidden(L, nD, d, forb, cap);
    if (nf < 0) { free(forb); return -3; }
    int *last = (int *)malloc(sizeof(int) * (nf > 0 ? nf : 1));
    for (int f = 0; f < nf; ++f) {
        last[f] = 0;
        for (int j = 0; j < nD; ++j) if (forb[f * MAXD + j] != 0) last[f] = j;
    }
    for (int nc = 2; nc <= max_nc; ++nc) {
        int s[MAXD] = {0, 0, 0, 0};
        if (search_rec(s, 0, nD, nc, forb, last, nf)) {
            *n_c = nc;
            for (int j = 0; j < nD; ++j) sigma[j] = s[j];
            free(last);
            free(forb);
            return 0;
        }
    }
    free(last);
    free(forb);
    return -1;
}
