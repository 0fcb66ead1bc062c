/* Host driver for the sanitizer build (AddressSanitizer +
 * UndefinedBehaviorSanitizer) of the CPU oracle: on seeded random graphs it
 * runs the brute force, the elimination in all four algebras, the
 * polynomial elimination and the plan follower on a left-deep tree (with and
 * without sliced indices), and checks that they agree.  The sanitizers abort
 * on a memory error or undefined behaviour; the exit status counts failed
 * agreements. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_brute_force(int nv, int ne, const int32_t* edges, const double* w, int nbeta, const double* betas,
                    double* max_size, uint64_t* count_at_max, uint64_t* total, uint64_t* size_hist, double* z,
                    double* logz, int sets_cap, uint64_t* sets, int* n_sets, uint64_t fix_mask, uint64_t fix_val);
int orc_eliminate(int nv, int ne, const int32_t* edges, const double* w, int sr, double beta, int max_width,
                  double* size, uint64_t* limbs, double* zval, double* logz, int* width_out);
int orc_eliminate_poly(int nv, int ne, const int32_t* edges, int max_width, uint64_t* coeffs, int* degree,
                       int* width_out);
int orc_follow_plan(int nv, int ne, const int32_t* edges, const double* w, int sr, double beta, int nleaf,
                    int ninner, const int32_t* fac_off, const int32_t* fac, const int32_t* left,
                    const int32_t* right, const int32_t* idx_off, const int32_t* idx, int nsliced,
                    const int32_t* sliced, int64_t slice_begin, int64_t slice_end, int max_rank, double* size,
                    uint64_t* limbs, double* zval, double* logz);

static uint64_t g_state = 88172645463325252ull;
static uint64_t rnd(void) { /* xorshift64 */
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return g_state;
}

static int bad = 0;
#define CHECK(c)                                                     \
    do {                                                             \
        if (!(c)) {                                                  \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            bad++;                                                   \
        }                                                            \
    } while (0)

int main(void) {
    for (int round = 0; round < 30; round++) {
        const int nv = 3 + (int)(rnd() % 14);
        int32_t edges[2 * 120];
        int ne = 0;
        for (int a = 0; a < nv; a++)
            for (int b = a + 1; b < nv && ne < 120; b++)
                if (rnd() % 4 == 0) {
                    edges[2 * ne] = a;
                    edges[2 * ne + 1] = b;
                    ne++;
                }
        double w[32];
        for (int v = 0; v < nv; v++) w[v] = (double)(1 + rnd() % 3);
        const double* wp = round % 2 ? w : NULL;
        const double beta = 0.7;
        double mx, z, lz;
        uint64_t cmax, tot, hist[40];
        int nsets = 0;
        CHECK(orc_brute_force(nv, ne, edges, wp, 1, &beta, &mx, &cmax, &tot, hist, &z, &lz, 0, NULL, &nsets, 0, 0) == 0);
        double size, zv, lzv;
        uint64_t limbs[4];
        int width;
        CHECK(orc_eliminate(nv, ne, edges, wp, 0, 0.0, 26, &size, limbs, &zv, &lzv, &width) == 0);
        CHECK(size == mx);
        CHECK(orc_eliminate(nv, ne, edges, wp, 1, 0.0, 26, &size, limbs, &zv, &lzv, &width) == 0);
        CHECK(size == mx && limbs[0] == cmax);
        CHECK(orc_eliminate(nv, ne, edges, wp, 2, 0.0, 26, &size, limbs, &zv, &lzv, &width) == 0);
        CHECK(limbs[0] == tot);
        CHECK(orc_eliminate(nv, ne, edges, wp, 3, beta, 26, &size, limbs, &zv, &lzv, &width) == 0);
        CHECK(fabs(zv - z) <= 1e-12 * z);
        uint64_t coeffs[40 * 4];
        int degree = 0;
        CHECK(orc_eliminate_poly(nv, ne, edges, 20, coeffs, &degree, &width) == 0);
        for (int k = 0; k <= degree; k++) CHECK(coeffs[4 * k] == hist[k]);
        /* a left-deep tree over one leaf per edge and one per vertex; index
         * lists by the einsum rule (an index stays while it occurs outside) */
        const int nleaf = ne + nv, ninner = nleaf - 1, nn = nleaf + ninner;
        int32_t fac_off[300], fac[300], left[300], right[300], idx_off[700], idx[20000];
        for (int l = 0; l <= nleaf; l++) fac_off[l] = l;
        for (int e = 0; e < ne; e++) fac[e] = e;
        for (int v = 0; v < nv; v++) fac[ne + v] = -v - 1;
        int occ_total[32] = {0};
        for (int e = 0; e < ne; e++) {
            occ_total[edges[2 * e]]++;
            occ_total[edges[2 * e + 1]]++;
        }
        for (int v = 0; v < nv; v++) occ_total[v]++;
        int occ[32] = {0}, pos = 0;
        idx_off[0] = 0;
        for (int x = 0; x < nn; x++) {
            if (x < nleaf) {
                int c = fac[x];
                int vs[2], k = 0;
                if (c >= 0) {
                    vs[k++] = edges[2 * c];
                    vs[k++] = edges[2 * c + 1];
                } else {
                    vs[k++] = -c - 1;
                }
                if (k == 2 && vs[0] > vs[1]) {
                    int t = vs[0];
                    vs[0] = vs[1];
                    vs[1] = t;
                }
                for (int q = 0; q < k; q++)
                    if (occ_total[vs[q]] > 1) idx[pos++] = vs[q];
            } else {
                const int t = x - nleaf;
                left[t] = t == 0 ? 0 : nleaf + t - 1;
                right[t] = t + 1;
                const int leaf = t + 1;
                int c = fac[leaf];
                if (c >= 0) {
                    occ[edges[2 * c]]++;
                    occ[edges[2 * c + 1]]++;
                } else {
                    occ[-c - 1]++;
                }
                if (t == 0) {
                    int c0 = fac[0];
                    if (c0 >= 0) {
                        occ[edges[2 * c0]]++;
                        occ[edges[2 * c0 + 1]]++;
                    } else {
                        occ[-c0 - 1]++;
                    }
                }
                for (int v = 0; v < nv; v++)
                    if (occ[v] > 0 && occ[v] < occ_total[v]) idx[pos++] = v;
            }
            idx_off[x + 1] = pos;
        }
        for (int sr = 0; sr < 4; sr++) {
            for (int ns = 0; ns <= 2; ns += 2) {
                const int32_t sliced[2] = {0, nv - 1};
                CHECK(orc_follow_plan(nv, ne, edges, wp, sr, beta, nleaf, ninner, fac_off, fac, left, right, idx_off,
                                      idx, ns, sliced, 0, 0, 26, &size, limbs, &zv, &lzv) == 0);
                if (sr == 0) CHECK(size == mx);
                if (sr == 1) CHECK(size == mx && limbs[0] == cmax);
                if (sr == 2) CHECK(limbs[0] == tot);
                if (sr == 3) CHECK(fabs(zv - z) <= 1e-12 * z);
            }
        }
    }
    printf("oracle driver: %d failed checks\n", bad);
    return bad ? 1 : 0;
}
