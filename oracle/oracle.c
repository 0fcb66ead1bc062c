/*
 * oracle.c -- plain, slow CPU reference for the generic tensor-network method
 * applied to the (weighted) independent-set problem.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this file.  It shares no code,
 * header, table or constant generator with the GPU library, and the GPU
 * library never loads it.
 *
 * What it computes (paper Sec. 3.1 eq. for the energy model and partition
 * function; Sec. 3.2 for the independent-set energy H(G,n) = -sum_v w_v n_v +
 * inf * sum_(u,v) n_u n_v; Sec. 5 property table):
 *
 *   SizeMax        max_{S independent} w(S)                     (tropical algebra)
 *   CountingMax    (SizeMax, #{S : w(S) = SizeMax})             (counting tropical)
 *   CountingAll    #{S independent}  = Z(beta = 0)              (integers)
 *   Partition fn   Z(beta) = sum_{S independent} exp(beta w(S)) (reals)
 *
 * Three programs, each independent of the others:
 *   O1  orc_brute_force   enumerate all 2^n subsets (the definitions above)
 *   O2  orc_eliminate     variable elimination with its own heuristic order,
 *                         over dense factor tables in exact semiring arithmetic;
 *       orc_eliminate_poly  the same over polynomial-valued tables: the
 *                         independence polynomial (Sec. 5.3 GraphPolynomial)
 *       orc_eliminate_sg, orc_brute_force_sg  the spin glass of Sec. 2
 *                         (energy H = sum J s s + sum h s, Sec. 6.4 buckyball)
 *       orc_brute_force_topk, orc_brute_force_sg_topk  the k largest values
 *                         with multiplicity (SizeMax(k)) by enumeration
 *       orc_brute_force_count_top, orc_brute_force_sg_count_top  the number
 *                         of configurations at the k highest integer values
 *                         top, top - 1, ... (CountingMax(k)) by enumeration
 *   O3  orc_follow_plan   evaluate a given binary contraction tree (Sec. 4.1),
 *                         one literal einsum loop per node, with optional
 *                         sliced indices (Sec. 4.2, TreeSA slicing)
 *
 * Element arithmetic: sizes and partition functions in long double (64-bit
 * mantissa, exponent range to 1e4932: no rescaling needed); counts as exact
 * 256-bit unsigned integers with an overflow flag.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EOVERFLOW (-4)
#define ORC_ETOOBIG (-5)

/* Semiring tags.  Sec. 5 property table: Tropical <-> SizeMax,
 * CountingTropical <-> CountingMax, Real <-> CountingAll / PartitionFunction. */
enum { SR_TROPICAL = 0, SR_COUNTING_TROPICAL = 1, SR_COUNT = 2, SR_PARTITION = 3 };

/* ---------------------------------------------------------------- u256 --- */

typedef struct {
    uint64_t w[4]; /* little-endian 64-bit limbs */
} u256;

static int g_overflow; /* set by any u256 operation whose result needs > 256 bits */

static u256 u256_from(uint64_t x) {
    u256 r;
    r.w[0] = x;
    r.w[1] = r.w[2] = r.w[3] = 0;
    return r;
}

static u256 u256_add(u256 a, u256 b) {
    u256 r;
    unsigned __int128 carry = 0;
    for (int i = 0; i < 4; i++) {
        unsigned __int128 s = (unsigned __int128)a.w[i] + b.w[i] + carry;
        r.w[i] = (uint64_t)s;
        carry = s >> 64;
    }
    if (carry) g_overflow = 1;
    return r;
}

/* schoolbook product; any non-zero limb beyond 256 bits flags overflow */
static u256 u256_mul(u256 a, u256 b) {
    uint64_t t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 4; i++) {
        unsigned __int128 carry = 0;
        for (int j = 0; j < 4; j++) {
            unsigned __int128 p = (unsigned __int128)a.w[i] * b.w[j] + t[i + j] + carry;
            t[i + j] = (uint64_t)p;
            carry = p >> 64;
        }
        t[i + 4] += (uint64_t)carry;
    }
    if (t[4] | t[5] | t[6] | t[7]) g_overflow = 1;
    u256 r;
    memcpy(r.w, t, sizeof r.w);
    return r;
}

/* -------------------------------------------------------- semiring ------ */

/* One element type for all four algebras: n carries the tropical size or the
 * real value of the partition function, c carries counts. */
typedef struct {
    long double n;
    u256 c;
} elem;

static inline elem e_zero(int sr) { /* additive identity */
    elem e;
    e.c = u256_from(0);
    e.n = (sr == SR_TROPICAL || sr == SR_COUNTING_TROPICAL) ? -INFINITY : 0.0L;
    return e;
}

static inline elem e_one(int sr) { /* multiplicative identity */
    elem e;
    e.c = u256_from(1);
    e.n = (sr == SR_TROPICAL || sr == SR_COUNTING_TROPICAL) ? 0.0L : 1.0L;
    if (sr == SR_TROPICAL) e.c = u256_from(0);
    return e;
}

static inline elem e_add(int sr, elem a, elem b) { /* the semiring's "+" */
    elem r = a;
    switch (sr) {
    case SR_TROPICAL: /* + is max */
        r.n = a.n >= b.n ? a.n : b.n;
        break;
    case SR_COUNTING_TROPICAL: /* larger size wins; equal sizes add counts */
        if (a.n > b.n) r = a;
        else if (b.n > a.n) r = b;
        else {
            r.n = a.n;
            r.c = u256_add(a.c, b.c);
        }
        break;
    case SR_COUNT:
        r.c = u256_add(a.c, b.c);
        break;
    default: /* SR_PARTITION */
        r.n = a.n + b.n;
        break;
    }
    return r;
}

static inline elem e_mul(int sr, elem a, elem b) { /* the semiring's "*" */
    elem r = a;
    switch (sr) {
    case SR_TROPICAL: /* * is + ; -inf absorbs */
        r.n = a.n + b.n;
        break;
    case SR_COUNTING_TROPICAL:
        r.n = a.n + b.n;
        r.c = u256_mul(a.c, b.c);
        break;
    case SR_COUNT:
        r.c = u256_mul(a.c, b.c);
        break;
    default:
        r.n = a.n * b.n;
        break;
    }
    return r;
}

/* x^w, the weight entry of a vertex tensor W = (1, x^w) with x = e^beta
 * (Sec. 3.2).  In the tropical algebras x^w is the size w itself. */
static elem e_weight(int sr, double w, double beta) {
    elem e = e_one(sr);
    switch (sr) {
    case SR_TROPICAL:
    case SR_COUNTING_TROPICAL:
        e.n = (long double)w;
        break;
    case SR_COUNT:
        break; /* x = 1 */
    default:
        e.n = expl((long double)beta * (long double)w);
        break;
    }
    return e;
}

/* Edge tensor B(n_u, n_v) = [[1, 1], [1, 0]]  (Sec. 3.2). */
static elem e_edge(int sr, int nu, int nv) { return (nu && nv) ? e_zero(sr) : e_one(sr); }

/* Vertex tensor W(n_v) = [1, x^w]  (Sec. 3.2). */
static elem e_vertex(int sr, int nv, double w, double beta) {
    return nv ? e_weight(sr, w, beta) : e_one(sr);
}

static void put_result(int sr, elem e, double* size, uint64_t* limbs, double* zval, double* logz) {
    if (size) *size = (double)e.n;
    if (limbs) memcpy(limbs, e.c.w, sizeof e.c.w);
    if (sr == SR_PARTITION) {
        if (zval) *zval = (double)e.n;
        if (logz) *logz = (double)logl(e.n);
    }
}

/* ================================================================ O1 ===== */
/*
 * Brute force, straight from the definitions: every subset S of V (bit v of
 * the mask = n_v) is independent iff no edge has both ends in S.
 * Conditioning (fixed vertices of the Sec. 5 network object): only subsets
 * with (S & fix_mask) == fix_val are counted.
 *
 * Outputs (NULL to skip): maximum weight, number of subsets reaching it,
 * total number of independent sets, per-cardinality histogram (the
 * independence polynomial coefficients c_k, Sec. 6.2), Z(beta) for each beta
 * (Kahan-compensated long double sums), and up to sets_cap of the maximum
 * independent sets as bit masks.
 */
int orc_brute_force(int nv, int ne, const int32_t* edges, const double* w, int nbeta,
                    const double* betas, double* max_size, uint64_t* count_at_max,
                    uint64_t* total, uint64_t* size_hist, double* z, double* logz,
                    int sets_cap, uint64_t* sets, int* n_sets, uint64_t fix_mask, uint64_t fix_val) {
    if (nv < 0 || nv > 30 || ne < 0) return ORC_EINVAL;
    uint64_t* nbr = calloc((size_t)(nv > 0 ? nv : 1), sizeof(uint64_t));
    if (!nbr) return ORC_ENOMEM;
    for (int e = 0; e < ne; e++) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= nv || v >= nv || u == v) {
            free(nbr);
            return ORC_EINVAL;
        }
        nbr[u] |= 1ull << v;
        nbr[v] |= 1ull << u;
    }
    long double best = -INFINITY;
    uint64_t nbest = 0, ntot = 0;
    long double zs[64], zc[64];
    if (nbeta > 64) {
        free(nbr);
        return ORC_EINVAL;
    }
    for (int b = 0; b < nbeta; b++) zs[b] = zc[b] = 0.0L;
    if (size_hist)
        for (int k = 0; k <= nv; k++) size_hist[k] = 0;
    int nfound = 0;
    uint64_t nsub = 1ull << nv;
    for (uint64_t S = 0; S < nsub; S++) {
        if ((S & fix_mask) != fix_val) continue;
        int ok = 1;
        for (int v = 0; v < nv && ok; v++)
            if (((S >> v) & 1) && (S & nbr[v])) ok = 0;
        if (!ok) continue;
        long double ws = 0.0L;
        int card = 0;
        for (int v = 0; v < nv; v++)
            if ((S >> v) & 1) {
                ws += w ? (long double)w[v] : 1.0L;
                card++;
            }
        ntot++;
        if (size_hist) size_hist[card]++;
        for (int b = 0; b < nbeta; b++) { /* Kahan summation of e^{beta w(S)} */
            long double term = expl((long double)betas[b] * ws) - zc[b];
            long double t = zs[b] + term;
            zc[b] = (t - zs[b]) - term;
            zs[b] = t;
        }
        if (ws > best) {
            best = ws;
            nbest = 0;
            nfound = 0;
        }
        if (ws == best) {
            nbest++;
            if (sets && nfound < sets_cap) sets[nfound++] = S;
        }
    }
    free(nbr);
    if (max_size) *max_size = (double)best;
    if (count_at_max) *count_at_max = nbest;
    if (total) *total = ntot;
    for (int b = 0; b < nbeta; b++) {
        if (z) z[b] = (double)zs[b];
        if (logz) logz[b] = (double)logl(zs[b]);
    }
    if (n_sets) *n_sets = nfound;
    return ORC_OK;
}

/* ================================================================ O2 ===== */
/*
 * Variable (bucket) elimination.  The network is the product of edge tensors
 * B(n_u, n_v) and vertex tensors W(n_v) summed over all n (Sec. 3.2).  Each
 * vertex is summed out in turn: multiply every factor that mentions it into
 * one table over the union of their scopes and add over the vertex's two
 * values.  The order is this file's own heuristic order on the
 * interaction graph (see elimination_order).  Nothing here depends on a
 * contraction tree.
 */

typedef struct {
    int nvars;
    int* vars; /* ascending vertex ids; bit t of an entry index is vars[t] */
    elem* tab; /* 2^nvars entries */
    int alive;
} factor;

static int contains(const int* a, int n, int x) {
    for (int i = 0; i < n; i++)
        if (a[i] == x) return 1;
    return 0;
}

/*
 * Elimination order: three plain heuristics on the interaction graph -- greedy
 * min-fill, greedy min-degree, and the natural vertex order -- and keep the one
 * whose largest eliminated neighbourhood (the induced width) is smallest.  Ties
 * inside a heuristic go to the lower vertex id.  The order changes only the
 * cost of the elimination, never its result.
 */
static int order_by(int nv, int ne, const int32_t* edges, int mode, int* order, int* width) {
    unsigned char* adj = calloc((size_t)nv * (size_t)nv + 1, 1);
    unsigned char* gone = calloc((size_t)nv + 1, 1);
    int* nb = malloc(sizeof(int) * (size_t)(nv + 1));
    if (!adj || !gone || !nb) {
        free(adj);
        free(gone);
        free(nb);
        return ORC_ENOMEM;
    }
    for (int e = 0; e < ne; e++) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        adj[(size_t)u * nv + v] = adj[(size_t)v * nv + u] = 1;
    }
    int maxdeg = 0;
    for (int step = 0; step < nv; step++) {
        int bestv = -1;
        long bestfill = 0, bestdeg = 0;
        for (int v = 0; v < nv; v++) {
            if (gone[v]) continue;
            if (mode == 2) { /* natural order */
                bestv = v;
                break;
            }
            int d = 0;
            for (int u = 0; u < nv; u++)
                if (!gone[u] && adj[(size_t)v * nv + u]) nb[d++] = u;
            long fill = 0;
            for (int a = 0; a < d; a++)
                for (int b = a + 1; b < d; b++)
                    if (!adj[(size_t)nb[a] * nv + nb[b]]) fill++;
            long k1 = mode == 0 ? fill : d, k2 = mode == 0 ? d : fill;
            if (bestv < 0 || k1 < bestfill || (k1 == bestfill && k2 < bestdeg)) {
                bestv = v;
                bestfill = k1;
                bestdeg = k2;
            }
        }
        int d = 0;
        for (int u = 0; u < nv; u++)
            if (!gone[u] && adj[(size_t)bestv * nv + u]) nb[d++] = u;
        for (int a = 0; a < d; a++)
            for (int b = a + 1; b < d; b++)
                adj[(size_t)nb[a] * nv + nb[b]] = adj[(size_t)nb[b] * nv + nb[a]] = 1;
        if (d > maxdeg) maxdeg = d;
        gone[bestv] = 1;
        order[step] = bestv;
    }
    free(nb);
    free(adj);
    free(gone);
    *width = maxdeg;
    return ORC_OK;
}

static int elimination_order(int nv, int ne, const int32_t* edges, int* order, int* width) {
    int* cand = malloc(sizeof(int) * (size_t)(nv + 1));
    if (!cand) return ORC_ENOMEM;
    int best = -1;
    for (int mode = 0; mode < 3; mode++) {
        int wdt = 0;
        if (order_by(nv, ne, edges, mode, cand, &wdt) != ORC_OK) {
            free(cand);
            return ORC_ENOMEM;
        }
        if (best < 0 || wdt < best) {
            best = wdt;
            memcpy(order, cand, sizeof(int) * (size_t)nv);
        }
    }
    free(cand);
    *width = best;
    return ORC_OK;
}

/* positions of factor f's variables inside a larger scope */
static void positions(const factor* f, const int* scope, int nscope, int* pos) {
    for (int t = 0; t < f->nvars; t++)
        for (int s = 0; s < nscope; s++)
            if (scope[s] == f->vars[t]) pos[t] = s;
}

/* entry of a factor at an assignment of the larger scope (bit s = scope[s]) */
static size_t project(const factor* f, const int* pos, uint64_t assign) {
    size_t idx = 0;
    for (int t = 0; t < f->nvars; t++) idx |= (size_t)((assign >> pos[t]) & 1) << t;
    return idx;
}

/* g = sum over the eliminated vertex (at bit vpos of the bucket scope) of the
 * product of the bucket's factors */
static inline __attribute__((always_inline)) void sum_out(int sr, factor* fs, const int* bucket, int nb,
                                                          const int* pos, int nv, int vpos, factor* g,
                                                          size_t nout) {
    for (size_t y = 0; y < nout; y++) {
        /* insert v's value at bit position vpos of the full scope */
        uint64_t lo = y & (((uint64_t)1 << vpos) - 1), hi = (y >> vpos) << (vpos + 1);
        elem acc = e_zero(sr);
        for (int xv = 0; xv < 2; xv++) {
            uint64_t x = hi | ((uint64_t)xv << vpos) | lo;
            elem prod = e_one(sr);
            for (int b = 0; b < nb; b++) {
                factor* f = &fs[bucket[b]];
                prod = e_mul(sr, prod, f->tab[project(f, pos + (size_t)b * (size_t)(nv + 1), x)]);
            }
            acc = e_add(sr, acc, prod);
        }
        g->tab[y] = acc;
    }
}

static int cmp_int(const void* a, const void* b) {
    int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

/*
 * O2 entry point.  Returns the root element of the whole network in algebra
 * sr (beta used by SR_PARTITION only).  max_width bounds the largest
 * intermediate scope (the table has 2^(width+1) entries while being built).
 */
static int eliminate_impl(int nv, int ne, const int32_t* edges, const double* w, const double* J,
                          const double* hf, int model, int sr, double beta, int max_width, double* size,
                          uint64_t* limbs, double* zval, double* logz, int* width_out) {
    if (nv < 0 || ne < 0 || sr < 0 || sr > 3) return ORC_EINVAL;
    for (int e = 0; e < ne; e++) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= nv || v >= nv || u == v) return ORC_EINVAL;
    }
    g_overflow = 0;
    int nf = ne + nv;
    factor* fs = calloc((size_t)(nf + nv + 1), sizeof(factor));
    int* order = malloc(sizeof(int) * (size_t)(nv + 1));
    if (!fs || !order) {
        free(fs);
        free(order);
        return ORC_ENOMEM;
    }
    int width = 0;
    if (nv > 0 && elimination_order(nv, ne, edges, order, &width) != ORC_OK) {
        free(fs);
        free(order);
        return ORC_ENOMEM;
    }
    if (width_out) *width_out = width;
    if (width > max_width) {
        free(fs);
        free(order);
        return ORC_ETOOBIG;
    }
    int nfac = 0;
    for (int e = 0; e < ne; e++) { /* edge tensors */
        factor* f = &fs[nfac++];
        int u = edges[2 * e], v = edges[2 * e + 1];
        f->nvars = 2;
        f->vars = malloc(2 * sizeof(int));
        f->vars[0] = u < v ? u : v;
        f->vars[1] = u < v ? v : u;
        f->tab = malloc(4 * sizeof(elem));
        for (int a = 0; a < 4; a++) {
            if (model == 0) {
                f->tab[a] = e_edge(sr, a & 1, (a >> 1) & 1);
            } else { /* spin glass: x^(-J s_u s_v), s = 2n - 1 */
                int su = 2 * (a & 1) - 1, sv = 2 * ((a >> 1) & 1) - 1;
                f->tab[a] = e_weight(sr, -(J ? J[e] : 1.0) * su * sv, beta);
            }
        }
        f->alive = 1;
    }
    for (int v = 0; v < nv; v++) { /* vertex tensors */
        factor* f = &fs[nfac++];
        f->nvars = 1;
        f->vars = malloc(sizeof(int));
        f->vars[0] = v;
        f->tab = malloc(2 * sizeof(elem));
        for (int a = 0; a < 2; a++) /* spin glass: x^(-h s_v) */
            f->tab[a] = model == 0 ? e_vertex(sr, a, w ? w[v] : 1.0, beta)
                                   : e_weight(sr, -(hf ? hf[v] : 0.0) * (2 * a - 1), beta);
        f->alive = 1;
    }
    int status = ORC_OK;
    int* scope = malloc(sizeof(int) * (size_t)(nv + 1));
    int* bucket = malloc(sizeof(int) * (size_t)(nfac + nv + 1));
    int* pos = malloc(sizeof(int) * (size_t)(nfac + nv + 1) * (size_t)(nv + 1));
    for (int step = 0; step < nv && status == ORC_OK; step++) {
        int v = order[step];
        int nb = 0, ns = 0;
        for (int i = 0; i < nfac; i++) {
            if (!fs[i].alive || !contains(fs[i].vars, fs[i].nvars, v)) continue;
            bucket[nb++] = i;
            for (int t = 0; t < fs[i].nvars; t++)
                if (!contains(scope, ns, fs[i].vars[t])) scope[ns++] = fs[i].vars[t];
        }
        qsort(scope, (size_t)ns, sizeof(int), cmp_int);
        int vpos = 0;
        while (scope[vpos] != v) vpos++;
        factor* g = &fs[nfac];
        g->nvars = ns - 1;
        g->vars = malloc(sizeof(int) * (size_t)(ns > 1 ? ns - 1 : 1));
        for (int s = 0, t = 0; s < ns; s++)
            if (s != vpos) g->vars[t++] = scope[s];
        size_t nout = (size_t)1 << g->nvars;
        g->tab = malloc(sizeof(elem) * nout);
        if (!g->tab) {
            status = ORC_ENOMEM;
            break;
        }
        for (int b = 0; b < nb; b++) positions(&fs[bucket[b]], scope, ns, pos + (size_t)b * (size_t)(nv + 1));
        switch (sr) { /* one specialised copy of the loop per algebra */
        case SR_TROPICAL: sum_out(SR_TROPICAL, fs, bucket, nb, pos, nv, vpos, g, nout); break;
        case SR_COUNTING_TROPICAL: sum_out(SR_COUNTING_TROPICAL, fs, bucket, nb, pos, nv, vpos, g, nout); break;
        case SR_COUNT: sum_out(SR_COUNT, fs, bucket, nb, pos, nv, vpos, g, nout); break;
        default: sum_out(SR_PARTITION, fs, bucket, nb, pos, nv, vpos, g, nout); break;
        }
        for (int b = 0; b < nb; b++) {
            factor* f = &fs[bucket[b]];
            f->alive = 0;
            free(f->tab);
            free(f->vars);
            f->tab = NULL;
            f->vars = NULL;
        }
        g->alive = 1;
        nfac++;
    }
    elem root = e_one(sr);
    for (int i = 0; i < nfac; i++) {
        if (!fs[i].alive) continue;
        if (status == ORC_OK) root = e_mul(sr, root, fs[i].tab[0]); /* all scopes empty now */
        free(fs[i].tab);
        free(fs[i].vars);
    }
    free(scope);
    free(bucket);
    free(pos);
    free(fs);
    free(order);
    if (status != ORC_OK) return status;
    put_result(sr, root, size, limbs, zval, logz);
    return g_overflow ? ORC_EOVERFLOW : ORC_OK;
}

int orc_eliminate(int nv, int ne, const int32_t* edges, const double* w, int sr, double beta,
                  int max_width, double* size, uint64_t* limbs, double* zval, double* logz,
                  int* width_out) {
    return eliminate_impl(nv, ne, edges, w, NULL, NULL, 0, sr, beta, max_width, size, limbs, zval, logz,
                          width_out);
}

/*
 * O2 for the spin glass of Sec. 2 (H(sigma) = sum_(i,j) J_ij s_i s_j +
 * sum_i h_i s_i, s in {-1, 1}; index value n = (s + 1) / 2): edge tensors
 * x^(-J s_u s_v), vertex tensors x^(-h s).  The tropical algebras maximise
 * -H (size = -min H, count = number of ground states); the real algebra gives
 * Z(beta) = sum_sigma e^(-beta H).  J, h may be NULL (all 1 / all 0).
 */
int orc_eliminate_sg(int nv, int ne, const int32_t* edges, const double* J, const double* h, int sr,
                     double beta, int max_width, double* size, uint64_t* limbs, double* zval, double* logz,
                     int* width_out) {
    return eliminate_impl(nv, ne, edges, NULL, J, h, 1, sr, beta, max_width, size, limbs, zval, logz,
                          width_out);
}

/* O1 for the spin glass: every configuration s in {-1,1}^n (bit v of the mask
 * is n_v, s_v = 2 n_v - 1); the minimum energy, its multiplicity and
 * Z(beta) = sum e^(-beta H) for each beta (Kahan sums); with fixed spins,
 * only configurations with (m & fix_mask) == fix_val. */
int orc_brute_force_sg(int nv, int ne, const int32_t* edges, const double* J, const double* h, int nbeta,
                       const double* betas, double* emin, uint64_t* count_min, double* z, double* logz,
                       uint64_t fix_mask, uint64_t fix_val) {
    if (nv < 0 || nv > 30 || ne < 0 || nbeta < 0 || nbeta > 64) return ORC_EINVAL;
    for (int e = 0; e < ne; e++) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= nv || v >= nv || u == v) return ORC_EINVAL;
    }
    long double best = INFINITY, zs[64], zc[64];
    uint64_t nbest = 0;
    for (int b = 0; b < nbeta; b++) zs[b] = zc[b] = 0.0L;
    for (uint64_t m = 0; m < (1ull << nv); m++) {
        if ((m & fix_mask) != fix_val) continue;
        long double H = 0.0L;
        for (int e = 0; e < ne; e++) {
            int su = (int)((m >> edges[2 * e]) & 1) * 2 - 1, sv = (int)((m >> edges[2 * e + 1]) & 1) * 2 - 1;
            H += (long double)(J ? J[e] : 1.0) * su * sv;
        }
        for (int v = 0; v < nv; v++) H += (long double)(h ? h[v] : 0.0) * (int)(((m >> v) & 1) * 2 - 1);
        if (H < best) {
            best = H;
            nbest = 0;
        }
        if (H == best) nbest++;
        for (int b = 0; b < nbeta; b++) {
            long double term = expl(-(long double)betas[b] * H) - zc[b];
            long double t = zs[b] + term;
            zc[b] = (t - zs[b]) - term;
            zs[b] = t;
        }
    }
    if (emin) *emin = (double)best;
    if (count_min) *count_min = nbest;
    for (int b = 0; b < nbeta; b++) {
        if (z) z[b] = (double)zs[b];
        if (logz) logz[b] = (double)logl(zs[b]);
    }
    return ORC_OK;
}

/* The k largest values over all configurations, with multiplicity (SizeMax(k)
 * of the Sec. 5 table), by enumeration: independent sets and their total
 * weight, or spin configurations and -H.  Subsets that disagree with the
 * fixings are skipped.  out: k values, largest first, -INFINITY where fewer
 * than k configurations exist. */
static void topk_insert(double* top, int k, double v) {
    if (v <= top[k - 1]) return;
    int i = k - 1;
    while (i > 0 && top[i - 1] < v) {
        top[i] = top[i - 1];
        i--;
    }
    top[i] = v;
}

int orc_brute_force_topk(int nv, int ne, const int32_t* edges, const double* w, int k, double* out,
                         uint64_t fix_mask, uint64_t fix_val) {
    if (nv < 0 || nv > 30 || ne < 0 || k < 1 || k > 64) return ORC_EINVAL;
    uint64_t nbr[64] = {0};
    for (int e = 0; e < ne; e++) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= nv || v >= nv || u == v) return ORC_EINVAL;
        nbr[u] |= 1ull << v;
        nbr[v] |= 1ull << u;
    }
    for (int i = 0; i < k; i++) out[i] = -INFINITY;
    for (uint64_t S = 0; S < (1ull << nv); S++) {
        if ((S & fix_mask) != fix_val) continue;
        int ok = 1;
        for (int v = 0; v < nv && ok; v++)
            if (((S >> v) & 1) && (S & nbr[v])) ok = 0;
        if (!ok) continue;
        long double ws = 0.0L;
        for (int v = 0; v < nv; v++)
            if ((S >> v) & 1) ws += w ? (long double)w[v] : 1.0L;
        topk_insert(out, k, (double)ws);
    }
    return ORC_OK;
}

int orc_brute_force_sg_topk(int nv, int ne, const int32_t* edges, const double* J, const double* h, int k,
                            double* out, uint64_t fix_mask, uint64_t fix_val) {
    if (nv < 0 || nv > 30 || ne < 0 || k < 1 || k > 64) return ORC_EINVAL;
    for (int e = 0; e < ne; e++) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= nv || v >= nv || u == v) return ORC_EINVAL;
    }
    for (int i = 0; i < k; i++) out[i] = -INFINITY;
    for (uint64_t m = 0; m < (1ull << nv); m++) {
        if ((m & fix_mask) != fix_val) continue;
        long double H = 0.0L;
        for (int e = 0; e < ne; e++) {
            int su = (int)((m >> edges[2 * e]) & 1) * 2 - 1, sv = (int)((m >> edges[2 * e + 1]) & 1) * 2 - 1;
            H += (long double)(J ? J[e] : 1.0) * su * sv;
        }
        for (int v = 0; v < nv; v++) H += (long double)(h ? h[v] : 0.0) * (int)(((m >> v) & 1) * 2 - 1);
        topk_insert(out, k, (double)-H);
    }
    return ORC_OK;
}

/* --------------------------------------------------- O2 over polynomials --- */
/*
 * The independence polynomial I(G, x) = sum_k c_k x^k, c_k = #{S independent :
 * |S| = k} (Sec. 5.3, GraphPolynomial; Sec. 6.2).  Same elimination as above,
 * but every table entry is a polynomial in x with exact 256-bit coefficients:
 * the vertex tensor is [1, x], the edge tensor [[1,1],[1,0]], "+" adds
 * polynomials and "*" multiplies them.  Unit weights only.  Each factor keeps
 * the largest degree any of its entries can have (the number of vertex
 * tensors absorbed into it, at most nv).
 */
typedef struct {
    int nvars;
    int* vars;
    int deg;   /* entries are polynomials of degree <= deg */
    u256* tab; /* 2^nvars entries of deg+1 coefficients each */
    int alive;
} pfactor;

static void poly_mul_into(const u256* a, int da, const u256* b, int db, u256* out, int dout) {
    for (int k = 0; k <= dout; k++) out[k] = u256_from(0);
    for (int i = 0; i <= da; i++) {
        if (!(a[i].w[0] | a[i].w[1] | a[i].w[2] | a[i].w[3])) continue;
        for (int j = 0; j <= db && i + j <= dout; j++) out[i + j] = u256_add(out[i + j], u256_mul(a[i], b[j]));
    }
}

int orc_eliminate_poly(int nv, int ne, const int32_t* edges, int max_width, uint64_t* coeffs, int* degree,
                       int* width_out) {
    if (nv < 0 || ne < 0) return ORC_EINVAL;
    for (int e = 0; e < ne; e++) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= nv || v >= nv || u == v) return ORC_EINVAL;
    }
    g_overflow = 0;
    int* order = malloc(sizeof(int) * (size_t)(nv + 1));
    pfactor* fs = calloc((size_t)(ne + 2 * nv + 1), sizeof(pfactor));
    if (!order || !fs) {
        free(order);
        free(fs);
        return ORC_ENOMEM;
    }
    int width = 0;
    if (nv > 0 && elimination_order(nv, ne, edges, order, &width) != ORC_OK) {
        free(order);
        free(fs);
        return ORC_ENOMEM;
    }
    if (width_out) *width_out = width;
    if (width > max_width) {
        free(order);
        free(fs);
        return ORC_ETOOBIG;
    }
    int nfac = 0;
    for (int e = 0; e < ne; e++) { /* [[1,1],[1,0]] */
        pfactor* f = &fs[nfac++];
        int u = edges[2 * e], v = edges[2 * e + 1];
        f->nvars = 2;
        f->vars = malloc(2 * sizeof(int));
        f->vars[0] = u < v ? u : v;
        f->vars[1] = u < v ? v : u;
        f->deg = 0;
        f->tab = malloc(4 * sizeof(u256));
        for (int a = 0; a < 4; a++) f->tab[a] = u256_from(a == 3 ? 0 : 1);
        f->alive = 1;
    }
    for (int v = 0; v < nv; v++) { /* [1, x] */
        pfactor* f = &fs[nfac++];
        f->nvars = 1;
        f->vars = malloc(sizeof(int));
        f->vars[0] = v;
        f->deg = 1;
        f->tab = malloc(4 * sizeof(u256)); /* entry 0: 1 + 0x, entry 1: 0 + 1x */
        f->tab[0] = u256_from(1);
        f->tab[1] = u256_from(0);
        f->tab[2] = u256_from(0);
        f->tab[3] = u256_from(1);
        f->alive = 1;
    }
    int status = ORC_OK;
    int* scope = malloc(sizeof(int) * (size_t)(nv + 1));
    int* bucket = malloc(sizeof(int) * (size_t)(nfac + nv + 1));
    int* pos = malloc(sizeof(int) * (size_t)(nfac + nv + 1) * (size_t)(nv + 1));
    u256* prod = malloc(sizeof(u256) * (size_t)(nv + 1));
    u256* tmp = malloc(sizeof(u256) * (size_t)(nv + 1));
    for (int step = 0; step < nv && status == ORC_OK; step++) {
        int v = order[step];
        int nb = 0, ns = 0, dg = 0;
        for (int i = 0; i < nfac; i++) {
            if (!fs[i].alive || !contains(fs[i].vars, fs[i].nvars, v)) continue;
            bucket[nb++] = i;
            dg += fs[i].deg;
            for (int t = 0; t < fs[i].nvars; t++)
                if (!contains(scope, ns, fs[i].vars[t])) scope[ns++] = fs[i].vars[t];
        }
        if (dg > nv) dg = nv;
        qsort(scope, (size_t)ns, sizeof(int), cmp_int);
        int vpos = 0;
        while (scope[vpos] != v) vpos++;
        pfactor* g = &fs[nfac];
        g->nvars = ns - 1;
        g->deg = dg;
        g->vars = malloc(sizeof(int) * (size_t)(ns > 1 ? ns - 1 : 1));
        for (int s = 0, t = 0; s < ns; s++)
            if (s != vpos) g->vars[t++] = scope[s];
        size_t nout = (size_t)1 << g->nvars;
        g->tab = calloc(nout * (size_t)(dg + 1), sizeof(u256));
        if (!g->tab) {
            status = ORC_ENOMEM;
            break;
        }
        for (int b = 0; b < nb; b++) { /* positions of each bucket factor's variables in the scope */
            pfactor* f = &fs[bucket[b]];
            for (int t = 0; t < f->nvars; t++)
                for (int s2 = 0; s2 < ns; s2++)
                    if (scope[s2] == f->vars[t]) pos[(size_t)b * (size_t)(nv + 1) + t] = s2;
        }
        for (size_t y = 0; y < nout; y++) {
            uint64_t lo = y & (((uint64_t)1 << vpos) - 1), hi = (y >> vpos) << (vpos + 1);
            u256* acc = g->tab + y * (size_t)(dg + 1);
            for (int xv = 0; xv < 2; xv++) {
                uint64_t x = hi | ((uint64_t)xv << vpos) | lo;
                int dp = 0;
                prod[0] = u256_from(1);
                for (int b = 0; b < nb; b++) {
                    pfactor* f = &fs[bucket[b]];
                    size_t idx = 0;
                    for (int t = 0; t < f->nvars; t++)
                        idx |= (size_t)((x >> pos[(size_t)b * (size_t)(nv + 1) + t]) & 1) << t;
                    int dn = dp + f->deg > dg ? dg : dp + f->deg;
                    poly_mul_into(prod, dp, f->tab + idx * (size_t)(f->deg + 1), f->deg, tmp, dn);
                    memcpy(prod, tmp, sizeof(u256) * (size_t)(dn + 1));
                    dp = dn;
                }
                for (int k = 0; k <= dp; k++) acc[k] = u256_add(acc[k], prod[k]);
            }
        }
        for (int b = 0; b < nb; b++) {
            pfactor* f = &fs[bucket[b]];
            f->alive = 0;
            free(f->tab);
            free(f->vars);
            f->tab = NULL;
            f->vars = NULL;
        }
        g->alive = 1;
        nfac++;
    }
    /* product of the remaining scalars (empty scopes) */
    int dr = 0;
    prod[0] = u256_from(1);
    for (int i = 0; i < nfac; i++) {
        if (!fs[i].alive) continue;
        if (status == ORC_OK) {
            int dn = dr + fs[i].deg > nv ? nv : dr + fs[i].deg;
            poly_mul_into(prod, dr, fs[i].tab, fs[i].deg, tmp, dn);
            memcpy(prod, tmp, sizeof(u256) * (size_t)(dn + 1));
            dr = dn;
        }
        free(fs[i].tab);
        free(fs[i].vars);
    }
    if (status == ORC_OK) {
        int d = dr;
        while (d > 0 && !(prod[d].w[0] | prod[d].w[1] | prod[d].w[2] | prod[d].w[3])) d--;
        for (int k = 0; k <= nv; k++)
            for (int l = 0; l < 4; l++) coeffs[4 * k + l] = k <= dr ? prod[k].w[l] : 0;
        if (degree) *degree = d;
    }
    free(prod);
    free(tmp);
    free(scope);
    free(bucket);
    free(pos);
    free(fs);
    free(order);
    if (status != ORC_OK) return status;
    return g_overflow ? ORC_EOVERFLOW : ORC_OK;
}

/* ================================================================ O3 ===== */
/*
 * Plan following.  A contraction tree (Sec. 4.1: leaves are the input tensors,
 * each inner node contracts two tensors into one) is given as data:
 *
 *   nodes 0 .. nleaf-1            leaves; leaf l holds the factors
 *                                 fac[fac_off[l] .. fac_off[l+1]) where a code
 *                                 c >= 0 is edge c and c < 0 is vertex -c-1
 *   nodes nleaf .. nleaf+ninner-1 inner nodes with children left[], right[]
 *                                 (ids smaller than the node's own id)
 *   idx[idx_off[x] .. idx_off[x+1])  the output indices of node x (vertex ids)
 *   sliced[0 .. nsliced)           indices fixed per slice (Sec. 4.2: slicing
 *                                 loops over a subset of indices and combines
 *                                 the slice results at the end); slice s sets
 *                                 sliced[k] to bit k of s.  A range
 *                                 [slice_begin, slice_end) sums those slices
 *                                 only (0, 0: all)
 *
 * The root (last node) must have no output indices.  Before evaluating, the
 * tree is checked against the einsum rule: an index stays open at a node iff
 * it also occurs outside that node's subtree; each factor occurs once.
 * Evaluation: every leaf is the product of its factors summed over its
 * indices that are not output; every inner node computes
 *     C[c] = (+)_{summed indices} A[a] (*) B[b]
 * by looping over every assignment of the node's index union.
 */

typedef struct {
    int n;
    int* v;
} iset;

static int iset_has(const iset* s, int x) { return contains(s->v, s->n, x); }

int orc_follow_plan(int nv, int ne, const int32_t* edges, const double* w, int sr, double beta,
                    int nleaf, int ninner, const int32_t* fac_off, const int32_t* fac,
                    const int32_t* left, const int32_t* right, const int32_t* idx_off,
                    const int32_t* idx, int nsliced, const int32_t* sliced, int64_t slice_begin,
                    int64_t slice_end, int max_rank, double* size, uint64_t* limbs, double* zval,
                    double* logz) {
    if (nv < 0 || ne < 0 || nleaf < 1 || ninner < 0 || sr < 0 || sr > 3) return ORC_EINVAL;
    int nn = nleaf + ninner;
    g_overflow = 0;
    /* --- every factor exactly once ---------------------------------------- */
    int* seen = calloc((size_t)(ne + nv + 1), sizeof(int));
    for (int l = 0; l < nleaf; l++)
        for (int q = fac_off[l]; q < fac_off[l + 1]; q++) {
            int c = fac[q];
            int slot = c >= 0 ? c : ne + (-c - 1);
            if ((c >= 0 && c >= ne) || (c < 0 && -c - 1 >= nv)) {
                free(seen);
                return ORC_EINVAL;
            }
            seen[slot]++;
        }
    for (int s = 0; s < ne + nv; s++)
        if (seen[s] != 1) {
            free(seen);
            return ORC_EINVAL;
        }
    /* --- leaf scopes, subtree membership and the open-index rule ---------- */
    /* occurrences of each vertex index over all leaves' factor scopes */
    int* occ_total = calloc((size_t)(nv + 1), sizeof(int));
    iset* lscope = calloc((size_t)nleaf, sizeof(iset));
    for (int l = 0; l < nleaf; l++) {
        lscope[l].v = malloc(sizeof(int) * (size_t)(2 * (fac_off[l + 1] - fac_off[l]) + 1));
        for (int q = fac_off[l]; q < fac_off[l + 1]; q++) {
            int c = fac[q];
            int us[2], nu = 0;
            if (c >= 0) {
                us[nu++] = edges[2 * c];
                us[nu++] = edges[2 * c + 1];
            } else
                us[nu++] = -c - 1;
            for (int a = 0; a < nu; a++)
                if (!iset_has(&lscope[l], us[a])) lscope[l].v[lscope[l].n++] = us[a];
        }
        for (int a = 0; a < lscope[l].n; a++) occ_total[lscope[l].v[a]]++;
    }
    int status = ORC_OK;
    int* parent = malloc(sizeof(int) * (size_t)nn);
    for (int x = 0; x < nn; x++) parent[x] = -1;
    for (int t = 0; t < ninner; t++) {
        int x = nleaf + t;
        if (left[t] < 0 || right[t] < 0 || left[t] >= x || right[t] >= x || left[t] == right[t] ||
            parent[left[t]] >= 0 || parent[right[t]] >= 0) {
            status = ORC_EINVAL;
            break;
        }
        parent[left[t]] = parent[right[t]] = x;
    }
    for (int x = 0; x < nn - 1 && status == ORC_OK; x++)
        if (parent[x] < 0) status = ORC_EINVAL; /* every node but the root is used */
    if (status == ORC_OK && idx_off[nn] - idx_off[nn - 1] != 0) status = ORC_EINVAL;
    /* leaf sets below each node */
    int* cnt = calloc((size_t)(nv + 1), sizeof(int));
    for (int x = 0; x < nn && status == ORC_OK; x++) {
        /* occurrences of each index inside x's subtree: walk leaves up */
        for (int u = 0; u < nv; u++) cnt[u] = 0;
        for (int l = 0; l < nleaf; l++) {
            int y = l;
            while (y >= 0 && y != x) y = parent[y];
            if (y != x) continue;
            for (int a = 0; a < lscope[l].n; a++) cnt[lscope[l].v[a]]++;
        }
        int nout = idx_off[x + 1] - idx_off[x];
        int expect = 0;
        for (int u = 0; u < nv; u++) {
            int open = cnt[u] > 0 && cnt[u] < occ_total[u];
            expect += open;
            int listed = contains(idx + idx_off[x], nout, u);
            if (open != listed) status = ORC_EINVAL;
        }
        if (expect != nout) status = ORC_EINVAL;
    }
    free(cnt);
    for (int s = 0; s < nsliced && status == ORC_OK; s++)
        if (sliced[s] < 0 || sliced[s] >= nv) status = ORC_EINVAL;
    for (int x = 0; x < nn && status == ORC_OK; x++) {
        int r = 0;
        for (int q = idx_off[x]; q < idx_off[x + 1]; q++)
            r += !contains(sliced, nsliced, idx[q]);
        if (r > max_rank) status = ORC_ETOOBIG;
    }
    if (status != ORC_OK) {
        for (int l = 0; l < nleaf; l++) free(lscope[l].v);
        free(lscope);
        free(occ_total);
        free(parent);
        free(seen);
        return status;
    }

    /* --- evaluate, slice by slice ------------------------------------------ */
    /* value[u] = the value of index u in the current assignment (-1 if free) */
    int* value = malloc(sizeof(int) * (size_t)(nv + 1));
    elem** tab = calloc((size_t)nn, sizeof(elem*));
    iset* kept = calloc((size_t)nn, sizeof(iset)); /* output indices minus sliced ones */
    for (int x = 0; x < nn; x++) {
        kept[x].v = malloc(sizeof(int) * (size_t)(idx_off[x + 1] - idx_off[x] + 1));
        for (int q = idx_off[x]; q < idx_off[x + 1]; q++)
            if (!contains(sliced, nsliced, idx[q])) kept[x].v[kept[x].n++] = idx[q];
    }
    int* free_idx = malloc(sizeof(int) * (size_t)(nv + 1));
    elem total = e_zero(sr);
    uint64_t nslices = (uint64_t)1 << nsliced;
    /* slices [slice_begin, slice_end) only; 0, 0 means all of them */
    uint64_t sl_lo = 0, sl_hi = nslices;
    if (slice_begin != 0 || slice_end != 0) {
        if (slice_begin < 0 || slice_end <= slice_begin || (uint64_t)slice_end > nslices) status = ORC_EINVAL;
        sl_lo = (uint64_t)slice_begin;
        sl_hi = (uint64_t)slice_end;
    }
    for (uint64_t sl = sl_lo; sl < sl_hi && status == ORC_OK; sl++) {
        for (int u = 0; u < nv; u++) value[u] = -1;
        for (int s = 0; s < nsliced; s++) value[sliced[s]] = (int)((sl >> s) & 1);
        for (int x = 0; x < nn && status == ORC_OK; x++) {
            size_t nout = (size_t)1 << kept[x].n;
            tab[x] = malloc(sizeof(elem) * nout);
            if (!tab[x]) {
                status = ORC_ENOMEM;
                break;
            }
            /* summed indices at this node: the node's index union, minus the
             * output indices, minus the sliced indices */
            int nfree = 0;
            if (x < nleaf) {
                for (int a = 0; a < lscope[x].n; a++) {
                    int u = lscope[x].v[a];
                    if (!iset_has(&kept[x], u) && value[u] < 0) free_idx[nfree++] = u;
                }
            } else {
                int L = left[x - nleaf], R = right[x - nleaf];
                for (int a = 0; a < kept[L].n; a++)
                    if (!iset_has(&kept[x], kept[L].v[a]) && !contains(free_idx, nfree, kept[L].v[a]))
                        free_idx[nfree++] = kept[L].v[a];
                for (int a = 0; a < kept[R].n; a++)
                    if (!iset_has(&kept[x], kept[R].v[a]) && !contains(free_idx, nfree, kept[R].v[a]))
                        free_idx[nfree++] = kept[R].v[a];
            }
            for (size_t c = 0; c < nout; c++) {
                for (int a = 0; a < kept[x].n; a++) value[kept[x].v[a]] = (int)((c >> a) & 1);
                elem acc = e_zero(sr);
                for (uint64_t s = 0; s < ((uint64_t)1 << nfree); s++) {
                    for (int a = 0; a < nfree; a++) value[free_idx[a]] = (int)((s >> a) & 1);
                    elem prod = e_one(sr);
                    if (x < nleaf) {
                        for (int q = fac_off[x]; q < fac_off[x + 1]; q++) {
                            int f = fac[q];
                            if (f >= 0)
                                prod = e_mul(sr, prod,
                                             e_edge(sr, value[edges[2 * f]], value[edges[2 * f + 1]]));
                            else
                                prod = e_mul(sr, prod,
                                             e_vertex(sr, value[-f - 1], w ? w[-f - 1] : 1.0, beta));
                        }
                    } else {
                        int ch[2] = {left[x - nleaf], right[x - nleaf]};
                        for (int k = 0; k < 2; k++) {
                            size_t off = 0;
                            for (int a = 0; a < kept[ch[k]].n; a++)
                                off |= (size_t)value[kept[ch[k]].v[a]] << a;
                            prod = e_mul(sr, prod, tab[ch[k]][off]);
                        }
                    }
                    acc = e_add(sr, acc, prod);
                }
                tab[x][c] = acc;
            }
            for (int a = 0; a < nfree; a++) value[free_idx[a]] = -1;
            for (int a = 0; a < kept[x].n; a++) value[kept[x].v[a]] = -1;
            if (x >= nleaf) {
                free(tab[left[x - nleaf]]);
                free(tab[right[x - nleaf]]);
                tab[left[x - nleaf]] = tab[right[x - nleaf]] = NULL;
            }
        }
        if (status == ORC_OK) total = e_add(sr, total, tab[nn - 1][0]);
        for (int x = 0; x < nn; x++) {
            free(tab[x]);
            tab[x] = NULL;
        }
    }
    for (int x = 0; x < nn; x++) free(kept[x].v);
    for (int l = 0; l < nleaf; l++) free(lscope[l].v);
    free(kept);
    free(tab);
    free(value);
    free(free_idx);
    free(lscope);
    free(occ_total);
    free(parent);
    free(seen);
    if (status != ORC_OK) return status;
    put_result(sr, total, size, limbs, zval, logz);
    return g_overflow ? ORC_EOVERFLOW : ORC_OK;
}

/* CountingMax(k) of the Sec. 5 table by enumeration: the largest value over
 * all configurations (independent sets: total weight; spin glass: -H) and the
 * number of configurations at each value top - d, d < k.  Integer weights
 * only (the values are then integers); counts are exact (n <= 30). */
static int count_top_values(const long long* vals, const unsigned char* ok, uint64_t nconf, int k, long long* top,
                            uint64_t* counts) {
    int any = 0;
    long long best = 0;
    for (uint64_t m = 0; m < nconf; m++)
        if (ok[m] && (!any || vals[m] > best)) {
            best = vals[m];
            any = 1;
        }
    for (int d = 0; d < k; d++) counts[d] = 0;
    if (!any) return 0;
    for (uint64_t m = 0; m < nconf; m++)
        if (ok[m] && best - vals[m] < k) counts[best - vals[m]]++;
    *top = best;
    return 1;
}

static int is_integral(const double* x, int n) {
    for (int i = 0; x && i < n; i++)
        if (x[i] != floor(x[i]) || fabs(x[i]) > 65536.0) return 0;
    return 1;
}

int orc_brute_force_count_top(int nv, int ne, const int32_t* edges, const double* w, int k, int64_t* top,
                              uint64_t* counts, int* found, uint64_t fix_mask, uint64_t fix_val) {
    if (nv < 0 || nv > 24 || ne < 0 || k < 1 || k > 64 || !is_integral(w, nv)) return ORC_EINVAL;
    uint64_t nbr[64] = {0};
    for (int e = 0; e < ne; e++) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= nv || v >= nv || u == v) return ORC_EINVAL;
        nbr[u] |= 1ull << v;
        nbr[v] |= 1ull << u;
    }
    const uint64_t nconf = 1ull << nv;
    long long* vals = (long long*)malloc(sizeof(long long) * nconf);
    unsigned char* ok = (unsigned char*)malloc(nconf);
    if (!vals || !ok) {
        free(vals);
        free(ok);
        return ORC_EINVAL;
    }
    for (uint64_t S = 0; S < nconf; S++) {
        int good = (S & fix_mask) == fix_val;
        for (int v = 0; v < nv && good; v++)
            if (((S >> v) & 1) && (S & nbr[v])) good = 0;
        long long ws = 0;
        for (int v = 0; v < nv; v++)
            if ((S >> v) & 1) ws += w ? (long long)w[v] : 1;
        ok[S] = (unsigned char)good;
        vals[S] = ws;
    }
    long long t = 0;
    *found = count_top_values(vals, ok, nconf, k, &t, counts);
    *top = t;
    free(vals);
    free(ok);
    return ORC_OK;
}

int orc_brute_force_sg_count_top(int nv, int ne, const int32_t* edges, const double* J, const double* h, int k,
                                 int64_t* top, uint64_t* counts, int* found, uint64_t fix_mask, uint64_t fix_val) {
    if (nv < 0 || nv > 24 || ne < 0 || k < 1 || k > 64 || !is_integral(J, ne) || !is_integral(h, nv))
        return ORC_EINVAL;
    for (int e = 0; e < ne; e++) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= nv || v >= nv || u == v) return ORC_EINVAL;
    }
    const uint64_t nconf = 1ull << nv;
    long long* vals = (long long*)malloc(sizeof(long long) * nconf);
    unsigned char* ok = (unsigned char*)malloc(nconf);
    if (!vals || !ok) {
        free(vals);
        free(ok);
        return ORC_EINVAL;
    }
    for (uint64_t m = 0; m < nconf; m++) {
        long long H = 0;
        for (int e = 0; e < ne; e++) {
            int su = (int)((m >> edges[2 * e]) & 1) * 2 - 1, sv = (int)((m >> edges[2 * e + 1]) & 1) * 2 - 1;
            H += (long long)(J ? J[e] : 1.0) * su * sv;
        }
        for (int v = 0; v < nv; v++) H += (long long)(h ? h[v] : 0.0) * (int)(((m >> v) & 1) * 2 - 1);
        ok[m] = (unsigned char)((m & fix_mask) == fix_val);
        vals[m] = -H;
    }
    long long t = 0;
    *found = count_top_values(vals, ok, nconf, k, &t, counts);
    *top = t;
    free(vals);
    free(ok);
    return ORC_OK;
}
