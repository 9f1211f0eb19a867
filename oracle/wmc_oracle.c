/*
 * CPU oracle for literal-weighted model counting.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library may include, link or
 * call this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or helper with the
 * GPU path.
 *
 * What it computes (Definition 1, literal-weighted model count):
 *     W(phi) = sum over tau in {0,1}^X of phi(tau) * prod_x W(x, tau(x)).
 *
 * Two exact reorganisations of that sum are implemented here:
 *
 *   O1  oracle_brute   - the definition written out: enumerate every
 *                        assignment, test every clause, multiply the n
 *                        literal weights, add with Neumaier compensation.
 *   O2  oracle_bucket  - variable (bucket) elimination in FP64: for each
 *                        variable x in an elimination order, multiply every
 *                        factor that mentions x (clause indicator tables and
 *                        the weight vector [W(x,0), W(x,1)]) over the union
 *                        of their scopes, sum x out, and keep the message.
 *                        Each message is renormalised by a power of two taken
 *                        from its largest magnitude and carries an int64
 *                        exponent, so values far below the double range
 *                        (lattices reach ~1e-280 and below) stay exact up to
 *                        ordinary rounding.
 *
 * Readings (the paper is silent on these; see the design notes):
 *   - a variable in no clause contributes W(x,0)+W(x,1);
 *   - duplicate literals collapse; a clause holding x and not-x is always true;
 *   - the empty clause is always false, so W = 0;
 *   - duplicate clauses are kept (0/1 factors are idempotent).
 *
 * Parity is pinned in the test-suite against brute force, closed forms
 * (empty formula, single clause, the psi family, the Figure 1 formula),
 * exact integer counts and invariants, never against the GPU library.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_INVALID 1
#define OR_NOMEM 2
#define OR_TOO_BIG 3

/* ------------------------------------------------------------------ */
/* shared input checks (oracle-local)                                   */
/* ------------------------------------------------------------------ */
static int check_clauses(int32_t n, int64_t m, const int64_t *cptr, const int32_t *lits) {
    if (n < 0 || m < 0) return OR_INVALID;
    if (m > 0 && (!cptr || (cptr[m] > 0 && !lits))) return OR_INVALID;
    for (int64_t c = 0; c < m; ++c) {
        if (cptr[c + 1] < cptr[c]) return OR_INVALID;
        for (int64_t j = cptr[c]; j < cptr[c + 1]; ++j) {
            int32_t l = lits[j];
            if (l == 0 || l > n || l < -n) return OR_INVALID;
        }
    }
    return OR_OK;
}

static int check_input(int32_t n, int64_t m, const int64_t *cptr, const int32_t *lits,
                       const double *w) {
    if (n > 0 && !w) return OR_INVALID;
    return check_clauses(n, m, cptr, lits);
}

/* Neumaier-compensated running sum */
typedef struct { double s, c; } nsum;
static void nsum_add(nsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

/* ------------------------------------------------------------------ */
/* O1: brute force over all 2^n assignments (n <= 30)                   */
/* ------------------------------------------------------------------ */
int oracle_brute(int32_t n, int64_t m, const int64_t *cptr, const int32_t *lits,
                 const double *w, double *out) {
    int st = check_input(n, m, cptr, lits, w);
    if (st) return st;
    if (n > 30) return OR_TOO_BIG;
    uint32_t *pos = (uint32_t *)calloc((size_t)(m ? m : 1), sizeof(uint32_t));
    uint32_t *neg = (uint32_t *)calloc((size_t)(m ? m : 1), sizeof(uint32_t));
    if (!pos || !neg) { free(pos); free(neg); return OR_NOMEM; }
    for (int64_t c = 0; c < m; ++c)
        for (int64_t j = cptr[c]; j < cptr[c + 1]; ++j) {
            int32_t l = lits[j];
            if (l > 0) pos[c] |= 1u << (l - 1);
            else neg[c] |= 1u << (-l - 1);
        }
    /* fixed chunking so the rounding does not depend on the thread count */
    const int chunk_bits = n > 12 ? 12 : n;
    const int64_t n_chunks = (int64_t)1 << (n - chunk_bits);
    double *part = (double *)malloc(sizeof(double) * (size_t)n_chunks * 2);
    if (!part) { free(pos); free(neg); return OR_NOMEM; }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t ch = 0; ch < n_chunks; ++ch) {
        nsum acc = {0.0, 0.0};
        for (int64_t k = 0; k < ((int64_t)1 << chunk_bits); ++k) {
            uint32_t tau = (uint32_t)((ch << chunk_bits) | k);
            int sat = 1;
            for (int64_t c = 0; c < m; ++c) {
                if (((pos[c] & tau) | (neg[c] & ~tau)) == 0) { sat = 0; break; }
            }
            if (!sat) continue;
            double p = 1.0;
            for (int32_t x = 0; x < n; ++x) p *= w[2 * x + ((tau >> x) & 1u)];
            nsum_add(&acc, p);
        }
        part[2 * ch] = acc.s;
        part[2 * ch + 1] = acc.c;
    }
    nsum tot = {0.0, 0.0};
    for (int64_t ch = 0; ch < n_chunks; ++ch) {
        nsum_add(&tot, part[2 * ch]);
        nsum_add(&tot, part[2 * ch + 1]);
    }
    *out = tot.s + tot.c;
    free(part);
    free(pos);
    free(neg);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* O2: FP64 bucket elimination with power-of-two renormalisation        */
/* ------------------------------------------------------------------ */
typedef struct {
    int nv;          /* scope size */
    int32_t *vars;   /* ascending variable ids (1-based); bit i of an index <-> vars[i] */
    double *t;       /* 2^nv entries */
    int64_t e;       /* true value = t * 2^e */
    int alive;
} factor;

static void factor_free(factor *f) {
    free(f->vars);
    free(f->t);
    f->vars = NULL;
    f->t = NULL;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Renormalise a table so that its largest magnitude lies in [0.5, 1). */
static void renormalise(double *t, int64_t size, int64_t *e) {
    double mx = 0.0;
    for (int64_t i = 0; i < size; ++i) {
        double a = fabs(t[i]);
        if (a > mx) mx = a;
    }
    if (mx == 0.0 || !isfinite(mx)) return;
    int k;
    frexp(mx, &k);
    for (int64_t i = 0; i < size; ++i) t[i] = ldexp(t[i], -k);
    *e += k;
}

/* Min-fill elimination order on the primal graph; ties go to the lowest id. */
static int minfill_order(int32_t n, int64_t m, const int64_t *cptr, const int32_t *lits,
                         int32_t *order) {
    if (n == 0) return OR_OK;
    unsigned char *adj = (unsigned char *)calloc((size_t)n * (size_t)n, 1);
    unsigned char *done = (unsigned char *)calloc((size_t)n, 1);
    int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!adj || !done || !nb) { free(adj); free(done); free(nb); return OR_NOMEM; }
    for (int64_t c = 0; c < m; ++c)
        for (int64_t i = cptr[c]; i < cptr[c + 1]; ++i)
            for (int64_t j = cptr[c]; j < cptr[c + 1]; ++j) {
                int a = abs(lits[i]) - 1, b = abs(lits[j]) - 1;
                if (a != b) adj[(size_t)a * n + b] = 1;
            }
    for (int32_t step = 0; step < n; ++step) {
        int32_t best = -1;
        int64_t best_fill = -1;
        for (int32_t v = 0; v < n; ++v) {
            if (done[v]) continue;
            int k = 0;
            for (int32_t u = 0; u < n; ++u)
                if (!done[u] && adj[(size_t)v * n + u]) nb[k++] = u;
            int64_t fill = 0;
            for (int a = 0; a < k; ++a)
                for (int b = a + 1; b < k; ++b)
                    if (!adj[(size_t)nb[a] * n + nb[b]]) ++fill;
            if (best < 0 || fill < best_fill) { best = v; best_fill = fill; }
        }
        int k = 0;
        for (int32_t u = 0; u < n; ++u)
            if (!done[u] && adj[(size_t)best * n + u]) nb[k++] = u;
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
                if (a != b) adj[(size_t)nb[a] * n + nb[b]] = 1;
        done[best] = 1;
        order[step] = best + 1;
    }
    free(adj);
    free(done);
    free(nb);
    return OR_OK;
}

/*
 * order: NULL for the oracle's own min-fill order, else a permutation of 1..n.
 * max_log2: largest message scope allowed (returns OR_TOO_BIG beyond it).
 * Result: W = *out_mant * 2^(*out_exp), with |mant| in [0.5, 1) or exactly 0.
 * out_width (optional): largest message scope seen.
 */
int oracle_bucket(int32_t n, int64_t m, const int64_t *cptr, const int32_t *lits,
                  const double *w, const int32_t *order_in, int32_t max_log2,
                  double *out_mant, int64_t *out_exp, int32_t *out_width) {
    int st = check_input(n, m, cptr, lits, w);
    if (st) return st;
    if (max_log2 <= 0 || max_log2 > 34) max_log2 = 34;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    if (!order) return OR_NOMEM;
    if (order_in) {
        unsigned char *seen = (unsigned char *)calloc((size_t)(n ? n : 1), 1);
        if (!seen) { free(order); return OR_NOMEM; }
        for (int32_t i = 0; i < n; ++i) {
            int32_t v = order_in[i];
            if (v < 1 || v > n || seen[v - 1]) { free(seen); free(order); return OR_INVALID; }
            seen[v - 1] = 1;
            order[i] = v;
        }
        free(seen);
    } else {
        st = minfill_order(n, m, cptr, lits, order);
        if (st) { free(order); return st; }
    }

    /* factors: m clause indicators, then n weight vectors */
    int64_t cap = m + n + 1;
    factor *fs = (factor *)calloc((size_t)(cap + n + 1), sizeof(factor));
    if (!fs) { free(order); return OR_NOMEM; }
    int64_t nf = 0;
    int32_t width = 0;
    for (int64_t c = 0; c < m; ++c) {
        int64_t len = cptr[c + 1] - cptr[c];
        int32_t *vs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(len ? len : 1));
        if (!vs) { st = OR_NOMEM; goto fail; }
        int k = 0;
        for (int64_t j = cptr[c]; j < cptr[c + 1]; ++j) {
            int32_t v = abs(lits[j]);
            int dup = 0;
            for (int q = 0; q < k; ++q) dup |= (vs[q] == v);
            if (!dup) vs[k++] = v;
        }
        qsort(vs, (size_t)k, sizeof(int32_t), cmp_i32);
        if (k > 30) { free(vs); st = OR_TOO_BIG; goto fail; }
        factor *f = &fs[nf++];
        f->nv = k;
        f->vars = vs;
        f->e = 0;
        f->alive = 1;
        f->t = (double *)malloc(sizeof(double) * ((size_t)1 << k));
        if (!f->t) { st = OR_NOMEM; goto fail; }
        for (int64_t a = 0; a < ((int64_t)1 << k); ++a) {
            int sat = 0;
            for (int64_t j = cptr[c]; j < cptr[c + 1] && !sat; ++j) {
                int32_t l = lits[j];
                int q = 0;
                while (vs[q] != abs(l)) ++q;
                int val = (int)((a >> q) & 1);
                if ((l > 0 && val == 1) || (l < 0 && val == 0)) sat = 1;
            }
            f->t[a] = sat ? 1.0 : 0.0;
        }
    }
    for (int32_t x = 1; x <= n; ++x) {
        factor *f = &fs[nf++];
        f->nv = 1;
        f->vars = (int32_t *)malloc(sizeof(int32_t));
        f->t = (double *)malloc(2 * sizeof(double));
        if (!f->vars || !f->t) { st = OR_NOMEM; goto fail; }
        f->vars[0] = x;
        f->t[0] = w[2 * (x - 1)];
        f->t[1] = w[2 * (x - 1) + 1];
        f->e = 0;
        f->alive = 1;
    }

    int64_t *bucket = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cap + n + 1));
    int32_t *uni = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!bucket || !uni) { free(bucket); free(uni); st = OR_NOMEM; goto fail; }

    for (int32_t step = 0; step < n; ++step) {
        int32_t x = order[step];
        int nb = 0;
        int nu = 0;
        for (int64_t i = 0; i < nf; ++i) {
            factor *f = &fs[i];
            if (!f->alive) continue;
            int has = 0;
            for (int q = 0; q < f->nv; ++q) has |= (f->vars[q] == x);
            if (!has) continue;
            bucket[nb++] = i;
            for (int q = 0; q < f->nv; ++q) {
                int dup = 0;
                for (int u = 0; u < nu; ++u) dup |= (uni[u] == f->vars[q]);
                if (!dup) uni[nu++] = f->vars[q];
            }
        }
        qsort(uni, (size_t)nu, sizeof(int32_t), cmp_i32);
        int px = 0;
        while (uni[px] != x) ++px;
        int r = nu - 1;
        if (r > width) width = r;
        if (r > max_log2) { st = OR_TOO_BIG; free(bucket); free(uni); goto fail; }

        /* position of each bucket factor's variables inside the union scope */
        int **posu = (int **)malloc(sizeof(int *) * (size_t)nb);
        if (!posu) { st = OR_NOMEM; free(bucket); free(uni); goto fail; }
        int64_t esum = 0;
        for (int b = 0; b < nb; ++b) {
            factor *f = &fs[bucket[b]];
            posu[b] = (int *)malloc(sizeof(int) * (size_t)(f->nv ? f->nv : 1));
            for (int q = 0; q < f->nv; ++q) {
                int u = 0;
                while (uni[u] != f->vars[q]) ++u;
                posu[b][q] = u;
            }
            esum += f->e;
        }
        int64_t osize = (int64_t)1 << r;
        double *out = (double *)malloc(sizeof(double) * (size_t)osize);
        int32_t *ovars = (int32_t *)malloc(sizeof(int32_t) * (size_t)(r ? r : 1));
        if (!out || !ovars) {
            free(out); free(ovars);
            for (int b = 0; b < nb; ++b) free(posu[b]);
            free(posu); free(bucket); free(uni);
            st = OR_NOMEM;
            goto fail;
        }
        for (int u = 0, q = 0; u < nu; ++u)
            if (u != px) ovars[q++] = uni[u];

#pragma omp parallel for schedule(static)
        for (int64_t o = 0; o < osize; ++o) {
            int64_t lo = o & (((int64_t)1 << px) - 1);
            int64_t hi = (o >> px) << (px + 1);
            double s = 0.0;
            for (int64_t xv = 0; xv < 2; ++xv) {
                int64_t a = hi | (xv << px) | lo;   /* assignment over the union scope */
                double p = 1.0;
                for (int b = 0; b < nb; ++b) {
                    factor *f = &fs[bucket[b]];
                    int64_t idx = 0;
                    for (int q = 0; q < f->nv; ++q) idx |= ((a >> posu[b][q]) & 1) << q;
                    p *= f->t[idx];
                }
                s += p;
            }
            out[o] = s;
        }
        for (int b = 0; b < nb; ++b) {
            free(posu[b]);
            factor_free(&fs[bucket[b]]);
            fs[bucket[b]].alive = 0;
        }
        free(posu);
        factor *g = &fs[nf++];
        g->nv = r;
        g->vars = ovars;
        g->t = out;
        g->e = esum;
        g->alive = 1;
        renormalise(g->t, osize, &g->e);
    }
    free(bucket);
    free(uni);

    /* every surviving factor is now a scalar */
    {
        double mant = 1.0;
        int64_t ex = 0;
        for (int64_t i = 0; i < nf; ++i) {
            factor *f = &fs[i];
            if (!f->alive) continue;
            mant *= f->t[0];
            ex += f->e;
            if (mant == 0.0) { ex = 0; break; }
            int k;
            mant = frexp(mant, &k);
            ex += k;
        }
        if (mant == 0.0) ex = 0;
        *out_mant = mant;
        *out_exp = ex;
        if (out_width) *out_width = width;
    }
    for (int64_t i = 0; i < nf; ++i) factor_free(&fs[i]);
    free(fs);
    free(order);
    return OR_OK;

fail:
    for (int64_t i = 0; i < nf; ++i) factor_free(&fs[i]);
    free(fs);
    free(order);
    return st;
}

/* The oracle's own min-fill order (exported so tests can feed it back in). */
int oracle_minfill(int32_t n, int64_t m, const int64_t *cptr, const int32_t *lits,
                   int32_t *order) {
    int st = check_clauses(n, m, cptr, lits);
    if (st) return st;
    return minfill_order(n, m, cptr, lits, order);
}
