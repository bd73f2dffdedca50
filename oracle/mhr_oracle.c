/*
 * CPU oracle for exact three-hop top-K path search.  TEST INFRASTRUCTURE
 * ONLY: the tests, the smoke check and the benchmark's CPU-baseline leg use
 * it; the product path never calls it.  It shares no code with the GPU
 * library.
 *
 * What it computes (the plain definition; every step in FP64):
 *  - Canonical graph: the input triples (h, r, t) of the problem statement
 *    (section 3.1, the three inputs) sorted and with identical triples
 *    removed.  Edges are directed h -> t.
 *  - Edge weight, one of two scorers:
 *    DistMult: the score x(u,r,v) = sum_i (X[u,i]*Y[r,i])*X[v,i], summed in
 *      ascending i, passed through the log-sigmoid
 *      w = min(x,0) - log1p(exp(-|x|)).  (The paper only says edge weights
 *      come from learned vertex and relation embeddings, section 1; this is
 *      the reading the project takes for its main workloads.)
 *    TransE-L1: the paper's own score (section 3.3, the person and
 *      affiliation scoring algorithms): the L1 distance
 *      x(u,r,v) = sum_i |(X[u,i] + Y[r,i]) - X[v,i]| of the head plus the
 *      relation from the tail, summed in ascending i, subtracted from the
 *      constant gamma (1.0 in the paper): w = gamma - x.
 *  - Paths: every walk s -r1-> a -r2-> b -r3-> t of exactly three edges
 *    (the three-hop query of section 3.1); a and b may repeat s, t or each
 *    other.  Score S = w1 + w2 + w3, the exact sum rounded once to FP64
 *    (so two paths whose weights are the same multiset score equal).
 *  - Order: S descending, then a, b, r1, r2, r3 ascending (a total order);
 *    the result is the first min(K, |P|) paths, the top-K ranked list the
 *    generic algorithm (section 5) returns.
 *
 * Enumeration: for each out-edge (s, r1, a), each out-edge (a, r2, b), the
 * out-edges of b with tail t are found by binary search in b's row (rows
 * are sorted by (tail, relation)), and every r3 is emitted.  All paths of a
 * query are collected and sorted; nothing is pruned.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    uint32_t n, R;
    uint64_t m;          /* distinct triples */
    uint64_t *rowptr;    /* n + 1 */
    uint32_t *tail;      /* m, sorted by (tail, rel) within each row */
    uint32_t *rel;       /* m */
} og_graph;

typedef struct {
    double s;
    uint32_t a, b, r1, r2, r3;
} og_path;

/* ------------------------------------------------------------------ */
/* graph                                                                */
/* ------------------------------------------------------------------ */

typedef struct { uint32_t u, v, r; } og_triple;

static int cmp_triple(const void *x, const void *y)
{
    const og_triple *p = (const og_triple *)x, *q = (const og_triple *)y;
    if (p->u != q->u) return p->u < q->u ? -1 : 1;
    if (p->v != q->v) return p->v < q->v ? -1 : 1;
    if (p->r != q->r) return p->r < q->r ? -1 : 1;
    return 0;
}

/* Returns the canonical graph, or NULL if an id is out of range or memory
 * runs out. */
og_graph *og_graph_build(uint32_t n, uint32_t R, uint64_t m,
                         const uint32_t *head, const uint32_t *rel,
                         const uint32_t *tail)
{
    og_triple *t = (og_triple *)malloc((m ? m : 1) * sizeof(og_triple));
    if (!t) return NULL;
    for (uint64_t i = 0; i < m; ++i) {
        if (head[i] >= n || tail[i] >= n || rel[i] >= R) { free(t); return NULL; }
        t[i].u = head[i]; t[i].v = tail[i]; t[i].r = rel[i];
    }
    qsort(t, m, sizeof(og_triple), cmp_triple);
    uint64_t k = 0;
    for (uint64_t i = 0; i < m; ++i)
        if (k == 0 || cmp_triple(&t[k - 1], &t[i]) != 0) t[k++] = t[i];

    og_graph *g = (og_graph *)calloc(1, sizeof(og_graph));
    g->n = n; g->R = R; g->m = k;
    g->rowptr = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    g->tail = (uint32_t *)malloc((k ? k : 1) * sizeof(uint32_t));
    g->rel = (uint32_t *)malloc((k ? k : 1) * sizeof(uint32_t));
    if (!g->rowptr || !g->tail || !g->rel) { free(t); return NULL; }
    for (uint64_t i = 0; i < k; ++i) {
        g->rowptr[t[i].u + 1]++;
        g->tail[i] = t[i].v;
        g->rel[i] = t[i].r;
    }
    for (uint32_t u = 0; u < n; ++u) g->rowptr[u + 1] += g->rowptr[u];
    free(t);
    return g;
}

void og_graph_free(og_graph *g)
{
    if (!g) return;
    free(g->rowptr); free(g->tail); free(g->rel); free(g);
}

uint64_t og_graph_edges(const og_graph *g) { return g->m; }

/* Copies the canonical CSR out (rowptr n+1, tail m, rel m). */
void og_graph_export(const og_graph *g, uint64_t *rowptr, uint32_t *tail, uint32_t *rel)
{
    memcpy(rowptr, g->rowptr, ((size_t)g->n + 1) * sizeof(uint64_t));
    memcpy(tail, g->tail, g->m * sizeof(uint32_t));
    memcpy(rel, g->rel, g->m * sizeof(uint32_t));
}

/* ------------------------------------------------------------------ */
/* edge weight                                                          */
/* ------------------------------------------------------------------ */

double og_logsigmoid(double x)
{
    return fmin(x, 0.0) - log1p(exp(-fabs(x)));
}

/* Scorer selection: 0 = DistMult + log-sigmoid, 1 = TransE-L1 with gamma. */
enum { OG_DISTMULT = 0, OG_TRANSE_L1 = 1 };
typedef struct { int kind; double gamma; } og_scorer;

/* TransE-L1 distance of (u, r, v): sum over i ascending of
 * |(X[u,i] + Y[r,i]) - X[v,i]|, every operation in FP64. */
static double og_l1(uint32_t d, const float *X, const float *Y,
                    uint32_t u, uint32_t r, uint32_t v)
{
    const float *xu = X + (size_t)u * d, *yr = Y + (size_t)r * d, *xv = X + (size_t)v * d;
    double acc = 0.0;
    for (uint32_t i = 0; i < d; ++i)
        acc += fabs(((double)xu[i] + (double)yr[i]) - (double)xv[i]);
    return acc;
}

/* DistMult score of (u, r, v): sum over i ascending of (X[u,i]*Y[r,i])*X[v,i]. */
static double og_x(uint32_t d, const float *X, const float *Y,
                   uint32_t u, uint32_t r, uint32_t v)
{
    const float *xu = X + (size_t)u * d, *yr = Y + (size_t)r * d, *xv = X + (size_t)v * d;
    double acc = 0.0;
    for (uint32_t i = 0; i < d; ++i)
        acc += ((double)xu[i] * (double)yr[i]) * (double)xv[i];
    return acc;
}

/* The scorer's raw value x (DistMult score or L1 distance) of (u, r, v). */
static double og_raw(og_scorer sc, uint32_t d, const float *X, const float *Y,
                     uint32_t u, uint32_t r, uint32_t v)
{
    return sc.kind == OG_TRANSE_L1 ? og_l1(d, X, Y, u, r, v) : og_x(d, X, Y, u, r, v);
}

/* The edge weight from the raw value. */
static double og_weight(og_scorer sc, double x)
{
    return sc.kind == OG_TRANSE_L1 ? sc.gamma - x : og_logsigmoid(x);
}

static double og_edge_weight(og_scorer sc, uint32_t d, const float *X, const float *Y,
                             uint32_t u, uint32_t r, uint32_t v)
{
    return og_weight(sc, og_raw(sc, d, X, Y, u, r, v));
}

/* Raw values and weights of ne arbitrary edges (u[i], r[i], v[i]). */
void og_edge_weights_s(int scorer, double gamma, uint32_t d, const float *X, const float *Y,
                       uint64_t ne, const uint32_t *u, const uint32_t *r, const uint32_t *v,
                       double *out_x, double *out_w)
{
    og_scorer sc = {scorer, gamma};
    for (uint64_t i = 0; i < ne; ++i) {
        double x = og_raw(sc, d, X, Y, u[i], r[i], v[i]);
        if (out_x) out_x[i] = x;
        out_w[i] = og_weight(sc, x);
    }
}

void og_edge_weights(uint32_t d, const float *X, const float *Y, uint64_t ne,
                     const uint32_t *u, const uint32_t *r, const uint32_t *v,
                     double *out_x, double *out_w)
{
    og_edge_weights_s(OG_DISTMULT, 0.0, d, X, Y, ne, u, r, v, out_x, out_w);
}

/* ------------------------------------------------------------------ */
/* path score: the sum of three weights, correctly rounded              */
/* ------------------------------------------------------------------ */

/* Correctly rounded sum of n doubles (n small), after Shewchuk, "Adaptive
 * Precision Floating-Point Arithmetic and Fast Robust Geometric Predicates"
 * (1997): the running sum is kept as a list of non-overlapping partials
 * built with error-free two-sums; the partials are then added from the
 * largest, and a half-way case at the last step is settled by the sign of
 * the next partial (round half to even on the exact sum).  The result
 * depends only on the multiset of inputs, so paths whose weights are
 * permutations of each other get bit-identical scores. */
double og_fsum(const double *v, int n)
{
    double p[8];
    int np = 0;
    for (int k = 0; k < n; ++k) {
        double x = v[k];
        int i = 0;
        for (int j = 0; j < np; ++j) {
            double y = p[j];
            if (fabs(x) < fabs(y)) { double t = x; x = y; y = t; }
            double hi = x + y;
            double lo = y - (hi - x);
            if (lo != 0.0) p[i++] = lo;
            x = hi;
        }
        p[i++] = x;
        np = i;
    }
    if (np == 0) return 0.0;
    int j = np - 1;
    double hi = p[j], lo = 0.0;
    while (j > 0) {
        double x = hi, y = p[--j];
        hi = x + y;
        double yr = hi - x;
        lo = y - yr;
        if (lo != 0.0) break;
    }
    if (j > 0 && ((lo < 0.0 && p[j - 1] < 0.0) || (lo > 0.0 && p[j - 1] > 0.0))) {
        double y = lo * 2.0;
        double x = hi + y;
        double yr = x - hi;
        if (y == yr) hi = x;
    }
    return hi;
}

static double og_path_score(double w1, double w2, double w3)
{
    double v[3] = {w1, w2, w3};
    return og_fsum(v, 3);
}

/* ------------------------------------------------------------------ */
/* top-K paths                                                          */
/* ------------------------------------------------------------------ */

/* The total order: score descending, then a, b, r1, r2, r3 ascending. */
static int cmp_path(const void *x, const void *y)
{
    const og_path *p = (const og_path *)x, *q = (const og_path *)y;
    if (p->s != q->s) return p->s > q->s ? -1 : 1;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    if (p->r1 != q->r1) return p->r1 < q->r1 ? -1 : 1;
    if (p->r2 != q->r2) return p->r2 < q->r2 ? -1 : 1;
    if (p->r3 != q->r3) return p->r3 < q->r3 ? -1 : 1;
    return 0;
}

/* First index in [lo, hi) of row entries whose tail is >= key. */
static uint64_t lower_tail(const uint32_t *tail, uint64_t lo, uint64_t hi, uint32_t key)
{
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (tail[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

typedef struct { og_path *p; uint64_t n, cap; int oom; } og_vec;

static void vec_push(og_vec *v, og_path x)
{
    if (v->oom) return;
    if (v->n == v->cap) {
        uint64_t nc = v->cap ? v->cap * 2 : 1024;
        og_path *np = (og_path *)realloc(v->p, nc * sizeof(og_path));
        if (!np) { v->oom = 1; return; }
        v->p = np; v->cap = nc;
    }
    v->p[v->n++] = x;
}

/* One query: all paths s -> a -> b -> t, sorted; keeps the first K.
 * Returns the number of paths |P(s,t)|, or UINT64_MAX on allocation failure. */
static uint64_t og_query(const og_graph *g, og_scorer sc, uint32_t d, const float *X, const float *Y,
                         uint32_t s, uint32_t t, uint32_t K, og_path *out, uint32_t *count)
{
    og_vec v = {0};
    for (uint64_t e1 = g->rowptr[s]; e1 < g->rowptr[s + 1]; ++e1) {
        uint32_t a = g->tail[e1], r1 = g->rel[e1];
        double w1 = og_edge_weight(sc, d, X, Y, s, r1, a);
        for (uint64_t e2 = g->rowptr[a]; e2 < g->rowptr[a + 1]; ++e2) {
            uint32_t b = g->tail[e2], r2 = g->rel[e2];
            uint64_t lo = lower_tail(g->tail, g->rowptr[b], g->rowptr[b + 1], t);
            uint64_t e3 = lo;
            if (e3 >= g->rowptr[b + 1] || g->tail[e3] != t) continue;
            double w2 = og_edge_weight(sc, d, X, Y, a, r2, b);
            for (; e3 < g->rowptr[b + 1] && g->tail[e3] == t; ++e3) {
                uint32_t r3 = g->rel[e3];
                double w3 = og_edge_weight(sc, d, X, Y, b, r3, t);
                og_path p;
                p.s = og_path_score(w1, w2, w3);
                p.a = a; p.b = b; p.r1 = r1; p.r2 = r2; p.r3 = r3;
                vec_push(&v, p);
            }
        }
    }
    if (v.oom) { free(v.p); *count = 0; return UINT64_MAX; }
    if (v.n) qsort(v.p, v.n, sizeof(og_path), cmp_path);
    uint64_t keep = v.n < K ? v.n : K;
    if (keep) memcpy(out, v.p, keep * sizeof(og_path));
    *count = (uint32_t)keep;
    uint64_t total = v.n;
    free(v.p);
    return total;
}

/* Batch of queries; OpenMP over queries (dynamic schedule).  out has
 * nq * kmax records; k[q] <= kmax.  Returns 0, or -1 on a bad argument or
 * allocation failure. */
int og_topk_s(const og_graph *g, int scorer, double gamma, uint32_t d, const float *X,
              const float *Y, uint32_t nq, const uint32_t *src, const uint32_t *dst,
              const uint32_t *k, uint32_t kmax, int nthreads,
              og_path *out, uint32_t *out_count, uint64_t *out_total)
{
    og_scorer sc = {scorer, gamma};
    if (scorer != OG_DISTMULT && scorer != OG_TRANSE_L1) return -1;
    for (uint32_t q = 0; q < nq; ++q)
        if (src[q] >= g->n || dst[q] >= g->n || k[q] == 0 || k[q] > kmax) return -1;
    int fail = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t q = 0; q < (int64_t)nq; ++q) {
        uint64_t tot = og_query(g, sc, d, X, Y, src[q], dst[q], k[q],
                                out + (size_t)q * kmax, &out_count[q]);
        if (tot == UINT64_MAX) fail = 1;
        out_total[q] = tot;
    }
    return fail ? -1 : 0;
}

int og_topk(const og_graph *g, uint32_t d, const float *X, const float *Y,
            uint32_t nq, const uint32_t *src, const uint32_t *dst,
            const uint32_t *k, uint32_t kmax, int nthreads,
            og_path *out, uint32_t *out_count, uint64_t *out_total)
{
    return og_topk_s(g, OG_DISTMULT, 0.0, d, X, Y, nq, src, dst, k, kmax, nthreads,
                     out, out_count, out_total);
}

int og_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Candidate scan (the paper's three-hop Turing-award pipeline,         */
/* section 3.2 and the person / affiliation scoring of section 3.3)    */
/* ------------------------------------------------------------------ */

typedef struct { double s; uint32_t id; } og_cand;

/* Score descending, then candidate id ascending (a total order). */
static int cmp_cand(const void *x, const void *y)
{
    const og_cand *p = (const og_cand *)x, *q = (const og_cand *)y;
    if (p->s != q->s) return p->s > q->s ? -1 : 1;
    if (p->id != q->id) return p->id < q->id ? -1 : 1;
    return 0;
}

/* For each query q: the TransE-L1 score of every candidate c of the list,
 * gamma - sum_i |(X[head[q],i] + Y[rel[q],i]) - X[c,i]| (candidate as the
 * tail, FP64, ascending i), and the best min(K, ncand) candidates under
 * (score descending, id ascending).  out_id / out_s hold nq * K entries.
 * Returns 0, or -1 on allocation failure. */
int og_scan_topk(uint32_t d, const float *X, const float *Y, uint32_t nq,
                 const uint32_t *head, const uint32_t *rel, const uint32_t *cand,
                 uint32_t ncand, uint32_t K, double gamma,
                 uint32_t *out_id, double *out_s)
{
    int fail = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t q = 0; q < (int64_t)nq; ++q) {
        og_cand *all = (og_cand *)malloc((ncand ? ncand : 1) * sizeof(og_cand));
        if (!all) { fail = 1; continue; }
        og_scorer sc = {OG_TRANSE_L1, gamma};
        for (uint32_t i = 0; i < ncand; ++i) {
            all[i].id = cand[i];
            all[i].s = og_edge_weight(sc, d, X, Y, head[q], rel[q], cand[i]);
        }
        qsort(all, ncand, sizeof(og_cand), cmp_cand);
        uint32_t keep = ncand < K ? ncand : K;
        for (uint32_t k = 0; k < K; ++k) {
            out_id[(size_t)q * K + k] = k < keep ? all[k].id : 0xFFFFFFFFu;
            out_s[(size_t)q * K + k] = k < keep ? all[k].s : -HUGE_VAL;
        }
        free(all);
    }
    return fail ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Generic multi-hop search (section 5: the level-by-level expansion   */
/* with a per-parent top-K, paths to the target recorded as found)     */
/* ------------------------------------------------------------------ */

#define OG_MAX_HOPS 8

typedef struct {
    double s;
    uint32_t len;                   /* edges */
    uint32_t v[OG_MAX_HOPS];        /* v[0..len): the vertices after the source */
    uint32_t r[OG_MAX_HOPS];
} og_bpath;

/* Score descending, then the vertex sequence lexicographically (a proper
 * prefix first), then the relation sequence. */
static int cmp_bpath(const og_bpath *p, const og_bpath *q)
{
    if (p->s != q->s) return p->s > q->s ? -1 : 1;
    uint32_t n = p->len < q->len ? p->len : q->len;
    for (uint32_t i = 0; i < n; ++i)
        if (p->v[i] != q->v[i]) return p->v[i] < q->v[i] ? -1 : 1;
    if (p->len != q->len) return p->len < q->len ? -1 : 1;
    for (uint32_t i = 0; i < p->len; ++i)
        if (p->r[i] != q->r[i]) return p->r[i] < q->r[i] ? -1 : 1;
    return 0;
}

static int cmp_bpath_q(const void *x, const void *y)
{
    return cmp_bpath((const og_bpath *)x, (const og_bpath *)y);
}

typedef struct { og_bpath *p; uint64_t n, cap; int oom; } og_bvec;

static void bvec_push(og_bvec *v, const og_bpath *x)
{
    if (v->oom) return;
    if (v->n == v->cap) {
        uint64_t nc = v->cap ? v->cap * 2 : 64;
        og_bpath *np = (og_bpath *)realloc(v->p, nc * sizeof(og_bpath));
        if (!np) { v->oom = 1; return; }
        v->p = np; v->cap = nc;
    }
    v->p[v->n++] = *x;
}

/* One query of the generic search.  A path starts as the source alone with
 * score 0.  At each of the H levels every current path is extended by every
 * out-edge (horizon, r, nb) of its last vertex whose head nb is not on the
 * path yet; the extension's score is the path's score plus w(horizon, r, nb)
 * (scores add along the path).  An extension that reaches the target is
 * recorded as a result and not extended further; of the others, each parent
 * passes its best K (under the order above) to the next level.  The result
 * is the best K recorded paths.  Returns the number recorded, or UINT64_MAX
 * on allocation failure. */
static uint64_t og_beam_query(const og_graph *g, og_scorer sc, uint32_t d, const float *X, const float *Y,
                              uint32_t s, uint32_t t, uint32_t H, uint32_t K, og_bpath *out, uint32_t *count)
{
    og_bvec curr = {0}, next = {0}, res = {0}, kids = {0};
    og_bpath root;
    memset(&root, 0, sizeof(root));
    bvec_push(&curr, &root);
    for (uint32_t level = 0; level < H; ++level) {
        next.n = 0;
        for (uint64_t pi = 0; pi < curr.n; ++pi) {
            const og_bpath *par = &curr.p[pi];
            uint32_t h = par->len ? par->v[par->len - 1] : s;
            kids.n = 0;
            for (uint64_t e = g->rowptr[h]; e < g->rowptr[h + 1]; ++e) {
                uint32_t nb = g->tail[e], r = g->rel[e];
                int on_path = nb == s;
                for (uint32_t i = 0; i < par->len; ++i) on_path |= par->v[i] == nb;
                if (on_path) continue;
                og_bpath x = *par;
                x.v[x.len] = nb;
                x.r[x.len] = r;
                x.len += 1;
                x.s = par->s + og_edge_weight(sc, d, X, Y, h, r, nb);
                if (nb == t) bvec_push(&res, &x);
                else bvec_push(&kids, &x);
            }
            if (kids.n) qsort(kids.p, kids.n, sizeof(og_bpath), cmp_bpath_q);
            for (uint64_t i = 0; i < kids.n && i < K; ++i) bvec_push(&next, &kids.p[i]);
        }
        og_bvec tmp = curr; curr = next; next = tmp;
    }
    uint64_t total = res.n;
    int oom = curr.oom | next.oom | res.oom | kids.oom;
    if (!oom && res.n) qsort(res.p, res.n, sizeof(og_bpath), cmp_bpath_q);
    uint32_t keep = (uint32_t)(res.n < K ? res.n : K);
    if (!oom && keep) memcpy(out, res.p, keep * sizeof(og_bpath));
    *count = oom ? 0 : keep;
    free(curr.p); free(next.p); free(res.p); free(kids.p);
    return oom ? UINT64_MAX : total;
}

/* Batch of queries (OpenMP over queries).  H in 1..OG_MAX_HOPS.  out holds
 * nq * K paths.  Returns 0, or -1 on a bad argument or allocation failure. */
int og_beam(const og_graph *g, int scorer, double gamma, uint32_t d, const float *X, const float *Y,
            uint32_t nq, const uint32_t *src, const uint32_t *dst, uint32_t H, uint32_t K,
            og_bpath *out, uint32_t *out_count, uint64_t *out_recorded)
{
    if (H < 1 || H > OG_MAX_HOPS || K < 1) return -1;
    for (uint32_t q = 0; q < nq; ++q)
        if (src[q] >= g->n || dst[q] >= g->n) return -1;
    og_scorer sc = {scorer, gamma};
    int fail = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t q = 0; q < (int64_t)nq; ++q) {
        uint64_t tot = og_beam_query(g, sc, d, X, Y, src[q], dst[q], H, K, out + (size_t)q * K, &out_count[q]);
        if (tot == UINT64_MAX) fail = 1;
        out_recorded[q] = tot;
    }
    return fail ? -1 : 0;
}
