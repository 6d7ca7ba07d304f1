/*
 * Plain sequential FP64 oracle for MPLP++ dual block-coordinate ascent.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the solver library links, calls or
 * imports this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP path.
 *
 * Paper: Tourani, Shekhovtsov, Rother, Savchynskyy, "MPLP++: Fast, Parallel
 * Dual Block-Coordinate Ascent for Dense Graphical Models" (ECCV 2018).
 *
 * What it computes, in the paper's own terms and order:
 *  - the state is the reparametrized cost vector theta^phi itself (Eq. 2):
 *    Tu[u][s] for every node and Te[e][s][t] for every edge, starting from
 *    phi = 0, i.e. from the input costs;
 *  - one BCA update on edge uv (Sec. 4, "Block Coordinate Ascent Updates")
 *    forms the aggregated cost g = Te + Tu_u + Tu_v, computes new node
 *    unaries with the mapping (H) (or (M), (U)), and writes back
 *    Te := g - Tu_u_new - Tu_v_new;
 *  - the (H) mapping is evaluated in its literal four-line form: the MPLP
 *    halves of the row and column minima, then the correction of v, then the
 *    correction of u with the new v;
 *  - an iteration applies the update to every edge once, matching by
 *    matching, in the order of the edge schedule of Alg. 1 (Sec. 6);
 *  - the dual bound is Eq. (3), the primal rounding Eq. (5), the energy
 *    Eq. (1), and a brute-force MAP enumerates all labellings.
 *
 * Readings taken where the paper is silent:
 *  - edges are stored as (u, v) with u < v; a table given for (v, u) is
 *    transposed on input (Sec. 3 "Notation");
 *  - the schedule of a complete graph is the round-robin (circle) 1-factor-
 *    ization; any other graph gets greedy maximal matchings that scan the
 *    remaining edges in ascending (u, v) order (Alg. 1 with a greedy
 *    matching); edges of one matching are listed in ascending (u, v) order;
 *  - rounding (Eq. 5) visits nodes in ascending order and breaks ties
 *    toward the smallest label;
 *  - non-finite costs are rejected.
 *
 * OpenMP (optional) only spreads the edges of one matching over threads;
 * the edges of a matching touch disjoint data (Sec. 6), so the result is
 * bitwise the same for any thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

enum { RULE_H = 0, RULE_M = 1, RULE_U = 2 };

/* ------------------------------------------------------------------ */
/* Input canonicalization (Sec. 3: uv in E means u < v).               */
/* ------------------------------------------------------------------ */

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/* Copies edges and tables so that every edge reads (u, v) with u < v and its
 * table is indexed [label of u][label of v].  Rejects bad indices, self
 * loops, duplicate pairs and non-finite costs. */
int orc_canonicalize(int n, int L, int64_t m, const int32_t* edges_in, const double* unaries,
                     const double* pw_in, int32_t* edges_out, double* pw_out) {
    if (n < 1 || L < 1 || m < 0) return ORC_EINVAL;
    if (m > (int64_t)n * (n - 1) / 2) return ORC_EINVAL;
    for (int64_t i = 0; i < (int64_t)n * L; ++i)
        if (!isfinite(unaries[i])) return ORC_EINVAL;
    int64_t* keys = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!keys) return ORC_ENOMEM;
    for (int64_t e = 0; e < m; ++e) {
        int a = edges_in[2 * e], b = edges_in[2 * e + 1];
        if (a < 0 || a >= n || b < 0 || b >= n || a == b) { free(keys); return ORC_EINVAL; }
        int u = a < b ? a : b, v = a < b ? b : a;
        edges_out[2 * e] = u;
        edges_out[2 * e + 1] = v;
        keys[e] = (int64_t)u * n + v;
        const double* src = pw_in + (size_t)e * L * L;
        double* dst = pw_out + (size_t)e * L * L;
        for (int s = 0; s < L; ++s)
            for (int t = 0; t < L; ++t) {
                /* rows of the stored table belong to the lower node */
                double x = (a < b) ? src[(size_t)s * L + t] : src[(size_t)t * L + s];
                if (!isfinite(x)) { free(keys); return ORC_EINVAL; }
                dst[(size_t)s * L + t] = x;
            }
    }
    qsort(keys, (size_t)m, sizeof(int64_t), cmp_i64);
    for (int64_t e = 1; e < m; ++e)
        if (keys[e] == keys[e - 1]) { free(keys); return ORC_EINVAL; }
    free(keys);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Edge schedule (Sec. 6, Alg. 1: repeatedly take a matching of the     */
/* remaining edges and push it to the queue).                          */
/* ------------------------------------------------------------------ */

static int64_t g_n_for_sort;
static const int32_t* g_edges_for_sort;
static int cmp_edge_idx(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    int64_t kx = (int64_t)g_edges_for_sort[2 * x] * g_n_for_sort + g_edges_for_sort[2 * x + 1];
    int64_t ky = (int64_t)g_edges_for_sort[2 * y] * g_n_for_sort + g_edges_for_sort[2 * y + 1];
    return (kx > ky) - (kx < ky);
}

/* Writes step_ptr[0..S] and order[0..m-1] (edge indices); returns S or an
 * error.  step_ptr must hold m + 2 entries (S <= m + 1 is always enough). */
int orc_schedule(int n, int64_t m, const int32_t* edges, int32_t* step_ptr, int32_t* order) {
    if (n < 1 || m < 0) return ORC_EINVAL;
    if (m == 0) { step_ptr[0] = 0; return 0; }
    /* index of each unordered pair, -1 if absent (plain n x n table) */
    int32_t* id = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * n);
    if (!id) return ORC_ENOMEM;
    for (int64_t i = 0; i < (int64_t)n * n; ++i) id[i] = -1;
    for (int64_t e = 0; e < m; ++e) id[(size_t)edges[2 * e] * n + edges[2 * e + 1]] = (int32_t)e;

    int S = 0;
    int64_t pos = 0;
    g_n_for_sort = n;
    g_edges_for_sort = edges;
    if (m == (int64_t)n * (n - 1) / 2) {
        /* complete graph: round-robin 1-factorization.  N = n (even) or
         * n + 1 (odd, node n is a dummy whose edges are dropped).  Round r
         * pairs node N-1 with r and (r+k) with (r-k) modulo N-1. */
        int N = (n % 2 == 0) ? n : n + 1;
        for (int r = 0; r < N - 1; ++r) {
            step_ptr[S] = (int32_t)pos;
            int64_t start = pos;
            int a = N - 1, b = r;
            if (a < n && b < n) {
                int u = a < b ? a : b, v = a < b ? b : a;
                order[pos++] = id[(size_t)u * n + v];
            }
            for (int k = 1; k < N / 2; ++k) {
                a = (r + k) % (N - 1);
                b = ((r - k) % (N - 1) + (N - 1)) % (N - 1);
                if (a < n && b < n) {
                    int u = a < b ? a : b, v = a < b ? b : a;
                    order[pos++] = id[(size_t)u * n + v];
                }
            }
            qsort(order + start, (size_t)(pos - start), sizeof(int32_t), cmp_edge_idx);
            ++S;
        }
        step_ptr[S] = (int32_t)pos;
    } else {
        /* greedy maximal matchings over the remaining edges in (u, v) order */
        int32_t* rem = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
        int32_t* busy = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        if (!rem || !busy) { free(rem); free(busy); free(id); return ORC_ENOMEM; }
        int64_t nrem = 0;
        for (int u = 0; u < n; ++u)
            for (int v = u + 1; v < n; ++v)
                if (id[(size_t)u * n + v] >= 0) rem[nrem++] = id[(size_t)u * n + v];
        while (nrem > 0) {
            for (int i = 0; i < n; ++i) busy[i] = 0;
            step_ptr[S] = (int32_t)pos;
            int64_t keep = 0;
            for (int64_t i = 0; i < nrem; ++i) {
                int32_t e = rem[i];
                int u = edges[2 * e], v = edges[2 * e + 1];
                if (!busy[u] && !busy[v]) {
                    busy[u] = busy[v] = 1;
                    order[pos++] = e;
                } else {
                    rem[keep++] = e;
                }
            }
            nrem = keep;
            ++S;
        }
        step_ptr[S] = (int32_t)pos;
        free(rem);
        free(busy);
    }
    free(id);
    return S;
}

/* ------------------------------------------------------------------ */
/* Alternative schedule: the colour classes of an edge colouring with   */
/* at most Delta + 1 colours (Vizing's bound, by Misra and Gries'       */
/* constructive proof), one matching per colour.  Every choice is fixed */
/* so that the schedule depends on the edge set only:                   */
/*  - edges are coloured one by one in ascending (u, v), u < v; the fan */
/*    is centred at u and starts at v;                                  */
/*  - a free colour of a node is always its smallest free colour;       */
/*  - the fan grows, while it can, by the neighbour y of u (not yet in  */
/*    the fan) whose edge u-y carries the smallest colour that is free  */
/*    at the fan's current last node;                                   */
/*  - with c free at u and d free at the fan's last node, the maximal   */
/*    path leaving u by its d edge and then alternating c, d, ... has   */
/*    its two colours exchanged;                                        */
/*  - the fan is then cut after its first node where d is free (and up  */
/*    to which it is still a fan), each edge of that prefix takes the   */
/*    colour of the next one, and the cut node's edge gets d.           */
/* Complete graphs keep the round-robin schedule.                      */
/* ------------------------------------------------------------------ */

typedef struct {
    int n, C;
    int32_t* owner;   /* owner[x * C + c]: the node joined to x by colour c, or -1 */
    int32_t* colour;  /* colour of edge id, or -1 */
    const int32_t* edges;
    const int32_t* id;  /* id[u * n + v], u < v */
} colouring;

static int32_t edge_between(const colouring* k, int a, int b) {
    int u = a < b ? a : b, v = a < b ? b : a;
    return k->id[(size_t)u * k->n + v];
}
static int is_free(const colouring* k, int x, int c) { return k->owner[(size_t)x * k->C + c] < 0; }
static int smallest_free(const colouring* k, int x) {
    int c = 0;
    while (!is_free(k, x, c)) ++c;
    return c;
}
static void paint(colouring* k, int a, int b, int c) {
    int32_t e = edge_between(k, a, b);
    int old = k->colour[e];
    if (old >= 0) {
        k->owner[(size_t)a * k->C + old] = -1;
        k->owner[(size_t)b * k->C + old] = -1;
    }
    k->colour[e] = c;
    if (c >= 0) {
        k->owner[(size_t)a * k->C + c] = b;
        k->owner[(size_t)b * k->C + c] = a;
    }
}

static void colour_one_edge(colouring* k, int u, int v, int32_t* fan, char* infan, int32_t* path) {
    int len = 0;
    fan[len++] = v;
    infan[v] = 1;
    for (;;) {
        int x = fan[len - 1], grown = 0;
        for (int c = 0; c < k->C && !grown; ++c) {
            if (!is_free(k, x, c)) continue;
            int y = k->owner[(size_t)u * k->C + c];
            if (y < 0 || infan[y]) continue;
            fan[len++] = y;
            infan[y] = 1;
            grown = 1;
        }
        if (!grown) break;
    }
    for (int i = 0; i < len; ++i) infan[fan[i]] = 0;
    int c = smallest_free(k, u);
    int d = smallest_free(k, fan[len - 1]);
    if (c != d) {
        /* collect the path's nodes, then exchange its colours */
        int np = 0, x = u, want = d;
        path[np++] = u;
        while (!is_free(k, x, want)) {
            int y = k->owner[(size_t)x * k->C + want];
            path[np++] = y;
            x = y;
            want = (want == d) ? c : d;
        }
        /* uncolour all path edges first, then recolour each with the other colour */
        int* was = (int*)malloc(sizeof(int) * (size_t)(np > 1 ? np - 1 : 1));
        for (int i = 0; i + 1 < np; ++i) {
            was[i] = k->colour[edge_between(k, path[i], path[i + 1])];
            paint(k, path[i], path[i + 1], -1);
        }
        for (int i = 0; i + 1 < np; ++i) paint(k, path[i], path[i + 1], was[i] == c ? d : c);
        free(was);
    }
    int w = -1;
    for (int i = 0; i < len; ++i) {
        if (i > 0) {
            int ci = k->colour[edge_between(k, u, fan[i])];
            if (ci < 0 || !is_free(k, fan[i - 1], ci)) break;
        }
        if (is_free(k, fan[i], d)) { w = i; break; }
    }
    if (w < 0) w = 0; /* not reached for a proper colouring */
    for (int i = 0; i < w; ++i) {
        int cn = k->colour[edge_between(k, u, fan[i + 1])];
        paint(k, u, fan[i + 1], -1);
        paint(k, u, fan[i], cn);
    }
    paint(k, u, fan[w], d);
}

/* Same contract as orc_schedule; kind 0 = orc_schedule's rule, 1 = the
 * colouring above (complete graphs: round-robin either way). */
int orc_schedule_kind(int n, int64_t m, const int32_t* edges, int kind, int32_t* step_ptr, int32_t* order) {
    if (kind == 0 || m == 0 || m == (int64_t)n * (n - 1) / 2) return orc_schedule(n, m, edges, step_ptr, order);
    if (kind != 1 || n < 1 || m < 0) return ORC_EINVAL;
    int32_t* id = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * n);
    int32_t* deg = (int32_t*)calloc((size_t)n, sizeof(int32_t));
    if (!id || !deg) { free(id); free(deg); return ORC_ENOMEM; }
    for (int64_t i = 0; i < (int64_t)n * n; ++i) id[i] = -1;
    int maxdeg = 0;
    for (int64_t e = 0; e < m; ++e) {
        id[(size_t)edges[2 * e] * n + edges[2 * e + 1]] = (int32_t)e;
        if (++deg[edges[2 * e]] > maxdeg) maxdeg = deg[edges[2 * e]];
        if (++deg[edges[2 * e + 1]] > maxdeg) maxdeg = deg[edges[2 * e + 1]];
    }
    colouring k;
    k.n = n;
    k.C = maxdeg + 1;
    k.edges = edges;
    k.id = id;
    k.owner = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * k.C);
    k.colour = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    int32_t* fan = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* path = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    char* infan = (char*)calloc((size_t)n, 1);
    if (!k.owner || !k.colour || !fan || !path || !infan) {
        free(id); free(deg); free(k.owner); free(k.colour); free(fan); free(path); free(infan);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < (int64_t)n * k.C; ++i) k.owner[i] = -1;
    for (int64_t e = 0; e < m; ++e) k.colour[e] = -1;
    for (int u = 0; u < n; ++u)
        for (int v = u + 1; v < n; ++v)
            if (id[(size_t)u * n + v] >= 0) colour_one_edge(&k, u, v, fan, infan, path);
    /* one round per colour, edges ascending (u, v) inside a round */
    int S = 0;
    int64_t pos = 0;
    for (int c = 0; c < k.C; ++c) {
        int64_t start = pos;
        for (int u = 0; u < n; ++u)
            for (int v = u + 1; v < n; ++v) {
                int32_t e = id[(size_t)u * n + v];
                if (e >= 0 && k.colour[e] == c) order[pos++] = e;
            }
        if (pos > start) step_ptr[S++] = (int32_t)start;
    }
    step_ptr[S] = (int32_t)pos;
    free(id); free(deg); free(k.owner); free(k.colour); free(fan); free(path); free(infan);
    return pos == m ? S : ORC_EINVAL;
}

/* ------------------------------------------------------------------ */
/* BCA updates on one edge (Sec. 4).  Te is the edge's reparametrized   */
/* L x L table, Tu_u / Tu_v the current reparametrized unaries of its   */
/* two nodes; g, hu, hv are scratch.                                    */
/* ------------------------------------------------------------------ */

static void aggregate(int L, const double* Te, const double* Tu_u, const double* Tu_v, double* g) {
    for (int s = 0; s < L; ++s)
        for (int t = 0; t < L; ++t) g[(size_t)s * L + t] = Te[(size_t)s * L + t] + Tu_u[s] + Tu_v[t];
}

static void write_back(int L, double* Te, double* Tu_u, double* Tu_v, const double* g,
                       const double* hu, const double* hv) {
    for (int s = 0; s < L; ++s)
        for (int t = 0; t < L; ++t) Te[(size_t)s * L + t] = g[(size_t)s * L + t] - hu[s] - hv[t];
    for (int s = 0; s < L; ++s) Tu_u[s] = hu[s];
    for (int t = 0; t < L; ++t) Tu_v[t] = hv[t];
}

/* (M): half of the row minima of g to u, half of the column minima to v. */
static void mplp_halves(int L, const double* g, double* hu, double* hv) {
    for (int s = 0; s < L; ++s) {
        double mn = INFINITY;
        for (int t = 0; t < L; ++t) mn = fmin(mn, g[(size_t)s * L + t]);
        hu[s] = 0.5 * mn;
    }
    for (int t = 0; t < L; ++t) {
        double mn = INFINITY;
        for (int s = 0; s < L; ++s) mn = fmin(mn, g[(size_t)s * L + t]);
        hv[t] = 0.5 * mn;
    }
}

static void update_edge(int rule, int L, double* Te, double* Tu_u, double* Tu_v, double* g, double* hu,
                        double* hv) {
    aggregate(L, Te, Tu_u, Tu_v, g);
    if (rule == RULE_U) {
        double mn = INFINITY;
        for (size_t i = 0; i < (size_t)L * L; ++i) mn = fmin(mn, g[i]);
        for (int s = 0; s < L; ++s) hu[s] = 0.5 * mn;
        for (int t = 0; t < L; ++t) hv[t] = 0.5 * mn;
    } else {
        mplp_halves(L, g, hu, hv);
        if (rule == RULE_H) {
            /* (H), second line: v takes what is left in each column */
            for (int t = 0; t < L; ++t) {
                double mn = INFINITY;
                for (int s = 0; s < L; ++s) mn = fmin(mn, g[(size_t)s * L + t] - hv[t] - hu[s]);
                hv[t] = hv[t] + mn;
            }
            /* (H), third line: u takes what is left in each row, new hv */
            for (int s = 0; s < L; ++s) {
                double mn = INFINITY;
                for (int t = 0; t < L; ++t) mn = fmin(mn, g[(size_t)s * L + t] - hv[t] - hu[s]);
                hu[s] = hu[s] + mn;
            }
        }
    }
    write_back(L, Te, Tu_u, Tu_v, g, hu, hv);
}

/* One update on a single edge; exposed for the worked-example tests. */
int orc_update(int rule, int L, double* Te, double* Tu_u, double* Tu_v) {
    if (L < 1 || rule < RULE_H || rule > RULE_U) return ORC_EINVAL;
    double* g = (double*)malloc(sizeof(double) * ((size_t)L * L + 2 * (size_t)L));
    if (!g) return ORC_ENOMEM;
    update_edge(rule, L, Te, Tu_u, Tu_v, g, g + (size_t)L * L, g + (size_t)L * L + L);
    free(g);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Dual bound, Eq. (3).                                                 */
/* ------------------------------------------------------------------ */

double orc_dual(int n, int L, int64_t m, const double* Tu, const double* Te) {
    double d = 0.0;
    for (int u = 0; u < n; ++u) {
        double mn = INFINITY;
        for (int s = 0; s < L; ++s) mn = fmin(mn, Tu[(size_t)u * L + s]);
        d += mn;
    }
    for (int64_t e = 0; e < m; ++e) {
        double mn = INFINITY;
        const double* T = Te + (size_t)e * L * L;
        for (size_t i = 0; i < (size_t)L * L; ++i) mn = fmin(mn, T[i]);
        d += mn;
    }
    return d;
}

/* ------------------------------------------------------------------ */
/* Iterations (Def. "BCA-iteration", Sec. 5; schedule of Sec. 6).       */
/* ------------------------------------------------------------------ */

int orc_run(int n, int L, int64_t m, const int32_t* edges, int S, const int32_t* step_ptr,
            const int32_t* order, double* Tu, double* Te, int rule, int iters, double* trace,
            int nthreads) {
    if (n < 1 || L < 1 || m < 0 || iters < 0 || rule < RULE_H || rule > RULE_U) return ORC_EINVAL;
    if (nthreads < 1) nthreads = 1;
    size_t per = (size_t)L * L + 2 * (size_t)L;
    double* scratch = (double*)malloc(sizeof(double) * per * (size_t)nthreads);
    if (!scratch) return ORC_ENOMEM;
    for (int it = 0; it < iters; ++it) {
        for (int k = 0; k < S; ++k) {
            int64_t lo = step_ptr[k], hi = step_ptr[k + 1];
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static)
#endif
            for (int64_t i = lo; i < hi; ++i) {
                int tid = 0;
#ifdef _OPENMP
                tid = omp_get_thread_num();
#endif
                double* g = scratch + per * (size_t)tid;
                int32_t e = order[i];
                int u = edges[2 * e], v = edges[2 * e + 1];
                update_edge(rule, L, Te + (size_t)e * L * L, Tu + (size_t)u * L, Tu + (size_t)v * L, g,
                            g + (size_t)L * L, g + (size_t)L * L + L);
            }
        }
        if (trace) trace[it] = orc_dual(n, L, m, Tu, Te);
    }
    free(scratch);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Directional derivative of the dual after K iterations (not in the    */
/* paper; the reference for the adjoint).  D_K is piecewise linear in   */
/* the input costs: every quantity of (H) is a sum, a difference, a     */
/* half or a minimum of earlier ones.  Forward-mode differentiation     */
/* carries, next to each value x of the run, its derivative dx along a  */
/* direction (du on the unaries, dp on the tables): sums and halves     */
/* pass derivatives through, and a minimum takes the derivative of the  */
/* entry that attains it, the lowest index on ties.  The values are     */
/* computed by the same operations as update_edge, so the run is        */
/* bitwise the plain one.                                               */
/* ------------------------------------------------------------------ */

/* (H) on one edge with derivatives: g and dg are the aggregated cost and
 * its derivative; hu, hv, dhu, dhv the new unaries and their derivatives. */
static void update_edge_tangent(int L, double* Te, double* Tu_u, double* Tu_v, double* dTe, double* dTu_u,
                                double* dTu_v, double* g, double* dg, double* hu, double* hv, double* dhu,
                                double* dhv) {
    aggregate(L, Te, Tu_u, Tu_v, g);
    aggregate(L, dTe, dTu_u, dTu_v, dg);
    /* MPLP halves: hu(s) = min_t g(s,t) / 2, hv(t) = min_s g(s,t) / 2 */
    for (int s = 0; s < L; ++s) {
        double mn = INFINITY, best = INFINITY;
        int at = 0;
        for (int t = 0; t < L; ++t) {
            double x = g[(size_t)s * L + t];
            mn = fmin(mn, x);
            if (x < best) { best = x; at = t; }
        }
        hu[s] = 0.5 * mn;
        dhu[s] = 0.5 * dg[(size_t)s * L + at];
    }
    for (int t = 0; t < L; ++t) {
        double mn = INFINITY, best = INFINITY;
        int at = 0;
        for (int s = 0; s < L; ++s) {
            double x = g[(size_t)s * L + t];
            mn = fmin(mn, x);
            if (x < best) { best = x; at = s; }
        }
        hv[t] = 0.5 * mn;
        dhv[t] = 0.5 * dg[(size_t)at * L + t];
    }
    /* second line of (H): hv(t) += min_s [g(s,t) - hv(t) - hu(s)]; the
     * derivative of the sum is dg(s*,t) - dhu(s*), the old dhv cancels */
    for (int t = 0; t < L; ++t) {
        double mn = INFINITY, best = INFINITY;
        int at = 0;
        for (int s = 0; s < L; ++s) {
            double x = g[(size_t)s * L + t] - hv[t] - hu[s];
            mn = fmin(mn, x);
            if (x < best) { best = x; at = s; }
        }
        dhv[t] = dhv[t] + (dg[(size_t)at * L + t] - dhv[t] - dhu[at]);
        hv[t] = hv[t] + mn;
    }
    /* third line: hu(s) += min_t [g(s,t) - hv(t) - hu(s)] with the new hv */
    for (int s = 0; s < L; ++s) {
        double mn = INFINITY, best = INFINITY;
        int at = 0;
        for (int t = 0; t < L; ++t) {
            double x = g[(size_t)s * L + t] - hv[t] - hu[s];
            mn = fmin(mn, x);
            if (x < best) { best = x; at = t; }
        }
        dhu[s] = dhu[s] + (dg[(size_t)s * L + at] - dhv[at] - dhu[s]);
        hu[s] = hu[s] + mn;
    }
    write_back(L, Te, Tu_u, Tu_v, g, hu, hv);
    write_back(L, dTe, dTu_u, dTu_v, dg, dhu, dhv);
}

/* Runs `iters` (H) iterations like orc_run, carrying the derivatives dTu
 * [n][L] and dTe [m][L][L] (on entry: the direction, tables oriented as Te),
 * and writes to *dD the derivative of D_K = sum_u min_s Tu(u, s) + sum_e
 * min Te(e): each node term contributes dTu at its minimizing label (lowest
 * on ties).  The edge terms contribute nothing: after an edge's (H) update
 * every row minimum of its reparametrized table is zero (Sec. 4, after (H)),
 * for any input, so for iters >= 1 each edge term is identically zero as a
 * function of the costs. */
int orc_run_tangent(int n, int L, int64_t m, const int32_t* edges, int S, const int32_t* step_ptr,
                    const int32_t* order, double* Tu, double* Te, double* dTu, double* dTe, int iters,
                    double* dD, int nthreads) {
    if (n < 1 || L < 1 || m < 0 || iters < 0 || !dD) return ORC_EINVAL;
    if (nthreads < 1) nthreads = 1;
    size_t per = 2 * (size_t)L * L + 4 * (size_t)L;
    double* scratch = (double*)malloc(sizeof(double) * per * (size_t)nthreads);
    if (!scratch) return ORC_ENOMEM;
    for (int it = 0; it < iters; ++it) {
        for (int k = 0; k < S; ++k) {
            int64_t lo = step_ptr[k], hi = step_ptr[k + 1];
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static)
#endif
            for (int64_t i = lo; i < hi; ++i) {
                int tid = 0;
#ifdef _OPENMP
                tid = omp_get_thread_num();
#endif
                double* g = scratch + per * (size_t)tid;
                double* dg = g + (size_t)L * L;
                double* h = dg + (size_t)L * L;
                int32_t e = order[i];
                int u = edges[2 * e], v = edges[2 * e + 1];
                update_edge_tangent(L, Te + (size_t)e * L * L, Tu + (size_t)u * L, Tu + (size_t)v * L,
                                    dTe + (size_t)e * L * L, dTu + (size_t)u * L, dTu + (size_t)v * L, g, dg, h,
                                    h + L, h + 2 * L, h + 3 * L);
            }
        }
    }
    double d = 0.0;
    for (int u = 0; u < n; ++u) {
        int at = 0;
        for (int s = 1; s < L; ++s)
            if (Tu[(size_t)u * L + s] < Tu[(size_t)u * L + at]) at = s;
        d += dTu[(size_t)u * L + at];
    }
    *dD = d;
    free(scratch);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Primal rounding, Eq. (5), and energy, Eq. (1).                       */
/* ------------------------------------------------------------------ */

int orc_decode(int n, int L, int64_t m, const int32_t* edges, const double* Tu, const double* Te,
               int32_t* labels) {
    double* cost = (double*)malloc(sizeof(double) * (size_t)L);
    if (!cost) return ORC_ENOMEM;
    for (int u = 0; u < n; ++u) {
        for (int x = 0; x < L; ++x) cost[x] = Tu[(size_t)u * L + x];
        for (int64_t e = 0; e < m; ++e) {
            if (edges[2 * e + 1] != u) continue;       /* edge (v, u) with v < u */
            int v = edges[2 * e];
            const double* row = Te + (size_t)e * L * L + (size_t)labels[v] * L;
            for (int x = 0; x < L; ++x) cost[x] += row[x];
        }
        int best = 0;
        for (int x = 1; x < L; ++x)
            if (cost[x] < cost[best]) best = x;
        labels[u] = best;
    }
    free(cost);
    return ORC_OK;
}

double orc_energy(int n, int L, int64_t m, const int32_t* edges, const double* unaries,
                  const double* pairwise, const int32_t* labels) {
    double en = 0.0;
    for (int u = 0; u < n; ++u) en += unaries[(size_t)u * L + labels[u]];
    for (int64_t e = 0; e < m; ++e) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        en += pairwise[(size_t)e * L * L + (size_t)labels[u] * L + labels[v]];
    }
    return en;
}

/* Exhaustive MAP over all L^n labellings (node 0 varies fastest); the first
 * minimizer in that order is returned in best. */
double orc_bruteforce(int n, int L, int64_t m, const int32_t* edges, const double* unaries,
                      const double* pairwise, int32_t* best) {
    int32_t* y = (int32_t*)calloc((size_t)n, sizeof(int32_t));
    if (!y) return NAN;
    double best_e = INFINITY;
    for (;;) {
        double en = orc_energy(n, L, m, edges, unaries, pairwise, y);
        if (en < best_e) {
            best_e = en;
            memcpy(best, y, sizeof(int32_t) * (size_t)n);
        }
        int i = 0;
        while (i < n && ++y[i] == L) y[i++] = 0;
        if (i == n) break;
    }
    free(y);
    return best_e;
}

int orc_openmp_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
