/*
 * CPU ORACLE -- test infrastructure only.
 *
 * A plain, slow, deliberately unoptimised bucket eliminator used to check the
 * device library.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header or table with the device
 * library.
 *
 * What it computes (Fioretto, Pontelli, Yeoh, Dechter, "Accelerating Exact and
 * Approximate Inference for (Distributed) Discrete Optimization with GPUs"):
 *   - Bucket Elimination (Sec. 2.1, Alg. 1) and Mini-Bucket Elimination
 *     (Sec. 2.2, Alg. 2) on a WCSP <X, D, C> (Sec. 2): for every variable, in
 *     reverse order, the functions of its bucket are AGGREGATED into one table
 *     over the union of their scopes (sum, Sec. 2 "aggregation") and the
 *     variable is then ELIMINATED (min-projection, Sec. 2 "elimination"); with
 *     mini-buckets the bucket is first partitioned so that each part's union
 *     scope holds at most `ibound` variables.
 *   - the value assignment phase (Alg. 1/2, second loop) and the cost of the
 *     resulting assignment (an upper bound for MBE, Sec. 2.2).
 *   - MPE on belief networks (Sec. 3) as min-sum over -ln p in double.
 *   - DPOP (Sec. 4.1) is BE along a pseudo-tree order; the caller checks that
 *     each message scope equals the agent's separator.
 *   - the sum-product variant the paper names as future work (Sec. 10:
 *     weighted counting, partition function, probability of evidence), on
 *     double costs c = -ln phi: eliminating x turns a table a(s, x) into
 *     -ln sum_x exp(-a(s, x)) instead of min_x a(s, x), so BE returns
 *     -ln Z with Z = sum over all assignments of prod phi.  With mini-buckets
 *     (R18) the first mini-bucket of a bucket sums and the others take the
 *     minimum (the maximum of phi): sum_x prod_k F_k <= (sum_x F_1) *
 *     prod_{k>1} max_x F_k, so the result is a lower bound of -ln Z.
 *
 * Readings of the paper taken here (the paper is silent or inconsistent):
 *   R1 a function goes to the bucket of the variable of its scope that comes
 *      LAST in the order (eliminated first), as the worked example does.
 *   R2 `ibound` bounds |union of scopes| of a mini-bucket INCLUDING the
 *      eliminated variable.
 *   R3 partition: if the whole bucket fits, one mini-bucket; otherwise the
 *      functions, sorted by (decreasing arity, increasing id), go first-fit into
 *      mini-buckets tried in creation order.  Input functions have ids 0..m-1,
 *      messages get m, m+1, ... in creation order.
 *   R4 value ties go to the smallest value.
 *   R5 a variable's value minimises the sum of ALL functions placed in its
 *      bucket (inputs and received messages).
 *   R6 integer infinity is INT32_MAX; a (+) b = min(INF, a + b) for a, b >= 0.
 *   R7 a mini-bucket output goes to the bucket of the last-in-order variable
 *      of its scope; an empty-scope output is added to the constant.
 *   R8 elimination writes a new table (never in place).
 *  R10 table rows are plain row-major mixed radix over the scope, first scope
 *      variable most significant (the bucket-table of Sec. 6.1, with the hash
 *      of Eq. (3) read as digit_j(r) = floor(r / prod of later domains) mod d_j).
 *  R12 scopes are kept sorted by increasing position in the order, so the
 *      eliminated variable is the last (fastest) one (Sec. 6.2).
 *  R18 sum-product with mini-buckets: the mini-bucket created first sums over
 *      the eliminated variable, every other one minimises; the value phase is
 *      unchanged (each variable takes the value of least bucket cost), and
 *      the cost of that assignment bounds -ln Z from above.  A variable in no
 *      function's scope adds -ln |D_v| to the constant (its values each
 *      weigh 1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_INF ((int32_t)0x7fffffff)

/* ------------------------------------------------------------------------ */
/* saturating integer addition (R6)                                          */
/* ------------------------------------------------------------------------ */
static int32_t sat_add(int32_t a, int32_t b)
{
    int64_t s = (int64_t)a + (int64_t)b;
    return s >= OR_INF ? OR_INF : (int32_t)s;
}

int32_t or_sat_add(int32_t a, int32_t b) { return sat_add(a, b); }

/* ------------------------------------------------------------------------ */
/* a cost function: scope listed in increasing order position               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int id;
    int arity;
    int *scope;       /* variable ids */
    int64_t size;     /* number of rows = product of domains */
    int32_t *ti;      /* integer costs, or NULL */
    double *td;       /* double costs, or NULL */
} ofn;

typedef struct { int n, cap; int *v; } ilist;

static void il_push(ilist *l, int x)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 8;
        l->v = (int *)realloc(l->v, sizeof(int) * (size_t)l->cap);
    }
    l->v[l->n++] = x;
}

/* one recorded mini-bucket: which functions it aggregated and what it sent  */
typedef struct {
    int var;          /* eliminated variable */
    int k;            /* index of the mini-bucket inside its bucket */
    int n_members;
    int *members;     /* function ids, in aggregation order */
    int out_id;       /* id given to the output (-1 if it went to the constant) */
    int out_arity;
    int *out_scope;
    int64_t out_size;
    int32_t *out_ti;
    double *out_td;
} ominib;

typedef struct {
    int n;
    int is_double;
    double lb;        /* bound: the constant after all eliminations */
    double ub;        /* cost of the assignment found */
    int *assign;
    int n_mb;
    int cap_mb;
    ominib *mb;
    int n_buckets_used;
    int max_union;    /* largest |union scope| over all mini-buckets processed */
} or_result;

/* ------------------------------------------------------------------------ */
/* row <-> assignment (R10)                                                  */
/* ------------------------------------------------------------------------ */

/* index of the row of f selected by the full assignment val[] (by var id)   */
static int64_t row_of(const ofn *f, const int *dom, const int *val)
{
    int64_t r = 0;
    for (int j = 0; j < f->arity; ++j)
        r = r * dom[f->scope[j]] + val[f->scope[j]];
    return r;
}

/* advance the assignment of the variables in scope[0..a-1] like an odometer,
 * last variable fastest; returns 0 once it wraps around */
static int odometer_next(int a, const int *scope, const int *dom, int *val)
{
    for (int j = a - 1; j >= 0; --j) {
        int u = scope[j];
        if (++val[u] < dom[u]) return 1;
        val[u] = 0;
    }
    return 0;
}

/* map every row of an "output" table over out_scope to the row of an input
 * table over in_scope (a subset of out_scope): the bucket-table index
 * correspondence of Sec. 6.3, Eq. (3).  Exported so that the worked example
 * of Sec. 6.3 can be checked directly. */
int or_map_rows(int n_vars, const int *dom, int out_arity, const int *out_scope,
                int in_arity, const int *in_scope, int64_t *map_out)
{
    int *val = (int *)calloc((size_t)n_vars, sizeof(int));
    ofn f;
    f.arity = in_arity;
    f.scope = (int *)in_scope;
    int64_t r = 0;
    do {
        map_out[r++] = row_of(&f, dom, val);
    } while (odometer_next(out_arity, out_scope, dom, val));
    free(val);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* graph helpers                                                             */
/* ------------------------------------------------------------------------ */
static unsigned char *primal_graph(int n, int m, const int *arity, const int *scope_flat)
{
    unsigned char *adj = (unsigned char *)calloc((size_t)n * n, 1);
    int off = 0;
    for (int f = 0; f < m; ++f) {
        for (int a = 0; a < arity[f]; ++a)
            for (int b = 0; b < arity[f]; ++b) {
                int x = scope_flat[off + a], y = scope_flat[off + b];
                if (x != y) adj[(size_t)x * n + y] = 1;
            }
        off += arity[f];
    }
    return adj;
}

static int degree(const unsigned char *adj, const unsigned char *alive, int n, int v)
{
    int d = 0;
    for (int u = 0; u < n; ++u)
        if (alive[u] && adj[(size_t)v * n + u]) ++d;
    return d;
}

static int fill_in(const unsigned char *adj, const unsigned char *alive, int n, int v)
{
    int f = 0;
    for (int a = 0; a < n; ++a) {
        if (!alive[a] || !adj[(size_t)v * n + a]) continue;
        for (int b = a + 1; b < n; ++b)
            if (alive[b] && adj[(size_t)v * n + b] && !adj[(size_t)a * n + b]) ++f;
    }
    return f;
}

/* Greedy elimination orders.  The variable chosen first is eliminated first,
 * i.e. it takes the LAST position of the order.
 *   heuristic 0 (min-degree): fewest neighbours in the current graph; ties to
 *                             the lowest id.
 *   heuristic 1 (min-fill):   fewest new edges; ties to fewest neighbours,
 *                             then the lowest id.
 * Eliminating a vertex connects its remaining neighbours pairwise. */
static void greedy_order(int n, unsigned char *adj, int heuristic, int *order)
{
    unsigned char *alive = (unsigned char *)malloc((size_t)n);
    memset(alive, 1, (size_t)n);
    for (int p = n - 1; p >= 0; --p) {
        int best = -1, bf = 0, bd = 0;
        for (int v = 0; v < n; ++v) {
            if (!alive[v]) continue;
            int d = degree(adj, alive, n, v);
            int f = heuristic == 1 ? fill_in(adj, alive, n, v) : 0;
            int better;
            if (best < 0) better = 1;
            else if (heuristic == 1) better = (f < bf) || (f == bf && d < bd);
            else better = d < bd;
            if (better) { best = v; bf = f; bd = d; }
        }
        order[p] = best;
        for (int a = 0; a < n; ++a) {
            if (!alive[a] || !adj[(size_t)best * n + a]) continue;
            for (int b = 0; b < n; ++b)
                if (b != a && alive[b] && adj[(size_t)best * n + b])
                    adj[(size_t)a * n + b] = 1;
        }
        alive[best] = 0;
    }
    free(alive);
}

/* DFS pseudo-tree (Sec. 2, pseudo-tree definition): every component is rooted
 * at its highest-degree vertex (ties: lowest id) and the DFS enters unvisited
 * neighbours by decreasing degree (ties: lowest id).  order = pre-order,
 * parent[root] = -1.  Degrees are those of the primal graph. */
static int dfs_visit(int n, const unsigned char *adj, const int *deg, int v, int par,
                     int *parent, unsigned char *seen, int *order, int pos)
{
    seen[v] = 1;
    parent[v] = par;
    order[pos++] = v;
    for (;;) {
        int best = -1;
        for (int u = 0; u < n; ++u)
            if (!seen[u] && adj[(size_t)v * n + u] && (best < 0 || deg[u] > deg[best]))
                best = u;
        if (best < 0) break;
        pos = dfs_visit(n, adj, deg, best, v, parent, seen, order, pos);
    }
    return pos;
}

static void dfs_order(int n, const unsigned char *adj, int *order, int *parent)
{
    int *deg = (int *)malloc(sizeof(int) * (size_t)n);
    unsigned char *seen = (unsigned char *)calloc((size_t)n, 1);
    unsigned char *all = (unsigned char *)malloc((size_t)n);
    memset(all, 1, (size_t)n);
    for (int v = 0; v < n; ++v) deg[v] = degree(adj, all, n, v);
    int pos = 0;
    while (pos < n) {
        int root = -1;
        for (int v = 0; v < n; ++v)
            if (!seen[v] && (root < 0 || deg[v] > deg[root])) root = v;
        pos = dfs_visit(n, adj, deg, root, -1, parent, seen, order, pos);
    }
    free(deg); free(seen); free(all);
}

/* The paper's own ordering (Sec. 6.2): x_i precedes x_j when x_i has fewer
 * neighbours; ties to the lowest id.  The last variable is eliminated first. */
static void degree_sort_order(int n, const unsigned char *adj, int *order)
{
    unsigned char *all = (unsigned char *)malloc((size_t)n);
    memset(all, 1, (size_t)n);
    int *deg = (int *)malloc(sizeof(int) * (size_t)n);
    for (int v = 0; v < n; ++v) { deg[v] = degree(adj, all, n, v); order[v] = v; }
    for (int i = 1; i < n; ++i) {              /* insertion sort, stable */
        int x = order[i], j = i - 1;
        while (j >= 0 && deg[order[j]] > deg[x]) { order[j + 1] = order[j]; --j; }
        order[j + 1] = x;
    }
    free(all); free(deg);
}

/* heuristic: 0 min-degree, 1 min-fill, 2 DFS pseudo-tree (pre-order, parent
 * written to parent_out), 3 the paper's static degree order */
int or_order(int n, int m, const int *arity, const int *scope_flat, int heuristic,
             int *order_out, int *parent_out)
{
    if (n <= 0) return 0;
    unsigned char *adj = primal_graph(n, m, arity, scope_flat);
    if (heuristic == 0 || heuristic == 1) greedy_order(n, adj, heuristic, order_out);
    else if (heuristic == 2) dfs_order(n, adj, order_out, parent_out);
    else if (heuristic == 3) degree_sort_order(n, adj, order_out);
    else { free(adj); return -1; }
    if (heuristic != 2 && parent_out)
        for (int v = 0; v < n; ++v) parent_out[v] = -1;
    free(adj);
    return 0;
}

/* Induced width along an order (Sec. 2, Def. 1): process variables from the
 * last position to the first; the width of a variable is the number of its
 * earlier neighbours in the induced graph, and those neighbours are then
 * connected pairwise. */
int or_induced_width(int n, int m, const int *arity, const int *scope_flat, const int *order)
{
    unsigned char *adj = primal_graph(n, m, arity, scope_flat);
    int *pos = (int *)malloc(sizeof(int) * (size_t)n);
    for (int p = 0; p < n; ++p) pos[order[p]] = p;
    int w = 0;
    for (int p = n - 1; p >= 0; --p) {
        int v = order[p], width = 0;
        for (int u = 0; u < n; ++u)
            if (adj[(size_t)v * n + u] && pos[u] < p) ++width;
        if (width > w) w = width;
        for (int a = 0; a < n; ++a) {
            if (!adj[(size_t)v * n + a] || pos[a] >= p) continue;
            for (int b = 0; b < n; ++b)
                if (b != a && adj[(size_t)v * n + b] && pos[b] < p) adj[(size_t)a * n + b] = 1;
        }
    }
    free(adj); free(pos);
    return w;
}

/* Separator of every agent (Sec. 4): the ancestors of a_i that are linked in
 * the primal graph with a_i or with one of its descendants.  sep_out is an
 * n x n 0/1 matrix, row i = sep(a_i). */
int or_separators(int n, int m, const int *arity, const int *scope_flat,
                  const int *parent, unsigned char *sep_out)
{
    unsigned char *adj = primal_graph(n, m, arity, scope_flat);
    memset(sep_out, 0, (size_t)n * n);
    for (int i = 0; i < n; ++i) {
        /* ancestors of i */
        unsigned char *anc = (unsigned char *)calloc((size_t)n, 1);
        for (int a = parent[i]; a >= 0; a = parent[a]) anc[a] = 1;
        /* i and its descendants: every d with i on its ancestor chain */
        for (int d = 0; d < n; ++d) {
            int inside = 0;
            for (int a = d; a >= 0; a = parent[a])
                if (a == i) { inside = 1; break; }
            if (!inside) continue;
            for (int u = 0; u < n; ++u)
                if (anc[u] && adj[(size_t)d * n + u]) sep_out[(size_t)i * n + u] = 1;
        }
        free(anc);
    }
    free(adj);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* helpers on functions                                                      */
/* ------------------------------------------------------------------------ */
static int64_t table_size(int a, const int *scope, const int *dom)
{
    int64_t s = 1;
    for (int j = 0; j < a; ++j) s *= dom[scope[j]];
    return s;
}

static void sort_scope_by_pos(int a, int *scope, const int *pos)
{
    for (int i = 1; i < a; ++i) {
        int x = scope[i], j = i - 1;
        while (j >= 0 && pos[scope[j]] > pos[x]) { scope[j + 1] = scope[j]; --j; }
        scope[j + 1] = x;
    }
}

/* union of the scopes of a list of functions, sorted by order position */
static int union_scope(int nf, ofn *const *fs, const int *pos, int n, int *out)
{
    unsigned char *in = (unsigned char *)calloc((size_t)n, 1);
    int a = 0;
    for (int i = 0; i < nf; ++i)
        for (int j = 0; j < fs[i]->arity; ++j)
            if (!in[fs[i]->scope[j]]) { in[fs[i]->scope[j]] = 1; out[a++] = fs[i]->scope[j]; }
    free(in);
    sort_scope_by_pos(a, out, pos);
    return a;
}

static int union_size2(const int *sa, int a, const ofn *f, int n)
{
    unsigned char *in = (unsigned char *)calloc((size_t)n, 1);
    int c = 0;
    for (int j = 0; j < a; ++j) if (!in[sa[j]]) { in[sa[j]] = 1; ++c; }
    for (int j = 0; j < f->arity; ++j) if (!in[f->scope[j]]) { in[f->scope[j]] = 1; ++c; }
    free(in);
    return c;
}

/* ------------------------------------------------------------------------ */
/* the solver                                                                */
/* ------------------------------------------------------------------------ */
void or_result_free(or_result *r);

/*
 * n, dom           : variables and domain sizes
 * m, arity, scope_flat : the input functions; scopes concatenated, listed in
 *                    any order; table rows follow the scope AS GIVEN (R10)
 * ti_flat / td_flat: concatenated tables (int32 costs, or doubles)
 * kind             : 0 int32 costs, 1 double costs, 2 double probabilities
 *                    (cost = -ln p, Sec. 3: MPE as min-sum)
 * order            : order[p] = variable at position p; elimination runs from
 *                    p = n-1 down to 0
 * ibound           : mini-bucket bound (<= 0 means unbounded, i.e. BE)
 */
static int solve_impl(int n, const int *dom, int m, const int *arity, const int *scope_flat,
                      const int32_t *ti_flat, const double *td_flat, int kind, const int *order,
                      int ibound, const int *ov, int n_ov, int sum, or_result **out);

int or_solve_parts(int n, const int *dom, int m, const int *arity, const int *scope_flat,
                   const int32_t *ti_flat, const double *td_flat, int kind,
                   const int *order, int ibound, const int *ov, int n_ov, or_result **out)
{
    return solve_impl(n, dom, m, arity, scope_flat, ti_flat, td_flat, kind, order, ibound, ov, n_ov, 0, out);
}

/* The sum-product variant (double costs only, kind 1 or 2): see the header
 * comment and R18.  Returns -3 for integer costs. */
int or_solve_sum(int n, const int *dom, int m, const int *arity, const int *scope_flat,
                 const double *td_flat, int kind, const int *order, int ibound, or_result **out)
{
    if (kind == 0) return -3;
    return solve_impl(n, dom, m, arity, scope_flat, NULL, td_flat, kind, order, ibound, NULL, 0, 1, out);
}

int or_solve(int n, const int *dom, int m, const int *arity, const int *scope_flat,
             const int32_t *ti_flat, const double *td_flat, int kind,
             const int *order, int ibound, or_result **out)
{
    return or_solve_parts(n, dom, m, arity, scope_flat, ti_flat, td_flat, kind, order, ibound,
                          NULL, 0, out);
}

/*
 * Same as or_solve, except that the partition of some buckets is given:
 * ov holds n_ov triples (variable, part index, function id); the parts of
 * bucket v are the listed functions grouped by part index, in the listed
 * order.  The partition step of Alg. 2 admits any partition whose parts hold at most
 * `ibound` variables; as in R3, a single function with more than `ibound`
 * variables forms a part of its own.  A given partition with a part of
 * several functions over the bound (ibound > 0), or that does not cover the
 * bucket exactly, makes the call return -2.
 */
static int solve_impl(int n, const int *dom, int m, const int *arity, const int *scope_flat,
                      const int32_t *ti_flat, const double *td_flat, int kind, const int *order,
                      int ibound, const int *ov, int n_ov, int sum, or_result **out)
{
    int is_double = kind != 0;
    or_result *res = (or_result *)calloc(1, sizeof(or_result));
    res->n = n;
    res->is_double = is_double;
    res->assign = (int *)calloc((size_t)(n > 0 ? n : 1), sizeof(int));

    int *pos = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int p = 0; p < n; ++p) pos[order[p]] = p;

    int cap_f = m + 16, n_f = 0;
    ofn **fn = (ofn **)malloc(sizeof(ofn *) * (size_t)cap_f);
    ilist *bucket = (ilist *)calloc((size_t)(n > 0 ? n : 1), sizeof(ilist));

    int32_t ci = 0;       /* the constant (functions with empty scope) */
    double cd = 0.0;

    /* normalisation (Sec. 6.1 / R12): scope sorted by position, table permuted */
    int soff = 0;
    int64_t toff = 0;
    for (int f = 0; f < m; ++f) {
        int a = arity[f];
        const int *sc = scope_flat + soff;
        int64_t size = table_size(a, sc, dom);
        ofn *g = (ofn *)calloc(1, sizeof(ofn));
        g->id = f;
        g->arity = a;
        g->scope = (int *)malloc(sizeof(int) * (size_t)(a > 0 ? a : 1));
        memcpy(g->scope, sc, sizeof(int) * (size_t)a);
        sort_scope_by_pos(a, g->scope, pos);
        g->size = size;
        if (is_double) g->td = (double *)malloc(sizeof(double) * (size_t)size);
        else g->ti = (int32_t *)malloc(sizeof(int32_t) * (size_t)size);
        /* walk the rows of the original layout; write each to its new row */
        ofn orig;
        orig.arity = a;
        orig.scope = (int *)sc;
        int *val = (int *)calloc((size_t)(n > 0 ? n : 1), sizeof(int));
        int64_t r = 0;
        do {
            int64_t src = row_of(&orig, dom, val);
            int64_t dst = row_of(g, dom, val);
            if (kind == 0) g->ti[dst] = ti_flat[toff + src];
            else if (kind == 1) g->td[dst] = td_flat[toff + src];
            else g->td[dst] = -log(td_flat[toff + src]);
            ++r;
        } while (odometer_next(a, sc, dom, val));
        free(val);
        soff += a;
        toff += size;
        fn[n_f++] = g;
        if (a == 0) {
            if (is_double) cd += g->td[0]; else ci = sat_add(ci, g->ti[0]);
        } else {
            il_push(&bucket[g->scope[a - 1]], g->id);   /* R1 */
        }
    }

    int *U = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *val = (int *)calloc((size_t)(n > 0 ? n : 1), sizeof(int));
    int next_id = m;

    /* variable elimination phase: positions n-1 down to 0 (Alg. 1/2, first loop) */
    for (int p = n - 1; p >= 0; --p) {
        int v = order[p];
        ilist *B = &bucket[v];
        if (B->n == 0) {                                    /* R15 */
            /* sum-product: a variable no function mentions multiplies Z by
             * |D_v| (each of its values has weight 1) */
            if (sum) cd += -log((double)dom[v]);
            continue;
        }
        res->n_buckets_used++;

        /* the bucket's functions */
        ofn **bf = (ofn **)malloc(sizeof(ofn *) * (size_t)B->n);
        for (int i = 0; i < B->n; ++i) bf[i] = fn[B->v[i]];

        /* partition into mini-buckets (the partition step of Alg. 2; R2, R3) */
        int n_mb = 0;
        int *mb_of = (int *)malloc(sizeof(int) * (size_t)B->n);   /* mini-bucket of bf[i] */
        int **mb_scope = (int **)malloc(sizeof(int *) * (size_t)B->n);
        int *mb_a = (int *)malloc(sizeof(int) * (size_t)B->n);
        int *sorted = (int *)malloc(sizeof(int) * (size_t)B->n);
        int whole = union_scope(B->n, bf, pos, n, U);
        int given = 0;
        for (int t = 0; t < n_ov; ++t) if (ov[3 * t] == v) { given = 1; break; }
        if (given) {
            /* the caller's partition: parts in order of first mention */
            int *part_id = (int *)malloc(sizeof(int) * (size_t)B->n);
            for (int i = 0; i < B->n; ++i) part_id[i] = -1;
            int *seen_part = (int *)malloc(sizeof(int) * (size_t)(n_ov + 1));
            int n_seen = 0, bad = 0, t_sorted = 0;
            for (int t = 0; t < n_ov; ++t) {
                if (ov[3 * t] != v) continue;
                int pk = ov[3 * t + 1], fid = ov[3 * t + 2], k = -1;
                for (int q = 0; q < n_seen; ++q) if (seen_part[q] == pk) { k = q; break; }
                if (k < 0) { seen_part[n_seen] = pk; k = n_seen++; }
                int i;
                for (i = 0; i < B->n; ++i) if (bf[i]->id == fid) break;
                if (i == B->n || part_id[i] >= 0) { bad = 1; break; }
                part_id[i] = k;
                sorted[t_sorted++] = i;
            }
            for (int i = 0; i < B->n; ++i) if (part_id[i] < 0) bad = 1;
            n_mb = n_seen;
            for (int i = 0; i < B->n && !bad; ++i) mb_of[i] = part_id[i];
            for (int k = 0; k < n_mb && !bad; ++k) {
                ofn **mf = (ofn **)malloc(sizeof(ofn *) * (size_t)B->n);
                int nm = 0;
                for (int i = 0; i < B->n; ++i) if (part_id[i] == k) mf[nm++] = bf[i];
                /* a part of several functions must fit the bound; a single
                 * function wider than the bound stands alone (R3) */
                if (ibound > 0 && nm > 1 && union_scope(nm, mf, pos, n, U) > ibound) bad = 1;
                free(mf);
            }
            for (int k = 0; k < n_mb; ++k) mb_scope[k] = NULL;
            free(part_id);
            free(seen_part);
            if (bad) {
                free(mb_of); free(mb_scope); free(mb_a); free(sorted); free(bf);
                or_result_free(res);
                return -2;
            }
        } else if (ibound <= 0 || whole <= ibound) {
            for (int i = 0; i < B->n; ++i) { mb_of[i] = 0; sorted[i] = i; }
            n_mb = 1;
            mb_scope[0] = NULL;
        } else {
            for (int i = 0; i < B->n; ++i) sorted[i] = i;
            for (int i = 1; i < B->n; ++i) {   /* sort by (-arity, id) */
                int x = sorted[i], j = i - 1;
                while (j >= 0 && (bf[sorted[j]]->arity < bf[x]->arity ||
                                  (bf[sorted[j]]->arity == bf[x]->arity &&
                                   bf[sorted[j]]->id > bf[x]->id))) {
                    sorted[j + 1] = sorted[j]; --j;
                }
                sorted[j + 1] = x;
            }
            for (int t = 0; t < B->n; ++t) {
                int i = sorted[t];
                int k;
                for (k = 0; k < n_mb; ++k)
                    if (union_size2(mb_scope[k], mb_a[k], bf[i], n) <= ibound) break;
                if (k == n_mb) {
                    mb_scope[k] = (int *)malloc(sizeof(int) * (size_t)n);
                    mb_a[k] = 0;
                    ++n_mb;
                }
                /* add f's variables to the mini-bucket scope */
                for (int j = 0; j < bf[i]->arity; ++j) {
                    int u = bf[i]->scope[j], have = 0;
                    for (int q = 0; q < mb_a[k]; ++q) if (mb_scope[k][q] == u) { have = 1; break; }
                    if (!have) mb_scope[k][mb_a[k]++] = u;
                }
                mb_of[i] = k;
            }
        }

        /* aggregate and eliminate every mini-bucket, in creation order */
        for (int k = 0; k < n_mb; ++k) {
            ofn **mf = (ofn **)malloc(sizeof(ofn *) * (size_t)B->n);
            int nm = 0;
            for (int t = 0; t < B->n; ++t)
                if (mb_of[sorted[t]] == k) mf[nm++] = bf[sorted[t]];
            int a = union_scope(nm, mf, pos, n, U);     /* v is U[a-1] */
            if (a > res->max_union) res->max_union = a;
            int64_t jsize = table_size(a, U, dom);

            /* Aggregation (Sec. 2; Sec. 6.3): a zero table over U, then every
             * function of the mini-bucket is added into it, one at a time */
            int32_t *ji = NULL;
            double *jd = NULL;
            if (is_double) jd = (double *)calloc((size_t)jsize, sizeof(double));
            else ji = (int32_t *)calloc((size_t)jsize, sizeof(int32_t));
            for (int i = 0; i < nm; ++i) {
                for (int j = 0; j < a; ++j) val[U[j]] = 0;
                int64_t r = 0;
                do {
                    int64_t src = row_of(mf[i], dom, val);
                    if (is_double) jd[r] += mf[i]->td[src];
                    else ji[r] = sat_add(ji[r], mf[i]->ti[src]);
                    ++r;
                } while (odometer_next(a, U, dom, val));
            }

            /* Elimination (Sec. 2; Sec. 6.4): v is the last scope variable, so
             * the rows for its values are consecutive; keep the minimum */
            int dv = dom[v];
            int64_t osize = jsize / dv;
            ominib rec;
            memset(&rec, 0, sizeof rec);
            rec.var = v;
            rec.k = k;
            rec.n_members = nm;
            rec.members = (int *)malloc(sizeof(int) * (size_t)(nm > 0 ? nm : 1));
            for (int i = 0; i < nm; ++i) rec.members[i] = mf[i]->id;
            rec.out_arity = a - 1;
            rec.out_scope = (int *)malloc(sizeof(int) * (size_t)(a > 1 ? a - 1 : 1));
            memcpy(rec.out_scope, U, sizeof(int) * (size_t)(a - 1));
            rec.out_size = osize;
            if (is_double) {
                rec.out_td = (double *)malloc(sizeof(double) * (size_t)osize);
                for (int64_t s = 0; s < osize; ++s) {
                    double best = jd[s * dv];
                    for (int x = 1; x < dv; ++x)
                        if (jd[s * dv + x] < best) best = jd[s * dv + x];
                    if (sum && k == 0 && !isinf(best)) {
                        /* sum-product: -ln sum_x exp(-a_x), written as
                         * best - ln sum_x exp(-(a_x - best)) so that the
                         * largest term is exp(0) = 1 (R18: first mini-bucket) */
                        double z = 0.0;
                        for (int x = 0; x < dv; ++x) z += exp(-(jd[s * dv + x] - best));
                        best = best - log(z);
                    }
                    rec.out_td[s] = best;
                }
            } else {
                rec.out_ti = (int32_t *)malloc(sizeof(int32_t) * (size_t)osize);
                for (int64_t s = 0; s < osize; ++s) {
                    int32_t best = ji[s * dv];
                    for (int x = 1; x < dv; ++x)
                        if (ji[s * dv + x] < best) best = ji[s * dv + x];
                    rec.out_ti[s] = best;
                }
            }
            free(ji);
            free(jd);

            /* placement of the new function (Alg. 1 / Alg. 2; R7) */
            if (a - 1 == 0) {
                rec.out_id = -1;
                if (is_double) cd += rec.out_td[0]; else ci = sat_add(ci, rec.out_ti[0]);
            } else {
                ofn *g = (ofn *)calloc(1, sizeof(ofn));
                g->id = next_id++;
                g->arity = a - 1;
                g->scope = (int *)malloc(sizeof(int) * (size_t)(a - 1));
                memcpy(g->scope, U, sizeof(int) * (size_t)(a - 1));
                g->size = osize;
                if (is_double) {
                    g->td = (double *)malloc(sizeof(double) * (size_t)osize);
                    memcpy(g->td, rec.out_td, sizeof(double) * (size_t)osize);
                } else {
                    g->ti = (int32_t *)malloc(sizeof(int32_t) * (size_t)osize);
                    memcpy(g->ti, rec.out_ti, sizeof(int32_t) * (size_t)osize);
                }
                if (n_f == cap_f) {
                    cap_f *= 2;
                    fn = (ofn **)realloc(fn, sizeof(ofn *) * (size_t)cap_f);
                }
                fn[n_f++] = g;                 /* fn[id] == function with that id */
                rec.out_id = g->id;
                il_push(&bucket[g->scope[g->arity - 1]], g->id);
            }
            if (res->n_mb == res->cap_mb) {
                res->cap_mb = res->cap_mb ? 2 * res->cap_mb : 16;
                res->mb = (ominib *)realloc(res->mb, sizeof(ominib) * (size_t)res->cap_mb);
            }
            res->mb[res->n_mb++] = rec;
            free(mf);
        }
        for (int k = 0; k < n_mb; ++k) if (mb_scope[k]) free(mb_scope[k]);
        free(mb_of); free(mb_scope); free(mb_a); free(sorted); free(bf);
    }

    res->lb = is_double ? cd : (double)ci;

    /* value assignment phase (Alg. 1/2, second loop; R4, R5) */
    for (int v = 0; v < n; ++v) val[v] = 0;
    for (int p = 0; p < n; ++p) {
        int v = order[p];
        ilist *B = &bucket[v];
        int best_x = 0;
        int32_t best_i = 0;
        double best_d = 0.0;
        for (int x = 0; x < dom[v]; ++x) {
            val[v] = x;
            int32_t si = 0;
            double sd = 0.0;
            for (int i = 0; i < B->n; ++i) {
                ofn *g = fn[B->v[i]];
                int64_t r = row_of(g, dom, val);
                if (is_double) sd += g->td[r]; else si = sat_add(si, g->ti[r]);
            }
            if (x == 0 || (is_double ? sd < best_d : si < best_i)) {
                best_x = x; best_i = si; best_d = sd;
            }
        }
        val[v] = best_x;
        res->assign[v] = best_x;
    }

    /* cost of the assignment over the input functions (upper bound, Sec. 2.2) */
    {
        int32_t ui = 0;
        double ud = 0.0;
        for (int f = 0; f < m; ++f) {
            int64_t r = row_of(fn[f], dom, val);
            if (is_double) ud += fn[f]->td[r]; else ui = sat_add(ui, fn[f]->ti[r]);
        }
        res->ub = is_double ? ud : (double)ui;
    }

    for (int f = 0; f < n_f; ++f) {
        free(fn[f]->scope); free(fn[f]->ti); free(fn[f]->td); free(fn[f]);
    }
    free(fn);
    for (int v = 0; v < n; ++v) free(bucket[v].v);
    free(bucket); free(U); free(val); free(pos);
    *out = res;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* result accessors                                                          */
/* ------------------------------------------------------------------------ */
double or_result_lb(const or_result *r) { return r->lb; }
double or_result_ub(const or_result *r) { return r->ub; }
int or_result_max_union(const or_result *r) { return r->max_union; }
void or_result_assignment(const or_result *r, int *out)
{
    memcpy(out, r->assign, sizeof(int) * (size_t)r->n);
}
int or_result_num_minibuckets(const or_result *r) { return r->n_mb; }

/* header of mini-bucket i: var, k, n_members, out_id, out_arity, out_size */
void or_result_mb_info(const or_result *r, int i, int *var, int *k, int *n_members,
                       int *out_id, int *out_arity, int64_t *out_size)
{
    const ominib *b = &r->mb[i];
    *var = b->var; *k = b->k; *n_members = b->n_members;
    *out_id = b->out_id; *out_arity = b->out_arity; *out_size = b->out_size;
}

void or_result_mb_data(const or_result *r, int i, int *members, int *out_scope,
                       int32_t *out_ti, double *out_td)
{
    const ominib *b = &r->mb[i];
    if (members) memcpy(members, b->members, sizeof(int) * (size_t)b->n_members);
    if (out_scope) memcpy(out_scope, b->out_scope, sizeof(int) * (size_t)b->out_arity);
    if (out_ti && b->out_ti) memcpy(out_ti, b->out_ti, sizeof(int32_t) * (size_t)b->out_size);
    if (out_td && b->out_td) memcpy(out_td, b->out_td, sizeof(double) * (size_t)b->out_size);
}

void or_result_free(or_result *r)
{
    if (!r) return;
    for (int i = 0; i < r->n_mb; ++i) {
        free(r->mb[i].members); free(r->mb[i].out_scope);
        free(r->mb[i].out_ti); free(r->mb[i].out_td);
    }
    free(r->mb);
    free(r->assign);
    free(r);
}
